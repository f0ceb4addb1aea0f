// Launchers of the six-component spectral equilibrium norm (eq. (43)): plain,
// with an anchor's divergence spectrum added, or storing that spectrum (the
// operators of the six-component form: MS, MS with eq. (15)'s Nyquist rule,
// centered; WP and ROT use the displacement form and never come here).
#include <type_traits>

#include "fe_passes.h"

namespace fe {

template <typename T, typename TS>
int launch_xeta6(const cpx<T>* S, Dims d, const cpx<T>* twx, WaveTables<T> wt, double* partials, int op, int mode,
                 cpx<TS>* base, hipStream_t s) {
  int nblk = 0;
  dispatch_length(d.nx, [&](auto NC) {
    constexpr int N = decltype(NC)::value;
    using C = LineCfg<T, N, 6>;
    nblk = x_blocks<T, N>(d, 6);
    const dim3 grid(nblk), block(C::NT);
    if constexpr (!std::is_same<T, TS>::value) {
      // float64 anchor spectrum stored for a float32 plan (MS, MSS, C)
      if (mode != XETA_STORE) return;
      if (op == OP_MS)
        hipLaunchKernelGGL((k_xeta6<T, N, OP_MS, XETA_STORE, TS>), grid, block, 0, s, S, d, twx, wt, partials, base);
      else if (op == OP_MSS)
        hipLaunchKernelGGL((k_xeta6<T, N, OP_MSS, XETA_STORE, TS>), grid, block, 0, s, S, d, twx, wt, partials, base);
      else
        hipLaunchKernelGGL((k_xeta6<T, N, OP_C, XETA_STORE, TS>), grid, block, 0, s, S, d, twx, wt, partials, base);
    } else {
      if (mode == XETA_PLAIN) {
        switch (op) {
          case OP_MS: hipLaunchKernelGGL((k_xeta6<T, N, OP_MS, XETA_PLAIN, TS>), grid, block, 0, s, S, d, twx, wt, partials, base); break;
          case OP_C: hipLaunchKernelGGL((k_xeta6<T, N, OP_C, XETA_PLAIN, TS>), grid, block, 0, s, S, d, twx, wt, partials, base); break;
          case OP_MSS: hipLaunchKernelGGL((k_xeta6<T, N, OP_MSS, XETA_PLAIN, TS>), grid, block, 0, s, S, d, twx, wt, partials, base); break;
          default: break;  // WP and ROT never take the six-component path
        }
      } else if constexpr (sizeof(T) == 4) {  // a float32 correction on a float64 anchor (MS, MSS, C)
        if (mode != XETA_BASE) return;
        if (op == OP_MS)
          hipLaunchKernelGGL((k_xeta6<T, N, OP_MS, XETA_BASE, TS>), grid, block, 0, s, S, d, twx, wt, partials, base);
        else if (op == OP_MSS)
          hipLaunchKernelGGL((k_xeta6<T, N, OP_MSS, XETA_BASE, TS>), grid, block, 0, s, S, d, twx, wt, partials, base);
        else
          hipLaunchKernelGGL((k_xeta6<T, N, OP_C, XETA_BASE, TS>), grid, block, 0, s, S, d, twx, wt, partials, base);
      }
    }
  });
  return nblk;
}

template <typename T>
int Launch<T>::xeta6(const cpx<T>* S, Dims d, const cpx<T>* twx, WaveTables<T> wt, double* partials, int op,
                     hipStream_t s) {
  return launch_xeta6<T, T>(S, d, twx, wt, partials, op, XETA_PLAIN, nullptr, s);
}

template int Launch<float>::xeta6(const cpx<float>*, Dims, const cpx<float>*, WaveTables<float>, double*, int,
                                  hipStream_t);
template int Launch<double>::xeta6(const cpx<double>*, Dims, const cpx<double>*, WaveTables<double>, double*, int,
                                   hipStream_t);

// float: plain and with the anchor's divergence spectrum; double: plain;
// (double, float): the anchor's spectrum written from float64 arithmetic
template int launch_xeta6<float, float>(const cpx<float>*, Dims, const cpx<float>*, WaveTables<float>, double*, int,
                                        int, cpx<float>*, hipStream_t);
template int launch_xeta6<double, float>(const cpx<double>*, Dims, const cpx<double>*, WaveTables<double>, double*,
                                         int, int, cpx<float>*, hipStream_t);

}  // namespace fe
