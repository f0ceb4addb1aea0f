// Launcher of the six-component x pass: transform along x, Green operator,
// inverse transform (the operators of the six-component form: MS, MS with
// eq. (15)'s Nyquist rule, centered; WP and ROT use the displacement form).
#include "fe_passes.h"

namespace fe {

template <typename T>
void Launch<T>::xgreen6(cpx<T>* S, Dims d, const cpx<T>* twx, WaveTables<T> wt, GreenConst<T> g, int op,
                        hipStream_t s) {
  dispatch_length(d.nx, [&](auto NC) {
    constexpr int N = decltype(NC)::value;
    using C = LineCfg<T, N, 6>;
    const dim3 grid(x_blocks<T, N>(d, 6)), block(C::NT);
    switch (op) {
      case OP_MS: hipLaunchKernelGGL((k_xgreen6<T, N, OP_MS>), grid, block, 0, s, S, d, twx, wt, g); break;
      case OP_C: hipLaunchKernelGGL((k_xgreen6<T, N, OP_C>), grid, block, 0, s, S, d, twx, wt, g); break;
      case OP_MSS: hipLaunchKernelGGL((k_xgreen6<T, N, OP_MSS>), grid, block, 0, s, S, d, twx, wt, g); break;
      default: break;  // WP and ROT never take the six-component path
    }
  });
}

template void Launch<float>::xgreen6(cpx<float>*, Dims, const cpx<float>*, WaveTables<float>, GreenConst<float>, int,
                                     hipStream_t);
template void Launch<double>::xgreen6(cpx<double>*, Dims, const cpx<double>*, WaveTables<double>,
                                      GreenConst<double>, int, hipStream_t);
}  // namespace fe
