// Launchers of the six-component x passes: Green operator (every operator) and
// the spectral equilibrium norm.
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
      case OP_WP: hipLaunchKernelGGL((k_xgreen6<T, N, OP_WP>), grid, block, 0, s, S, d, twx, wt, g); break;
      case OP_C: hipLaunchKernelGGL((k_xgreen6<T, N, OP_C>), grid, block, 0, s, S, d, twx, wt, g); break;
      default: hipLaunchKernelGGL((k_xgreen6<T, N, OP_ROT>), grid, block, 0, s, S, d, twx, wt, g); break;
    }
  });
}

template <typename T>
int Launch<T>::xeta6(const cpx<T>* S, Dims d, const cpx<T>* twx, WaveTables<T> wt, double* partials, int op,
                     hipStream_t s) {
  int nblk = 0;
  dispatch_length(d.nx, [&](auto NC) {
    constexpr int N = decltype(NC)::value;
    using C = LineCfg<T, N, 6>;
    nblk = x_blocks<T, N>(d, 6);
    const dim3 grid(nblk), block(C::NT);
    switch (op) {
      case OP_MS: hipLaunchKernelGGL((k_xeta6<T, N, OP_MS>), grid, block, 0, s, S, d, twx, wt, partials); break;
      case OP_WP: hipLaunchKernelGGL((k_xeta6<T, N, OP_WP>), grid, block, 0, s, S, d, twx, wt, partials); break;
      case OP_C: hipLaunchKernelGGL((k_xeta6<T, N, OP_C>), grid, block, 0, s, S, d, twx, wt, partials); break;
      default: hipLaunchKernelGGL((k_xeta6<T, N, OP_ROT>), grid, block, 0, s, S, d, twx, wt, partials); break;
    }
  });
  return nblk;
}

template void Launch<float>::xgreen6(cpx<float>*, Dims, const cpx<float>*, WaveTables<float>, GreenConst<float>, int,
                                     hipStream_t);
template void Launch<double>::xgreen6(cpx<double>*, Dims, const cpx<double>*, WaveTables<double>,
                                      GreenConst<double>, int, hipStream_t);
template int Launch<float>::xeta6(const cpx<float>*, Dims, const cpx<float>*, WaveTables<float>, double*, int,
                                  hipStream_t);
template int Launch<double>::xeta6(const cpx<double>*, Dims, const cpx<double>*, WaveTables<double>, double*, int,
                                   hipStream_t);

}  // namespace fe
