// Launchers of the x pass with the displacement-form Green operator (WP, ROT).
#include "fe_passes.h"

namespace fe {

template <typename T>
void Launch<T>::xgreen3(cpx<T>* S, Dims d, const cpx<T>* twx, WaveTables<T> wt, GreenConst<T> g, int op,
                        hipStream_t s, Batch bt, const GreenConst<T>* gs, int nsamp) {
  dispatch_length(d.nx, [&](auto NC) {
    constexpr int N = decltype(NC)::value;
    using C = LineCfg<T, N, 3>;
    const dim3 grid(x_blocks<T, N>(d, 3), nsamp), block(C::NT);
    if (op == OP_ROT)
      hipLaunchKernelGGL((k_xgreen3<T, N, OP_ROT>), grid, block, 0, s, S, d, twx, wt, g, bt, gs);
    else
      hipLaunchKernelGGL((k_xgreen3<T, N, OP_WP>), grid, block, 0, s, S, d, twx, wt, g, bt, gs);
  });
}

template void Launch<float>::xgreen3(cpx<float>*, Dims, const cpx<float>*, WaveTables<float>, GreenConst<float>, int,
                                     hipStream_t, Batch, const GreenConst<float>*, int);
template void Launch<double>::xgreen3(cpx<double>*, Dims, const cpx<double>*, WaveTables<double>,
                                      GreenConst<double>, int, hipStream_t, Batch, const GreenConst<double>*, int);

}  // namespace fe
