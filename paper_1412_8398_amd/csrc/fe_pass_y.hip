// Launchers of the y transform pass (all supported lengths, float and double).
#include "fe_passes.h"

namespace fe {

template <typename T>
void Launch<T>::yfft(cpx<T>* S, int ncomp, Dims d, const cpx<T>* twy, int inverse, hipStream_t s) {
  dispatch_length(d.ny, [&](auto NC) {
    constexpr int N = decltype(NC)::value;
    using C = StridedCfg<T, N>;
    const int ntx = (d.nx + C::TX - 1) / C::TX;
    const dim3 grid(ntx * d.H * ncomp), block(C::NT);
    if (inverse)
      hipLaunchKernelGGL((k_ypass<T, N, true>), grid, block, 0, s, S, d, twy);
    else
      hipLaunchKernelGGL((k_ypass<T, N, false>), grid, block, 0, s, S, d, twy);
  });
}

template void Launch<float>::yfft(cpx<float>*, int, Dims, const cpx<float>*, int, hipStream_t);
template void Launch<double>::yfft(cpx<double>*, int, Dims, const cpx<double>*, int, hipStream_t);

}  // namespace fe
