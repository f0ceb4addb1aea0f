// Launchers of the y transform pass (all supported lengths, float and double).
#include "fe_passes.h"

namespace fe {

template <typename T>
void Launch<T>::yfft(cpx<T>* S, int ncomp, Dims d, const cpx<T>* twy, int inverse, hipStream_t s, Batch bt,
                     int nsamp) {
  dispatch_length(d.ny, [&](auto NC) {
    constexpr int N = decltype(NC)::value;
    using C = StridedCfg<T, N, true>;
    const int ntx = (d.nx + C::TX - 1) / C::TX;
    const dim3 grid(ntx * d.H * ncomp, nsamp), block(C::NT);
    if (inverse)
      hipLaunchKernelGGL((k_ypass<T, N, true>), grid, block, 0, s, S, d, twy, bt);
    else
      hipLaunchKernelGGL((k_ypass<T, N, false>), grid, block, 0, s, S, d, twy, bt);
  });
}

template void Launch<float>::yfft(cpx<float>*, int, Dims, const cpx<float>*, int, hipStream_t, Batch, int);
template void Launch<double>::yfft(cpx<double>*, int, Dims, const cpx<double>*, int, hipStream_t, Batch, int);

}  // namespace fe
