// Launchers of the z real-to-complex / complex-to-real passes.
#include "fe_passes.h"

namespace fe {

template <typename T>
void Launch<T>::zr2c(const T* R, cpx<T>* S, int ncomp, Dims d, const cpx<T>* twz, hipStream_t s, Batch bt,
                     int nsamp) {
  dispatch_z_length(d.nz, [&](auto NC) {
    constexpr int N = decltype(NC)::value;
    using C = StridedCfg<T, N>;
    const int ntx = (d.nx / 2 + C::TX - 1) / C::TX;
    hipLaunchKernelGGL((k_zr2c<T, N>), dim3(ntx * d.ny * ncomp, nsamp), dim3(C::NT), 0, s, R, S, d, twz, bt);
  });
}

template <typename T>
void Launch<T>::zc2r(const cpx<T>* S, T* R, int ncomp, Dims d, const cpx<T>* twz, hipStream_t s, Batch bt,
                     int nsamp) {
  dispatch_z_length(d.nz, [&](auto NC) {
    constexpr int N = decltype(NC)::value;
    using C = StridedCfg<T, N>;
    const int ntx = (d.nx / 2 + C::TX - 1) / C::TX;
    hipLaunchKernelGGL((k_zc2r<T, N>), dim3(ntx * d.ny * ncomp, nsamp), dim3(C::NT), 0, s, S, R, d, twz, bt);
  });
}

template void Launch<float>::zr2c(const float*, cpx<float>*, int, Dims, const cpx<float>*, hipStream_t, Batch, int);
template void Launch<double>::zr2c(const double*, cpx<double>*, int, Dims, const cpx<double>*, hipStream_t, Batch,
                                   int);
template void Launch<float>::zc2r(const cpx<float>*, float*, int, Dims, const cpx<float>*, hipStream_t, Batch, int);
template void Launch<double>::zc2r(const cpx<double>*, double*, int, Dims, const cpx<double>*, hipStream_t, Batch,
                                   int);

}  // namespace fe
