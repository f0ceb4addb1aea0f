// Persistent batched solve: one cooperative launch runs every pass of every
// iteration of many independent samples (the displacement form, float32
// fields, float64 reductions), with the per-sample convergence decisions and
// the retirement of converged samples on the device.
//
// The grid is sized to be fully resident.  Each pass (divergence, z forward,
// y forward, x with the Green operator, y inverse, z inverse, update) is a
// set of virtual workgroups, the pass's tiles over all active samples; the
// resident workgroups stride through them, then the grid synchronises.  The
// workgroup bodies are those of the per-pass kernels (fe_passes.h,
// fe_stencil.h) with the same tiles and the same partial-sum slots, and eta is
// reduced by the same fixed-order body, so every sample follows exactly the
// iteration of a single-sample fe_solve with refinement off.  After the update
// one workgroup per active sample reduces its partial sums, evaluates eta of
// eq. (43) and applies the stop rules; one workgroup then compacts the active
// lists.  Every workgroup reads the active count after the same grid barrier,
// so all leave the loop together; a sample retires at its iteration cap at
// the latest, and the loop is bounded by that cap.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

#include "../../include/fe.h"
#include "fe_batch.h"
#include "fe_passes.h"
#include "fe_stencil.h"

namespace fe {

namespace {

constexpr int kBatchThreads = 256;
constexpr int kBatchDX = 32, kBatchDY = 8;  // update tile (SmallTile<float>)
constexpr int kStallWindow = 100;           // no 5% gain in eta over this many iterations: float32 floor

enum { BP_DIV = 0, BP_ZR2C, BP_YFWD, BP_XGREEN, BP_YINV, BP_ZC2R, BP_UPDATE };

// LDS of the largest body over the compiled lengths: strided tiles hold
// N TX complex values (at most 32 KiB), the x pass LPB LINE (its components
// take turns through the buffer; at most 26 KiB).
template <int N>
constexpr size_t batch_lds_of() {
  using Z = StridedCfg<float, N>;
  using Y = StridedCfg<float, N, true>;
  constexpr size_t z = (size_t)Z::ROWS * Z::TX, y = (size_t)Y::ROWS * Y::TX;
  constexpr size_t x = (size_t)LineCfg<float, N, 3>::LPB * LineCfg<float, N, 3>::LINE;
  return sizeof(cpx<float>) * (z > y ? (z > x ? z : x) : (y > x ? y : x));
}
constexpr size_t cmax(size_t a, size_t b) { return a > b ? a : b; }
constexpr size_t kBatchLds =
    cmax(cmax(cmax(batch_lds_of<16>(), batch_lds_of<24>()), cmax(batch_lds_of<32>(), batch_lds_of<48>())),
         cmax(cmax(batch_lds_of<64>(), batch_lds_of<96>()), cmax(batch_lds_of<128>(),
                                                                  sizeof(UpdLds<float, kBatchDX, kBatchDY>))));
static_assert(sizeof(DivLds<float, kBatchDX, kBatchDY>) <= kBatchLds, "divergence tile LDS");
// four resident workgroups per CU (16 waves): the launch bounds cap the
// registers at 128 per lane, and the LDS of four must fit the CU's 160 KiB
constexpr int kBatchWavesPerSimd = 3;
static_assert(kBatchWavesPerSimd * (kBatchLds + 8 * 16 * sizeof(double)) <= 160 * 1024, "four workgroups per CU");

template <class F>
__device__ __forceinline__ void with_batch_length(int n, F&& f) {
  switch (n) {
    case 16: f(std::integral_constant<int, 16>()); break;
    case 24: f(std::integral_constant<int, 24>()); break;
    case 32: f(std::integral_constant<int, 32>()); break;
    case 48: f(std::integral_constant<int, 48>()); break;
    case 64: f(std::integral_constant<int, 64>()); break;
    case 96: f(std::integral_constant<int, 96>()); break;
    case 128: f(std::integral_constant<int, 128>()); break;
    default: break;  // the host admits these lengths only
  }
}

__device__ __forceinline__ int blocks_of(const BatchClassDev& c, int pass) {
  switch (pass) {
    case BP_DIV:
    case BP_UPDATE: return c.bu;
    case BP_ZR2C:
    case BP_ZC2R: return c.bz;
    case BP_XGREEN: return c.bx;
    default: return c.by;
  }
}

// Pointers into device memory pass to the pass functions as global-space
// pointers (gptr), converted back to generic inside: the compiler then emits
// global_* instead of flat_* loads and stores for them (a generic pointer
// parameter, or one read from the batch descriptor, gives flat accesses,
// and a flat access also counts against the LDS wait counter, so every LDS
// wait of an FFT exchange would wait for the loads in flight as well).
template <typename P>
using gptr = __attribute__((address_space(1))) P*;
template <typename P>
__device__ __forceinline__ gptr<P> to_g(P* p) {
  return (gptr<P>)p;
}
template <typename P>
__device__ __forceinline__ P* un_g(gptr<P> p) {
  return (P*)p;
}

// The bodies of each pass and length in functions of their own, so that the
// register allocation of one does not load the others (inlined into one
// kernel they would share, and spill, the largest set).  Small structures
// by value: a reference would put them in the caller's scratch memory.
template <int N>
__device__ __noinline__ void pass_zr2c(gptr<const float> R, gptr<cpx<float>> S, Dims d, gptr<const cpx<float>> tw,
                                       cpx<float>* lds, int b) {
  zr2c_body<float, N>(un_g(R), un_g(S), d, un_g(tw), lds, b);
}
template <int N>
__device__ __noinline__ void pass_zc2r(gptr<const cpx<float>> S, gptr<float> R, Dims d, gptr<const cpx<float>> tw,
                                       cpx<float>* lds, int b) {
  zc2r_body<float, N>(un_g(S), un_g(R), d, un_g(tw), lds, b);
}
template <int N, bool INV>
__device__ __noinline__ void pass_y(gptr<cpx<float>> S, Dims d, gptr<const cpx<float>> tw, cpx<float>* lds, int b) {
  ypass_body<float, N, INV>(un_g(S), d, un_g(tw), lds, b);
}
// (the x pass keeps generic pointers: it has no loads in flight during its
// LDS exchanges, and global ones let the scheduler raise its registers
// beyond the kernel's budget)
template <int N, int OP>
__device__ __noinline__ void pass_x(cpx<float>* S, Dims d, const cpx<float>* tw, WaveTables<float> wt,
                                    const GreenConst<float>* gp, cpx<float>* lds, int b) {
  xgreen3_body<float, N, OP, true>(S, d, tw, wt, *gp, lds, b);
}
template <int OP>
__device__ __noinline__ void pass_div(unsigned char* smem, gptr<const float> eps, gptr<const uint8_t> phase,
                                      gptr<const PhaseCoef<float>> coef, gptr<float> D, gptr<double> out7, Dims d,
                                      int zchunk, int tile) {
  auto& L = *reinterpret_cast<DivLds<float, kBatchDX, kBatchDY>*>(smem);
  div_body<kBatchDX, kBatchDY, float, float, float, OP>(L, un_g(eps), un_g(phase), un_g(coef), un_g(D),
                                                        (float*)nullptr, (const float*)nullptr, un_g(out7), d,
                                                        zchunk, tile);
}
template <int OP, bool AS>
__device__ __noinline__ void pass_update(unsigned char* smem, gptr<const float> U, gptr<const float> eps_in,
                                         gptr<float> eps_out, gptr<const uint8_t> phase,
                                         gptr<const PhaseCoef<float>> coef, int ncoef,
                                         gptr<const GreenConst<float>> gp, gptr<float> D, gptr<double> out7, Dims d,
                                         int zchunk, int tile) {
  auto& L = *reinterpret_cast<UpdLds<float, kBatchDX, kBatchDY>*>(smem);
  const GreenConst<float> g = *un_g(gp);
  update_div_body<kBatchDX, kBatchDY, float, OP, AS, false, true>(
      L, un_g(U), un_g(eps_in), un_g(eps_out), un_g(phase), un_g(coef), ncoef, g, (const float*)nullptr, un_g(D),
      (const float*)nullptr, un_g(out7), d, zchunk, tile);
}

// every virtual workgroup of one pass over the active samples
template <int OP, bool AS>
__device__ void run_pass(BatchDev* bd, int pass, unsigned char* smem) {
  long long total = 0;
  for (int c = 0; c < bd->ncls; ++c) total += (long long)bd->cls[c].nact * blocks_of(bd->cls[c], pass);
  cpx<float>* lds = reinterpret_cast<cpx<float>*>(smem);
  for (long long v = blockIdx.x; v < total; v += gridDim.x) {
    int c = 0;
    long long off = v;
    for (;;) {
      const long long nb = (long long)bd->cls[c].nact * blocks_of(bd->cls[c], pass);
      if (off < nb) break;
      off -= nb;
      ++c;
    }
    const BatchClassDev& C = bd->cls[c];
    const int per = blocks_of(C, pass);
    const int slot = (int)(off / per), b = (int)(off % per);
    const long long smp = C.act[slot];
    const int par = bd->st[C.first + smp].parity;
    const Dims d = C.d;
    const long long N = d.N, spec = spec_size(d);
    float* R = C.R[par] + smp * 3 * N;
    cpx<float>* S = C.S + smp * 3 * spec;
    switch (pass) {
      case BP_DIV:
        pass_div<OP>(smem, to_g<const float>(C.eps[par] + smp * 6 * N), to_g(C.phase + smp * N),
                     to_g(C.coef + smp * C.ncoef), to_g(R), to_g(C.partials + (smp * per + b) * 7), d, C.zchunk,
                     xcd_block(b, per));
        break;
      case BP_ZR2C:
        with_batch_length(d.nz, [&](auto NC) { pass_zr2c<decltype(NC)::value>(to_g<const float>(R), to_g(S), d, to_g(C.tw[2]), lds, b); });
        break;
      case BP_YFWD:
        with_batch_length(d.ny, [&](auto NC) { pass_y<decltype(NC)::value, false>(to_g(S), d, to_g(C.tw[1]), lds, b); });
        break;
      case BP_XGREEN:
        with_batch_length(d.nx, [&](auto NC) {
          pass_x<decltype(NC)::value, OP>(S, d, C.tw[0], C.wt, C.gcon + smp, lds, b);
        });
        break;
      case BP_YINV:
        with_batch_length(d.ny, [&](auto NC) { pass_y<decltype(NC)::value, true>(to_g(S), d, to_g(C.tw[1]), lds, b); });
        break;
      case BP_ZC2R:
        with_batch_length(d.nz, [&](auto NC) { pass_zc2r<decltype(NC)::value>(to_g<const cpx<float>>(S), to_g(R), d, to_g(C.tw[2]), lds, b); });
        break;
      default:  // BP_UPDATE: eps^(k+1) and the divergence of its tau into the other parity
        pass_update<OP, AS>(smem, to_g<const float>(R), to_g<const float>(C.eps[par] + smp * 6 * N),
                            to_g(C.eps[par ^ 1] + smp * 6 * N), to_g(C.phase + smp * N), to_g(C.coef + smp * C.ncoef),
                            C.ncoef < 256 ? C.ncoef : 256, to_g(C.gcon + smp), to_g(C.R[par ^ 1] + smp * 3 * N),
                            to_g(C.partials + (smp * per + b) * 7), d, C.zchunk, xcd_block(b, per));
        break;
    }
    __syncthreads();  // the next virtual workgroup rewrites the LDS
  }
}

// no fused multiply-adds: the same roundings as the host's eta of a single solve
__device__ __forceinline__ double frob6(const double* s) {
#pragma clang fp contract(off)
  return sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2] + 2.0 * (s[3] * s[3] + s[4] * s[4] + s[5] * s[5]));
}

// eta of every active sample from its partial sums, and the stop rules of
// fe_solve_batched (after an update: the sample advanced one iteration)
__device__ void decide(BatchDev* bd, bool advanced, double* red) {
  int total = 0;
  for (int c = 0; c < bd->ncls; ++c) total += bd->cls[c].nact;
  for (int j = blockIdx.x; j < total; j += gridDim.x) {
    int c = 0, off = j;
    while (off >= bd->cls[c].nact) {
      off -= bd->cls[c].nact;
      ++c;
    }
    const BatchClassDev& C = bd->cls[c];
    const long long smp = C.act[off];
    double acc[8];
    reduce_body(C.partials + smp * C.bu * 7, C.bu, 7, acc, red);
    if (threadIdx.x == 0) {
      BatchState& st = bd->st[C.first + smp];
      if (advanced) {
        st.iterations += 1;
        st.parity ^= 1;
      }
      const int k = st.iterations;
      const double n = (double)C.d.N;
      for (int i = 0; i < 6; ++i) st.mean[i] = acc[1 + i] / n;
      const double eta = sqrt(acc[0] / n) / frob6(st.mean);
      st.eta = eta;
      if (!isfinite(eta)) {
        st.status = FE_DIVERGED;
      } else if (eta <= bd->tol) {
        st.status = FE_OK;
      } else if (k >= bd->max_iter) {
        st.status = FE_NOT_CONVERGED;
      } else {
        st.rising = eta > st.prev ? st.rising + 1 : 0;
        st.prev = eta;
        if (bd->diverge_window > 0 && st.rising >= bd->diverge_window) {
          st.status = FE_DIVERGED;
        } else if (eta < 0.95 * st.best) {
          st.best = eta;
          st.best_k = k;
        } else if (k - st.best_k >= kStallWindow) {
          st.status = FE_NOT_CONVERGED;
        }
      }
    }
    __syncthreads();  // red is reused by the next sample
  }
}

// workgroup 0 keeps the running samples of each class, in order: per chunk
// of 256 entries, a running flag per thread and its exclusive prefix
// (ballots within a wave, then the waves in order)
__device__ void compact(BatchDev* bd, int* wsum) {
  if (blockIdx.x != 0) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int total = 0;
  for (int c = 0; c < bd->ncls; ++c) {
    BatchClassDev& C = bd->cls[c];
    const int n = C.nact;
    int kept = 0;
    for (int base = 0; base < n; base += kBatchThreads) {
      const int s = base + (int)threadIdx.x;
      const int smp = s < n ? C.act[s] : 0;
      const bool run = s < n && bd->st[C.first + smp].status == kBatchRunning;
      const unsigned long long m = __ballot(run);
      const int below = __popcll(m & ((1ull << lane) - 1ull));
      if (lane == 0) wsum[wave] = __popcll(m);
      __syncthreads();
      int before = kept;
      for (int w = 0; w < wave; ++w) before += wsum[w];
      int chunk = 0;
      for (int w = 0; w < kBatchThreads / 64; ++w) chunk += wsum[w];
      __syncthreads();  // every C.act read of this chunk, and wsum, before the writes
      if (run) C.act[before + below] = smp;
      kept += chunk;
    }
    if (threadIdx.x == 0) C.nact = kept;
    total += kept;
  }
  if (threadIdx.x == 0) bd->ctrl[0] = total;
}

// Barrier over the whole grid of a cooperative launch (every workgroup
// resident): workgroup w's k-th arrival adds 1 to a 64-bit counter and
// waits until it reaches k * gridDim.x.  Each wave waits for its own stores
// to complete, then one thread per workgroup writes back the L2 (release at
// device scope: the stores become visible to the other XCDs), arrives,
// spins, and invalidates the caches it reads through (acquire).  A wait that
// outlasts a few seconds (a grid that is not resident) sets ctrl[1] and
// returns false; the kernel then ends.
constexpr unsigned kBarrierPolls = 1u << 22;
__device__ bool grid_barrier(BatchDev* bd, unsigned long long& target) {
  __shared__ int ok;
  target += gridDim.x;
  __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(bd->bar, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    unsigned polls = 0;
    while (__hip_atomic_load(bd->bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target &&
           __hip_atomic_load(bd->ctrl + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
      if (++polls == kBarrierPolls) {
        __hip_atomic_store(bd->ctrl + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    ok = __hip_atomic_load(bd->ctrl + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
  }
  __syncthreads();
  return ok;
}

template <int OP, bool AS>
__global__ __launch_bounds__(kBatchThreads, kBatchWavesPerSimd) void k_batch_persistent(BatchDev* bd) {
  __shared__ __align__(16) unsigned char smem[kBatchLds];
  __shared__ double red[8 * 16];
  __shared__ int wsum[kBatchThreads / 64];
  unsigned long long target = 0;
  // eta^0: the divergence of eps_bar (parity 0)
  run_pass<OP, AS>(bd, BP_DIV, smem);
  if (!grid_barrier(bd, target)) return;
  decide(bd, false, red);
  if (!grid_barrier(bd, target)) return;
  compact(bd, wsum);
  if (!grid_barrier(bd, target)) return;
  const int cap = bd->max_iter + 1;  // every sample retires at its cap at the latest
  for (int it = 0; it < cap && bd->ctrl[0] > 0; ++it) {
    for (int pass = BP_ZR2C; pass <= BP_UPDATE; ++pass) {
      run_pass<OP, AS>(bd, pass, smem);
      if (!grid_barrier(bd, target)) return;
    }
    decide(bd, true, red);
    if (!grid_barrier(bd, target)) return;
    compact(bd, wsum);
    if (!grid_barrier(bd, target)) return;
  }
}

}  // namespace

void batch_class_layout(const Dims& d, int* bz, int* by, int* bx, int* bu, int* zchunk) {
  dispatch_length(d.nz, [&](auto NC) {
    using C = StridedCfg<float, decltype(NC)::value>;
    *bz = ((d.nx / 2 + C::TX - 1) / C::TX) * d.ny * 3;
  });
  dispatch_length(d.ny, [&](auto NC) {
    using C = StridedCfg<float, decltype(NC)::value, true>;
    *by = ((d.nx + C::TX - 1) / C::TX) * d.H * 3;
  });
  dispatch_length(d.nx, [&](auto NC) { *bx = x_blocks<float, decltype(NC)::value>(d, 3); });
  const DivGrid gd = div_grid<kBatchDX, kBatchDY>(d);
  *bu = gd.blocks;
  *zchunk = gd.zchunk;
}

template <int OP, bool AS>
static int grid_of() {
  int dev = 0, per_cu = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
  if (!prop.cooperativeLaunch) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_persistent<OP, AS>, kBatchThreads, 0) !=
      hipSuccess)
    return 0;
  return per_cu * prop.multiProcessorCount;
}

int batch_persistent_grid(int op, bool accel) {
  if (op == OP_ROT) return accel ? grid_of<OP_ROT, true>() : grid_of<OP_ROT, false>();
  return accel ? grid_of<OP_WP, true>() : grid_of<OP_WP, false>();
}

template <int OP, bool AS>
static hipError_t launch_of(BatchDev* dev, int grid, hipStream_t s) {
  void* args[] = {&dev};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_batch_persistent<OP, AS>), dim3(grid),
                                    dim3(kBatchThreads), args, 0, s);
}

hipError_t launch_batch_persistent(int op, bool accel, BatchDev* dev, int grid, hipStream_t s) {
  if (op == OP_ROT) return accel ? launch_of<OP_ROT, true>(dev, grid, s) : launch_of<OP_ROT, false>(dev, grid, s);
  return accel ? launch_of<OP_WP, true>(dev, grid, s) : launch_of<OP_WP, false>(dev, grid, s);
}

}  // namespace fe
