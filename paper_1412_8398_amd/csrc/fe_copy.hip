// Streaming device copy: the attainable-bandwidth reference that the solver's
// passes are measured against (include/fe.h: fe_stream_copy).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/fe.h"
#include "fe_error.h"

using namespace fe;

namespace {

typedef unsigned int v4u __attribute__((ext_vector_type(4)));  // one 16-byte vector

constexpr int kCopyThreads = 512;
constexpr int kCopyUnroll = 4;  // 16-byte vectors per thread, kCopyThreads apart

// Each workgroup moves kCopyUnroll * kCopyThreads * 16 bytes: all loads issue
// before the first store, every access is a whole 16-byte vector and a
// wavefront covers 1 KiB per access (fully coalesced).
template <bool NT>
__global__ __launch_bounds__(kCopyThreads) void k_copy16(const v4u* __restrict__ src, v4u* __restrict__ dst,
                                                         long long n) {
  const long long base = (long long)blockIdx.x * kCopyThreads * kCopyUnroll + threadIdx.x;
  v4u v[kCopyUnroll];
#pragma unroll
  for (int u = 0; u < kCopyUnroll; ++u) {
    const long long j = base + (long long)u * kCopyThreads;
    if (j < n) v[u] = NT ? __builtin_nontemporal_load(src + j) : src[j];
  }
#pragma unroll
  for (int u = 0; u < kCopyUnroll; ++u) {
    const long long j = base + (long long)u * kCopyThreads;
    if (j < n) {
      if (NT)
        __builtin_nontemporal_store(v[u], dst + j);
      else
        dst[j] = v[u];
    }
  }
}

// In place (dst == src): every thread rewrites the vectors it has just read,
// so the pointers may alias (no __restrict__).
template <bool NT>
__global__ __launch_bounds__(kCopyThreads) void k_rewrite16(v4u* p, long long n) {
  const long long base = (long long)blockIdx.x * kCopyThreads * kCopyUnroll + threadIdx.x;
  v4u v[kCopyUnroll];
#pragma unroll
  for (int u = 0; u < kCopyUnroll; ++u) {
    const long long j = base + (long long)u * kCopyThreads;
    if (j < n) v[u] = NT ? __builtin_nontemporal_load(p + j) : p[j];
  }
#pragma unroll
  for (int u = 0; u < kCopyUnroll; ++u) {
    const long long j = base + (long long)u * kCopyThreads;
    if (j < n) {
      if (NT)
        __builtin_nontemporal_store(v[u], p + j);
      else
        p[j] = v[u];
    }
  }
}

}  // namespace

extern "C" fe_status fe_stream_copy(void* dst, const void* src, size_t bytes, int32_t nontemporal, void* hip_stream) {
  if (!dst || !src) return fail(FE_ERR_INVALID_ARG, "dst or src is NULL");
  if (bytes % 16 != 0) return fail(FE_ERR_INVALID_ARG, "bytes must be a multiple of 16");
  if ((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) % 16 != 0)
    return fail(FE_ERR_INVALID_ARG, "dst and src must be 16-byte aligned");
  const char* s = static_cast<const char*>(src);
  const char* d = static_cast<const char*>(dst);
  if (s != d && s < d + bytes && d < s + bytes) return fail(FE_ERR_INVALID_ARG, "dst and src overlap");
  const long long n = (long long)(bytes / 16);
  if (n == 0) return FE_OK;
  const long long per_block = (long long)kCopyThreads * kCopyUnroll;
  const long long blocks = (n + per_block - 1) / per_block;
  if (blocks > 0x7fffffffLL) return fail(FE_ERR_UNSUPPORTED, "copy too large");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (s == d) {
    if (nontemporal)
      hipLaunchKernelGGL(k_rewrite16<true>, dim3((unsigned)blocks), dim3(kCopyThreads), 0, st, static_cast<v4u*>(dst), n);
    else
      hipLaunchKernelGGL(k_rewrite16<false>, dim3((unsigned)blocks), dim3(kCopyThreads), 0, st, static_cast<v4u*>(dst), n);
  } else if (nontemporal)
    hipLaunchKernelGGL(k_copy16<true>, dim3((unsigned)blocks), dim3(kCopyThreads), 0, st,
                       static_cast<const v4u*>(src), static_cast<v4u*>(dst), n);
  else
    hipLaunchKernelGGL(k_copy16<false>, dim3((unsigned)blocks), dim3(kCopyThreads), 0, st,
                       static_cast<const v4u*>(src), static_cast<v4u*>(dst), n);
  HIP_TRY(hipGetLastError());
  return FE_OK;
}
