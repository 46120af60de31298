// Measurement probes: the two ceilings the update is priced against, measured
// on the device rather than taken from a datasheet. Neither is a step of the
// method.
//  - a streaming copy: the HBM rate a kernel that reads and writes
//    contiguous memory once can reach;
//  - random no-return 32-bit atomic ORs into a buffer of cube size: the rate
//    at which the one-thread-per-packet scheme of Sec. 4.1 can set bits,
//    whatever it spends on hashing (the addresses are precomputed).
#include "../../include/cbaa_probe.h"
#include "cbaa_internal.hpp"

namespace cbaa {
namespace {

constexpr int kProbeBlock = 256;
constexpr int kCopyUnroll = 4;

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <bool NT>
__global__ __launch_bounds__(kProbeBlock) void k_probe_copy(const u32x4* __restrict__ src,
                                                            u32x4* __restrict__ dst, uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * kProbeBlock;
  uint64_t i = (uint64_t)blockIdx.x * kProbeBlock + threadIdx.x;
  for (; i + (kCopyUnroll - 1) * stride < n; i += kCopyUnroll * stride) {
    u32x4 v[kCopyUnroll];
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u)
      v[u] = NT ? __builtin_nontemporal_load(src + i + u * stride) : src[i + u * stride];
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
      if (NT) __builtin_nontemporal_store(v[u], dst + i + u * stride);
      else dst[i + u * stride] = v[u];
    }
  }
  for (; i < n; i += stride) dst[i] = src[i];
}

// Word indices in [0, 2^log2_words): the top bits of a mixed counter.
__global__ __launch_bounds__(kProbeBlock) void k_probe_addresses(uint32_t* addr, uint64_t n,
                                                                 uint32_t log2_words,
                                                                 uint32_t seed) {
  const uint64_t stride = (uint64_t)gridDim.x * kProbeBlock;
  for (uint64_t i = (uint64_t)blockIdx.x * kProbeBlock + threadIdx.x; i < n; i += stride) {
    const uint32_t h = fmix32((uint32_t)i ^ fmix32((uint32_t)(i >> 32) + seed));
    addr[i] = log2_words ? h >> (32 - log2_words) : 0u;
  }
}

// Each thread takes four precomputed indices (one 16-byte load) and ORs one
// bit into each word with a device-scope atomic whose result is unused. The
// indices are masked to the buffer (a power of two of words), so any index
// content stays in bounds.
__global__ __launch_bounds__(kProbeBlock) void k_probe_atomic_or(uint32_t* buf, uint32_t mask,
                                                                 const uint4* __restrict__ addr,
                                                                 uint64_t quads) {
  const uint64_t stride = (uint64_t)gridDim.x * kProbeBlock;
  for (uint64_t i = (uint64_t)blockIdx.x * kProbeBlock + threadIdx.x; i < quads; i += stride) {
    uint4 a = addr[i];
    a.x &= mask;
    a.y &= mask;
    a.z &= mask;
    a.w &= mask;
    const uint32_t bit = (uint32_t)i & 31u;
    __hip_atomic_fetch_or(buf + a.x, 1u << bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_or(buf + a.y, 1u << ((bit + 8) & 31u), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_or(buf + a.z, 1u << ((bit + 16) & 31u), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_or(buf + a.w, 1u << ((bit + 24) & 31u), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

uint32_t grid_for(uint64_t items, uint32_t cap) {
  const uint64_t b = (items + kProbeBlock - 1) / kProbeBlock;
  return (uint32_t)(b < cap ? (b ? b : 1) : cap);
}

int launched(const char* what) {
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? CBAA_OK : hip_fail(e, what);
}

}  // namespace
}  // namespace cbaa

using namespace cbaa;

extern "C" {

int cbaa_probe_copy(void* d_dst, const void* d_src, uint64_t bytes, uint32_t blocks,
                    uint32_t flags, void* stream) {
  if (!d_dst || !d_src || ((uintptr_t)d_dst & 15u) || ((uintptr_t)d_src & 15u) || (bytes & 15u) ||
      blocks > (1u << 20) || (flags & ~CBAA_PROBE_NONTEMPORAL)) {
    set_error("copy probe needs non-null 16-byte aligned buffers, a multiple of 16 bytes, at "
              "most 2^20 blocks and known flags");
    return CBAA_EINVAL;
  }
  if (bytes == 0) return CBAA_OK;
  const uint64_t n = bytes / 16;
  // default: 8 blocks of 256 threads per CU on 256 CUs, striding over the buffer
  const uint32_t grid = grid_for(n, blocks ? blocks : 2048);
  if (flags & CBAA_PROBE_NONTEMPORAL)
    hipLaunchKernelGGL(k_probe_copy<true>, dim3(grid), dim3(kProbeBlock), 0, (hipStream_t)stream,
                       (const u32x4*)d_src, (u32x4*)d_dst, n);
  else
    hipLaunchKernelGGL(k_probe_copy<false>, dim3(grid), dim3(kProbeBlock), 0, (hipStream_t)stream,
                       (const u32x4*)d_src, (u32x4*)d_dst, n);
  return launched("copy probe launch");
}

int cbaa_probe_addresses(uint32_t* d_addr, uint64_t n, uint32_t log2_words, uint32_t seed,
                         void* stream) {
  if (!d_addr || log2_words > 32 || ((uintptr_t)d_addr & 3u)) {
    set_error("address probe needs a non-null 4-byte aligned buffer and log2_words <= 32");
    return CBAA_EINVAL;
  }
  if (n == 0) return CBAA_OK;
  hipLaunchKernelGGL(k_probe_addresses, dim3(grid_for(n, 8192)), dim3(kProbeBlock), 0,
                     (hipStream_t)stream, d_addr, n, log2_words, seed);
  return launched("address probe launch");
}

int cbaa_probe_atomic_or(uint32_t* d_buf, uint64_t words, const uint32_t* d_addr, uint64_t n,
                         void* stream) {
  if (!d_buf || !d_addr || ((uintptr_t)d_addr & 15u) || ((uintptr_t)d_buf & 3u) || (n & 3u) ||
      words == 0 || words > (1ull << 32) || (words & (words - 1))) {
    set_error("atomic probe needs non-null buffers (indices 16-byte aligned), a power-of-two "
              "word count up to 2^32 and n a multiple of 4");
    return CBAA_EINVAL;
  }
  if (n == 0) return CBAA_OK;
  hipLaunchKernelGGL(k_probe_atomic_or, dim3(grid_for(n / 4, 8192)), dim3(kProbeBlock), 0,
                     (hipStream_t)stream, d_buf, (uint32_t)(words - 1), (const uint4*)d_addr,
                     n / 4);
  return launched("atomic probe launch");
}

}  // extern "C"
