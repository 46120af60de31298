// Local-server kernels: cube initialisation, the per-pair update of Alg. 1
// with direct device-scope atomics, and the global server's OR-merge.
#include "cbaa_internal.hpp"

namespace cbaa {

namespace {

constexpr int kBlock = 256;
constexpr uint32_t kMaxBlocks = 256u * 16u;  // 16 resident blocks of 256 per CU, 256 CUs

inline uint32_t grid_for(uint64_t items, uint32_t per_block) {
  uint64_t b = (items + per_block - 1) / per_block;
  if (b > kMaxBlocks) b = kMaxBlocks;
  return b == 0 ? 1u : (uint32_t)b;
}

// Zero fill with 16-byte stores (used instead of a runtime memset so the call
// stays valid inside captured graphs).
__global__ __launch_bounds__(kBlock) void k_fill_zero(uint4* p, uint64_t n16) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
}

// A new cube: zero bits, and a whole valid header (reserved words zero).
__global__ __launch_bounds__(kBlock) void k_cube_init(Dims d, uint64_t* bits) {
  uint4* p = (uint4*)bits;
  const uint64_t n16 = d.words / 2;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
  if (blockIdx.x == 0 && threadIdx.x == 0) header_set(header_of(bits), d, CBAA_CUBE_VALID);
}

// The direct path's cubes keep a valid header only if they have one.
__global__ void k_touch_headers(Dims d, uint64_t* c0, uint64_t* c1) {
  if (threadIdx.x == 0 && c0) header_touch(c0, d);
  if (threadIdx.x == 1 && c1) header_touch(c1, d);
}

// Sets the A bits of one (host, peer) pair: bit H_bv(peer) of the host's
// column in every array of its sketch. 32-bit no-return atomic OR on the half
// of the 64-bit word that holds the bit.
template <int NRA, int NVA>
__device__ inline void set_pair_bits(const Dims& d, uint32_t* cube32, uint32_t host, uint32_t peer) {
  constexpr int A = NRA + NVA;
  uint32_t slot[A];
  const uint32_t cs = host_slots<NRA, NVA>(d, host, slot);
  const uint32_t b = bit_of_peer(d, peer);
  const uint64_t row = ((uint64_t)cs * d.R + (b >> 6)) * d.W;
  const uint32_t half = (b >> 5) & 1u;
  const uint32_t mask = 1u << (b & 31u);
#pragma unroll
  for (int a = 0; a < A; ++a)
    __hip_atomic_fetch_or(cube32 + 2 * (row + slot[a]) + half, mask, __ATOMIC_RELAXED,
                          __HIP_MEMORY_SCOPE_AGENT);
}

// Alg. 1 over a batch, one pair per thread per grid-stride step. With two
// cubes, cube0 is keyed by the source and cube1 by the destination.
template <int NRA, int NVA, bool TWO>
__global__ __launch_bounds__(kBlock) void k_update_direct(Dims d, uint32_t* cube0, uint32_t* cube1,
                                                          const uint2* __restrict__ pairs,
                                                          uint64_t n, int side) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
    const uint2 p = pairs[k];
    const uint32_t host = side == CBAA_SIDE_SRC ? p.x : p.y;
    const uint32_t peer = side == CBAA_SIDE_SRC ? p.y : p.x;
    set_pair_bits<NRA, NVA>(d, cube0, host, peer);
    if (TWO) set_pair_bits<NRA, NVA>(d, cube1, peer, host);
  }
}

struct MergeSources {
  const uint4* p[8];
};

// dst = (accumulate ? dst : 0) | OR of k <= 8 sources, 16 bytes per lane.
// The first thread also writes dst's header: valid only if every source (and,
// when accumulating, dst's own earlier pass) carries this configuration's
// valid header. A source that is dst is placed first, and its header is read
// before it is written, by the same thread.
__global__ __launch_bounds__(kBlock) void k_merge_or(Dims d, uint4* dst, MergeSources s, int k,
                                                     uint64_t n16, int accumulate) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    bool ok = !accumulate || header_ok(header_of((const uint64_t*)dst), d);
    for (int j = 0; j < k; ++j) ok = ok && header_ok(header_of((const uint64_t*)s.p[j]), d);
    header_set(header_of((uint64_t*)dst), d, ok ? CBAA_CUBE_VALID : CBAA_CUBE_MIXED);
  }
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) {
    uint4 v = accumulate ? load_stream(dst + i) : make_uint4(0u, 0u, 0u, 0u);
    for (int j = 0; j < k; ++j) {
      const uint4 w = load_stream(s.p[j] + i);
      v.x |= w.x;
      v.y |= w.y;
      v.z |= w.z;
      v.w |= w.w;
    }
    store_stream(dst + i, v);
  }
}

template <bool TWO>
int dispatch_direct(const Dims& d, uint32_t* c0, uint32_t* c1, const uint2* pairs, uint64_t n,
                    int side, hipStream_t s) {
  const uint32_t grid = grid_for(n, kBlock);
#define CBAA_UPD(NRA, NVA)                                                                      \
  if (d.n_ra == NRA && d.n_va == NVA) {                                                         \
    hipLaunchKernelGGL((k_update_direct<NRA, NVA, TWO>), dim3(grid), dim3(kBlock), 0, s, d, c0, \
                       c1, pairs, n, side);                                                     \
    hipError_t e = hipGetLastError();                                                           \
    return e == hipSuccess ? CBAA_OK : hip_fail(e, "update kernel launch");                    \
  }
  CBAA_UPD(2, 0) CBAA_UPD(2, 1) CBAA_UPD(2, 2)
  CBAA_UPD(3, 0) CBAA_UPD(3, 1) CBAA_UPD(3, 2)
  CBAA_UPD(4, 0) CBAA_UPD(4, 1) CBAA_UPD(4, 2)
#undef CBAA_UPD
  set_error("no update kernel for n_ra=%u n_va=%u", d.n_ra, d.n_va);
  return CBAA_ECONFIG;
}

}  // namespace

int launch_fill_zero(uint64_t* p, uint64_t words, hipStream_t s) {
  const uint64_t n16 = words / 2;  // cubes are a whole number of 16-byte units
  hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(n16, kBlock)), dim3(kBlock), 0, s, (uint4*)p, n16);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? CBAA_OK : hip_fail(e, "fill kernel launch");
}

int launch_cube_init(const Dims& d, uint64_t* bits, hipStream_t s) {
  hipLaunchKernelGGL(k_cube_init, dim3(grid_for(d.words / 2, kBlock)), dim3(kBlock), 0, s, d, bits);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? CBAA_OK : hip_fail(e, "cube init launch");
}

int launch_update_direct(const Dims& d, uint64_t* cube0, uint64_t* cube1, const uint32_t* pairs,
                         uint64_t n, int side, hipStream_t s) {
  hipLaunchKernelGGL(k_touch_headers, dim3(1), dim3(64), 0, s, d, cube0, cube1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "header launch");
  if (cube1)
    return dispatch_direct<true>(d, (uint32_t*)cube0, (uint32_t*)cube1, (const uint2*)pairs, n,
                                 CBAA_SIDE_SRC, s);
  return dispatch_direct<false>(d, (uint32_t*)cube0, nullptr, (const uint2*)pairs, n, side, s);
}

int launch_merge_or(const Dims& d, uint64_t* dst, const uint64_t* const* srcs, int k,
                    hipStream_t s) {
  // Put a source that aliases dst first, so it is read before dst is written.
  const uint64_t* order[64];
  const uint64_t** ord = order;
  const uint64_t** heap = nullptr;
  if (k > 64) ord = heap = new const uint64_t*[k];
  int n = 0;
  for (int i = 0; i < k; ++i)
    if (srcs[i] == dst) ord[n++] = srcs[i];
  for (int i = 0; i < k; ++i)
    if (srcs[i] != dst) ord[n++] = srcs[i];
  const uint64_t n16 = d.words / 2;
  int rc = CBAA_OK;
  for (int base = 0; base < k && rc == CBAA_OK; base += 8) {
    MergeSources ms{};
    int m = k - base < 8 ? k - base : 8;
    for (int j = 0; j < m; ++j) ms.p[j] = (const uint4*)ord[base + j];
    hipLaunchKernelGGL(k_merge_or, dim3(grid_for(n16, kBlock)), dim3(kBlock), 0, s, d, (uint4*)dst,
                       ms, m, n16, base > 0 ? 1 : 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) rc = hip_fail(e, "merge kernel launch");
  }
  delete[] heap;
  return rc;
}

// The partitioned (LDS-tiled) update lives in cbaa_partition.hip.

}  // namespace cbaa
