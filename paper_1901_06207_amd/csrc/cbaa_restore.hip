// Global-server kernels: per-column zero counts, per-sketch eps and threshold,
// hot-column lists (Alg. 2), the hot-column tuple check (Alg. 3) with union
// column verification, reassembly of the IP, the Thm. 2 estimate, and the
// ordering of the restored list.
#include <math.h>

#include "cbaa_internal.hpp"

namespace cbaa {

namespace {

constexpr int kScanBlock = 256;
constexpr int kPrepBlock = 1024;
constexpr int kJoinBlock = 256;
constexpr int kSortChunk = 4096;   // entries sorted per block in LDS
constexpr int kSortBlock = 1024;

inline uint64_t align256(uint64_t x) { return (x + 255u) & ~uint64_t(255u); }

// Scratch carve-up shared by restore and estimate.
struct RestoreScratch {
  uint16_t* zeros;  // [S][W]
  uint32_t* ones;   // [S][A]
  double* eps;      // [S]
  int32_t* zmax;    // [S]
  uint32_t* hcnt;   // [S][n_ra]
  uint16_t* hot;    // [S][n_ra][maxc_ra]
  cbaa_host* stage; // [capacity]
  uint64_t* keys;   // [capacity]
  uint64_t bytes;
};

RestoreScratch carve(const Dims& d, void* base, uint64_t capacity) {
  RestoreScratch r;
  uint64_t off = 0;
  char* b = (char*)base;
  auto take = [&](uint64_t bytes) {
    char* p = b ? b + off : nullptr;
    off += align256(bytes);
    return (void*)p;
  };
  r.zeros = (uint16_t*)take((uint64_t)d.S * d.W * 2);
  r.ones = (uint32_t*)take((uint64_t)d.S * d.A * 4);
  r.eps = (double*)take((uint64_t)d.S * 8);
  r.zmax = (int32_t*)take((uint64_t)d.S * 4);
  r.hcnt = (uint32_t*)take((uint64_t)d.S * d.n_ra * 4);
  r.hot = (uint16_t*)take((uint64_t)d.S * d.n_ra * d.maxc_ra * 2);
  r.stage = (cbaa_host*)take(capacity * sizeof(cbaa_host));
  r.keys = (uint64_t*)take(capacity * 8);
  r.bytes = off;
  return r;
}

__device__ inline uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ inline uint32_t lane_id() { return __lane_id(); }

// ---- per-column zero counts ---------------------------------------------
// Thread (cs, w..w+1): popcounts of two neighbouring columns' words over all
// R row blocks; a wave reads 1 KiB contiguous per row block.
__global__ __launch_bounds__(kScanBlock) void k_column_zeros(Dims d, const uint4* __restrict__ cube,
                                                             uint32_t* __restrict__ zeros2) {
  const uint32_t cs = blockIdx.y;
  const uint32_t pair = blockIdx.x * kScanBlock + threadIdx.x;  // column pair index
  const uint32_t half_w = d.W / 2;
  if (pair >= half_w) return;
  uint32_t c0 = 0, c1 = 0;
  const uint4* p = cube + ((uint64_t)cs * d.R) * half_w + pair;
  uint32_t rb = 0;
  for (; rb + 4 <= d.R; rb += 4) {
    const uint4 v0 = p[(uint64_t)(rb + 0) * half_w];
    const uint4 v1 = p[(uint64_t)(rb + 1) * half_w];
    const uint4 v2 = p[(uint64_t)(rb + 2) * half_w];
    const uint4 v3 = p[(uint64_t)(rb + 3) * half_w];
    c0 += __popc(v0.x) + __popc(v0.y) + __popc(v1.x) + __popc(v1.y) + __popc(v2.x) + __popc(v2.y) +
          __popc(v3.x) + __popc(v3.y);
    c1 += __popc(v0.z) + __popc(v0.w) + __popc(v1.z) + __popc(v1.w) + __popc(v2.z) + __popc(v2.w) +
          __popc(v3.z) + __popc(v3.w);
  }
  for (; rb < d.R; ++rb) {
    uint4 v = p[(uint64_t)rb * half_w];
    c0 += __popc(v.x) + __popc(v.y);
    c1 += __popc(v.z) + __popc(v.w);
  }
  zeros2[(uint64_t)cs * half_w + pair] = (d.g - c0) | ((d.g - c1) << 16);
}

// Block-wide sum of per-thread counts (each below 2^32 in total per wave).
__device__ inline uint64_t block_sum(uint32_t v, uint64_t* lds) {
  const uint32_t w = wave_sum(v);
  const int wid = threadIdx.x / kWave;
  __syncthreads();
  if (lane_id() == 0) lds[wid] = w;
  __syncthreads();
  uint64_t t = 0;
  for (int i = 0; i < (int)(blockDim.x / kWave); ++i) t += lds[i];
  __syncthreads();
  return t;
}

// One block per sketch: array fills, eps (Thm. 1 with measured fills), Zmax,
// and, if `lists`, the ascending hot-column list of every RA (Alg. 2).
__global__ __launch_bounds__(kPrepBlock) void k_prepare(Dims d, const uint16_t* __restrict__ zeros,
                                                        uint32_t* ones, double* eps, int32_t* zmax,
                                                        uint32_t* hcnt, uint16_t* hot, double x,
                                                        int rule, int lists,
                                                        cbaa_restore_stats* stats) {
  __shared__ uint64_t red[kPrepBlock / kWave];
  __shared__ uint32_t wave_cnt[kPrepBlock / kWave];
  __shared__ int32_t s_zmax;
  __shared__ uint64_t s_ones[CBAA_MAX_ARRAYS];
  const uint32_t cs = blockIdx.x;
  const uint16_t* z = zeros + (uint64_t)cs * d.W;

  for (uint32_t a = 0; a < d.A; ++a) {
    uint32_t zs = 0;  // at most 64 columns of at most 2^15 zeros per thread
    for (uint32_t j = threadIdx.x; j < d.ncol[a]; j += blockDim.x) zs += z[d.aoff[a] + j];
    const uint64_t tot = block_sum(zs, red);
    if (threadIdx.x == 0) s_ones[a] = (uint64_t)d.ncol[a] * d.g - tot;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double g = (double)d.g;
    double e = 1.0;
    for (uint32_t a = 0; a < d.A; ++a) {
      ones[cs * d.A + a] = (uint32_t)s_ones[a];
      e = e * ((double)s_ones[a] / ((double)d.ncol[a] * g));
    }
    double zf;
    if (rule == CBAA_THR_PAPER)
      zf = (g + g * e) * x - g * e;
    else
      zf = (g - g * e) * x;
    const int32_t zm = zf < 0.0 ? -1 : (int32_t)floor(zf);
    if (eps) eps[cs] = e;
    if (zmax) zmax[cs] = zm;
    s_zmax = zm;
  }
  __syncthreads();
  if (!lists) return;
  const int32_t zm = s_zmax;
  const int wid = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  uint64_t hot_total = 0;
  for (uint32_t i = 0; i < d.n_ra; ++i) {
    uint16_t* out = hot + ((uint64_t)cs * d.n_ra + i) * d.maxc_ra;
    uint32_t base = 0;
    for (uint32_t t0 = 0; t0 < d.ncol[i]; t0 += blockDim.x) {
      const uint32_t j = t0 + threadIdx.x;
      const bool pred = j < d.ncol[i] && (int32_t)z[d.aoff[i] + j] <= zm;
      const uint64_t bal = __ballot(pred);
      const uint32_t before = __popcll(bal & ((1ull << lane_id()) - 1ull));
      if (lane_id() == 0) wave_cnt[wid] = __popcll(bal);
      __syncthreads();
      uint32_t woff = 0, total = 0;
      for (int w = 0; w < nw; ++w) {
        if (w < wid) woff += wave_cnt[w];
        total += wave_cnt[w];
      }
      if (pred) out[base + woff + before] = (uint16_t)j;
      base += total;
      __syncthreads();
    }
    if (threadIdx.x == 0) hcnt[cs * d.n_ra + i] = base;
    hot_total += base;
  }
  if (threadIdx.x == 0 && stats)
    __hip_atomic_fetch_add(&stats->hot_columns, hot_total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_reset_stats(cbaa_restore_stats* st) {
  if (threadIdx.x == 0) {
    st->n_hosts = 0;
    st->hot_columns = 0;
    st->partial_checked = 0;
    st->tuples_checked = 0;
  }
}

// ---- tuple join and union-column verification (Alg. 3) ------------------
//
// One wave owns one hot column hc0 of RA 0 and walks the tuples that extend
// it, RA by RA: candidates of RA l are screened 64 at a time by the CP check
// of Alg. 3 against hc_{l-1} (and, for the last RA, against hc_0), then the
// AND of the columns chosen so far is counted. Because AND can only add zero
// bits, a partial tuple whose AND already has more than Zmax zeros cannot
// complete to an accepted tuple and is dropped: the accepted set is exactly
// Alg. 3's. Lane q of the wave holds row blocks q, q+64, ...

template <int RPL>
struct Col {
  uint64_t w[RPL];
};

template <int RPL>
__device__ inline void load_col(const Dims& d, const uint64_t* __restrict__ cube, uint32_t cs,
                                uint32_t slot, Col<RPL>& c) {
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    const uint32_t rb = lane_id() + q * kWave;
    c.w[q] = rb < d.R ? cube[((uint64_t)cs * d.R + rb) * d.W + slot] : ~0ull;
  }
}

template <int RPL>
__device__ inline uint32_t col_zeros(const Dims& d, const Col<RPL>& c) {
  uint32_t ones = 0;
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    const uint32_t rb = lane_id() + q * kWave;
    ones += rb < d.R ? (uint32_t)__popcll(c.w[q]) : 0u;
  }
  return d.g - wave_sum(ones);
}

struct JoinArgs {
  const uint64_t* cube;
  const uint16_t* hot;
  const uint32_t* hcnt;
  const int32_t* zmax;
  const double* eps;
  cbaa_host* stage;
  uint64_t capacity;
  cbaa_restore_stats* stats;
};

template <int NRA, int NVA>
__device__ inline void emit_host(const Dims& d, const JoinArgs& ja, uint32_t cs, uint32_t lp,
                                 uint32_t z) {
  if (lane_id() == 0) {
    const uint64_t idx =
        __hip_atomic_fetch_add(&ja.stats->n_hosts, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (idx < ja.capacity) {
      const double g = (double)d.g;
      const double e = ja.eps[cs];
      uint32_t zc = z;
      uint8_t flags = 0;
      if (zc == 0) {
        zc = 1;
        flags |= CBAA_FLAG_SATURATED;
      }
      double est = -g * log((double)zc / (g - g * e));
      if (est < 0.0) est = 0.0;
      cbaa_host h;
      h.ip = fmix32_inverse((lp << d.r) | cs) ^ d.seed_mangle;
      h.zeros = (uint16_t)z;
      h.cs = (uint8_t)cs;
      h.flags = flags;
      h.est = est;
      ja.stage[idx] = h;
    }
  }
}

template <int NRA, int NVA, int RPL, int LEVEL>
__device__ void extend(const Dims& d, const JoinArgs& ja, uint32_t cs, int32_t zm,
                       uint32_t (&t)[NRA], const Col<RPL>& acc, uint32_t& n_partial,
                       uint32_t& n_tuples) {
  const uint32_t cnt = ja.hcnt[cs * NRA + LEVEL];
  const uint16_t* list = ja.hot + ((uint64_t)cs * NRA + LEVEL) * d.maxc_ra;
  const uint32_t prev = t[LEVEL - 1];
  const uint32_t want_lo = prev >> d.ep[LEVEL - 1];          // CP of hc_{l-1}
  const uint32_t cp_mask = low_mask(d.cp[LEVEL - 1]);
  const uint32_t want_hi = t[0] & low_mask(d.cp[NRA - 1]);   // first bits of hc_0
  for (uint32_t base = 0; base < cnt; base += kWave) {
    const uint32_t j = base + lane_id();
    const uint32_t cand = j < cnt ? list[j] : 0u;
    bool ok = j < cnt && (cand & cp_mask) == want_lo;
    if (LEVEL == NRA - 1) ok = ok && (cand >> d.ep[LEVEL]) == want_hi;
    uint64_t m = __ballot(ok);
    while (m) {
      const int l = __builtin_ctzll(m);
      m &= m - 1;
      const uint32_t h = (uint32_t)__builtin_amdgcn_readlane((int)cand, l);
      Col<RPL> c;
      load_col<RPL>(d, ja.cube, cs, d.aoff[LEVEL] + h, c);
#pragma unroll
      for (int q = 0; q < RPL; ++q) c.w[q] &= acc.w[q];
      t[LEVEL] = h;
      if constexpr (LEVEL < NRA - 1) {
        ++n_partial;
        if ((int32_t)col_zeros<RPL>(d, c) > zm) continue;
        extend<NRA, NVA, RPL, LEVEL + 1>(d, ja, cs, zm, t, c, n_partial, n_tuples);
      } else {
        // complete CP-valid tuple: LP = concatenation of the EPs
        uint32_t lp = 0;
#pragma unroll
        for (int i = 0; i < NRA; ++i) lp |= rotl_in(t[i] & low_mask(d.ep[i]), d.off[i], d.L);
#pragma unroll
        for (int v = 0; v < NVA; ++v) {
          Col<RPL> vc;
          load_col<RPL>(d, ja.cube, cs, d.aoff[NRA + v] + va_col(d, v, lp), vc);
#pragma unroll
          for (int q = 0; q < RPL; ++q) c.w[q] &= vc.w[q];
        }
        ++n_tuples;
        const uint32_t z = col_zeros<RPL>(d, c);
        if ((int32_t)z <= zm) emit_host<NRA, NVA>(d, ja, cs, lp, z);
      }
    }
  }
}

template <int NRA, int NVA, int RPL>
__global__ __launch_bounds__(kJoinBlock) void k_join(Dims d, JoinArgs ja) {
  __shared__ uint32_t pre[257];
  // prefix over sketches of |HC(0)|: flattened work list of (cs, hc0)
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (uint32_t cs = 0; cs < d.S; ++cs) {
      pre[cs] = acc;
      acc += ja.hcnt[cs * NRA + 0];
    }
    pre[d.S] = acc;
  }
  __syncthreads();
  const uint32_t total = pre[d.S];
  const uint32_t waves_per_block = kJoinBlock / kWave;
  const uint32_t gw = blockIdx.x * waves_per_block + threadIdx.x / kWave;
  const uint32_t nwaves = gridDim.x * waves_per_block;
  uint32_t n_partial = 0, n_tuples = 0;
  for (uint32_t item = gw; item < total; item += nwaves) {
    uint32_t lo = 0, hi = d.S;  // largest cs with pre[cs] <= item
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) / 2;
      if (pre[mid] <= item) lo = mid; else hi = mid;
    }
    const uint32_t cs = lo;
    const uint32_t hc0 = ja.hot[((uint64_t)cs * NRA + 0) * d.maxc_ra + (item - pre[cs])];
    const int32_t zm = ja.zmax[cs];
    uint32_t t[NRA];
    t[0] = hc0;
    Col<RPL> c0;
    load_col<RPL>(d, ja.cube, cs, d.aoff[0] + hc0, c0);
    extend<NRA, NVA, RPL, 1>(d, ja, cs, zm, t, c0, n_partial, n_tuples);
  }
  if (lane_id() == 0 && (n_partial | n_tuples)) {
    __hip_atomic_fetch_add(&ja.stats->partial_checked, (uint64_t)n_partial, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(&ja.stats->tuples_checked, (uint64_t)n_tuples, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ---- ordering of the restored list --------------------------------------
// Keys are (ip << 32 | stage index); restored IPs are distinct, the index
// keeps keys unique regardless. Each block sorts kSortChunk keys in LDS
// (bitonic); a second kernel ranks every key against the other chunks by
// binary search and scatters the entry to its final place.

__global__ __launch_bounds__(kSortBlock) void k_sort_chunks(const cbaa_host* stage,
                                                            const cbaa_restore_stats* stats,
                                                            uint64_t capacity, uint64_t* keys) {
  __shared__ uint64_t k[kSortChunk];
  const uint64_t n = stats->n_hosts < capacity ? stats->n_hosts : capacity;
  const uint64_t base = (uint64_t)blockIdx.x * kSortChunk;
  if (base >= n) return;
  for (int i = threadIdx.x; i < kSortChunk; i += kSortBlock) {
    const uint64_t g = base + i;
    k[i] = g < n ? (((uint64_t)stage[g].ip << 32) | (uint32_t)g) : ~0ull;
  }
  __syncthreads();
  for (int size = 2; size <= kSortChunk; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < kSortChunk / 2; i += kSortBlock) {
        const int lo = 2 * i - (i & (stride - 1));
        const int hi = lo + stride;
        const bool up = (lo & size) == 0;
        const uint64_t a = k[lo], b = k[hi];
        if ((a > b) == up) {
          k[lo] = b;
          k[hi] = a;
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < kSortChunk; i += kSortBlock) {
    const uint64_t g = base + i;
    if (g < n) keys[g] = k[i];
  }
}

__global__ __launch_bounds__(256) void k_rank_scatter(const cbaa_host* stage, const uint64_t* keys,
                                                      const cbaa_restore_stats* stats,
                                                      uint64_t capacity, cbaa_host* out) {
  const uint64_t n = stats->n_hosts < capacity ? stats->n_hosts : capacity;
  const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const uint64_t key = keys[g];
  const uint64_t my_chunk = g / kSortChunk;
  uint64_t rank = g - my_chunk * kSortChunk;
  const uint64_t nchunks = (n + kSortChunk - 1) / kSortChunk;
  for (uint64_t c = 0; c < nchunks; ++c) {
    if (c == my_chunk) continue;
    uint64_t lo = c * kSortChunk;
    uint64_t hi = lo + kSortChunk < n ? lo + kSortChunk : n;
    while (lo < hi) {  // count keys < key in chunk c
      const uint64_t mid = (lo + hi) / 2;
      if (keys[mid] < key) lo = mid + 1; else hi = mid;
    }
    rank += lo - c * kSortChunk;
  }
  out[rank] = stage[(uint32_t)key];
}

// ---- point estimates ------------------------------------------------------

template <int NRA, int NVA, int RPL>
__global__ __launch_bounds__(256) void k_estimate(Dims d, const uint64_t* __restrict__ cube,
                                                  const uint32_t* __restrict__ hosts, uint64_t n,
                                                  const double* __restrict__ eps, double* est,
                                                  uint16_t* zeros, uint16_t* layer) {
  constexpr int A = NRA + NVA;
  const uint64_t gw = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const uint64_t nw = ((uint64_t)gridDim.x * blockDim.x) / kWave;
  for (uint64_t k = gw; k < n; k += nw) {
    uint32_t slot[A];
    const uint32_t cs = host_slots<NRA, NVA>(d, hosts[k], slot);
    Col<RPL> u;
#pragma unroll
    for (int q = 0; q < RPL; ++q) u.w[q] = ~0ull;
#pragma unroll
    for (int a = 0; a < A; ++a) {
      Col<RPL> c;
      load_col<RPL>(d, cube, cs, slot[a], c);
      if (layer) {
        const uint32_t za = col_zeros<RPL>(d, c);
        if (lane_id() == 0) layer[k * A + a] = (uint16_t)za;
      }
#pragma unroll
      for (int q = 0; q < RPL; ++q) u.w[q] &= c.w[q];
    }
    const uint32_t z = col_zeros<RPL>(d, u);
    if (lane_id() == 0) {
      const double g = (double)d.g;
      const uint32_t zc = z == 0 ? 1u : z;
      double e = -g * log((double)zc / (g - g * eps[cs]));
      est[k] = e < 0.0 ? 0.0 : e;
      zeros[k] = (uint16_t)z;
    }
  }
}

int check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? CBAA_OK : hip_fail(e, what);
}

int run_scan(const Dims& d, const uint64_t* cube, uint16_t* zeros, hipStream_t s) {
  const uint32_t half_w = d.W / 2;
  dim3 grid((half_w + kScanBlock - 1) / kScanBlock, d.S);
  hipLaunchKernelGGL(k_column_zeros, grid, dim3(kScanBlock), 0, s, d, (const uint4*)cube,
                     (uint32_t*)zeros);
  return check_launch("column scan launch");
}

template <int NRA, int NVA>
int dispatch_rpl_join(const Dims& d, const JoinArgs& ja, hipStream_t s) {
  const uint32_t grid = 2048;  // 8 waves per CU on 256 CUs; waves stride over the work list
#define CBAA_JOIN(RPL)                                                                  \
  if (d.R <= RPL * kWave) {                                                             \
    hipLaunchKernelGGL((k_join<NRA, NVA, RPL>), dim3(grid / (kJoinBlock / kWave)),      \
                       dim3(kJoinBlock), 0, s, d, ja);                                  \
    return check_launch("join launch");                                                \
  }
  CBAA_JOIN(1) CBAA_JOIN(2) CBAA_JOIN(4) CBAA_JOIN(8)
#undef CBAA_JOIN
  return CBAA_ECONFIG;
}

template <int NRA, int NVA>
int dispatch_rpl_est(const Dims& d, const uint64_t* cube, const uint32_t* hosts, uint64_t n,
                     const double* eps, double* est, uint16_t* zeros, uint16_t* layer,
                     hipStream_t s) {
  uint64_t blocks = (n + 3) / 4;  // 4 waves per block
  if (blocks > 4096) blocks = 4096;
#define CBAA_EST(RPL)                                                                        \
  if (d.R <= RPL * kWave) {                                                                  \
    hipLaunchKernelGGL((k_estimate<NRA, NVA, RPL>), dim3((uint32_t)blocks), dim3(256), 0, s, \
                       d, cube, hosts, n, eps, est, zeros, layer);                           \
    return check_launch("estimate launch");                                                 \
  }
  CBAA_EST(1) CBAA_EST(2) CBAA_EST(4) CBAA_EST(8)
#undef CBAA_EST
  return CBAA_ECONFIG;
}

#define CBAA_ARRAY_DISPATCH(FN, ...)                                              \
  do {                                                                            \
    if (d.n_ra == 2 && d.n_va == 0) return FN<2, 0>(__VA_ARGS__);                 \
    if (d.n_ra == 2 && d.n_va == 1) return FN<2, 1>(__VA_ARGS__);                 \
    if (d.n_ra == 2 && d.n_va == 2) return FN<2, 2>(__VA_ARGS__);                 \
    if (d.n_ra == 3 && d.n_va == 0) return FN<3, 0>(__VA_ARGS__);                 \
    if (d.n_ra == 3 && d.n_va == 1) return FN<3, 1>(__VA_ARGS__);                 \
    if (d.n_ra == 3 && d.n_va == 2) return FN<3, 2>(__VA_ARGS__);                 \
    if (d.n_ra == 4 && d.n_va == 0) return FN<4, 0>(__VA_ARGS__);                 \
    if (d.n_ra == 4 && d.n_va == 1) return FN<4, 1>(__VA_ARGS__);                 \
    if (d.n_ra == 4 && d.n_va == 2) return FN<4, 2>(__VA_ARGS__);                 \
    return CBAA_ECONFIG;                                                          \
  } while (0)

int run_join(const Dims& d, const JoinArgs& ja, hipStream_t s) {
  CBAA_ARRAY_DISPATCH(dispatch_rpl_join, d, ja, s);
}

int run_est(const Dims& d, const uint64_t* cube, const uint32_t* hosts, uint64_t n,
            const double* eps, double* est, uint16_t* zeros, uint16_t* layer, hipStream_t s) {
  CBAA_ARRAY_DISPATCH(dispatch_rpl_est, d, cube, hosts, n, eps, est, zeros, layer, s);
}

}  // namespace

uint64_t restore_scratch_bytes(const Dims& d, uint64_t capacity) {
  return carve(d, nullptr, capacity).bytes;
}

int launch_column_zeros(const Dims& d, const uint64_t* cube, uint16_t* zeros, uint32_t* ones,
                        hipStream_t s) {
  int rc = run_scan(d, cube, zeros, s);
  if (rc != CBAA_OK) return rc;
  // array fills only: no threshold, no hot lists
  hipLaunchKernelGGL(k_prepare, dim3(d.S), dim3(kPrepBlock), 0, s, d, zeros, ones,
                     (double*)nullptr, (int32_t*)nullptr, (uint32_t*)nullptr,
                     (uint16_t*)nullptr, 1.0, 0, 0, (cbaa_restore_stats*)nullptr);
  return check_launch("fill reduction launch");
}

int launch_restore(const Dims& d, const uint64_t* cube, double x, int rule, void* scratch,
                   uint64_t capacity, cbaa_host* out, cbaa_restore_stats* stats, hipStream_t s) {
  RestoreScratch rs = carve(d, scratch, capacity);
  hipLaunchKernelGGL(k_reset_stats, dim3(1), dim3(64), 0, s, stats);
  int rc = check_launch("reset launch");
  if (rc == CBAA_OK) rc = run_scan(d, cube, rs.zeros, s);
  if (rc != CBAA_OK) return rc;
  hipLaunchKernelGGL(k_prepare, dim3(d.S), dim3(kPrepBlock), 0, s, d, rs.zeros, rs.ones, rs.eps,
                     rs.zmax, rs.hcnt, rs.hot, x, rule, 1, stats);
  if ((rc = check_launch("prepare launch")) != CBAA_OK) return rc;
  JoinArgs ja{cube, rs.hot, rs.hcnt, rs.zmax, rs.eps, rs.stage, capacity, stats};
  if ((rc = run_join(d, ja, s)) != CBAA_OK) return rc;
  if (capacity == 0) return CBAA_OK;
  const uint32_t nchunks = (uint32_t)((capacity + kSortChunk - 1) / kSortChunk);
  hipLaunchKernelGGL(k_sort_chunks, dim3(nchunks), dim3(kSortBlock), 0, s, rs.stage, stats,
                     capacity, rs.keys);
  if ((rc = check_launch("sort launch")) != CBAA_OK) return rc;
  hipLaunchKernelGGL(k_rank_scatter, dim3((uint32_t)((capacity + 255) / 256)), dim3(256), 0, s,
                     rs.stage, rs.keys, stats, capacity, out);
  return check_launch("scatter launch");
}

int launch_estimate(const Dims& d, const uint64_t* cube, const uint32_t* hosts, uint64_t n,
                    double* est, uint16_t* zeros, uint16_t* layer_zeros, void* scratch,
                    hipStream_t s) {
  RestoreScratch rs = carve(d, scratch, 0);
  int rc = run_scan(d, cube, rs.zeros, s);
  if (rc != CBAA_OK) return rc;
  hipLaunchKernelGGL(k_prepare, dim3(d.S), dim3(kPrepBlock), 0, s, d, rs.zeros, rs.ones, rs.eps,
                     rs.zmax, rs.hcnt, rs.hot, 1.0, CBAA_THR_THM2, 0,
                     (cbaa_restore_stats*)nullptr);
  if ((rc = check_launch("prepare launch")) != CBAA_OK) return rc;
  return run_est(d, cube, hosts, n, rs.eps, est, zeros, layer_zeros, s);
}

}  // namespace cbaa
