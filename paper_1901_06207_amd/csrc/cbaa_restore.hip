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
constexpr uint32_t kJoinWaves = 2048;    // join grid: 8 waves per CU on 256 CUs
constexpr uint32_t kSmallSort = 32768;   // lists up to this size are ranked all-pairs
constexpr uint32_t kBuckets = 65536;     // larger lists: buckets by the IP's top 16 bits
constexpr uint32_t kGatherCap = 1024;    // hot columns per (sketch, RA) list gathered
constexpr uint64_t kGatherBytes = 256ull << 20;

inline uint64_t align256(uint64_t x) { return (x + 255u) & ~uint64_t(255u); }

// Scratch carve-up shared by restore and estimate.
struct RestoreScratch {
  uint16_t* zeros;  // [S][W]
  uint32_t* ones;   // [S][A]
  double* eps;      // [S]
  int32_t* zmax;    // [S]
  uint32_t* hcnt;   // [S][n_ra]
  uint16_t* hot;    // [S][n_ra][maxc_ra]
  uint32_t* gfit;   // [S][n_ra] 1 if the list was gathered into hcol
  uint64_t* hcol;   // [S][n_ra][gcap][R] gathered hot columns, contiguous
  uint32_t gcap;    // hot columns per list the gather buffer holds
  uint32_t* rows;   // [S][A][g] columns of each array with each bit set (features)
  double* shared;   // [S] row-aware shared-bit mass (features)
  cbaa_host* stage; // [capacity]
  cbaa_host* wbuf;  // [kJoinWaves][kWave]: hosts each join wave found, by wave
  uint32_t* wcnt;   // [kJoinWaves]: how many of its slots each wave filled
  uint64_t* keys;   // [capacity]: index and IP of each entry, bucket-ordered
  uint32_t* bucket; // [2][kBuckets + 1]: starts, fills
  uint64_t* work;   // [1]: tuples the tuple check has examined (budget)
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
  r.gfit = (uint32_t*)take((uint64_t)d.S * d.n_ra * 4);
  const uint64_t per_col = (uint64_t)d.S * d.n_ra * d.R * 8;
  uint64_t gcap = kGatherBytes / per_col;
  if (gcap > kGatherCap) gcap = kGatherCap;
  if (gcap > d.maxc_ra) gcap = d.maxc_ra;
  r.gcap = (uint32_t)gcap;
  r.hcol = (uint64_t*)take(gcap * per_col);
  r.rows = (uint32_t*)take((uint64_t)d.S * d.A * d.g * 4);
  r.shared = (double*)take((uint64_t)d.S * 8);
  r.stage = (cbaa_host*)take(capacity * sizeof(cbaa_host));
  r.wbuf = (cbaa_host*)take((uint64_t)kJoinWaves * kWave * sizeof(cbaa_host));
  r.wcnt = (uint32_t*)take((uint64_t)kJoinWaves * 4);
  r.keys = (uint64_t*)take(capacity * 8);
  r.bucket = (uint32_t*)take(2ull * (kBuckets + 1) * 4);
  r.work = (uint64_t*)take(8);
  r.bytes = off;
  return r;
}

// Sum over the wave with DPP row shifts: after shifts by 1, 2, 4 and 8 lanes
// inside each row of 16, the last lane of a row holds the row's total (lanes
// whose source falls outside the row add 0); the four totals are read back as
// wave-uniform values. The result is the same in every lane.
__device__ inline uint32_t wave_sum(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);  // row_shr:1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);  // row_shr:2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);  // row_shr:4
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);  // row_shr:8
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 15) +
         (uint32_t)__builtin_amdgcn_readlane((int)v, 31) +
         (uint32_t)__builtin_amdgcn_readlane((int)v, 47) +
         (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

__device__ inline uint32_t lane_id() { return __lane_id(); }

// Inclusive prefix sum over the wave: DPP row shifts give the prefix inside
// each row of 16 lanes (as in wave_sum), then the totals of the rows before a
// lane's row are added from wave-uniform reads.
__device__ inline uint32_t wave_inclusive_scan(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);  // row_shr:1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);  // row_shr:2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);  // row_shr:4
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);  // row_shr:8
  const uint32_t r0 = (uint32_t)__builtin_amdgcn_readlane((int)v, 15);
  const uint32_t r1 = (uint32_t)__builtin_amdgcn_readlane((int)v, 31);
  const uint32_t r2 = (uint32_t)__builtin_amdgcn_readlane((int)v, 47);
  const uint32_t row = lane_id() >> 4;
  return v + (row > 0 ? r0 : 0u) + (row > 1 ? r1 : 0u) + (row > 2 ? r2 : 0u);
}

// ---- per-column zero counts ---------------------------------------------
// Thread (cs, w..w+1): popcounts of two neighbouring columns' words over all
// R row blocks (16 loads in flight); a wave reads 1 KiB contiguous per row
// block. Each array's one-bit total is accumulated into ones[cs][a] (zeroed
// beforehand) through an LDS partial per block.
__global__ __launch_bounds__(kScanBlock) void k_column_zeros(Dims d, const uint4* __restrict__ cube,
                                                             uint32_t* __restrict__ zeros2,
                                                             uint32_t* __restrict__ ones) {
  __shared__ uint32_t part[CBAA_MAX_ARRAYS];
  const uint32_t cs = blockIdx.y;
  if (threadIdx.x < CBAA_MAX_ARRAYS) part[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t pair = blockIdx.x * kScanBlock + threadIdx.x;  // column pair index
  const uint32_t half_w = d.W / 2;
  if (pair < half_w) {
    uint32_t c0 = 0, c1 = 0;
    const uint4* p = cube + ((uint64_t)cs * d.R) * half_w + pair;
    uint32_t rb = 0;
    constexpr uint32_t kU = 16;
    for (; rb + kU <= d.R; rb += kU) {
      uint4 v[kU];
#pragma unroll
      for (uint32_t u = 0; u < kU; ++u) v[u] = load_stream(p + (uint64_t)(rb + u) * half_w);
#pragma unroll
      for (uint32_t u = 0; u < kU; ++u) {
        c0 += __popc(v[u].x) + __popc(v[u].y);
        c1 += __popc(v[u].z) + __popc(v[u].w);
      }
    }
    for (; rb < d.R; ++rb) {
      const uint4 v = load_stream(p + (uint64_t)rb * half_w);
      c0 += __popc(v.x) + __popc(v.y);
      c1 += __popc(v.z) + __popc(v.w);
    }
    zeros2[(uint64_t)cs * half_w + pair] = (d.g - c0) | ((d.g - c1) << 16);
    // both columns lie in one array: array offsets are even
    const uint32_t w = 2 * pair;
    uint32_t a = 0;
    while (a + 1 < d.A && w >= d.aoff[a + 1]) ++a;
    atomicAdd(&part[a], c0 + c1);
  }
  __syncthreads();
  if (threadIdx.x < d.A && part[threadIdx.x])
    atomicAdd(&ones[cs * d.A + threadIdx.x], part[threadIdx.x]);
}

// The global server's OR-merge and the column scan in one pass: the same
// walk as k_column_zeros, each 16-byte unit being the OR of up to 16 source
// cubes, stored to dst (unless dst is null) and then counted. dst may be one
// of the sources: every unit is read from all sources by the thread that
// writes it.
constexpr int kMergeScanSources = 16;

struct MergeSrc {
  const uint4* p[kMergeScanSources];
};

// Where the restore reads cube words after the scan: the OR of k cubes
// (k = 1: one stored cube; k > 1: router cubes whose merge was not stored).
struct CubeSrc {
  const uint64_t* p[kMergeScanSources];
  int k;
};

__device__ inline uint64_t cube_word(const CubeSrc& c, uint64_t i) {
  // the first two sources are read with no branch between them (one cube:
  // the same word twice), so both loads are in flight together
  const uint64_t* p1 = c.k > 1 ? c.p[1] : c.p[0];
  uint64_t v = c.p[0][i] | p1[i];
  for (int j = 2; j < c.k; ++j) v |= c.p[j][i];
  return v;
}

__global__ __launch_bounds__(kScanBlock) void k_merge_scan(Dims d, MergeSrc src, int k, uint4* dst,
                                                           uint32_t* __restrict__ zeros2,
                                                           uint32_t* __restrict__ ones) {
  __shared__ uint32_t part[CBAA_MAX_ARRAYS];
  const uint32_t cs = blockIdx.y;
  if (threadIdx.x < CBAA_MAX_ARRAYS) part[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t pair = blockIdx.x * kScanBlock + threadIdx.x;  // column pair index
  const uint32_t half_w = d.W / 2;
  if (pair < half_w) {
    uint32_t c0 = 0, c1 = 0;
    const uint64_t first = ((uint64_t)cs * d.R) * half_w + pair;
    constexpr uint32_t kU = 8;
    for (uint32_t rb0 = 0; rb0 < d.R; rb0 += kU) {
      uint4 v[kU];
#pragma unroll
      for (uint32_t u = 0; u < kU; ++u) v[u] = make_uint4(0u, 0u, 0u, 0u);
      for (int j = 0; j < k; ++j) {
#pragma unroll
        for (uint32_t u = 0; u < kU; ++u) {
          if (rb0 + u >= d.R) break;
          const uint4 w = load_stream(src.p[j] + first + (uint64_t)(rb0 + u) * half_w);
          v[u].x |= w.x;
          v[u].y |= w.y;
          v[u].z |= w.z;
          v[u].w |= w.w;
        }
      }
#pragma unroll
      for (uint32_t u = 0; u < kU; ++u) {
        if (rb0 + u >= d.R) break;
        if (dst) store_stream(dst + first + (uint64_t)(rb0 + u) * half_w, v[u]);
        c0 += __popc(v[u].x) + __popc(v[u].y);
        c1 += __popc(v[u].z) + __popc(v[u].w);
      }
    }
    zeros2[(uint64_t)cs * half_w + pair] = (d.g - c0) | ((d.g - c1) << 16);
    const uint32_t w = 2 * pair;
    uint32_t a = 0;
    while (a + 1 < d.A && w >= d.aoff[a + 1]) ++a;
    atomicAdd(&part[a], c0 + c1);
  }
  __syncthreads();
  if (threadIdx.x < d.A && part[threadIdx.x])
    atomicAdd(&ones[cs * d.A + threadIdx.x], part[threadIdx.x]);
}

// Per-sketch eps (Thm. 1 with the measured fills) and Zmax, in fp64 with the
// operations in the order the oracle uses.
__device__ inline int32_t sketch_threshold(const Dims& d, const uint32_t* ones, uint32_t cs,
                                           double x, int rule, double* eps_out) {
  const double g = (double)d.g;
  double e = 1.0;
  for (uint32_t a = 0; a < d.A; ++a)
    e = e * ((double)ones[cs * d.A + a] / ((double)d.ncol[a] * g));
  double zf;
  if (rule == CBAA_THR_PAPER)
    zf = (g + g * e) * x - g * e;
  else
    zf = (g - g * e) * x;
  *eps_out = e;
  return zf < 0.0 ? -1 : (int32_t)floor(zf);
}

// Block (cs, i, part): Zmax of sketch cs and the ascending hot-column list of
// RA i (Alg. 2) by ordered ballot compaction; every part builds the list, part
// 0 stores it (and block (cs, 0, 0) stores eps, Zmax). A list of at most gcap
// columns is then copied column by column (R words strided by W in the cube)
// into a contiguous run of hcol, where the tuple join finds every hot column
// of the list in 512 B at the paper's g; gfit records whether it was. The
// copy is split over the parts, row block by row block, so that neighbouring
// threads read neighbouring hot columns of one row block.
constexpr uint32_t kPrepParts = 4;
__global__ __launch_bounds__(kPrepBlock) void k_prepare(Dims d, const uint16_t* __restrict__ zeros,
                                                        const uint32_t* __restrict__ ones,
                                                        double* eps, int32_t* zmax, uint32_t* hcnt,
                                                        uint16_t* hot, double x, int rule,
                                                        cbaa_restore_stats* stats,
                                                        CubeSrc cube, uint64_t* hcol,
                                                        uint32_t gcap, uint32_t* gfit) {
  __shared__ uint32_t wave_cnt[kPrepBlock / kWave];
  __shared__ uint16_t s_list[kGatherCap];
  const uint32_t cs = blockIdx.x;
  const uint32_t i = blockIdx.y;
  const bool lead = blockIdx.z == 0;
  double e;
  int32_t zm = sketch_threshold(d, ones, cs, x, rule, &e);
  // a cube read without this configuration's valid header restores nothing:
  // no column is hot
  if (stats && (stats->status & CBAA_STATUS_CONFIG)) zm = -1;
  if (lead && i == 0 && threadIdx.x == 0) {
    eps[cs] = e;
    zmax[cs] = zm;
  }
  if (!hot) return;
  const uint16_t* z = zeros + (uint64_t)cs * d.W + d.aoff[i];
  const int wid = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  uint16_t* out = hot + ((uint64_t)cs * d.n_ra + i) * d.maxc_ra;
  uint32_t base = 0;
  for (uint32_t t0 = 0; t0 < d.ncol[i]; t0 += blockDim.x) {
    const uint32_t j = t0 + threadIdx.x;
    const bool pred = j < d.ncol[i] && (int32_t)z[j] <= zm;
    const uint64_t bal = __ballot(pred);
    const uint32_t before = __popcll(bal & ((1ull << lane_id()) - 1ull));
    if (lane_id() == 0) wave_cnt[wid] = __popcll(bal);
    __syncthreads();
    uint32_t woff = 0, total = 0;
    for (int w = 0; w < nw; ++w) {
      if (w < wid) woff += wave_cnt[w];
      total += wave_cnt[w];
    }
    const uint32_t at = base + woff + before;
    if (pred) {
      if (lead) out[at] = (uint16_t)j;
      if (at < kGatherCap) s_list[at] = (uint16_t)j;
    }
    base += total;
    __syncthreads();
  }
  if (lead && threadIdx.x == 0) {
    hcnt[cs * d.n_ra + i] = base;
    if (stats)
      __hip_atomic_fetch_add(&stats->hot_columns, (uint64_t)base, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
  }
  if (!hcol) return;
  const bool fit = base <= gcap;   // base is the same in every thread
  if (lead && threadIdx.x == 0) gfit[cs * d.n_ra + i] = fit ? 1u : 0u;
  if (!fit) return;
  // s_list was written before the last barrier; gcap <= kGatherCap
  const uint64_t src = (uint64_t)cs * d.R * d.W + d.aoff[i];   // word index in the cube
  uint64_t* dst = hcol + ((uint64_t)cs * d.n_ra + i) * gcap * d.R;
  const uint32_t n = base * d.R;
  const uint32_t stride = gridDim.z * blockDim.x;
  constexpr int U = 4;   // loads in flight per thread
  uint32_t j = blockIdx.z * blockDim.x + threadIdx.x;
  for (; j + (U - 1) * stride < n; j += U * stride) {
    uint64_t v[U];
    uint32_t at[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t jj = j + u * stride;
      const uint32_t rb = jj / base, pos = jj - rb * base;
      v[u] = cube_word(cube, src + (uint64_t)rb * d.W + s_list[pos]);
      at[u] = pos * d.R + rb;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) dst[at[u]] = v[u];
  }
  for (; j < n; j += stride) {
    const uint32_t rb = j / base, pos = j - rb * base;
    dst[pos * d.R + rb] = cube_word(cube, src + (uint64_t)rb * d.W + s_list[pos]);
  }
}

// Zeroes the counters and the fill accumulators. With stats, it also checks
// the headers of the cubes the restore reads (status CBAA_STATUS_CONFIG if any
// lacks this configuration's valid one) and writes the header of the stored
// merge, if any (valid only when every source's is). A source that is the
// merge's destination has its header read before it is written, by the same
// thread.
__global__ void k_reset(Dims d, cbaa_restore_stats* st, uint32_t* ones, uint32_t n_ones,
                        uint64_t* work, CubeSrc src, uint64_t* dst) {
  if (st && threadIdx.x == 0) {
    st->n_hosts = 0;
    st->hot_columns = 0;
    st->partial_checked = 0;
    st->tuples_checked = 0;
    st->tuple_space = 0;
    bool ok = true;
    for (int j = 0; j < src.k; ++j) ok = ok && header_ok(header_of(src.p[j]), d);
    st->status = ok ? 0u : CBAA_STATUS_CONFIG;
    if (dst) header_set(header_of(dst), d, ok ? CBAA_CUBE_VALID : CBAA_CUBE_MIXED);
  }
  if (work && threadIdx.x == 0) *work = 0;
  for (uint32_t i = threadIdx.x; i < n_ones; i += blockDim.x) ones[i] = 0;
}

// ---- tuple join and union-column verification (Alg. 3) ------------------
//
// A wave takes work items, each a hot column hc0 of RA 0 with one 64-entry
// window of the RA 1 hot list, and walks the tuples that extend hc0 through
// that window, RA by RA: candidates of RA l are screened 64 at a time by the
// CP check
// of Alg. 3 against hc_{l-1} (and, for the last RA, against hc_0), then the
// AND of the columns chosen so far is counted. Because AND can only add zero
// bits, a partial tuple whose AND already has more than Zmax zeros cannot
// complete to an accepted tuple and is dropped: the accepted set is exactly
// Alg. 3's. Lane q of the wave holds row blocks q, q+64, ...
//
// The wave's time is a chain of dependent memory round trips, so the walk is
// arranged to keep that chain short:
// * the first kListRegs * 64 entries of every hot list are held in registers,
//   so the CP screens read no memory;
// * complete CP-valid tuples are not checked one prefix at a time but queued,
//   and a full queue is checked at once: the columns of all its tuples and the
//   scan's zero counts of their VA columns are loaded together, then the VA
//   columns of the tuples that pass;
// * the column loads of a candidate batch or of a queue have no branch
//   between them, so they are in flight together;
// * counts over the wave are summed with DPP row shifts, not LDS permutes.

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
__device__ inline void load_col(const Dims& d, const CubeSrc& cube, uint32_t cs, uint32_t slot,
                                Col<RPL>& c) {
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    const uint32_t rb = lane_id() + q * kWave;
    c.w[q] = rb < d.R ? cube_word(cube, ((uint64_t)cs * d.R + rb) * d.W + slot) : ~0ull;
  }
}

template <int RPL>
__device__ inline void and_col(Col<RPL>& a, const Col<RPL>& b) {
#pragma unroll
  for (int r = 0; r < RPL; ++r) a.w[r] &= b.w[r];
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
  CubeSrc cube;
  const uint16_t* zeros;  // [S][W] per-column zero counts of the scan
  const uint16_t* hot;
  const uint64_t* hcol;   // gathered hot columns ([S][n_ra][gcap][R])
  const uint32_t* gfit;   // [S][n_ra] list gathered
  uint32_t gcap;
  const uint32_t* hcnt;
  const int32_t* zmax;
  const double* eps;
  cbaa_host* stage;
  cbaa_host* wbuf;
  uint32_t* wcnt;
  uint64_t capacity;
  cbaa_restore_stats* stats;
  uint64_t* work;         // tuples examined so far, over all waves
  uint64_t max_checks;    // work budget
};

// Output entry of a restored host: IP reassembled from its sketch and LP
// (Alg. 3), Z of its union column, the Thm. 2 estimate.
__device__ inline cbaa_host make_host(const Dims& d, const JoinArgs& ja, uint32_t cs, uint32_t lp,
                                      uint32_t z) {
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
  return h;
}

// Hosts a wave has found and not yet written: entry k sits in lane k. One
// output counter shared by every wave serialises its increments (tens of ns
// each), so a wave takes slots from it only when all 64 lanes are full; what
// it holds at the end goes to its own region of wbuf, and k_compact appends
// the regions after the counter's slots.
struct Found {
  uint32_t lp, z, cs;  // this lane's entry
  uint32_t n;          // wave-uniform
};

__device__ inline void write_found(const Dims& d, const JoinArgs& ja, Found& f) {
  uint64_t base = 0;
  if (lane_id() == 0)
    base = __hip_atomic_fetch_add(&ja.stats->n_hosts, (uint64_t)f.n, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
  base = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(base >> 32)) << 32) |
         (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)base);
  const uint64_t idx = base + lane_id();
  if (lane_id() < f.n && idx < ja.capacity) ja.stage[idx] = make_host(d, ja, f.cs, f.lp, f.z);
  f.n = 0;
}

__device__ inline void emit_host(const Dims& d, const JoinArgs& ja, Found& f, uint32_t cs,
                                 uint32_t lp, uint32_t z) {
  if (lane_id() == f.n) {
    f.lp = lp;
    f.z = z;
    f.cs = cs;
  }
  if (++f.n == (uint32_t)kWave) write_found(d, ja, f);
}

// Column `col` at position `pos` of the hot list of RA `level` in sketch cs:
// from the gathered copy (G: every list of the restore fit the gather
// buffer) or straight from the cube. G is a compile-time choice so that a
// batch's loads have no branch between them and are in flight together.
template <int RPL, bool G>
__device__ inline void load_hot(const Dims& d, const JoinArgs& ja, uint32_t cs, uint32_t level,
                                uint32_t pos, uint32_t col, Col<RPL>& c) {
  if constexpr (G) {
    const uint64_t* src = ja.hcol + (((uint64_t)cs * d.n_ra + level) * ja.gcap + pos) * d.R;
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const uint32_t rb = lane_id() + q * kWave;
      c.w[q] = rb < d.R ? src[rb] : ~0ull;
    }
  } else {
    load_col<RPL>(d, ja.cube, cs, d.aoff[level] + col, c);
  }
}

// Candidates of an intermediate RA that pass the CP screen are taken kBatch
// (BatchLen<RPL>: 2 when a column takes 8 registers per lane)
// at a time so their column loads are in flight together; complete tuples
// are queued kQueue<RPL> at a time (fewer when a column takes more
// registers per lane).
template <int RPL>
struct BatchLen {
  static constexpr int value = RPL >= 8 ? 2 : 4;
};
constexpr int kListRegs = 4;
template <int RPL>
struct QueueLen {
  static constexpr int value = RPL <= 2 ? 4 : (RPL == 4 ? 2 : 1);
};

// Everything one wave keeps while it walks the tuples of one hc0.
template <int NRA, int RPL>
struct Walk {
  static constexpr int Q = QueueLen<RPL>::value;
  uint32_t cs;
  int32_t zm;
  Col<RPL> c0;                       // column hc0, whole
  uint32_t cnt[NRA];                 // |HC(i)|
  const uint16_t* list[NRA];         // HC(i) in ascending order
  uint32_t reg[NRA][kListRegs];      // HC(i)[lane + 64 k], k < kListRegs
  uint32_t b1_lo, b1_hi;             // this item's window of HC(1) positions
  uint32_t t[NRA];                   // columns of the tuple being extended
  uint32_t tp[NRA];                  // their positions in HC(i)
  uint32_t qc[Q][NRA];               // queued complete tuples in slots
  uint32_t qp[Q][NRA];               // [0, nq): columns and positions (RA 0 unused)
  int nq;
  uint32_t n_partial, n_tuples;
  uint32_t pending;                  // tuples examined since the last report
  bool stop;                         // the work budget is spent: unwind
  Found found;
};

// Work budget, counted in tuples examined: partial tuples whose AND is
// counted and complete CP-valid tuples (queued for the VA test and the union
// column). At the start of every 64-candidate round of a hot list, a wave
// that has examined kBudgetStep or more tuples since its last report adds
// them to the shared counter; when the total passes the budget, the wave
// stops (the rounds, the kept-candidate loop and the item loop test `stop`)
// and the restore is flagged incomplete. A round examines at most 64 tuples
// before the next round of some list starts, so every wave that keeps working
// notices within kBudgetStep + 64 tuples and the grid drains soon after.
constexpr uint32_t kBudgetStep = 256;
template <int NRA, int RPL>
__device__ inline void spend(const JoinArgs& ja, Walk<NRA, RPL>& w) {
  if (w.pending < kBudgetStep) return;
  uint64_t before = 0;
  if (lane_id() == 0)
    before = __hip_atomic_fetch_add(ja.work, (uint64_t)w.pending, __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT);
  before = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(before >> 32)) << 32) |
           (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)before);
  if (before + w.pending > ja.max_checks) {
    w.stop = true;
    if (lane_id() == 0)
      __hip_atomic_fetch_or(&ja.stats->status, (uint64_t)CBAA_STATUS_BUDGET, __ATOMIC_RELAXED,
                            __HIP_MEMORY_SCOPE_AGENT);
  }
  w.pending = 0;
}

// Screens HC(LEVEL) 64 entries at a time: `round(cand, valid, base)` is
// called with entry base + lane of the list. The first kListRegs rounds take
// their entries from registers (shifted down one round at a time, so no
// register is ever picked by a run-time index), later rounds from memory.
// HC(1) is screened only inside the item's window [b1_lo, b1_hi).
template <int NRA, int RPL, int LEVEL, typename F>
__device__ __attribute__((always_inline)) void for_list(const JoinArgs& ja, Walk<NRA, RPL>& w,
                                                        F&& round) {
  uint32_t r[kListRegs];
#pragma unroll
  for (int k = 0; k < kListRegs; ++k) r[k] = w.reg[LEVEL][k];
  const uint32_t cnt = w.cnt[LEVEL];
  for (uint32_t base = 0; base < cnt; base += kWave) {
    spend(ja, w);
    if (w.stop) break;
    const uint32_t j = base + lane_id();
    uint32_t cand;
    if (base < (uint32_t)(kListRegs * kWave)) {
      cand = r[0];
#pragma unroll
      for (int k = 0; k + 1 < kListRegs; ++k) r[k] = r[k + 1];
    } else {
      if (LEVEL == 1 && base < w.b1_lo) continue;
      cand = j < cnt ? w.list[LEVEL][j] : 0u;
    }
    if (LEVEL == 1 && base >= w.b1_hi) break;
    if (LEVEL == 1 && base < w.b1_lo) continue;
    round(cand, j < cnt, base);
  }
}

// Checks every queued tuple: AND of its RA columns with hc0, the VA
// zero-count test, the VA columns, the count against Zmax, the output.
template <int NRA, int NVA, int RPL, bool G>
__device__ __attribute__((always_inline)) void check_queue(const Dims& d, const JoinArgs& ja, Walk<NRA, RPL>& w) {
  constexpr int Q = Walk<NRA, RPL>::Q;
  Col<RPL> acc[Q];
  uint32_t lp[Q];
  int32_t zva[Q];
  // every slot is loaded, the empty ones (q >= nq) repeating slot 0, so that
  // no branch separates the loads
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const bool live = q < w.nq;
    uint32_t col[NRA], pos[NRA];
#pragma unroll
    for (int i = 1; i < NRA; ++i) {
      col[i] = live ? w.qc[q][i] : w.qc[0][i];
      pos[i] = live ? w.qp[q][i] : w.qp[0][i];
    }
    // LP = concatenation of the EPs
    uint32_t x = rotl_in(w.t[0] & low_mask(d.ep[0]), d.off[0], d.L);
#pragma unroll
    for (int i = 1; i < NRA; ++i) x |= rotl_in(col[i] & low_mask(d.ep[i]), d.off[i], d.L);
    lp[q] = x;
    int32_t z = 0;
#pragma unroll
    for (int v = 0; v < NVA; ++v) {
      const int32_t zv = ja.zeros[(uint64_t)w.cs * d.W + d.aoff[NRA + v] + va_col(d, v, x)];
      z = zv > z ? zv : z;
    }
    zva[q] = z;
    acc[q] = w.c0;
#pragma unroll
    for (int i = 1; i < NRA; ++i) {
      Col<RPL> c;
      load_hot<RPL, G>(d, ja, w.cs, i, pos[i], col[i], c);
      and_col(acc[q], c);
    }
  }
  // the union column is contained in every VA column, so it has at least as
  // many zeros: a VA column over Zmax rejects the tuple before it is read
  Col<RPL> vc[Q][NVA > 0 ? NVA : 1];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    if (q >= w.nq) break;
    if (zva[q] > w.zm) continue;
#pragma unroll
    for (int v = 0; v < NVA; ++v)
      load_col<RPL>(d, ja.cube, w.cs, d.aoff[NRA + v] + va_col(d, v, lp[q]), vc[q][v]);
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    if (q >= w.nq) break;
    if (zva[q] > w.zm) continue;
#pragma unroll
    for (int v = 0; v < NVA; ++v) and_col(acc[q], vc[q][v]);
    ++w.n_tuples;
    const uint32_t z = col_zeros<RPL>(d, acc[q]);
    if ((int32_t)z <= w.zm) emit_host(d, ja, w.found, w.cs, lp[q], z);
  }
  w.nq = 0;
}

// Last RA: every CP-valid candidate completes a tuple, which is queued.
template <int NRA, int NVA, int RPL, bool G>
__device__ __attribute__((always_inline)) void extend_last(const Dims& d, const JoinArgs& ja, Walk<NRA, RPL>& w) {
  constexpr int L = NRA - 1;
  constexpr int Q = Walk<NRA, RPL>::Q;
  const uint32_t want_lo = w.t[L - 1] >> d.ep[L - 1];      // CP of hc_{l-1}
  const uint32_t cp_mask = low_mask(d.cp[L - 1]);
  const uint32_t want_hi = w.t[0] & low_mask(d.cp[L]);     // first bits of hc_0
  for_list<NRA, RPL, L>(ja, w, [&](uint32_t cand, bool valid, uint32_t base) {
    const bool ok = valid && (cand & cp_mask) == want_lo && (cand >> d.ep[L]) == want_hi;
    uint64_t m = __ballot(ok);
    while (m) {
      const int l = __builtin_ctzll(m);
      m &= m - 1;
      const uint32_t h = (uint32_t)__builtin_amdgcn_readlane((int)cand, l);
      // the queue shifts up one slot and the new tuple enters slot 0: no slot
      // is chosen by a run-time index
#pragma unroll
      for (int q = Q - 1; q > 0; --q) {
#pragma unroll
        for (int i = 1; i < NRA; ++i) {
          w.qc[q][i] = w.qc[q - 1][i];
          w.qp[q][i] = w.qp[q - 1][i];
        }
      }
#pragma unroll
      for (int i = 1; i < L; ++i) {
        w.qc[0][i] = w.t[i];
        w.qp[0][i] = w.tp[i];
      }
      w.qc[0][L] = h;
      w.qp[0][L] = base + (uint32_t)l;
      ++w.pending;
      if (++w.nq == Q) check_queue<NRA, NVA, RPL, G>(d, ja, w);
    }
  });
}

// Intermediate RA LEVEL (0 < LEVEL < NRA - 1): CP screen against hc_{l-1},
// then the AND with the prefix `acc`, pruned above Zmax.
template <int NRA, int NVA, int RPL, int LEVEL, bool G>
__device__ __attribute__((always_inline)) void extend(const Dims& d, const JoinArgs& ja, Walk<NRA, RPL>& w,
                       const Col<RPL>& acc) {
  constexpr int kBatch = BatchLen<RPL>::value;
  const uint32_t want_lo = w.t[LEVEL - 1] >> d.ep[LEVEL - 1];
  const uint32_t cp_mask = low_mask(d.cp[LEVEL - 1]);
  for_list<NRA, RPL, LEVEL>(ja, w, [&](uint32_t cand, bool valid, uint32_t base) {
    const bool ok = valid && (cand & cp_mask) == want_lo;
    uint64_t m = __ballot(ok);
    while (m) {
      uint32_t h[kBatch], pos[kBatch];
      int nb = 0;
#pragma unroll
      for (int q = 0; q < kBatch; ++q) {
        h[q] = 0;
        pos[q] = 0;
        if (m) {
          const int l = __builtin_ctzll(m);
          m &= m - 1;
          h[q] = (uint32_t)__builtin_amdgcn_readlane((int)cand, l);
          pos[q] = base + (uint32_t)l;
          nb = q + 1;
        }
      }
      // unused slots repeat slot 0, so the loads have no branch between them
#pragma unroll
      for (int q = 1; q < kBatch; ++q) {
        h[q] = q < nb ? h[q] : h[0];
        pos[q] = q < nb ? pos[q] : pos[0];
      }
      Col<RPL> c[kBatch];
#pragma unroll
      for (int q = 0; q < kBatch; ++q) load_hot<RPL, G>(d, ja, w.cs, LEVEL, pos[q], h[q], c[q]);
      uint32_t keep = 0;   // candidates whose partial AND is within Zmax
#pragma unroll
      for (int q = 0; q < kBatch; ++q) {
        if (q >= nb) break;
        and_col(c[q], acc);
        ++w.n_partial;
        ++w.pending;
        if ((int32_t)col_zeros<RPL>(d, c[q]) <= w.zm) keep |= 1u << q;
      }
      // the kept candidates are extended in order; each step shifts the
      // batch down one slot, so the one at hand is always slot 0 and the
      // deeper levels are emitted once, not once per slot
#pragma unroll 1
      for (int q = 0; q < nb; ++q) {
        if (w.stop) break;
        if (keep & 1u) {
          w.t[LEVEL] = h[0];
          w.tp[LEVEL] = pos[0];
          if constexpr (LEVEL + 1 < NRA - 1)
            extend<NRA, NVA, RPL, LEVEL + 1, G>(d, ja, w, c[0]);
          else
            extend_last<NRA, NVA, RPL, G>(d, ja, w);
        }
        keep >>= 1;
#pragma unroll
        for (int k = 0; k + 1 < kBatch; ++k) {
          c[k] = c[k + 1];
          h[k] = h[k + 1];
          pos[k] = pos[k + 1];
        }
      }
    }
  });
}

// The items of one wave (gw, gw + nwaves, ...) with hot columns read from
// the gathered copy (G) or from the cube.
template <int NRA, int NVA, int RPL, bool G>
__device__ __attribute__((always_inline)) void join_items(const Dims& d, const JoinArgs& ja,
                                                          Walk<NRA, RPL>& w, const uint32_t* pre,
                                                          uint32_t total0, uint32_t total,
                                                          uint32_t gw, uint32_t nwaves) {
  for (uint32_t item = gw; item < total; item += nwaves) {
    if (w.stop) break;
    const uint32_t win = item / total0, flat = item - win * total0;
    uint32_t lo = 0, hi = d.S;  // largest cs with pre[cs] <= flat
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) / 2;
      if (pre[mid] <= flat) lo = mid; else hi = mid;
    }
    w.cs = lo;
#pragma unroll
    for (int i = 0; i < NRA; ++i) {
      w.cnt[i] = ja.hcnt[w.cs * NRA + i];
      w.list[i] = ja.hot + ((uint64_t)w.cs * NRA + i) * d.maxc_ra;
    }
    w.b1_lo = win * kWave;
    w.b1_hi = w.b1_lo + kWave;
    if (w.b1_lo >= w.cnt[1]) continue;   // this sketch's HC(1) has fewer windows
    const uint32_t pos0 = flat - pre[w.cs];
    w.zm = ja.zmax[w.cs];
    w.t[0] = w.list[0][pos0];
    w.tp[0] = pos0;
#pragma unroll
    for (int i = 1; i < NRA; ++i) {
#pragma unroll
      for (int k = 0; k < kListRegs; ++k) {
        const uint32_t j = (uint32_t)k * kWave + lane_id();
        w.reg[i][k] = j < w.cnt[i] ? w.list[i][j] : 0u;
      }
    }
    load_hot<RPL, G>(d, ja, w.cs, 0, pos0, w.t[0], w.c0);
    w.nq = 0;
    if constexpr (NRA > 2)
      extend<NRA, NVA, RPL, 1, G>(d, ja, w, w.c0);
    else
      extend_last<NRA, NVA, RPL, G>(d, ja, w);
    if (w.nq) check_queue<NRA, NVA, RPL, G>(d, ja, w);
  }
}

template <int NRA, int NVA, int RPL>
__global__ __launch_bounds__(kJoinBlock) void k_join(Dims d, JoinArgs ja) {
  __shared__ uint32_t pre[257];
  __shared__ uint32_t s_rounds;
  // hot columns come from the gathered copy only if every list fit it
  uint32_t missed = 0;
  for (uint32_t i = lane_id(); i < d.S * NRA; i += kWave) missed |= ja.gfit[i] ^ 1u;
  const bool all_fit = __ballot(missed != 0) == 0;
  // Work items: (window of 64 positions of HC(1), cs, hc0), the window
  // outermost, so that the windows of one hc0 fall to different waves: a hot
  // column of RA 0 that extends to many tuples is spread over several waves.
  // pre: prefix over sketches of |HC(0)|; s_rounds: most windows of any HC(1).
  if (threadIdx.x == 0) {
    uint32_t acc = 0, rounds = 0;
    for (uint32_t cs = 0; cs < d.S; ++cs) {
      pre[cs] = acc;
      acc += ja.hcnt[cs * NRA + 0];
      const uint32_t r1 = (ja.hcnt[cs * NRA + 1] + kWave - 1) / kWave;
      rounds = r1 > rounds ? r1 : rounds;
    }
    pre[d.S] = acc;
    s_rounds = rounds;
    if (blockIdx.x == 0) {
      // tuples Alg. 3 would enumerate: sum over sketches of prod_i |HC(i)|
      uint64_t space = 0;
      for (uint32_t cs = 0; cs < d.S; ++cs) {
        uint64_t prod = 1;
        for (int i = 0; i < NRA; ++i) {
          const uint64_t c = ja.hcnt[cs * NRA + i];
          prod = (c != 0 && prod > ~0ull / c) ? ~0ull : prod * c;
        }
        space = space > ~0ull - prod ? ~0ull : space + prod;
      }
      ja.stats->tuple_space = space;
    }
  }
  __syncthreads();
  const uint32_t total0 = pre[d.S];
  const uint32_t total = total0 * s_rounds;
  const uint32_t waves_per_block = kJoinBlock / kWave;
  const uint32_t gw = blockIdx.x * waves_per_block + threadIdx.x / kWave;
  const uint32_t nwaves = gridDim.x * waves_per_block;
  Walk<NRA, RPL> w;
  w.n_partial = 0;
  w.n_tuples = 0;
  w.pending = 0;
  w.stop = false;
  w.found.n = 0;
  if (all_fit)
    join_items<NRA, NVA, RPL, true>(d, ja, w, pre, total0, total, gw, nwaves);
  else
    join_items<NRA, NVA, RPL, false>(d, ja, w, pre, total0, total, gw, nwaves);
  if (lane_id() < w.found.n)
    ja.wbuf[(uint64_t)gw * kWave + lane_id()] = make_host(d, ja, w.found.cs, w.found.lp, w.found.z);
  if (lane_id() == 0) ja.wcnt[gw] = w.found.n;
  if (lane_id() == 0 && (w.n_partial | w.n_tuples)) {
    __hip_atomic_fetch_add(&ja.stats->partial_checked, (uint64_t)w.n_partial, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(&ja.stats->tuples_checked, (uint64_t)w.n_tuples, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Appends every join wave's region of wbuf, in wave order, after the slots
// the waves took from the output counter, and sets the counter to the total.
// One block: the per-wave counts are prefixed (wave scans, then the wave
// totals), then each thread copies entries e, e + kCompactBlock, ..., finding
// the region of e by binary search.
constexpr int kCompactBlock = 1024;
__global__ __launch_bounds__(kCompactBlock) void k_compact(const cbaa_host* __restrict__ wbuf,
                                                           const uint32_t* __restrict__ wcnt,
                                                           cbaa_restore_stats* stats,
                                                           cbaa_host* stage, uint64_t capacity) {
  constexpr uint32_t kPer = kJoinWaves / kCompactBlock;
  constexpr uint32_t kWaves = kCompactBlock / kWave;
  static_assert(kPer * kCompactBlock == kJoinWaves, "regions split evenly over threads");
  __shared__ uint32_t wave_tot[kWaves];
  __shared__ uint32_t pre[kJoinWaves];   // first entry of each region
  __shared__ uint64_t s_flushed;         // slots the waves took while joining
  const uint32_t t = threadIdx.x, wid = t / kWave;
  uint32_t c[kPer], sum = 0;
#pragma unroll
  for (uint32_t k = 0; k < kPer; ++k) {
    c[k] = wcnt[t * kPer + k];
    sum += c[k];
  }
  if (t == 0) s_flushed = stats->n_hosts;
  const uint32_t incl = wave_inclusive_scan(sum);
  if (lane_id() == kWave - 1) wave_tot[wid] = incl;
  __syncthreads();
  uint32_t run = incl - sum, total = 0;
  for (uint32_t w = 0; w < kWaves; ++w) {
    const uint32_t x = wave_tot[w];
    if (w < wid) run += x;
    total += x;
  }
#pragma unroll
  for (uint32_t k = 0; k < kPer; ++k) {
    pre[t * kPer + k] = run;
    run += c[k];
  }
  __syncthreads();   // pre and s_flushed complete
  const uint64_t flushed = s_flushed;
  if (t == 0) stats->n_hosts = flushed + total;
  for (uint32_t e = t; e < total; e += kCompactBlock) {
    uint32_t lo = 0, hi = kJoinWaves;   // last region starting at or before e
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) / 2;
      if (pre[mid] <= e) lo = mid; else hi = mid;
    }
    const uint64_t idx = flushed + e;
    if (idx < capacity) stage[idx] = wbuf[(uint64_t)lo * kWave + (e - pre[lo])];
  }
}

// ---- ordering of the restored list --------------------------------------
// Keys are (ip << 32 | stage index); restored IPs are distinct, the index
// keeps keys unique regardless. The rank of a key is the number of smaller
// keys, and the entry is written there.

// Lists of at most kSmallSort entries: each wave takes kRankPerWave entries
// and counts, for each, the smaller keys over the whole list, which the
// block streams through LDS in tiles; each entry is written at its rank.
constexpr uint32_t kRankPerWave = 4;
constexpr uint32_t kRankTile = 2048;   // keys per LDS tile (16 KiB)
__global__ __launch_bounds__(256) void k_rank_small(const cbaa_host* __restrict__ stage,
                                                    const cbaa_restore_stats* stats,
                                                    uint64_t capacity, cbaa_host* out) {
  __shared__ uint64_t keys[kRankTile];
  const uint64_t n64 = stats->n_hosts < capacity ? stats->n_hosts : capacity;
  if (n64 > kSmallSort) return;
  const uint32_t n = (uint32_t)n64;
  const uint32_t e0 = (blockIdx.x * (256 / kWave) + threadIdx.x / kWave) * kRankPerWave;
  if (blockIdx.x * (256 / kWave) * kRankPerWave >= n) return;   // uniform over the block
  uint64_t mine[kRankPerWave];
  uint32_t less[kRankPerWave];
#pragma unroll
  for (uint32_t q = 0; q < kRankPerWave; ++q) {
    const uint32_t e = e0 + q;
    mine[q] = e < n ? (((uint64_t)stage[e].ip << 32) | e) : ~0ull;
    less[q] = 0;
  }
  for (uint32_t t0 = 0; t0 < n; t0 += kRankTile) {
    const uint32_t m = n - t0 < kRankTile ? n - t0 : kRankTile;
    __syncthreads();   // the previous tile is no longer read
    for (uint32_t j = threadIdx.x; j < m; j += 256)
      keys[j] = ((uint64_t)stage[t0 + j].ip << 32) | (t0 + j);
    __syncthreads();
    for (uint32_t j = lane_id(); j < m; j += kWave) {
      const uint64_t k = keys[j];
#pragma unroll
      for (uint32_t q = 0; q < kRankPerWave; ++q) less[q] += k < mine[q] ? 1u : 0u;
    }
  }
#pragma unroll
  for (uint32_t q = 0; q < kRankPerWave; ++q) {
    const uint32_t rank = wave_sum(less[q]);
    const uint32_t e = e0 + q;
    if (e < n && lane_id() == 0) out[rank] = stage[e];
  }
}

// Larger lists: a counting sort into 2^16 buckets by the IP's top 16 bits,
// then each entry is ranked inside its bucket (restored IPs are distinct; the
// stage index breaks ties all the same). Uniform IPs leave ~n/2^16 entries per
// bucket; one bucket never holds more than the 2^16 IPs of its /16.
__device__ inline uint64_t list_size(const cbaa_restore_stats* stats, uint64_t capacity) {
  return stats->n_hosts < capacity ? stats->n_hosts : capacity;
}

__global__ __launch_bounds__(256) void k_bucket_zero(const cbaa_restore_stats* stats,
                                                     uint64_t capacity, uint32_t* bucket) {
  if (list_size(stats, capacity) <= kSmallSort) return;
  for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < 2 * (kBuckets + 1); i += gridDim.x * 256)
    bucket[i] = 0;
}

__global__ __launch_bounds__(256) void k_bucket_count(const cbaa_host* __restrict__ stage,
                                                      const cbaa_restore_stats* stats,
                                                      uint64_t capacity, uint32_t* cnt) {
  const uint64_t n = list_size(stats, capacity);
  if (n <= kSmallSort) return;
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256)
    atomicAdd(&cnt[stage[i].ip >> 16], 1u);
}

// One block: counts -> exclusive starts in place (start[kBuckets] = n).
__global__ __launch_bounds__(1024) void k_bucket_scan(const cbaa_restore_stats* stats,
                                                      uint64_t capacity, uint32_t* cnt) {
  __shared__ uint32_t wsum[1024 / kWave];
  if (list_size(stats, capacity) <= kSmallSort) return;
  constexpr uint32_t kPer = kBuckets / 1024;
  uint32_t* c = cnt + threadIdx.x * kPer;
  uint32_t mine = 0;
  for (uint32_t i = 0; i < kPer; ++i) mine += c[i];
  uint32_t incl = mine;   // inclusive scan over the wave, then over waves
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t t = __shfl_up(incl, o, kWave);
    if (lane_id() >= (uint32_t)o) incl += t;
  }
  const uint32_t wid = threadIdx.x / kWave;
  if (lane_id() == kWave - 1) wsum[wid] = incl;
  __syncthreads();
  uint32_t before = 0, total = 0;
  for (uint32_t w = 0; w < 1024 / kWave; ++w) {
    if (w < wid) before += wsum[w];
    total += wsum[w];
  }
  uint32_t run = before + incl - mine;
  for (uint32_t i = 0; i < kPer; ++i) {
    const uint32_t v = c[i];
    c[i] = run;
    run += v;
  }
  if (threadIdx.x == 0) cnt[kBuckets] = total;
}

// keys[pos] = (IP << 32) | stage index, grouped by bucket (order inside a
// bucket is whatever the atomics give).
__global__ __launch_bounds__(256) void k_bucket_scatter(const cbaa_host* __restrict__ stage,
                                                        const cbaa_restore_stats* stats,
                                                        uint64_t capacity,
                                                        const uint32_t* __restrict__ start,
                                                        uint32_t* fill, uint64_t* keys) {
  const uint64_t n = list_size(stats, capacity);
  if (n <= kSmallSort) return;
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * 256) {
    const uint32_t ip = stage[i].ip;
    const uint32_t b = ip >> 16;
    keys[start[b] + atomicAdd(&fill[b], 1u)] = ((uint64_t)ip << 32) | (uint32_t)i;
  }
}

__global__ __launch_bounds__(256) void k_bucket_rank(const cbaa_host* __restrict__ stage,
                                                     const cbaa_restore_stats* stats,
                                                     uint64_t capacity,
                                                     const uint32_t* __restrict__ start,
                                                     const uint64_t* __restrict__ keys,
                                                     cbaa_host* out) {
  const uint64_t n = list_size(stats, capacity);
  if (n <= kSmallSort) return;
  for (uint64_t j = (uint64_t)blockIdx.x * 256 + threadIdx.x; j < n;
       j += (uint64_t)gridDim.x * 256) {
    const uint64_t key = keys[j];
    const uint32_t b = (uint32_t)(key >> 48);
    const uint32_t lo = start[b], hi = start[b + 1];
    uint32_t rank = 0;
    for (uint32_t k = lo; k < hi; ++k) rank += keys[k] < key ? 1u : 0u;
    out[lo + rank] = stage[(uint32_t)key];
  }
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

// Features of the learned estimator, in the log domain of the linear count:
// for each array a, f_a = ln(1 + g * u_a) with u_a = -ln(max(z_a, 1) / g)
// (z_a = zeros of the host's column of array a, so g * u_a is that column's
// own linear count); optionally the same for the union column with Thm. 2's
// correction, u = max(0, -ln(max(Z, 1) / (g - g*eps))), and g * eps.
__device__ inline float log_count_feature(double g, uint32_t z, double denom) {
  double u = -log((double)(z == 0 ? 1u : z) / denom);
  if (u < 0.0) u = 0.0;
  return (float)log1p(g * u);
}

template <int NRA, int NVA, int RPL>
__global__ __launch_bounds__(256) void k_features(Dims d, const uint64_t* __restrict__ cube,
                                                  const uint32_t* __restrict__ hosts, uint64_t n,
                                                  const double* __restrict__ eps,
                                                  const double* __restrict__ shared, uint32_t F,
                                                  float* x) {
  constexpr int A = NRA + NVA;
  const uint64_t gw = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const uint64_t nw = ((uint64_t)gridDim.x * blockDim.x) / kWave;
  const double g = (double)d.g;
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
      const uint32_t za = col_zeros<RPL>(d, c);
      if (lane_id() == 0) x[k * F + a] = log_count_feature(g, za, g);
#pragma unroll
      for (int q = 0; q < RPL; ++q) u.w[q] &= c.w[q];
    }
    const uint32_t z = col_zeros<RPL>(d, u);
    if (lane_id() == 0 && F >= (uint32_t)A + 2) {
      const double e = eps[cs];
      x[k * F + A] = log_count_feature(g, z, g - g * e);
      x[k * F + A + 1] = (float)(g * e);
    }
    if (lane_id() == 0 && F == (uint32_t)A + 4) {
      const double sh = shared[cs];
      x[k * F + A + 2] = log_count_feature(g, z, g - sh);
      x[k * F + A + 3] = (float)sh;
    }
  }
}

// ---- per-row fills (features) ------------------------------------------
// Block (cs, rb): for every array a and each of the 64 rows of row block rb,
// the number of a's columns with that bit set. A wave reads 64 neighbouring
// words (one per lane); for bit j, the ballot of "bit j set" restricted to the
// lanes of array a, popcounted, is that chunk's count, kept by lane j.
constexpr int kRowBlock = 256;

__global__ __launch_bounds__(kRowBlock) void k_row_ones(Dims d, const uint64_t* __restrict__ cube,
                                                        uint32_t* rows) {
  __shared__ uint32_t cnt[CBAA_MAX_ARRAYS * kWave];
  const uint32_t cs = blockIdx.x / d.R, rb = blockIdx.x % d.R;
  for (uint32_t i = threadIdx.x; i < d.A * kWave; i += kRowBlock) cnt[i] = 0;
  __syncthreads();
  const uint64_t* base = cube + ((uint64_t)cs * d.R + rb) * d.W;
  const uint32_t wid = threadIdx.x / kWave, lane = lane_id();
  for (uint32_t c0 = wid * kWave; c0 < d.W; c0 += kRowBlock) {
    const uint32_t w = c0 + lane;
    const bool valid = w < d.W;
    const uint64_t word = valid ? base[w] : 0ull;
    uint32_t arr = d.A;
    for (uint32_t a = 0; a < d.A; ++a)
      if (valid && w >= d.aoff[a] && w < d.aoff[a] + d.ncol[a]) arr = a;
    const uint32_t last = d.W - 1 - c0 < (uint32_t)(kWave - 1) ? d.W - 1 - c0 : (uint32_t)(kWave - 1);
    const uint32_t a_lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)arr);
    const uint32_t a_hi = (uint32_t)__builtin_amdgcn_readlane((int)arr, (int)last);
    for (uint32_t a = a_lo; a <= a_hi; ++a) {
      const uint64_t amask = __ballot(arr == a);
      uint32_t mine = 0;
      for (uint32_t j = 0; j < (uint32_t)kWave; ++j) {
        const uint32_t c = (uint32_t)__popcll(__ballot((word >> j) & 1ull) & amask);
        if (lane == j) mine = c;
      }
      if (mine) atomicAdd(&cnt[a * kWave + lane], mine);
    }
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < d.A * kWave; i += kRowBlock) {
    const uint32_t a = i / kWave, j = i % kWave;
    rows[((uint64_t)cs * d.A + a) * d.g + rb * kWave + j] = cnt[i];
  }
}

// Block cs: sum over rows of the product over arrays (in array order) of
// row_ones / c(a) -- the row-aware counterpart of g * eps.
__global__ __launch_bounds__(kRowBlock) void k_row_shared(Dims d, const uint32_t* __restrict__ rows,
                                                          double* shared) {
  __shared__ double part[kRowBlock];
  const uint32_t cs = blockIdx.x;
  double s = 0.0;
  for (uint32_t b = threadIdx.x; b < d.g; b += kRowBlock) {
    double q = 1.0;
    for (uint32_t a = 0; a < d.A; ++a)
      q = q * ((double)rows[((uint64_t)cs * d.A + a) * d.g + b] / (double)d.ncol[a]);
    s += q;
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (uint32_t o = kRowBlock / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) shared[cs] = part[0];
}

int check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? CBAA_OK : hip_fail(e, what);
}

// Zeroes the counters (stats and work may be null) and the fill accumulators,
// checks the cube's header (with stats), then scans the cube.
int run_scan(const Dims& d, const uint64_t* cube, uint16_t* zeros, uint32_t* ones,
             cbaa_restore_stats* stats, uint64_t* work, hipStream_t s) {
  CubeSrc one{};
  one.p[0] = cube;
  one.k = 1;
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(256), 0, s, d, stats, ones, d.S * d.A, work, one,
                     (uint64_t*)nullptr);
  int rc = check_launch("reset launch");
  if (rc != CBAA_OK) return rc;
  const uint32_t half_w = d.W / 2;
  dim3 grid((half_w + kScanBlock - 1) / kScanBlock, d.S);
  hipLaunchKernelGGL(k_column_zeros, grid, dim3(kScanBlock), 0, s, d, (const uint4*)cube,
                     (uint32_t*)zeros, ones);
  return check_launch("column scan launch");
}

template <int NRA, int NVA>
int dispatch_rpl_join(const Dims& d, const JoinArgs& ja, hipStream_t s) {
  const uint32_t grid = kJoinWaves;  // waves; they stride over the work list
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

template <int NRA, int NVA>
int dispatch_rpl_feat(const Dims& d, const uint64_t* cube, const uint32_t* hosts, uint64_t n,
                      const double* eps, const double* shared, uint32_t F, float* x,
                      hipStream_t s) {
  uint64_t blocks = (n + 3) / 4;
  if (blocks > 4096) blocks = 4096;
#define CBAA_FEAT(RPL)                                                                       \
  if (d.R <= RPL * kWave) {                                                                  \
    hipLaunchKernelGGL((k_features<NRA, NVA, RPL>), dim3((uint32_t)blocks), dim3(256), 0, s, \
                       d, cube, hosts, n, eps, shared, F, x);                                \
    return check_launch("features launch");                                                 \
  }
  CBAA_FEAT(1) CBAA_FEAT(2) CBAA_FEAT(4) CBAA_FEAT(8)
#undef CBAA_FEAT
  return CBAA_ECONFIG;
}

int run_feat(const Dims& d, const uint64_t* cube, const uint32_t* hosts, uint64_t n,
             const double* eps, const double* shared, uint32_t F, float* x, hipStream_t s) {
  CBAA_ARRAY_DISPATCH(dispatch_rpl_feat, d, cube, hosts, n, eps, shared, F, x, s);
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
  return run_scan(d, cube, zeros, ones, nullptr, nullptr, s);
}

namespace {

// After the column scan: thresholds, hot lists and their gather (Alg. 2).
int find_hot(const Dims& d, const CubeSrc& cube, double x, int rule, const RestoreScratch& rs,
             cbaa_restore_stats* stats, hipStream_t s) {
  hipLaunchKernelGGL(k_prepare, dim3(d.S, d.n_ra, kPrepParts), dim3(kPrepBlock), 0, s, d,
                     rs.zeros, rs.ones, rs.eps, rs.zmax, rs.hcnt, rs.hot, x, rule, stats, cube,
                     rs.hcol, rs.gcap, rs.gfit);
  return check_launch("prepare launch");
}

// After the hot lists: the tuple check (Alg. 3) and the ordering.
int join_and_order(const Dims& d, const CubeSrc& cube, uint64_t max_checks,
                   const RestoreScratch& rs, uint64_t capacity, cbaa_host* out,
                   cbaa_restore_stats* stats, hipStream_t s) {
  int rc;
  JoinArgs ja{cube,     rs.zeros,  rs.hot,  rs.hcol, rs.gfit,  rs.gcap,  rs.hcnt, rs.zmax,
              rs.eps,   rs.stage,  rs.wbuf, rs.wcnt, capacity, stats,    rs.work, max_checks};
  if ((rc = run_join(d, ja, s)) != CBAA_OK) return rc;
  hipLaunchKernelGGL(k_compact, dim3(1), dim3(kCompactBlock), 0, s, rs.wbuf, rs.wcnt, stats,
                     rs.stage, capacity);
  if ((rc = check_launch("compact launch")) != CBAA_OK) return rc;
  if (capacity == 0) return CBAA_OK;
  const uint64_t small = capacity < kSmallSort ? capacity : kSmallSort;
  const uint32_t per_block = (256 / kWave) * kRankPerWave;
  hipLaunchKernelGGL(k_rank_small, dim3((uint32_t)((small + per_block - 1) / per_block)), dim3(256),
                     0, s, rs.stage,
                     stats, capacity, out);
  if ((rc = check_launch("rank launch")) != CBAA_OK) return rc;
  // larger lists (each kernel returns at once when the list is small; none
  // is launched when the capacity itself is small)
  if (capacity <= kSmallSort) return CBAA_OK;
  uint64_t gb = (capacity + 255) / 256;
  if (gb > 8192) gb = 8192;
  uint32_t* start = rs.bucket;
  uint32_t* fill = rs.bucket + kBuckets + 1;
  hipLaunchKernelGGL(k_bucket_zero, dim3(256), dim3(256), 0, s, stats, capacity, rs.bucket);
  hipLaunchKernelGGL(k_bucket_count, dim3((uint32_t)gb), dim3(256), 0, s, rs.stage, stats, capacity,
                     start);
  hipLaunchKernelGGL(k_bucket_scan, dim3(1), dim3(1024), 0, s, stats, capacity, start);
  hipLaunchKernelGGL(k_bucket_scatter, dim3((uint32_t)gb), dim3(256), 0, s, rs.stage, stats,
                     capacity, start, fill, rs.keys);
  hipLaunchKernelGGL(k_bucket_rank, dim3((uint32_t)gb), dim3(256), 0, s, rs.stage, stats, capacity,
                     start, rs.keys, out);
  return check_launch("sort launches");
}

// Everything after the column scan.
int restore_after_scan(const Dims& d, const CubeSrc& cube, double x, int rule,
                       uint64_t max_checks, const RestoreScratch& rs, uint64_t capacity,
                       cbaa_host* out, cbaa_restore_stats* stats, hipStream_t s) {
  const int rc = find_hot(d, cube, x, rule, rs, stats, s);
  if (rc != CBAA_OK) return rc;
  return join_and_order(d, cube, max_checks, rs, capacity, out, stats, s);
}

// The sources the restore reads: the merged cube when stored, else the
// router cubes (OR-ed on every read).
bool restore_sources(const uint64_t* dst, const uint64_t* const* srcs, int k, CubeSrc& cs) {
  cs = CubeSrc{};
  if (dst) {
    cs.p[0] = dst;
    cs.k = 1;
    return true;
  }
  if (k > kMergeScanSources) {
    set_error("more than %d source cubes need a destination cube", kMergeScanSources);
    return false;
  }
  for (int j = 0; j < k; ++j) cs.p[j] = srcs[j];
  cs.k = k;
  return true;
}

}  // namespace

int launch_restore(const Dims& d, const uint64_t* cube, double x, int rule, uint64_t max_checks,
                   void* scratch, uint64_t capacity, cbaa_host* out, cbaa_restore_stats* stats,
                   hipStream_t s) {
  RestoreScratch rs = carve(d, scratch, capacity);
  int rc = run_scan(d, cube, rs.zeros, rs.ones, stats, rs.work, s);
  if (rc != CBAA_OK) return rc;
  CubeSrc one{};
  one.p[0] = cube;
  one.k = 1;
  return restore_after_scan(d, one, x, rule, max_checks, rs, capacity, out, stats, s);
}

int launch_merge_scan(const Dims& d, uint64_t* dst, const uint64_t* const* srcs, int k,
                      double x, int rule, void* scratch, uint64_t capacity,
                      cbaa_restore_stats* stats, hipStream_t s) {
  RestoreScratch rs = carve(d, scratch, capacity);
  CubeSrc cs;
  if (!restore_sources(dst, srcs, k, cs)) return CBAA_EINVAL;
  int rc;
  if (k > kMergeScanSources) {   // merge in passes first, then the plain scan
    if ((rc = launch_merge_or(d, dst, srcs, k, s)) != CBAA_OK) return rc;
    if ((rc = run_scan(d, dst, rs.zeros, rs.ones, stats, rs.work, s)) != CBAA_OK) return rc;
    return find_hot(d, cs, x, rule, rs, stats, s);
  }
  CubeSrc all{};
  for (int j = 0; j < k; ++j) all.p[j] = srcs[j];
  all.k = k;
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(256), 0, s, d, stats, rs.ones, d.S * d.A, rs.work, all,
                     dst);
  if ((rc = check_launch("reset launch")) != CBAA_OK) return rc;
  MergeSrc ms{};
  for (int j = 0; j < k; ++j) ms.p[j] = (const uint4*)srcs[j];
  const uint32_t half_w = d.W / 2;
  dim3 grid((half_w + kScanBlock - 1) / kScanBlock, d.S);
  hipLaunchKernelGGL(k_merge_scan, grid, dim3(kScanBlock), 0, s, d, ms, k, (uint4*)dst,
                     (uint32_t*)rs.zeros, rs.ones);
  if ((rc = check_launch("merge scan launch")) != CBAA_OK) return rc;
  return find_hot(d, cs, x, rule, rs, stats, s);
}

int launch_restore_scanned(const Dims& d, const uint64_t* dst, const uint64_t* const* srcs,
                           int k, uint64_t max_checks, void* scratch, uint64_t capacity,
                           cbaa_host* out, cbaa_restore_stats* stats, hipStream_t s) {
  RestoreScratch rs = carve(d, scratch, capacity);
  CubeSrc cs;
  if (!restore_sources(dst, srcs, k, cs)) return CBAA_EINVAL;
  return join_and_order(d, cs, max_checks, rs, capacity, out, stats, s);
}

int launch_merge_restore(const Dims& d, uint64_t* dst, const uint64_t* const* srcs, int k,
                         double x, int rule, uint64_t max_checks, void* scratch,
                         uint64_t capacity, cbaa_host* out, cbaa_restore_stats* stats,
                         hipStream_t s) {
  const int rc = launch_merge_scan(d, dst, srcs, k, x, rule, scratch, capacity, stats, s);
  if (rc != CBAA_OK) return rc;
  return launch_restore_scanned(d, dst, srcs, k, max_checks, scratch, capacity, out, stats, s);
}

int launch_estimate(const Dims& d, const uint64_t* cube, const uint32_t* hosts, uint64_t n,
                    double* est, uint16_t* zeros, uint16_t* layer_zeros, void* scratch,
                    hipStream_t s) {
  RestoreScratch rs = carve(d, scratch, 0);
  int rc = run_scan(d, cube, rs.zeros, rs.ones, nullptr, nullptr, s);
  if (rc != CBAA_OK) return rc;
  hipLaunchKernelGGL(k_prepare, dim3(d.S, 1), dim3(kPrepBlock), 0, s, d, rs.zeros, rs.ones,
                     rs.eps, rs.zmax, rs.hcnt, (uint16_t*)nullptr, 1.0, CBAA_THR_THM2,
                     (cbaa_restore_stats*)nullptr, CubeSrc{}, (uint64_t*)nullptr, 0u,
                     (uint32_t*)nullptr);
  if ((rc = check_launch("prepare launch")) != CBAA_OK) return rc;
  return run_est(d, cube, hosts, n, rs.eps, est, zeros, layer_zeros, s);
}

int launch_features(const Dims& d, const uint64_t* cube, const uint32_t* hosts, uint64_t n,
                    uint32_t F, float* x, void* scratch, hipStream_t s) {
  RestoreScratch rs = carve(d, scratch, 0);
  int rc = run_scan(d, cube, rs.zeros, rs.ones, nullptr, nullptr, s);
  if (rc != CBAA_OK) return rc;
  hipLaunchKernelGGL(k_prepare, dim3(d.S, 1), dim3(kPrepBlock), 0, s, d, rs.zeros, rs.ones,
                     rs.eps, rs.zmax, rs.hcnt, (uint16_t*)nullptr, 1.0, CBAA_THR_THM2,
                     (cbaa_restore_stats*)nullptr, CubeSrc{}, (uint64_t*)nullptr, 0u,
                     (uint32_t*)nullptr);
  if ((rc = check_launch("prepare launch")) != CBAA_OK) return rc;
  if (F == d.A + 4) {
    hipLaunchKernelGGL(k_row_ones, dim3(d.S * d.R), dim3(kRowBlock), 0, s, d, cube, rs.rows);
    if ((rc = check_launch("row fill launch")) != CBAA_OK) return rc;
    hipLaunchKernelGGL(k_row_shared, dim3(d.S), dim3(kRowBlock), 0, s, d, rs.rows, rs.shared);
    if ((rc = check_launch("row mass launch")) != CBAA_OK) return rc;
  }
  return run_feat(d, cube, hosts, n, rs.eps, rs.shared, F, x, s);
}

}  // namespace cbaa
