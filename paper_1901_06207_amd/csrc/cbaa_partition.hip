// Partitioned update. The bit-sets of a batch are binned by (cube, sketch,
// 64-bit row block) so that each bin's target -- one row block of every column
// of one sketch, W contiguous words (128 KiB at the paper's dimensions) -- can
// be assembled in LDS and written to the cube once, coalesced. This replaces
// A random device-scope atomics per pair and cube by a streamed 8-byte record
// per pair and cube.
//
// The same launches serve one edge router's batch or K routers' batches of
// uneven sizes at once (a stream table passed by value to every kernel):
//   1. sample      every 64th piece (16 Ki pairs) of each stream: records per
//                  bin in LDS counters, added into the stream's sampled counts
//   2. bases       per stream: each bin's region (its sampled count scaled to
//                  the stream, plus a margin for the sampling error) and the
//                  prefix of the regions; the bins' write cursors start at
//                  their bases. A bin's records are contiguous in its region.
//   3. scatter     persistent blocks (one per CU, 1024 threads) take scatter
//                  chunks (16 pairs per thread), kept in registers, from a
//                  shared counter; per cube, rank the chunk's records inside
//                  their bins in LDS, reserve each bin's run with one atomic
//                  add on its cursor, stage the records bin-sorted and write
//                  every run contiguously. The order of runs inside a bin is
//                  whatever the atomics give: the OR of the bits does not
//                  depend on it. Records past the end of a full region go to
//                  the stream's overflow list instead
//   4. fills       per stream: each region's fill, the exclusive prefix of
//                  the apply segments and the fresh row blocks to zero; the
//                  last stream to finish prefixes the apply items over streams
//   5. apply       persistent blocks take (stream, bin, segment) items from a
//                  shared counter (work stealing across streams): zero
//                  an LDS tile, OR the records' bits into it, flush non-zero
//                  words to the stream's cube with atomic ORs -- or, for a
//                  stream whose cubes start empty and a bin with one item,
//                  store the whole tile (the row block needs no zeroing)
// Fresh streams' row blocks that no single item owns (empty bins and bins
// split over several items) are zeroed before the apply. Last, the overflow
// list of each stream (empty unless the sample misjudged a bin) is OR-ed into
// its cubes with device-scope atomics, after every tile is in place.
// A record is the mangled inner IP and the outer IP's bit with the cube index
// in bit 31 (uint2); the apply step recomputes the columns from the mangled IP.
#include "cbaa_internal.hpp"

namespace cbaa {

namespace {

constexpr int kBlock = 1024;
constexpr uint32_t kMaxBins = 8192;      // bins of a stream (both cubes)
constexpr int kUnroll = 8;                // independent loads in flight per thread
constexpr int kApplyUnroll = 8;           // record loads in flight per apply thread
constexpr uint32_t kMaxTileWords = 16384; // 128 KiB LDS tile
// Scatter blocks of 1024 threads (16 waves, 128 registers per lane): a chunk
// of 16 pairs per thread stays in registers with no spill, and its 8-byte
// records fill 128 KiB of LDS next to 24 KiB of per-bin counters, run offsets
// and region ends for up to 1024 bins per cube. Cubes of up to 4096 bins
// (e.g. 32 sketches, or 8192-bit columns) take 11 pairs per thread beside
// 64 KiB.
constexpr int kScatterThreads = 1024;
constexpr uint32_t kSmallBins = 1024;     // bins per cube of the first shape
constexpr int kScatterPerSmall = 16;
constexpr int kScatterPerLarge = 11;
inline uint32_t scatter_chunk(uint32_t per_cube) {
  return (per_cube <= kSmallBins ? kScatterPerSmall : kScatterPerLarge) * kScatterThreads;
}
constexpr uint32_t kScatterBlocks = 256;  // persistent scatter grid (one per CU)
constexpr uint32_t kDefaultChunk = 16384;   // pairs per sampled piece
constexpr uint32_t kSplit = 65536;          // a long update is split in multiples of this
constexpr uint32_t kDefaultSeg = 65536;
constexpr uint32_t kDefaultApplyBlocks = 512;
constexpr uint32_t kNoRank = 0xFFFFu;
// Every kSampleStride-th piece of a stream is counted, from its first; a
// bin's region is its scaled sampled count e plus e/5 + 4 sqrt(e) + 64
// records. At 16 Ki-pair pieces that is 1/64 of the pairs, spread evenly over
// the stream, and ~500 sampled records per bin at the paper's dimensions: the
// margin is several standard errors of the sample.
constexpr uint32_t kSampleStride = 64;

inline uint64_t align256(uint64_t x) { return (x + 255u) & ~uint64_t(255u); }

struct StreamDesc {
  const uint2* pairs;
  uint64_t n;
  uint64_t* cube0;
  uint64_t* cube1;
  uint64_t rec_base;      // first record of this stream's regions
  uint32_t ovf_off;       // its overflow list, right after its regions
  uint64_t sampled;       // pairs in its sampled pieces
  uint32_t sample_begin;  // first global sampled piece
  uint32_t schunk_begin;  // first global scatter chunk
  uint32_t side;
  uint32_t fresh;         // cubes start empty: row blocks are stored, not OR-ed
};

struct Batch {
  uint32_t k;
  uint32_t nbins;         // per stream: n_cubes * S * R
  uint32_t total_samples; // sampled pieces of all streams
  uint32_t total_schunks; // scatter chunks of all streams
  uint32_t chunk;         // pairs per piece
  uint32_t schunk;        // pairs per scatter chunk
  uint32_t seg;           // records per apply item
  StreamDesc s[CBAA_MAX_BATCH];
};

struct Layout {
  uint32_t* tot;      // [k][nbins] sampled records per bin, later each region's fill
  uint32_t* next;     // [2] next apply item, next scatter chunk (right after tot)
  uint32_t* ovfn;     // [k] entries of each stream's overflow list (right after next)
  uint32_t* nclear;   // [2] fresh row blocks to zero, streams whose fills are done (after ovfn)
  uint32_t* clear;    // [k][nbins] fresh row blocks to zero: stream << 16 | bin
  uint32_t* cursor;   // [k][nbins] next free record of each bin (scatter)
  uint32_t* base;     // [k][nbins + 1] record offsets inside the stream
  uint32_t* segpre;   // [k][nbins + 1] apply items inside the stream
  uint32_t* items;    // [k + 1] apply items before each stream
  uint2* rec;         // per stream: the bins' regions (region_records), then the
                      // overflow list (n_cubes * n)
  uint64_t bytes;
};

struct Tuning {
  uint32_t chunk, seg, apply_blocks;
};

Tuning effective(const cbaa_tuning* t) {
  Tuning r;
  r.chunk = (t && t->chunk_pairs) ? t->chunk_pairs : kDefaultChunk;
  r.seg = (t && t->seg_records) ? t->seg_records : kDefaultSeg;
  r.apply_blocks = (t && t->apply_blocks) ? t->apply_blocks : kDefaultApplyBlocks;
  return r;
}

// Records the regions of a stream of n pairs can hold at most, whatever the
// sample: the scaled sampled counts sum to n per cube, so the regions sum to
// at most n_cubes n (1 + 1/5) + 4 sqrt(nbins n_cubes n) + 65 nbins (the last
// term also absorbs the device's rounding of square roots).
uint64_t region_records(uint64_t n, uint32_t n_cubes, uint32_t nbins) {
  const uint64_t r = (uint64_t)n_cubes * n;
  const uint64_t sq = (uint64_t)sqrt((double)nbins * (double)r) + 1;
  return r + r / 5 + 4 * sq + 65ull * nbins;
}

// A stream's regions and its overflow list are addressed with 32-bit offsets,
// and a bin's cursor may run past its region by the bin's whole count.
bool fits(uint64_t n, uint32_t n_cubes, uint32_t nbins) {
  return region_records(n, n_cubes, nbins) + (uint64_t)n_cubes * n < 0xFFFFFFFFull;
}

// Largest multiple of chunk that fits() (about 0.45 * 2^32 / n_cubes).
uint64_t max_stream_pairs(const Dims& d, int n_cubes, uint64_t chunk) {
  const uint32_t nbins = (uint32_t)n_cubes * d.S * d.R;
  uint64_t lo = 0, hi = (0xFFFFFFFFull / (uint64_t)n_cubes) / chunk;   // in chunks
  while (lo < hi) {
    const uint64_t mid = (lo + hi + 1) / 2;
    if (fits(mid * chunk, (uint32_t)n_cubes, nbins)) lo = mid; else hi = mid - 1;
  }
  return lo * chunk;
}

// Fills the batch's chunk and record bookkeeping and carves the scratch.
Layout plan(const Dims& d, int n_cubes, uint32_t chunk, Batch& b, void* base) {
  b.nbins = (uint32_t)n_cubes * d.S * d.R;
  b.chunk = chunk;
  b.schunk = scatter_chunk(d.S * d.R);
  uint32_t sp = 0, sch = 0;
  uint64_t rec = 0;
  for (uint32_t i = 0; i < b.k; ++i) {
    StreamDesc& s = b.s[i];
    s.sample_begin = sp;
    s.schunk_begin = sch;
    s.rec_base = rec;
    const uint64_t nch = (s.n + chunk - 1) / chunk;
    s.sampled = 0;
    for (uint64_t c = 0; c < nch; c += kSampleStride)
      s.sampled += s.n - c * chunk < chunk ? s.n - c * chunk : chunk;
    sp += (uint32_t)((nch + kSampleStride - 1) / kSampleStride);
    sch += (uint32_t)((s.n + b.schunk - 1) / b.schunk);
    s.ovf_off = s.n ? (uint32_t)region_records(s.n, (uint32_t)n_cubes, b.nbins) : 0u;
    rec += s.ovf_off + (uint64_t)n_cubes * s.n;
  }
  b.total_samples = sp;
  b.total_schunks = sch;
  Layout L;
  uint64_t off = 0;
  char* p = (char*)base;
  auto take = [&](uint64_t bytes) {
    char* q = p ? p + off : nullptr;
    off += align256(bytes);
    return (void*)q;
  };
  L.tot = (uint32_t*)take(((uint64_t)b.k * b.nbins + 2 + b.k + 2) * 4);
  L.next = L.tot + (uint64_t)b.k * b.nbins;
  L.ovfn = L.next + 2;
  L.nclear = L.ovfn + b.k;
  L.clear = (uint32_t*)take((uint64_t)b.k * b.nbins * 4);
  L.cursor = (uint32_t*)take((uint64_t)b.k * b.nbins * 4);
  L.base = (uint32_t*)take((uint64_t)b.k * (b.nbins + 1) * 4);
  L.segpre = (uint32_t*)take((uint64_t)b.k * (b.nbins + 1) * 4);
  L.items = (uint32_t*)take((uint64_t)(b.k + 1) * 4);
  L.rec = (uint2*)take(rec * 8);
  L.bytes = off;
  return L;
}

// Stream owning global sampled piece x: the last stream whose first piece is
// <= x (streams without pairs share their successor's start and are skipped
// by taking the last match).
__device__ inline uint32_t owner_of_sample(const Batch& b, uint32_t x) {
  uint32_t s = 0;
  for (uint32_t i = 1; i < b.k; ++i)
    if (b.s[i].sample_begin <= x) s = i;
  return s;
}

__device__ inline uint32_t owner_of_schunk(const Batch& b, uint32_t x) {
  uint32_t s = 0;
  for (uint32_t i = 1; i < b.k; ++i)
    if (b.s[i].schunk_begin <= x) s = i;
  return s;
}

__device__ inline uint32_t bin_of(const Dims& d, uint32_t k, uint32_t host, uint32_t peer,
                                  uint2& rec) {
  const uint32_t m = fmix32(host ^ d.seed_mangle);
  const uint32_t b = bit_of_peer(d, peer);
  rec = make_uint2(m, b | (k << 31));
  const uint32_t cs = m & low_mask(d.r);
  return ((((k << d.r) | cs) << (d.log2_g - 6)) | (b >> 6));   // (k S + cs) R + b / 64
}

__device__ inline uint32_t bin_of_record(const Dims& d, uint2 rec) {
  const uint32_t k = rec.y >> 31;
  const uint32_t b = rec.y & 0x7FFFFFFFu;
  return ((((k << d.r) | (rec.x & low_mask(d.r))) << (d.log2_g - 6)) | (b >> 6));
}

// Zeroes the bin totals and counters, and sets the streams' cube headers: a
// fresh stream's cubes get a valid header (they are rebuilt from empty), any
// other cube keeps a valid header only if it has one. Two threads touching a
// cube named by two streams write the same words.
__global__ void k_begin(Dims d, Batch b, uint32_t* p, uint32_t n) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x < 2 * b.k) {
    const StreamDesc& st = b.s[threadIdx.x / 2];
    uint64_t* cube = (threadIdx.x & 1) ? st.cube1 : st.cube0;
    if (cube) {
      if (st.fresh) header_set(header_of(cube), d, CBAA_CUBE_VALID);
      else header_touch(cube, d);
    }
  }
}

template <bool TWO>
__global__ __launch_bounds__(kBlock) void k_histogram(Dims d, Batch b, uint32_t* tot) {
  __shared__ uint32_t hist[kMaxBins];
  const uint32_t gs = blockIdx.x;
  const uint32_t si = owner_of_sample(b, gs);
  const StreamDesc& st = b.s[si];
  for (uint32_t i = threadIdx.x; i < b.nbins; i += kBlock) hist[i] = 0;
  __syncthreads();
  const uint64_t lo = (uint64_t)(gs - st.sample_begin) * kSampleStride * b.chunk;
  const uint64_t hi = lo + b.chunk < st.n ? lo + b.chunk : st.n;
  const int side = st.side;
  for (uint64_t k0 = lo + threadIdx.x; k0 < hi; k0 += (uint64_t)kBlock * kUnroll) {
    uint2 p[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const uint64_t k = k0 + (uint64_t)u * kBlock;
      p[u] = k < hi ? st.pairs[k] : make_uint2(0u, 0u);
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if (k0 + (uint64_t)u * kBlock >= hi) break;
      uint2 rec;
      const uint32_t h0 = side == CBAA_SIDE_SRC ? p[u].x : p[u].y;
      const uint32_t p0 = side == CBAA_SIDE_SRC ? p[u].y : p[u].x;
      atomicAdd(&hist[bin_of(d, 0, h0, p0, rec)], 1u);
      if (TWO) atomicAdd(&hist[bin_of(d, 1, p[u].y, p[u].x, rec)], 1u);
    }
  }
  __syncthreads();
  uint32_t* row = tot + (uint64_t)si * b.nbins;
  for (uint32_t i = threadIdx.x; i < b.nbins; i += kBlock) {
    const uint32_t v = hist[i];
    if (v) __hip_atomic_fetch_add(row + i, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Exclusive scan of per-thread values over a block of T threads.
template <int T = kBlock>
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* lds_waves, uint32_t& total) {
  const uint32_t lane = __lane_id();
  const uint32_t wid = threadIdx.x / kWave;
  uint32_t incl = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t t = __shfl_up(incl, o, kWave);
    if (lane >= (uint32_t)o) incl += t;
  }
  __syncthreads();
  if (lane == kWave - 1) lds_waves[wid] = incl;
  __syncthreads();
  uint32_t before = 0, tot = 0;
  for (uint32_t w = 0; w < T / kWave; ++w) {
    if (w < wid) before += lds_waves[w];
    tot += lds_waves[w];
  }
  total = tot;
  __syncthreads();
  return before + incl - v;
}

// Block si: each bin's region, from its sampled count e scaled to the stream
// (e = sampled * n / pairs sampled): e + e/5 + 4 sqrt(e) + 64 records, and
// the exclusive prefix of the regions (base, also the scatter's starting
// cursors).
__global__ __launch_bounds__(kBlock) void k_bases(Batch b, const uint32_t* __restrict__ tot,
                                                  uint32_t* base, uint32_t* cursor) {
  __shared__ uint32_t waves[kBlock / kWave];
  __shared__ uint32_t carry;
  const uint32_t si = blockIdx.x;
  const StreamDesc& st = b.s[si];
  const uint32_t* t = tot + (uint64_t)si * b.nbins;
  uint32_t* bs = base + (uint64_t)si * (b.nbins + 1);
  uint32_t* cu = cursor + (uint64_t)si * b.nbins;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (uint32_t b0 = 0; b0 < b.nbins; b0 += kBlock) {
    const uint32_t bin = b0 + threadIdx.x;
    uint32_t cap = 0;
    if (bin < b.nbins && st.n) {
      const uint64_t e = (uint64_t)t[bin] * st.n / st.sampled;
      cap = (uint32_t)(e + e / 5 + 4 * (uint64_t)sqrtf((float)e) + 64);
    }
    uint32_t sum;
    const uint32_t ex = block_exclusive_scan(cap, waves, sum);
    const uint32_t cr = carry;
    if (bin < b.nbins) {
      bs[bin] = cr + ex;
      cu[bin] = cr + ex;
    }
    __syncthreads();
    if (threadIdx.x == 0) carry = cr + sum;
    __syncthreads();
  }
  if (threadIdx.x == 0) bs[b.nbins] = carry;
}

// Block si, after the scatter: each region's fill (its cursor, capped at the
// region's end; the rest went to the overflow list), kept in tot, and the
// exclusive prefix of the apply segments the fills need (segpre). A fresh
// stream's bins that no single apply item will store whole (no records, or
// several items) go to the clear list. The last block to finish prefixes the
// streams' apply items.
__global__ __launch_bounds__(kBlock) void k_fills(Batch b, const uint32_t* __restrict__ base,
                                                  const uint32_t* __restrict__ cursor,
                                                  uint32_t* tot, uint32_t* segpre,
                                                  uint32_t* clear, uint32_t* nclear,
                                                  uint32_t* items) {
  __shared__ uint32_t waves[kBlock / kWave];
  __shared__ uint32_t carry;
  __shared__ bool last;
  const uint32_t si = blockIdx.x;
  const bool fresh = b.s[si].fresh != 0;
  const uint32_t* bs = base + (uint64_t)si * (b.nbins + 1);
  const uint32_t* cu = cursor + (uint64_t)si * b.nbins;
  uint32_t* t = tot + (uint64_t)si * b.nbins;
  uint32_t* sp = segpre + (uint64_t)si * (b.nbins + 1);
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (uint32_t b0 = 0; b0 < b.nbins; b0 += kBlock) {
    const uint32_t bin = b0 + threadIdx.x;
    uint32_t nseg = 0;
    if (bin < b.nbins) {
      const uint32_t end = bs[bin + 1], c = cu[bin];
      const uint32_t fill = (c < end ? c : end) - bs[bin];
      t[bin] = fill;
      nseg = (uint32_t)(((uint64_t)fill + b.seg - 1) / b.seg);
      if (fresh && nseg != 1)
        clear[__hip_atomic_fetch_add(nclear, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)] =
            (si << 16) | bin;
    }
    uint32_t sum;
    const uint32_t ex = block_exclusive_scan(nseg, waves, sum);
    const uint32_t cr = carry;
    if (bin < b.nbins) sp[bin] = cr + ex;
    __syncthreads();
    if (threadIdx.x == 0) carry = cr + sum;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    __hip_atomic_store(sp + b.nbins, carry, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // the stream's total is visible before the count of finished streams
    last = __hip_atomic_fetch_add(nclear + 1, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) ==
           b.k - 1;
  }
  __syncthreads();
  if (last && threadIdx.x == 0) {
    uint32_t acc = 0;
    for (uint32_t j = 0; j < b.k; ++j) {
      items[j] = acc;
      acc += __hip_atomic_load(segpre + (uint64_t)j * (b.nbins + 1) + b.nbins, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
    items[b.k] = acc;
  }
}

// The apply reads each record once and writes each fresh row block once:
// both with the non-temporal hint (the scatter's run writes, by contrast,
// need L2 to merge the runs of neighbouring chunks into whole lines).
typedef uint32_t u32x2_nt __attribute__((ext_vector_type(2)));
__device__ inline uint2 load_rec_nt(const uint2* p) {
  const u32x2_nt v = __builtin_nontemporal_load((const u32x2_nt*)p);
  return make_uint2(v.x, v.y);
}

__device__ inline uint32_t pack_rank(uint32_t rk, int u, uint32_t rank) {
  return rk | (rank << (16 * (u & 1)));
}

__device__ inline uint32_t unpack_rank(uint32_t rk, int u) { return (rk >> (16 * (u & 1))) & 0xFFFFu; }

// NB: the most bins per cube the LDS counters hold; PER: pairs per thread.
template <bool TWO, uint32_t NB, int PER>
__global__ __launch_bounds__(kScatterThreads) void k_scatter(Dims d, Batch b, uint32_t* cursor,
                                                    const uint32_t* __restrict__ base,
                                                    uint2* __restrict__ rec_all,
                                                    uint32_t* ovfn,
                                                    uint32_t* ctr) {
  __shared__ uint32_t s_next;
  __shared__ uint32_t s_over;   // some bin of this chunk and cube overflows
  constexpr int kPer = PER;
  constexpr uint32_t P = PER * kScatterThreads;
  // One LDS block, per-bin arrays first: a thread's bins in all of them are
  // one address register plus offsets the LDS instructions encode (< 64 KiB).
  // The first shape also keeps its stream's region ends here (8 KiB); the
  // second reads them with the cursor adds.
  constexpr bool kEndsInLds = NB <= kSmallBins;
  constexpr uint32_t kEndsWords = kEndsInLds ? 2 * NB : 0;
  // ... then the scan's per-wave sums, a counter that absorbs the ranks of
  // a short chunk's empty slots (so that every slot's LDS add is issued
  // unconditionally and the adds stay in flight together), and padding
  constexpr uint32_t kSpill = 4 * NB + kEndsWords + kScatterThreads / kWave;
  constexpr uint32_t kStageWord = kSpill + 2;
  static_assert(kStageWord % 2 == 0, "stage must be 8-byte aligned");
  __shared__ __align__(16) uint32_t lds[kStageWord + 2 * P];
  uint32_t* cnt = lds;              // counts, then the end of the run's in-region part
  uint32_t* start = lds + NB;       // first stage slot of each bin's run
  uint32_t* din = lds + 2 * NB;     // region position of a stage slot, minus the slot
  uint32_t* dov = lds + 3 * NB;     // overflow position of a stage slot, minus the slot
  uint32_t* ends = lds + 4 * NB;    // region ends of both cubes (first shape)
  uint32_t* waves = lds + 4 * NB + kEndsWords;
  uint32_t* spill = lds + kSpill;
  uint2* stage = (uint2*)(lds + kStageWord);
  uint32_t ends_of = 0xFFFFFFFFu;   // stream whose ends are in LDS
  // bins per thread in the count scan
  constexpr uint32_t kNpt = (NB + kScatterThreads - 1) / kScatterThreads;
  const uint32_t per_cube = d.S * d.R;   // bins of one cube (<= NB)
  uint2 p[kPer];
  auto load = [&](uint32_t gc) {
    const StreamDesc& st = b.s[owner_of_schunk(b, gc)];
    const uint64_t lo = (uint64_t)(gc - st.schunk_begin) * P;
    const uint32_t rem = st.n - lo < P ? (uint32_t)(st.n - lo) : P;
    const uint2* src = st.pairs + lo;
    // held as (inner, outer) of the first cube: a destination-keyed
    // one-cube stream swaps its pairs on load
    const bool swap = !TWO && st.side != CBAA_SIDE_SRC;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const uint32_t k = threadIdx.x + u * kScatterThreads;
      const uint2 v = k < rem ? src[k] : make_uint2(0u, 0u);
      p[u] = swap ? make_uint2(v.y, v.x) : v;
    }
  };
  // chunks are taken from a shared counter (work stealing); the next one is
  // claimed at the top of each chunk and loaded while the current chunk's
  // runs are written
  if (threadIdx.x == 0) s_next = __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  uint32_t gc_cur = s_next;
  __syncthreads();
  if (gc_cur < b.total_schunks) load(gc_cur);
  for (uint32_t gc = gc_cur; gc < b.total_schunks; gc = gc_cur) {
    if (threadIdx.x == 0) s_next = __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t si = owner_of_schunk(b, gc);
    const StreamDesc& st = b.s[si];
    uint2* rec = rec_all + st.rec_base;
    uint32_t* cur = cursor + (uint64_t)si * b.nbins;
    const uint32_t* bend = base + (uint64_t)si * (b.nbins + 1) + 1;   // region ends
    const uint64_t lo = (uint64_t)(gc - st.schunk_begin) * P;
    const uint32_t rem = st.n - lo < P ? (uint32_t)(st.n - lo) : P;
    if (kEndsInLds && si != ends_of) {   // uniform: si is the block's
      for (uint32_t i = threadIdx.x; i < b.nbins; i += kScatterThreads) ends[i] = bend[i];
      ends_of = si;
    }
#pragma unroll
    for (int k = 0; k < (TWO ? 2 : 1); ++k) {
      for (uint32_t i = threadIdx.x; i < per_cube; i += kScatterThreads) cnt[i] = 0;
      if (threadIdx.x == 0) s_over = 0;
      __syncthreads();
      uint32_t rk[(kPer + 1) / 2];
#pragma unroll
      for (int u = 0; u < (kPer + 1) / 2; ++u) rk[u] = 0;
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        uint32_t h0 = k == 0 ? p[u].x : p[u].y;
        uint32_t p0 = k == 0 ? p[u].y : p[u].x;
        // opaque to the compiler (no instruction): the staging pass below
        // hashes the pair again instead of keeping this pass's bins live
        // across the scan, which would spill
        asm volatile("" : "+v"(h0), "+v"(p0));
        uint2 r;
        const uint32_t bl = bin_of(d, k, h0, p0, r) - k * per_cube;
        const bool valid = threadIdx.x + u * kScatterThreads < rem;
        const uint32_t got = atomicAdd(valid ? &cnt[bl] : spill, 1u);
        const uint32_t rank = valid ? got : kNoRank;
        rk[u / 2] = pack_rank(rk[u / 2], u, rank);
      }
      __syncthreads();
      // local runs (exclusive prefix of the counts, kNpt consecutive bins per
      // thread) and global runs (one atomic add per non-empty bin on the
      // stream's cursor; a thread's adds are in flight together). The part
      // of a run past its region's end goes to the overflow list.
      // (the counts are read from LDS again rather than held in registers)
      uint32_t g[kNpt], e[kNpt], sum = 0;
#pragma unroll
      for (uint32_t j = 0; j < kNpt; ++j) {
        const uint32_t i = threadIdx.x * kNpt + j;
        const uint32_t c = i < per_cube ? cnt[i] : 0u;
        sum += c;
        g[j] = c ? __hip_atomic_fetch_add(cur + k * per_cube + i, c, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT)
                 : 0u;
        if (!kEndsInLds) e[j] = c ? bend[k * per_cube + i] : 0u;
      }
      uint32_t total;
      uint32_t run = block_exclusive_scan<kScatterThreads>(sum, waves, total);
#pragma unroll
      for (uint32_t j = 0; j < kNpt; ++j) {
        const uint32_t i = threadIdx.x * kNpt + j;
        const uint32_t c = i < per_cube ? cnt[i] : 0u;
        if (i < per_cube) {
          const uint32_t ej = kEndsInLds ? ends[k * per_cube + i] : e[j];
          const uint32_t room = g[j] < ej ? ej - g[j] : 0u;
          const uint32_t nin = c < room ? c : room;
          start[i] = run;
          cnt[i] = run + nin;
          din[i] = g[j] - run;
          dov[i] = c - nin;   // records past the region's end, placed below
          if (c != nin) s_over = 1;
        }
        run += c;
      }
      __syncthreads();
      if (s_over) {   // uniform; rare: the sample gave some bin too little room
#pragma unroll
        for (uint32_t j = 0; j < kNpt; ++j) {
          const uint32_t i = threadIdx.x * kNpt + j;
          const uint32_t nov = i < per_cube ? dov[i] : 0u;
          if (nov) {
            const uint32_t ob = __hip_atomic_fetch_add(ovfn + si, nov, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
            dov[i] = st.ovf_off + ob - cnt[i];
          }
        }
        __syncthreads();
      }
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const uint32_t rank = unpack_rank(rk[u / 2], u);
        if (rank == kNoRank) continue;
        const uint32_t h0 = k == 0 ? p[u].x : p[u].y;
        const uint32_t p0 = k == 0 ? p[u].y : p[u].x;
        uint2 r;
        const uint32_t bl = bin_of(d, k, h0, p0, r) - k * per_cube;
        stage[start[bl] + rank] = r;
      }
      __syncthreads();
      // the chunk's pairs are no longer needed: fetch the next chunk while
      // the runs are written
      if (k == (TWO ? 1 : 0)) {
        gc_cur = s_next;
        if (gc_cur < b.total_schunks) load(gc_cur);
      }
      const bool over = s_over != 0;   // uniform
      for (uint32_t t = threadIdx.x; t < total; t += kScatterThreads) {
        const uint2 v = stage[t];
        const uint32_t bl = bin_of_record(d, v) - k * per_cube;
        rec[(over && t >= cnt[bl] ? dov[bl] : din[bl]) + t] = v;
      }
      __syncthreads();
    }
  }
}

__device__ inline void clear_row_block(const Dims& d, const StreamDesc& st, uint32_t bin) {
  const uint32_t per_cube = d.S * d.R;
  uint64_t* cube = bin < per_cube ? st.cube0 : st.cube1;
  const uint32_t row = bin < per_cube ? bin : bin - per_cube;
  uint4* dst = (uint4*)(cube + (uint64_t)row * d.W);   // W is even, cubes 16-byte aligned
  for (uint32_t w = threadIdx.x; w < d.W / 2; w += 256) dst[w] = make_uint4(0u, 0u, 0u, 0u);
}

// Row blocks of fresh streams that the apply does not store whole (the clear
// list: bins with no records, or with several items, each OR-ed): zeroed
// before the apply. Blocks stride over the list.
__global__ __launch_bounds__(256) void k_clear_fresh(Dims d, Batch b,
                                                     const uint32_t* __restrict__ clear,
                                                     const uint32_t* __restrict__ nclear) {
  const uint32_t n = *nclear;
  for (uint32_t e = blockIdx.x; e < n; e += gridDim.x) {
    const uint32_t v = clear[e];
    clear_row_block(d, b.s[v >> 16], v & 0xFFFFu);
  }
}


// Largest x in [0, n) with tab[x] <= v (tab ascending, tab[0] <= v < tab[n]).
__device__ inline uint32_t upper_index(const uint32_t* tab, uint32_t n, uint32_t v) {
  uint32_t lo = 0, hi = n;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (tab[mid] <= v) lo = mid; else hi = mid;
  }
  return lo;
}

template <int NRA, int NVA>
__global__ __launch_bounds__(kBlock) void k_apply(Dims d, Batch b, const uint2* __restrict__ rec_all,
                                                  const uint32_t* __restrict__ base,
                                                  const uint32_t* __restrict__ fill,
                                                  const uint32_t* __restrict__ segpre,
                                                  const uint32_t* __restrict__ items,
                                                  uint32_t* next) {
  __shared__ __align__(16) uint64_t tile[kMaxTileWords];
  __shared__ uint32_t s_item;
  uint32_t* tile32 = (uint32_t*)tile;
  const uint32_t n_items = items[b.k];
  const uint32_t per_cube = d.S * d.R;
  for (;;) {
    // every thread has read the previous item (the body ends with a barrier)
    if (threadIdx.x == 0)
      s_item = __hip_atomic_fetch_add(next, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const uint32_t item = s_item;
    if (item >= n_items) break;
    const uint32_t si = upper_index(items, b.k, item);
    const StreamDesc& st = b.s[si];
    const uint32_t* bs = base + (uint64_t)si * (b.nbins + 1);
    const uint32_t* sp = segpre + (uint64_t)si * (b.nbins + 1);
    const uint32_t local = item - items[si];
    const uint32_t bin = upper_index(sp, b.nbins, local);
    const uint32_t seg = local - sp[bin];
    const uint64_t r0w = (uint64_t)bs[bin] + (uint64_t)seg * b.seg;
    const uint64_t end = (uint64_t)bs[bin] + fill[(uint64_t)si * b.nbins + bin];
    const uint32_t r0 = (uint32_t)r0w;
    const uint32_t r1 = (uint32_t)(r0w + b.seg < end ? r0w + b.seg : end);
    const uint2* rec = rec_all + st.rec_base;
    uint4* tile4 = (uint4*)tile;
    for (uint32_t w = threadIdx.x; w < d.W / 2; w += kBlock) tile4[w] = make_uint4(0u, 0u, 0u, 0u);
    __syncthreads();
    for (uint32_t i0 = r0 + threadIdx.x; i0 < r1; i0 += kBlock * kApplyUnroll) {
      uint2 rr[kApplyUnroll];
#pragma unroll
      for (int u = 0; u < kApplyUnroll; ++u) {
        const uint32_t i = i0 + u * kBlock;
        rr[u] = i < r1 ? load_rec_nt(rec + i) : make_uint2(0u, 0u);
      }
#pragma unroll
      for (int u = 0; u < kApplyUnroll; ++u) {
        if (i0 + u * kBlock >= r1) break;
        const uint2 r = rr[u];
        const uint32_t lp = r.x >> d.r;
        const uint32_t half = (r.y >> 5) & 1u;
        const uint32_t mask = 1u << (r.y & 31u);
#pragma unroll
        for (int a = 0; a < NRA; ++a) {
          const uint32_t slot = d.aoff[a] + (rotr_in(lp, d.off[a], d.L) & low_mask(d.cbn[a]));
          atomicOr(&tile32[2 * slot + half], mask);
        }
#pragma unroll
        for (int j = 0; j < NVA; ++j) {
          const uint32_t slot = d.aoff[NRA + j] + va_col(d, j, lp);
          atomicOr(&tile32[2 * slot + half], mask);
        }
      }
    }
    __syncthreads();
    uint64_t* cube = bin < per_cube ? st.cube0 : st.cube1;
    const uint32_t row = bin < per_cube ? bin : bin - per_cube;  // = cs * R + rb
    uint64_t* dst = cube + (uint64_t)row * d.W;
    if (st.fresh && sp[bin + 1] - sp[bin] == 1) {
      // sole writer of an empty row block: store it whole
      const uint4* t4 = (const uint4*)tile;
      uint4* d4 = (uint4*)dst;
      for (uint32_t w = threadIdx.x; w < d.W / 2; w += kBlock) store_stream(d4 + w, t4[w]);
    } else {
      for (uint32_t w = threadIdx.x; w < d.W; w += kBlock) {
        const uint64_t v = tile[w];
        if (v) __hip_atomic_fetch_or(dst + w, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    __syncthreads();
  }
}

// The records no region could take: each is OR-ed into its cube with A
// device-scope atomics (Alg. 1 as the direct path does it), after the apply
// has put every tile in place. Block (part, stream); nothing to do in the
// usual case.
template <int NRA, int NVA>
__global__ __launch_bounds__(256) void k_overflow(Dims d, Batch b, const uint2* __restrict__ rec_all,
                                                  const uint32_t* __restrict__ ovfn) {
  const uint32_t si = blockIdx.y;
  const StreamDesc& st = b.s[si];
  const uint32_t n = ovfn[si];
  const uint2* o = rec_all + st.rec_base + st.ovf_off;
  for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const uint2 r = o[i];
    const uint32_t row = r.y & 0x7FFFFFFFu;
    uint64_t* cube = (r.y >> 31) ? st.cube1 : st.cube0;
    const uint32_t cs = r.x & low_mask(d.r), lp = r.x >> d.r;
    uint64_t* blk = cube + ((uint64_t)cs * d.R + (row >> 6)) * d.W;
    const uint64_t bit = 1ull << (row & 63u);
#pragma unroll
    for (int a = 0; a < NRA; ++a)
      __hip_atomic_fetch_or(blk + d.aoff[a] + (rotr_in(lp, d.off[a], d.L) & low_mask(d.cbn[a])), bit,
                            __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
    for (int j = 0; j < NVA; ++j)
      __hip_atomic_fetch_or(blk + d.aoff[NRA + j] + va_col(d, j, lp), bit, __ATOMIC_RELAXED,
                            __HIP_MEMORY_SCOPE_AGENT);
  }
}

int check(const char* what) {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? CBAA_OK : hip_fail(e, what);
}

template <int NRA, int NVA>
int apply_dispatch(const Dims& d, const Batch& b, const Layout& L, uint32_t blocks, hipStream_t s) {
  hipLaunchKernelGGL((k_apply<NRA, NVA>), dim3(blocks), dim3(kBlock), 0, s, d, b, L.rec, L.base,
                     L.tot, L.segpre, L.items, L.next);
  int rc = check("apply launch");
  if (rc != CBAA_OK) return rc;
  hipLaunchKernelGGL((k_overflow<NRA, NVA>), dim3(256, b.k), dim3(256), 0, s, d, b, L.rec, L.ovfn);
  return check("overflow launch");
}

int run_apply(const Dims& d, const Batch& b, const Layout& L, uint32_t blocks, hipStream_t s) {
#define CBAA_APPLY(NRA, NVA) \
  if (d.n_ra == NRA && d.n_va == NVA) return apply_dispatch<NRA, NVA>(d, b, L, blocks, s);
  CBAA_APPLY(2, 0) CBAA_APPLY(2, 1) CBAA_APPLY(2, 2)
  CBAA_APPLY(3, 0) CBAA_APPLY(3, 1) CBAA_APPLY(3, 2)
  CBAA_APPLY(4, 0) CBAA_APPLY(4, 1) CBAA_APPLY(4, 2)
#undef CBAA_APPLY
  return CBAA_ECONFIG;
}

template <bool TWO>
int run(const Dims& d, Batch& b, const Layout& L, uint32_t apply_blocks, hipStream_t s) {
  int rc;
  bool any_fresh = false;
  for (uint32_t i = 0; i < b.k; ++i) any_fresh = any_fresh || b.s[i].fresh;
  // sampled counts, the apply's and the scatter's counters, overflow counts,
  // the clear list's length and the count of streams with their fills done
  const uint32_t nt = b.k * b.nbins + 2 + b.k + 2;
  hipLaunchKernelGGL(k_begin, dim3((nt + 255) / 256), dim3(256), 0, s, d, b, L.tot, nt);
  if ((rc = check("begin launch")) != CBAA_OK) return rc;
  if (b.total_samples == 0) {   // no pairs at all: fresh cubes are just emptied
    for (uint32_t i = 0; i < b.k && any_fresh; ++i) {
      if (!b.s[i].fresh) continue;
      if ((rc = launch_fill_zero(b.s[i].cube0, d.words, s)) != CBAA_OK) return rc;
      if (TWO && (rc = launch_fill_zero(b.s[i].cube1, d.words, s)) != CBAA_OK) return rc;
    }
    return CBAA_OK;
  }
  hipLaunchKernelGGL((k_histogram<TWO>), dim3(b.total_samples), dim3(kBlock), 0, s, d, b, L.tot);
  if ((rc = check("histogram launch")) != CBAA_OK) return rc;
  hipLaunchKernelGGL(k_bases, dim3(b.k), dim3(kBlock), 0, s, b, L.tot, L.base, L.cursor);
  if ((rc = check("bases launch")) != CBAA_OK) return rc;
  const uint32_t sgrid = b.total_schunks < kScatterBlocks ? b.total_schunks : kScatterBlocks;
  if (d.S * d.R <= kSmallBins)
    hipLaunchKernelGGL((k_scatter<TWO, kSmallBins, kScatterPerSmall>), dim3(sgrid),
                       dim3(kScatterThreads), 0, s, d, b, L.cursor, L.base, L.rec, L.ovfn,
                       L.next + 1);
  else
    hipLaunchKernelGGL((k_scatter<TWO, kMaxBins / 2, kScatterPerLarge>), dim3(sgrid),
                       dim3(kScatterThreads), 0, s, d, b, L.cursor, L.base, L.rec, L.ovfn,
                       L.next + 1);
  if ((rc = check("scatter launch")) != CBAA_OK) return rc;
  hipLaunchKernelGGL(k_fills, dim3(b.k), dim3(kBlock), 0, s, b, L.base, L.cursor, L.tot, L.segpre,
                     L.clear, L.nclear, L.items);
  if ((rc = check("fills launch")) != CBAA_OK) return rc;
  if (any_fresh) {
    hipLaunchKernelGGL(k_clear_fresh, dim3(256), dim3(256), 0, s, d, b, L.clear, L.nclear);
    if ((rc = check("clear launch")) != CBAA_OK) return rc;
  }
  return run_apply(d, b, L, apply_blocks, s);
}

}  // namespace

bool partitioned_supported(const Dims& d) {
  // LDS tile of one row block of a sketch; bins of two cubes in LDS counters
  return d.W <= kMaxTileWords && 2u * d.S * d.R <= kMaxBins;
}

bool tuning_valid(const cbaa_tuning* t) {
  if (!t) return true;
  const Tuning r = effective(t);
  // seg is bounded so that the segment arithmetic of the bases and the apply
  // (n + seg - 1, r0 + seg) stays inside 32 bits
  return r.chunk >= 1024 && r.chunk <= (1u << 22) && r.chunk % 1024 == 0 && r.seg >= 1024 &&
         r.seg <= (1u << 24) && r.apply_blocks >= 1 && r.apply_blocks <= 65536;
}

uint64_t batch_scratch_bytes(const Dims& d, const StreamSpec* specs, int k, int n_cubes,
                             const cbaa_tuning* t) {
  Batch b;
  b.k = (uint32_t)k;
  for (int i = 0; i < k; ++i) b.s[i].n = specs[i].n;
  return plan(d, n_cubes, effective(t).chunk, b, nullptr).bytes;
}

int launch_update_batch(const Dims& d, const StreamSpec* specs, int k, int n_cubes,
                        const cbaa_tuning* t, void* scratch, hipStream_t s) {
  const Tuning tu = effective(t);
  Batch b;
  b.k = (uint32_t)k;
  b.seg = tu.seg;
  for (int i = 0; i < k; ++i) {
    b.s[i].pairs = (const uint2*)specs[i].pairs;
    b.s[i].n = specs[i].n;
    b.s[i].cube0 = specs[i].cube0;
    b.s[i].cube1 = specs[i].cube1;
    b.s[i].side = (uint32_t)specs[i].side;
    b.s[i].fresh = specs[i].fresh ? 1u : 0u;
  }
  const Layout L = plan(d, n_cubes, tu.chunk, b, scratch);
  return n_cubes == 2 ? run<true>(d, b, L, tu.apply_blocks, s)
                      : run<false>(d, b, L, tu.apply_blocks, s);
}

bool partitioned_stream_fits(const Dims& d, uint64_t n_pairs, int n_cubes) {
  return fits(n_pairs, (uint32_t)n_cubes, (uint32_t)n_cubes * d.S * d.R);
}

uint64_t partitioned_scratch_bytes(const Dims& d, uint64_t n_pairs, int n_cubes) {
  StreamSpec sp{};
  const uint64_t nb = n_pairs == 0 ? 1 : n_pairs;
  const uint64_t cap = max_stream_pairs(d, n_cubes, kSplit);
  sp.n = nb > cap ? cap : nb;
  return batch_scratch_bytes(d, &sp, 1, n_cubes, nullptr);
}

uint64_t partitioned_min_scratch_bytes(const Dims& d, int n_cubes, uint64_t n_pairs) {
  StreamSpec sp{};
  sp.n = n_pairs < kSplit ? n_pairs : kSplit;
  return batch_scratch_bytes(d, &sp, 1, n_cubes, nullptr);
}

int launch_update_partitioned(const Dims& d, uint64_t* c0, uint64_t* c1, const uint32_t* pairs,
                              uint64_t n, int side, void* scratch, uint64_t scratch_bytes,
                              hipStream_t s) {
  const int nc = c1 ? 2 : 1;
  const uint64_t chunk = kSplit;
  // largest batch (whole chunks) that fits the scratch and 32-bit offsets
  const uint64_t cap = max_stream_pairs(d, nc, chunk);
  auto bytes_for = [&](uint64_t m) {
    StreamSpec sp{};
    sp.n = m;
    return batch_scratch_bytes(d, &sp, 1, nc, nullptr);
  };
  uint64_t nb;
  if (n <= cap && bytes_for(n) <= scratch_bytes) {
    nb = n;
  } else {
    uint64_t lo = 1, hi = (n + chunk - 1) / chunk;  // in chunks
    while (lo < hi) {
      const uint64_t mid = (lo + hi + 1) / 2;
      if (mid * chunk <= cap && bytes_for(mid * chunk) <= scratch_bytes) lo = mid;
      else hi = mid - 1;
    }
    nb = lo * chunk;
  }
  for (uint64_t off = 0; off < n; off += nb) {
    StreamSpec sp{};
    sp.pairs = pairs + 2 * off;
    sp.n = n - off < nb ? n - off : nb;
    sp.cube0 = c0;
    sp.cube1 = c1;
    sp.side = c1 ? CBAA_SIDE_SRC : side;
    const int rc = launch_update_batch(d, &sp, 1, nc, nullptr, scratch, s);
    if (rc != CBAA_OK) return rc;
  }
  return CBAA_OK;
}

}  // namespace cbaa
