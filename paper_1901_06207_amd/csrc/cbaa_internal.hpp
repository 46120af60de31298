// Internal definitions of libcbaa: configuration-derived dimensions passed to
// kernels by value, the mixers, and per-host index arithmetic of Alg. 1.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/cbaa.h"

namespace cbaa {

constexpr int kWave = 64;

// Everything a kernel needs to address a cube, derived once on the host.
struct Dims {
  uint32_t r, n_ra, n_va, A;  // A = n_ra + n_va arrays
  uint32_t L;                 // LP bits = 32 - r
  uint32_t log2_g, g;         // bits per column
  uint32_t R;                 // 64-bit row blocks per column = g / 64
  uint32_t S;                 // sketches = 2^r
  uint32_t W;                 // words per row block of a sketch = sum of c(a)
  uint32_t maxc_ra;           // largest RA column count
  uint32_t cbn[CBAA_MAX_ARRAYS];
  uint32_t ncol[CBAA_MAX_ARRAYS];
  uint32_t aoff[CBAA_MAX_ARRAYS];
  uint32_t off[CBAA_MAX_RA];  // RA field start inside LP
  uint32_t ep[CBAA_MAX_RA];   // |EP(i)|
  uint32_t cp[CBAA_MAX_RA];   // |CP(i)|
  uint32_t seed_mangle, seed_bv;
  uint32_t seed_va[CBAA_MAX_VA];
  uint64_t words;             // 64-bit words of bits per cube (after the header)
  uint64_t hash;              // cbaa_config_hash of the configuration
};

// ---- streaming access ----------------------------------------------------
// Whole-cube passes (merge, column scan) read and write with the
// non-temporal hint: the hundreds of MiB that pass through do not push out
// of L2 what kernels running beside them (a restore's tuple check) keep
// there.
typedef uint32_t u32x4_stream __attribute__((ext_vector_type(4)));
__device__ inline uint4 load_stream(const uint4* p) {
  const u32x4_stream v = __builtin_nontemporal_load((const u32x4_stream*)p);
  return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ inline void store_stream(uint4* p, uint4 v) {
  u32x4_stream w;
  w.x = v.x;
  w.y = v.y;
  w.z = v.z;
  w.w = v.w;
  __builtin_nontemporal_store(w, (u32x4_stream*)p);
}

// ---- cube header ---------------------------------------------------------
// Kernels receive the cube's bits; its header sits the 256 bytes before them.

constexpr uint64_t kHeaderWords = CBAA_HEADER_BYTES / 8;

__host__ __device__ inline uint64_t* header_of(uint64_t* bits) { return bits - kHeaderWords; }
__host__ __device__ inline const uint64_t* header_of(const uint64_t* bits) {
  return bits - kHeaderWords;
}

__device__ inline bool header_ok(const uint64_t* h, const Dims& d) {
  return h[0] == CBAA_CUBE_MAGIC && h[1] == d.hash && h[2] == d.words * 8u &&
         h[3] == (uint64_t)CBAA_ABI_VERSION;   // state VALID in the high half
}

// Writes a whole header: the four defined words (state VALID or MIXED) and
// the reserved words, which are zero.
__device__ inline void header_set(uint64_t* h, const Dims& d, uint32_t state) {
  h[0] = CBAA_CUBE_MAGIC;
  h[1] = d.hash;
  h[2] = d.words * 8u;
  h[3] = ((uint64_t)state << 32) | CBAA_ABI_VERSION;
  for (uint64_t w = 4; w < kHeaderWords; ++w) h[w] = 0;
}

// A cube about to receive more bits keeps a valid header only if it has one.
__device__ inline void header_touch(uint64_t* bits, const Dims& d) {
  uint64_t* h = header_of(bits);
  if (!header_ok(h, d)) header_set(h, d, CBAA_CUBE_MIXED);
}

// ---- mixers (published definitions, written out here) -----------------

// MurmurHash3 32-bit finalizer (fmix32).
__host__ __device__ inline uint32_t fmix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x85EBCA6Bu;
  x ^= x >> 13;
  x *= 0xC2B2AE35u;
  x ^= x >> 16;
  return x;
}

// Exact inverse of fmix32: the xorshifts are undone by re-applying the shift
// until it leaves the word, the multiplies by the modular inverses
// 0xC2B2AE35^-1 = 0x7ED1B41D and 0x85EBCA6B^-1 = 0xA5CB9243 (mod 2^32).
__host__ __device__ inline uint32_t fmix32_inverse(uint32_t y) {
  y ^= y >> 16;
  y *= 0x7ED1B41Du;
  y ^= (y >> 13) ^ (y >> 26);
  y *= 0xA5CB9243u;
  y ^= y >> 16;
  return y;
}

// hash-prospector "lowbias32" (C. Wellons).
__host__ __device__ inline uint32_t lowbias32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7FEB352Du;
  x ^= x >> 15;
  x *= 0x846CA68Bu;
  x ^= x >> 16;
  return x;
}

__host__ __device__ inline uint32_t low_mask(uint32_t bits) {
  return bits >= 32 ? 0xFFFFFFFFu : ((1u << bits) - 1u);
}

// Rotations inside the L-bit LP (L <= 31, 0 <= s < L).
__host__ __device__ inline uint32_t rotr_in(uint32_t x, uint32_t s, uint32_t L) {
  return ((x >> s) | (x << (L - s))) & low_mask(L);
}
__host__ __device__ inline uint32_t rotl_in(uint32_t x, uint32_t s, uint32_t L) {
  return ((x << s) | (x >> (L - s))) & low_mask(L);
}

// Bit of the column an outer IP sets (H_bv of Alg. 1).
__device__ inline uint32_t bit_of_peer(const Dims& d, uint32_t oip) {
  return lowbias32(oip ^ d.seed_bv) >> (32u - d.log2_g);
}

// Alg. 1 index math for one inner IP: sketch id (RP) and the word offset of
// each of its columns inside one row block of that sketch (A_off(a) + col).
template <int NRA, int NVA>
__device__ inline uint32_t host_slots(const Dims& d, uint32_t iip, uint32_t (&slot)[NRA + NVA]) {
  const uint32_t m = fmix32(iip ^ d.seed_mangle);
  const uint32_t lp = m >> d.r;
#pragma unroll
  for (int i = 0; i < NRA; ++i) slot[i] = d.aoff[i] + (rotr_in(lp, d.off[i], d.L) & low_mask(d.cbn[i]));
#pragma unroll
  for (int j = 0; j < NVA; ++j)
    slot[NRA + j] = d.aoff[NRA + j] + (lowbias32(lp ^ d.seed_va[j]) >> (32u - d.cbn[NRA + j]));
  return m & low_mask(d.r);
}

// VA column (without A_off) of an LP.
__device__ inline uint32_t va_col(const Dims& d, int j, uint32_t lp) {
  return lowbias32(lp ^ d.seed_va[j]) >> (32u - d.cbn[d.n_ra + j]);
}

// One stream of a partitioned batch (host side).
struct StreamSpec {
  const uint32_t* pairs;
  uint64_t n;
  uint64_t* cube0;
  uint64_t* cube1;
  int side;
  int fresh;  // cubes start empty (CBAA_BATCH_FRESH)
};

// ---- host-side helpers (cbaa_api.hip) ----------------------------------

bool make_dims(const cbaa_config* cfg, Dims* out);
void set_error(const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);

// Launchers implemented in the kernel files. Each returns CBAA_OK or CBAA_EHIP.
int launch_fill_zero(uint64_t* d, uint64_t words, hipStream_t s);
// Zeroes a cube's bits and writes its whole header (valid).
int launch_cube_init(const Dims& d, uint64_t* bits, hipStream_t s);
int launch_update_direct(const Dims& d, uint64_t* cube0, uint64_t* cube1, const uint32_t* pairs,
                         uint64_t n, int side, hipStream_t s);
int launch_update_partitioned(const Dims& d, uint64_t* cube0, uint64_t* cube1,
                              const uint32_t* pairs, uint64_t n, int side, void* scratch,
                              uint64_t scratch_bytes, hipStream_t s);
uint64_t partitioned_scratch_bytes(const Dims& d, uint64_t n_pairs, int n_cubes);
// Whether one stream of n_pairs pairs fits the partitioned path's 32-bit record offsets.
bool partitioned_stream_fits(const Dims& d, uint64_t n_pairs, int n_cubes);
uint64_t partitioned_min_scratch_bytes(const Dims& d, int n_cubes, uint64_t n_pairs);
bool partitioned_supported(const Dims& d);
bool tuning_valid(const cbaa_tuning* t);
uint64_t batch_scratch_bytes(const Dims& d, const StreamSpec* specs, int k, int n_cubes,
                             const cbaa_tuning* t);
int launch_update_batch(const Dims& d, const StreamSpec* specs, int k, int n_cubes,
                        const cbaa_tuning* t, void* scratch, hipStream_t s);
int launch_merge_or(const Dims& d, uint64_t* dst, const uint64_t* const* srcs, int k,
                    hipStream_t s);
int launch_column_zeros(const Dims& d, const uint64_t* cube, uint16_t* zeros, uint32_t* ones,
                        hipStream_t s);
uint64_t restore_scratch_bytes(const Dims& d, uint64_t capacity);
int launch_restore(const Dims& d, const uint64_t* cube, double x_theta, int rule,
                   uint64_t max_checks, void* scratch, uint64_t capacity, cbaa_host* out,
                   cbaa_restore_stats* stats, hipStream_t s);
// The two halves of launch_merge_restore: reset, OR-merge, column scan,
// thresholds and hot lists (Alg. 2); then the tuple check (Alg. 3) and the
// ordering from the scratch the first half filled.
int launch_merge_scan(const Dims& d, uint64_t* dst, const uint64_t* const* srcs, int k,
                      double x_theta, int rule, void* scratch, uint64_t capacity,
                      cbaa_restore_stats* stats, hipStream_t s);
int launch_restore_scanned(const Dims& d, const uint64_t* dst, const uint64_t* const* srcs,
                           int k, uint64_t max_checks, void* scratch, uint64_t capacity,
                           cbaa_host* out, cbaa_restore_stats* stats, hipStream_t s);
int launch_merge_restore(const Dims& d, uint64_t* dst, const uint64_t* const* srcs, int k,
                         double x_theta, int rule, uint64_t max_checks, void* scratch,
                         uint64_t capacity, cbaa_host* out, cbaa_restore_stats* stats,
                         hipStream_t s);
int launch_features(const Dims& d, const uint64_t* cube, const uint32_t* hosts, uint64_t n,
                    uint32_t F, float* x, void* scratch, hipStream_t s);
int launch_estimate(const Dims& d, const uint64_t* cube, const uint32_t* hosts, uint64_t n,
                    double* est, uint16_t* zeros, uint16_t* layer_zeros, void* scratch,
                    hipStream_t s);

}  // namespace cbaa
