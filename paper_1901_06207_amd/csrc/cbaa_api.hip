// C ABI entry points of libcbaa: argument checks, configuration-derived
// dimensions, and dispatch to the kernel launchers. Every compute step runs
// in the HIP kernels of the sibling files; this file only validates, sizes
// and enqueues.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>

#include "../../include/cbaa_mlp.h"
#include "cbaa_internal.hpp"

namespace cbaa {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
}

int hip_fail(hipError_t e, const char* what) {
  set_error("%s: %s (%d)", what, hipGetErrorString(e), (int)e);
  return CBAA_EHIP;
}

// Validation rules of cbaa_config_validate; fills the derived dimensions.
bool make_dims(const cbaa_config* c, Dims* o) {
  if (!c) {
    set_error("null configuration");
    return false;
  }
  if (c->r < 1 || c->r > 8) return set_error("r=%u outside [1,8]", c->r), false;
  if (c->n_ra < 2 || c->n_ra > CBAA_MAX_RA) return set_error("n_ra=%u outside [2,4]", c->n_ra), false;
  if (c->n_va > CBAA_MAX_VA) return set_error("n_va=%u above 2", c->n_va), false;
  if (c->log2_g < 6 || c->log2_g > 15) return set_error("log2_g=%u outside [6,15]", c->log2_g), false;
  Dims d;
  memset(&d, 0, sizeof d);
  d.r = c->r;
  d.n_ra = c->n_ra;
  d.n_va = c->n_va;
  d.A = c->n_ra + c->n_va;
  d.L = 32u - c->r;
  d.log2_g = c->log2_g;
  d.g = 1u << c->log2_g;
  d.R = d.g / 64u;
  d.S = 1u << c->r;
  uint64_t W = 0;
  for (uint32_t a = 0; a < d.A; ++a) {
    if (c->cbn[a] < 1 || c->cbn[a] > 16) return set_error("cbn[%u]=%u outside [1,16]", a, c->cbn[a]), false;
    d.cbn[a] = c->cbn[a];
    d.ncol[a] = 1u << c->cbn[a];
    d.aoff[a] = (uint32_t)W;
    W += d.ncol[a];
  }
  d.W = (uint32_t)W;
  for (uint32_t i = 0; i < d.n_ra; ++i) {
    if (c->cl_bs[i] < c->r || c->cl_bs[i] > 31)
      return set_error("cl_bs[%u]=%u outside [r,31]", i, c->cl_bs[i]), false;
    if (i > 0 && c->cl_bs[i] <= c->cl_bs[i - 1])
      return set_error("cl_bs must increase strictly"), false;
    if (c->cbn[i] > d.L) return set_error("cbn[%u]=%u exceeds the %u LP bits", i, c->cbn[i], d.L), false;
    d.off[i] = c->cl_bs[i] - c->r;
    if (d.ncol[i] > d.maxc_ra) d.maxc_ra = d.ncol[i];
  }
  for (uint32_t i = 0; i < d.n_ra; ++i) {
    uint32_t nx = (i + 1) % d.n_ra;
    uint32_t e = (d.off[nx] + d.L - d.off[i]) % d.L;
    d.ep[i] = e == 0 ? d.L : e;
  }
  for (uint32_t i = 0; i < d.n_ra; ++i) {
    int32_t cp = (int32_t)d.cbn[i] - (int32_t)d.ep[i];
    if (cp < 0) return set_error("|CP(%u)| < 0: LP bits not covered by RA columns", i), false;
    if ((uint32_t)cp > d.ep[(i + 1) % d.n_ra])
      return set_error("|CP(%u)|=%d exceeds |EP(%u)|", i, cp, (i + 1) % d.n_ra), false;
    d.cp[i] = (uint32_t)cp;
  }
  d.seed_mangle = c->seed_mangle;
  d.seed_bv = c->seed_bv;
  for (uint32_t j = 0; j < CBAA_MAX_VA; ++j) d.seed_va[j] = c->seed_va[j];
  d.words = (uint64_t)d.S * d.R * d.W;
  // FNV-1a over the defined fields' little-endian bytes (cbaa_config_hash)
  uint64_t h = 0xCBF29CE484222325ull;
  auto mix = [&](uint32_t v) {
    for (int k = 0; k < 4; ++k) {
      h ^= (v >> (8 * k)) & 0xFFu;
      h *= 0x100000001B3ull;
    }
  };
  mix(c->r);
  mix(c->n_ra);
  mix(c->n_va);
  mix(c->log2_g);
  for (uint32_t a = 0; a < d.A; ++a) mix(c->cbn[a]);
  for (uint32_t i = 0; i < d.n_ra; ++i) mix(c->cl_bs[i]);
  mix(c->seed_mangle);
  mix(c->seed_bv);
  for (uint32_t j = 0; j < d.n_va; ++j) mix(c->seed_va[j]);
  d.hash = h;
  *o = d;
  return true;
}

}  // namespace cbaa

using namespace cbaa;

#define CHECK_DIMS(cfg, d)                 \
  Dims d;                                  \
  if (!make_dims((cfg), &d)) return CBAA_ECONFIG

// The bits of a caller's cube (after its header).
static inline uint64_t* bits_of(void* cube) {
  return cube ? (uint64_t*)((char*)cube + CBAA_HEADER_BYTES) : nullptr;
}
static inline const uint64_t* bits_of(const void* cube) {
  return cube ? (const uint64_t*)((const char*)cube + CBAA_HEADER_BYTES) : nullptr;
}

#define REQUIRE(cond, ...)        \
  do {                            \
    if (!(cond)) {                \
      set_error(__VA_ARGS__);     \
      return CBAA_EINVAL;         \
    }                             \
  } while (0)

extern "C" {

uint32_t cbaa_abi_version(void) { return CBAA_ABI_VERSION; }

int cbaa_config_default(cbaa_config* out) {
  REQUIRE(out, "null output");
  memset(out, 0, sizeof *out);
  out->r = 4;
  out->n_ra = 3;
  out->n_va = 1;
  out->log2_g = 12;
  for (int a = 0; a < 4; ++a) out->cbn[a] = 12;
  out->cl_bs[0] = 4;
  out->cl_bs[1] = 14;
  out->cl_bs[2] = 23;
  out->seed_mangle = 0x243F6A88u;
  out->seed_bv = 0x85A308D3u;
  out->seed_va[0] = 0x13198A2Eu;
  out->seed_va[1] = 0x03707344u;
  return CBAA_OK;
}

int cbaa_config_validate(const cbaa_config* cfg) {
  CHECK_DIMS(cfg, d);
  (void)d;
  return CBAA_OK;
}

uint64_t cbaa_cube_bytes(const cbaa_config* cfg) {
  Dims d;
  if (!make_dims(cfg, &d)) return 0;
  return CBAA_HEADER_BYTES + d.words * 8u;
}

uint64_t cbaa_config_hash(const cbaa_config* cfg) {
  Dims d;
  if (!make_dims(cfg, &d)) return 0;
  return d.hash;
}

int cbaa_cube_check(const cbaa_config* cfg, const void* d_cube, void* stream) {
  CHECK_DIMS(cfg, d);
  REQUIRE(d_cube && ((uintptr_t)d_cube & 15u) == 0, "cube must be a non-null 16-byte aligned pointer");
  uint64_t h[4];
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(h, d_cube, sizeof h, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "header read");
  if (h[0] != CBAA_CUBE_MAGIC) return set_error("no cube header (magic missing)"), CBAA_ECONFIG;
  if (h[1] != d.hash) return set_error("cube built with another configuration"), CBAA_ECONFIG;
  if (h[2] != d.words * 8u) return set_error("cube size differs from the configuration's"), CBAA_ECONFIG;
  if ((uint32_t)h[3] != CBAA_ABI_VERSION) return set_error("cube header of ABI version %u", (uint32_t)h[3]), CBAA_ECONFIG;
  if ((h[3] >> 32) != CBAA_CUBE_VALID)
    return set_error("cube holds bits of another configuration or of a cube without a header"), CBAA_ECONFIG;
  return CBAA_OK;
}

uint64_t cbaa_update_scratch_bytes(const cbaa_config* cfg, uint64_t n_pairs, int n_cubes) {
  Dims d;
  if (!make_dims(cfg, &d) || (n_cubes != 1 && n_cubes != 2) || !partitioned_supported(d)) return 0;
  return partitioned_scratch_bytes(d, n_pairs, n_cubes);
}

uint64_t cbaa_restore_scratch_bytes(const cbaa_config* cfg, uint64_t capacity) {
  Dims d;
  if (!make_dims(cfg, &d)) return 0;
  return restore_scratch_bytes(d, capacity);
}

int cbaa_cube_init(const cbaa_config* cfg, void* d_cube, void* stream) {
  CHECK_DIMS(cfg, d);
  REQUIRE(d_cube && ((uintptr_t)d_cube & 15u) == 0, "cube must be a non-null 16-byte aligned pointer");
  return launch_cube_init(d, bits_of(d_cube), (hipStream_t)stream);
}

static int update_common(const Dims& d, void* c0, void* c1, const uint32_t* pairs, uint64_t n,
                         int side, void* scratch, uint64_t scratch_bytes, void* stream) {
  REQUIRE(c0 && ((uintptr_t)c0 & 15u) == 0, "cube must be a non-null 16-byte aligned pointer");
  REQUIRE(!c1 || ((uintptr_t)c1 & 15u) == 0, "second cube must be 16-byte aligned");
  REQUIRE(side == CBAA_SIDE_SRC || side == CBAA_SIDE_DST, "side must be CBAA_SIDE_SRC or _DST");
  if (n == 0) return CBAA_OK;
  REQUIRE(pairs && ((uintptr_t)pairs & 7u) == 0, "pairs must be a non-null 8-byte aligned pointer");
  REQUIRE(n < (1ull << 40), "n_pairs too large");
  hipStream_t s = (hipStream_t)stream;
  if (scratch == nullptr || scratch_bytes == 0 || !partitioned_supported(d))
    return launch_update_direct(d, bits_of(c0), bits_of(c1), pairs, n, side, s);
  if (scratch_bytes < partitioned_min_scratch_bytes(d, c1 ? 2 : 1, n)) {
    set_error("update scratch of %llu bytes is below the minimum %llu",
              (unsigned long long)scratch_bytes,
              (unsigned long long)partitioned_min_scratch_bytes(d, c1 ? 2 : 1, n));
    return CBAA_ESCRATCH;
  }
  REQUIRE(((uintptr_t)scratch & 255u) == 0, "scratch must be 256-byte aligned");
  return launch_update_partitioned(d, bits_of(c0), bits_of(c1), pairs, n, side, scratch,
                                   scratch_bytes, s);
}

int cbaa_update(const cbaa_config* cfg, void* d_cube, const uint32_t* d_pairs, uint64_t n_pairs,
                int side, void* d_scratch, uint64_t scratch_bytes, void* stream) {
  CHECK_DIMS(cfg, d);
  return update_common(d, d_cube, nullptr, d_pairs, n_pairs, side, d_scratch, scratch_bytes, stream);
}

int cbaa_update2(const cbaa_config* cfg, void* d_cube_src, void* d_cube_dst,
                 const uint32_t* d_pairs, uint64_t n_pairs, void* d_scratch,
                 uint64_t scratch_bytes, void* stream) {
  CHECK_DIMS(cfg, d);
  REQUIRE(d_cube_dst, "destination-keyed cube is null");
  REQUIRE(d_cube_src != d_cube_dst, "the two cubes must differ");
  return update_common(d, d_cube_src, d_cube_dst, d_pairs, n_pairs, CBAA_SIDE_SRC, d_scratch,
                       scratch_bytes, stream);
}

// Checks a stream table; returns the cube count (1 or 2) or a negative code.
static int check_streams(const Dims& d, const cbaa_stream_batch* h, int k, StreamSpec* out) {
  REQUIRE(h && k >= 1 && k <= CBAA_MAX_BATCH, "need 1..%d streams", CBAA_MAX_BATCH);
  if (!partitioned_supported(d)) {
    set_error("configuration outside the partitioned update's limits");
    return CBAA_ECONFIG;
  }
  const int nc = h[0].d_cube_dst ? 2 : 1;
  for (int i = 0; i < k; ++i) {
    const cbaa_stream_batch& s = h[i];
    REQUIRE((s.d_cube_dst != nullptr) == (nc == 2), "streams mix one- and two-cube updates");
    REQUIRE(s.d_cube && ((uintptr_t)s.d_cube & 15u) == 0, "stream %d: cube null or misaligned", i);
    REQUIRE(!s.d_cube_dst || ((uintptr_t)s.d_cube_dst & 15u) == 0,
            "stream %d: destination cube misaligned", i);
    REQUIRE(s.d_cube != s.d_cube_dst, "stream %d: the two cubes must differ", i);
    REQUIRE(nc == 2 || s.side == CBAA_SIDE_SRC || s.side == CBAA_SIDE_DST, "stream %d: bad side", i);
    REQUIRE(s.n_pairs == 0 || (s.d_pairs && ((uintptr_t)s.d_pairs & 7u) == 0),
            "stream %d: pairs null or misaligned", i);
    REQUIRE(partitioned_stream_fits(d, s.n_pairs, nc), "stream %d: too many pairs", i);
    REQUIRE((s.flags & ~CBAA_BATCH_FRESH) == 0, "stream %d: unknown flags", i);
    if (s.flags & CBAA_BATCH_FRESH)
      for (int j = 0; j < k; ++j) {
        if (j == i) continue;
        const void* mine[2] = {s.d_cube, s.d_cube_dst};
        for (const void* c : mine)
          REQUIRE(!c || (c != h[j].d_cube && c != h[j].d_cube_dst),
                  "stream %d: a fresh stream's cube is also named by stream %d", i, j);
      }
    out[i].fresh = (s.flags & CBAA_BATCH_FRESH) ? 1 : 0;
    out[i].pairs = s.d_pairs;
    out[i].n = s.n_pairs;
    out[i].cube0 = bits_of(s.d_cube);
    out[i].cube1 = bits_of(s.d_cube_dst);
    out[i].side = nc == 2 ? CBAA_SIDE_SRC : s.side;
  }
  return nc;
}

uint64_t cbaa_update_batch_scratch_bytes(const cbaa_config* cfg, const cbaa_stream_batch* h,
                                         int k, const cbaa_tuning* t) {
  Dims d;
  if (!make_dims(cfg, &d) || !tuning_valid(t)) return 0;
  StreamSpec sp[CBAA_MAX_BATCH];
  const int nc = check_streams(d, h, k, sp);
  if (nc < 0) return 0;
  return batch_scratch_bytes(d, sp, k, nc, t);
}

int cbaa_update_batch(const cbaa_config* cfg, const cbaa_stream_batch* h, int k,
                      const cbaa_tuning* t, void* d_scratch, uint64_t scratch_bytes,
                      void* stream) {
  CHECK_DIMS(cfg, d);
  REQUIRE(tuning_valid(t), "tuning out of range");
  StreamSpec sp[CBAA_MAX_BATCH];
  const int nc = check_streams(d, h, k, sp);
  if (nc < 0) return nc;
  const uint64_t need = batch_scratch_bytes(d, sp, k, nc, t);
  if (!d_scratch || scratch_bytes < need) {
    set_error("batch scratch of %llu bytes is below the required %llu",
              (unsigned long long)scratch_bytes, (unsigned long long)need);
    return CBAA_ESCRATCH;
  }
  REQUIRE(((uintptr_t)d_scratch & 255u) == 0, "scratch must be 256-byte aligned");
  return launch_update_batch(d, sp, k, nc, t, d_scratch, (hipStream_t)stream);
}

int cbaa_merge_or(const cbaa_config* cfg, void* d_dst, const void* const* h_srcs, int k,
                  void* stream) {
  CHECK_DIMS(cfg, d);
  REQUIRE(d_dst && ((uintptr_t)d_dst & 15u) == 0, "destination must be a non-null 16-byte aligned pointer");
  REQUIRE(h_srcs && k >= 1, "need at least one source cube");
  for (int i = 0; i < k; ++i)
    REQUIRE(h_srcs[i] && ((uintptr_t)h_srcs[i] & 15u) == 0, "source %d null or not 16-byte aligned", i);
  const uint64_t* stack[64];
  const uint64_t** b = k <= 64 ? stack : new const uint64_t*[k];
  for (int i = 0; i < k; ++i) b[i] = bits_of(h_srcs[i]);
  const int rc = launch_merge_or(d, bits_of(d_dst), b, k, (hipStream_t)stream);
  if (b != stack) delete[] b;
  return rc;
}

int cbaa_column_zeros(const cbaa_config* cfg, const void* d_cube, uint16_t* d_zeros,
                      uint32_t* d_ones, void* stream) {
  CHECK_DIMS(cfg, d);
  REQUIRE(d_cube && ((uintptr_t)d_cube & 15u) == 0, "cube must be 16-byte aligned");
  REQUIRE(d_zeros && d_ones, "null output");
  REQUIRE(((uintptr_t)d_zeros & 3u) == 0 && ((uintptr_t)d_ones & 3u) == 0,
          "outputs must be 4-byte aligned");
  return launch_column_zeros(d, bits_of(d_cube), d_zeros, d_ones, (hipStream_t)stream);
}

int cbaa_restore(const cbaa_config* cfg, const void* d_cube, double theta, int thr_rule,
                 uint64_t max_checks, void* d_scratch, uint64_t scratch_bytes, cbaa_host* d_out,
                 uint64_t capacity, cbaa_restore_stats* d_stats, void* stream) {
  CHECK_DIMS(cfg, d);
  REQUIRE(d_cube && ((uintptr_t)d_cube & 15u) == 0, "cube must be 16-byte aligned");
  REQUIRE(thr_rule == CBAA_THR_THM2 || thr_rule == CBAA_THR_PAPER, "unknown threshold rule");
  REQUIRE(theta >= 0.0 && isfinite(theta), "theta must be finite and non-negative");
  REQUIRE(d_stats, "null stats");
  REQUIRE(capacity == 0 || d_out, "null output with non-zero capacity");
  REQUIRE(capacity < (1ull << 32), "capacity must be below 2^32");
  REQUIRE(d_scratch && ((uintptr_t)d_scratch & 255u) == 0, "scratch must be 256-byte aligned");
  if (scratch_bytes < restore_scratch_bytes(d, capacity)) {
    set_error("restore scratch of %llu bytes is below the required %llu",
              (unsigned long long)scratch_bytes,
              (unsigned long long)restore_scratch_bytes(d, capacity));
    return CBAA_ESCRATCH;
  }
  // exp(-theta/g) is taken once here so that the threshold of every sketch
  // is computed from the same IEEE double on the device.
  const double x = exp(-theta / (double)d.g);
  return launch_restore(d, bits_of(d_cube), x, thr_rule,
                        max_checks ? max_checks : CBAA_DEFAULT_MAX_CHECKS, d_scratch, capacity,
                        d_out, d_stats, (hipStream_t)stream);
}

// Argument checks and launch of the window end, shared by cbaa_merge_restore
// (caller's scratch) and cbaa_merge_restore_noalloc (the library's array).
// Which part of the window end a call runs.
enum MergePhase { kBoth, kScanOnly, kRestoreOnly };

static int merge_restore_checked(const Dims& d, void* d_dst, const void* const* h_srcs, int k,
                                 double theta, int thr_rule, uint64_t max_checks, void* d_scratch,
                                 uint64_t scratch_bytes, cbaa_host* d_out, uint64_t capacity,
                                 cbaa_restore_stats* d_stats, void* stream,
                                 MergePhase phase = kBoth) {
  // a null destination (merge not stored) is served by the one-pass scan,
  // which takes up to 16 sources
  REQUIRE(((uintptr_t)d_dst & 15u) == 0, "destination must be 16-byte aligned");
  REQUIRE(h_srcs && k >= 1, "need at least one source cube");
  REQUIRE(d_dst || k <= 16, "more than 16 source cubes need a destination cube");
  for (int i = 0; i < k; ++i)
    REQUIRE(h_srcs[i] && ((uintptr_t)h_srcs[i] & 15u) == 0, "source %d null or not 16-byte aligned", i);
  REQUIRE(thr_rule == CBAA_THR_THM2 || thr_rule == CBAA_THR_PAPER, "unknown threshold rule");
  REQUIRE(theta >= 0.0 && isfinite(theta), "theta must be finite and non-negative");
  REQUIRE(d_stats, "null stats");
  REQUIRE(capacity == 0 || d_out, "null output with non-zero capacity");
  REQUIRE(capacity < (1ull << 32), "capacity must be below 2^32");
  REQUIRE(d_scratch && ((uintptr_t)d_scratch & 255u) == 0, "scratch must be 256-byte aligned");
  if (scratch_bytes < restore_scratch_bytes(d, capacity)) {
    set_error("restore scratch of %llu bytes is below the required %llu",
              (unsigned long long)scratch_bytes,
              (unsigned long long)restore_scratch_bytes(d, capacity));
    return CBAA_ESCRATCH;
  }
  const double x = exp(-theta / (double)d.g);
  const uint64_t* stack[64];
  const uint64_t** b = k <= 64 ? stack : new const uint64_t*[k];
  for (int i = 0; i < k; ++i) b[i] = bits_of(h_srcs[i]);
  const uint64_t mc = max_checks ? max_checks : CBAA_DEFAULT_MAX_CHECKS;
  const hipStream_t s = (hipStream_t)stream;
  const int rc =
      phase == kScanOnly
          ? launch_merge_scan(d, bits_of(d_dst), b, k, x, thr_rule, d_scratch, capacity, d_stats, s)
      : phase == kRestoreOnly
          ? launch_restore_scanned(d, bits_of(d_dst), b, k, mc, d_scratch, capacity, d_out,
                                   d_stats, s)
          : launch_merge_restore(d, bits_of(d_dst), b, k, x, thr_rule, mc, d_scratch, capacity,
                                 d_out, d_stats, s);
  if (b != stack) delete[] b;
  return rc;
}

int cbaa_merge_restore(const cbaa_config* cfg, void* d_dst, const void* const* h_srcs, int k,
                       double theta, int thr_rule, uint64_t max_checks, void* d_scratch,
                       uint64_t scratch_bytes, cbaa_host* d_out, uint64_t capacity,
                       cbaa_restore_stats* d_stats, void* stream) {
  CHECK_DIMS(cfg, d);
  return merge_restore_checked(d, d_dst, h_srcs, k, theta, thr_rule, max_checks, d_scratch,
                               scratch_bytes, d_out, capacity, d_stats, stream);
}

int cbaa_merge_scan(const cbaa_config* cfg, void* d_dst, const void* const* h_srcs, int k,
                    double theta, int thr_rule, uint64_t max_checks, void* d_scratch,
                    uint64_t scratch_bytes, cbaa_host* d_out, uint64_t capacity,
                    cbaa_restore_stats* d_stats, void* stream) {
  CHECK_DIMS(cfg, d);
  return merge_restore_checked(d, d_dst, h_srcs, k, theta, thr_rule, max_checks, d_scratch,
                               scratch_bytes, d_out, capacity, d_stats, stream, kScanOnly);
}

int cbaa_restore_scanned(const cbaa_config* cfg, void* d_dst, const void* const* h_srcs, int k,
                         double theta, int thr_rule, uint64_t max_checks, void* d_scratch,
                         uint64_t scratch_bytes, cbaa_host* d_out, uint64_t capacity,
                         cbaa_restore_stats* d_stats, void* stream) {
  CHECK_DIMS(cfg, d);
  return merge_restore_checked(d, d_dst, h_srcs, k, theta, thr_rule, max_checks, d_scratch,
                               scratch_bytes, d_out, capacity, d_stats, stream, kRestoreOnly);
}

}  // extern "C"

// Scratch of cbaa_merge_restore_noalloc. Each device holds its own copy of
// this array from the library's first use on it until the process ends. In
// host code the name is only a host-side stand-in, never a device address:
// the address comes from hipGetSymbolAddress, resolved once per device with
// that device current, and only that address is handed to kernels.
static __device__ __align__(256) uint64_t g_noalloc_scratch[CBAA_NOALLOC_SCRATCH_BYTES / 8];

namespace {

constexpr int kNoAllocDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kNoAllocDevices];

// Device address of the current device's copy of g_noalloc_scratch.
int noalloc_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kNoAllocDevices) {
    set_error("device %d beyond the %d the no-allocation scratch table covers", dev, kNoAllocDevices);
    return CBAA_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_noalloc_scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(no-allocation scratch)");
    if (!p) {
      set_error("hipGetSymbolAddress returned a null address for the no-allocation scratch");
      return CBAA_EHIP;
    }
    g_noalloc_ptr[dev] = p;
  }
  *out = g_noalloc_ptr[dev];
  return CBAA_OK;
}

}  // namespace

extern "C" {

int cbaa_merge_restore_noalloc(const cbaa_config* cfg, void* d_dst, const void* const* h_srcs,
                               int k, double theta, int thr_rule, uint64_t max_checks,
                               cbaa_host* d_out, uint64_t capacity, cbaa_restore_stats* d_stats,
                               void* stream) {
  CHECK_DIMS(cfg, d);
  // the source table stays on the stack: nothing on this path allocates
  REQUIRE(k <= 64, "at most 64 source cubes");
  REQUIRE(capacity < (1ull << 32), "capacity must be below 2^32");
  const uint64_t need = restore_scratch_bytes(d, capacity);
  if (need > CBAA_NOALLOC_SCRATCH_BYTES) {
    set_error("this configuration and capacity need %llu bytes of scratch, above the %llu of "
              "the no-allocation entry point; use cbaa_merge_restore with a caller buffer",
              (unsigned long long)need, (unsigned long long)CBAA_NOALLOC_SCRATCH_BYTES);
    return CBAA_ESCRATCH;
  }
  void* scratch = nullptr;
  const int rc = noalloc_scratch(&scratch);
  if (rc != CBAA_OK) return rc;
  return merge_restore_checked(d, d_dst, h_srcs, k, theta, thr_rule, max_checks, scratch,
                               CBAA_NOALLOC_SCRATCH_BYTES, d_out, capacity, d_stats, stream);
}

int cbaa_estimate(const cbaa_config* cfg, const void* d_cube, const uint32_t* d_hosts, uint64_t n,
                  double* d_est, uint16_t* d_zeros, uint16_t* d_layer_zeros, void* d_scratch,
                  uint64_t scratch_bytes, void* stream) {
  CHECK_DIMS(cfg, d);
  REQUIRE(d_cube && ((uintptr_t)d_cube & 15u) == 0, "cube must be 16-byte aligned");
  REQUIRE(d_scratch && ((uintptr_t)d_scratch & 255u) == 0, "scratch must be 256-byte aligned");
  if (scratch_bytes < restore_scratch_bytes(d, 0)) {
    set_error("estimate scratch too small");
    return CBAA_ESCRATCH;
  }
  if (n == 0) return CBAA_OK;
  REQUIRE(d_hosts && d_est && d_zeros, "null host list or output");
  REQUIRE(n < (1ull << 32), "n must be below 2^32");
  return launch_estimate(d, bits_of(d_cube), d_hosts, n, d_est, d_zeros, d_layer_zeros,
                         d_scratch, (hipStream_t)stream);
}

int cbaa_mlp_features(const cbaa_config* cfg, const void* d_cube, const uint32_t* d_hosts,
                      uint64_t n, uint32_t n_features, float* d_x, void* d_scratch,
                      uint64_t scratch_bytes, void* stream) {
  CHECK_DIMS(cfg, d);
  REQUIRE(d_cube && ((uintptr_t)d_cube & 15u) == 0, "cube must be 16-byte aligned");
  REQUIRE(n_features == d.A || n_features == d.A + 2 || n_features == d.A + 4,
          "n_features must be A, A + 2 or A + 4");
  REQUIRE(n_features <= 8, "at most 8 features");
  REQUIRE(d_scratch && ((uintptr_t)d_scratch & 255u) == 0, "scratch must be 256-byte aligned");
  if (scratch_bytes < restore_scratch_bytes(d, 0)) {
    set_error("features scratch too small");
    return CBAA_ESCRATCH;
  }
  if (n == 0) return CBAA_OK;
  REQUIRE(d_hosts && d_x, "null host list or output");
  REQUIRE(n < (1ull << 32), "n must be below 2^32");
  return launch_features(d, bits_of(d_cube), d_hosts, n, n_features, d_x, d_scratch,
                         (hipStream_t)stream);
}

const char* cbaa_strerror(int code) {
  switch (code) {
    case CBAA_OK: return "ok";
    case CBAA_EINVAL: return "invalid argument";
    case CBAA_ECONFIG: return "invalid configuration";
    case CBAA_ESCRATCH: return "scratch buffer too small";
    case CBAA_EHIP: return "HIP runtime error";
    default: return "unknown error";
  }
}

const char* cbaa_last_error(void) { return g_err; }

}  // extern "C"
