/*
 * CBAA oracle -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH.
 *
 * A plain, single-threaded, obviously-correct CPU implementation of what the
 * CBAA super-host detector computes (Xu, Ding, Hu: "GPU based Real-time Super
 * Hosts Detection at Distributed Edge Routers", arXiv 1901.06207):
 *
 *   - the per-pair cube update                      (Sec. 3.2, Alg. 1)
 *   - the OR-merge of local cubes                   (Sec. 3.3, opening paragraph)
 *   - per-column zero counts, per-array fill        (Sec. 3.3, Alg. 2; Sec. 4.2)
 *   - the shared-bit probability and threshold      (Thm. 1, Thm. 2, Sec. 3.3)
 *   - hot-column lists                              (Def. 3, Alg. 2)
 *   - the hot-column tuple check                    (Alg. 3, with the EP/CP
 *                                                    lengths of Sec. 3.3)
 *   - reassembly LP || RP and unmangling            (Sec. 3.1 mangling, end of Sec. 3.3)
 *   - the corrected linear-counting estimate        (Eq. 1, Thm. 2)
 *   - exact per-host distinct-peer counts           (Sec. 3.1 "exact way"; Sec. 5.1 baseline)
 *   - per-row fills and the row-aware shared-bit mass (an extension of Thm. 1
 *     used by the learned estimator; it reduces to g * eps when every row of
 *     an array is equally full)
 *
 * Only tests/, the smoke entry and the benchmark's CPU-baseline leg may load
 * this library. It shares no code with the HIP library: no header, no helper,
 * no table. Both sides implement the same documented definitions (hash
 * functions, cube memory layout) independently.
 *
 * Readings of places where the paper is silent or inconsistent (each one is
 * listed in the design notes):
 *   R-bits   bit 0 is the least significant bit; RP is bits 0..r-1 of the
 *            mangled IP, LP is bits r..31 shifted down.
 *   R-wrap   an RA field that runs past bit 31 wraps inside LP (index mod
 *            32-r), never into RP.
 *   R-EP     |EP(i)| = (o(i+1) - o(i)) mod (32-r), o(i) = CL_bs(i) - r, and
 *            |CP(i)| = cbn(i) - |EP(i)|.
 *   R-first  the "first |CP(i)| bits" of the next column index are its low bits.
 *   R-eps    eta is not observable; each array's fill ones/(c*g) stands for
 *            P_1(i) of Thm. 1, and eps is their product in array order.
 *   R-thr    default threshold rule THM2: Zmax = floor((g - g*eps) * exp(-theta/g)),
 *            which is what Thm. 2 gives for est >= theta. The printed rule of
 *            Sec. 3.3, (g + g*eps) * exp(-theta/g) - g*eps, is rule PAPER.
 *   R-cmp    a column is hot and a tuple accepted iff zeros <= Zmax (integer).
 *   R-merge  local cubes are merged by bitwise OR from all-zero cubes.
 *   R-est    Z = 0 is taken as Z = 1 with the SATURATED flag; est is clamped >= 0.
 *   R-hash   mangle M(x) = fmix32(x ^ seed_mangle) with fmix32 the published
 *            MurmurHash3 32-bit finalizer (an invertible mixer); H_bv and H_j
 *            take the top bits of lowbias32(x ^ seed), lowbias32 being
 *            C. Wellons' published hash-prospector mixer.
 *   R-layout the cube is 64-bit little-endian words; bit b of column col of
 *            array a in sketch cs lives in word
 *                ((cs * R + (b >> 6)) * W) + A_off(a) + col,   bit (b & 63),
 *            with R = g/64, W = sum of c(a), A_off(a) = sum of c(a') for a' < a.
 *
 * Floating point: fp64 throughout; build with -ffp-contract=off so no fused
 * multiply-add changes a rounding.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define REF_MAX_RA 4
#define REF_MAX_VA 2
#define REF_MAX_ARRAYS (REF_MAX_RA + REF_MAX_VA)

typedef struct ref_config {
  uint32_t r;                     /* 2^r cardinality sketches (Sec. 3.1) */
  uint32_t n_ra;                  /* |RA| */
  uint32_t n_va;                  /* |VA| */
  uint32_t log2_g;                /* g = 2^log2_g bits per column */
  uint32_t cbn[REF_MAX_ARRAYS];   /* c(i) = 2^cbn(i) columns; RAs first, then VAs */
  uint32_t cl_bs[REF_MAX_RA];     /* CL_bs(i): first IP bit of RA i's column index */
  uint32_t seed_mangle;
  uint32_t seed_bv;
  uint32_t seed_va[REF_MAX_VA];
} ref_config;

typedef struct ref_host {
  uint32_t ip;      /* restored, unmangled IPv4 address */
  uint16_t zeros;   /* Z: zero bits of the union column */
  uint8_t cs;       /* cardinality sketch id = RP */
  uint8_t flags;    /* bit 0: SATURATED (Z == 0) */
  double est;       /* Thm. 2 estimate */
} ref_host;

typedef struct ref_restore_stats {
  uint64_t hot_columns;   /* sum over sketches and RAs of |HC(i)| */
  uint64_t tuples;        /* tuples enumerated (product of list sizes) */
  uint64_t cp_valid;      /* tuples that pass every CP check */
  uint64_t accepted;      /* tuples whose union column passes the threshold */
} ref_restore_stats;

enum { REF_SIDE_SRC = 0, REF_SIDE_DST = 1 };
enum { REF_THR_THM2 = 0, REF_THR_PAPER = 1 };
enum { REF_FLAG_SATURATED = 1 };

/* ------------------------------------------------------------------ */
/* Derived quantities                                                   */
/* ------------------------------------------------------------------ */

static uint32_t n_arrays(const ref_config* c) { return c->n_ra + c->n_va; }
static uint32_t lp_bits(const ref_config* c) { return 32u - c->r; }
static uint64_t g_bits(const ref_config* c) { return 1ull << c->log2_g; }
static uint64_t n_cols(const ref_config* c, uint32_t a) { return 1ull << c->cbn[a]; }
static uint64_t row_blocks(const ref_config* c) { return g_bits(c) / 64u; }

static uint64_t slab_words(const ref_config* c) {
  uint64_t w = 0;
  for (uint32_t a = 0; a < n_arrays(c); ++a) w += n_cols(c, a);
  return w;
}

static uint64_t array_offset(const ref_config* c, uint32_t a) {
  uint64_t off = 0;
  for (uint32_t k = 0; k < a; ++k) off += n_cols(c, k);
  return off;
}

static uint32_t mask32(uint32_t bits) { return bits >= 32 ? 0xFFFFFFFFu : ((1u << bits) - 1u); }

/* o(i): offset of RA i's field inside LP (reading R-EP). */
static uint32_t ra_offset(const ref_config* c, uint32_t i) { return c->cl_bs[i] - c->r; }

/* |EP(i)| per the EP-length rule of Sec. 3.3, taken mod (32-r) (reading R-EP). */
static uint32_t ep_len(const ref_config* c, uint32_t i) {
  uint32_t L = lp_bits(c);
  uint32_t d = (ra_offset(c, (i + 1) % c->n_ra) + L - ra_offset(c, i)) % L;
  return d == 0 ? L : d;
}

/* |CP(i)| = cbn(i) - |EP(i)| (Sec. 3.3; the line of Alg. 3 that writes CL(i) reads as cbn(i)). */
static int32_t cp_len(const ref_config* c, uint32_t i) {
  return (int32_t)c->cbn[i] - (int32_t)ep_len(c, i);
}

/* Rotations inside the (32-r)-bit LP (reading R-wrap). */
static uint32_t rotr_lp(const ref_config* c, uint32_t x, uint32_t s) {
  uint32_t L = lp_bits(c);
  while (s >= L) s -= L;
  if (s == 0) return x & mask32(L);
  return ((x >> s) | (x << (L - s))) & mask32(L);
}

static uint32_t rotl_lp(const ref_config* c, uint32_t x, uint32_t s) {
  uint32_t L = lp_bits(c);
  while (s >= L) s -= L;
  if (s == 0) return x & mask32(L);
  return ((x << s) | (x >> (L - s))) & mask32(L);
}

/* Checks the oracle needs to stay in bounds; returns 0 if usable. */
int ref_config_check(const ref_config* c) {
  if (c->r < 1 || c->r > 8) return -1;
  if (c->n_ra < 2 || c->n_ra > REF_MAX_RA) return -1;
  if (c->n_va > REF_MAX_VA) return -1;
  if (c->log2_g < 6 || c->log2_g > 15) return -1;
  for (uint32_t a = 0; a < n_arrays(c); ++a)
    if (c->cbn[a] < 1 || c->cbn[a] > 16) return -1;
  for (uint32_t i = 0; i < c->n_ra; ++i) {
    if (c->cl_bs[i] < c->r || c->cl_bs[i] > 31) return -1;
    if (i > 0 && c->cl_bs[i] <= c->cl_bs[i - 1]) return -1;
    if (c->cbn[i] > lp_bits(c)) return -1;
  }
  for (uint32_t i = 0; i < c->n_ra; ++i) {
    int32_t cp = cp_len(c, i);
    if (cp < 0) return -1;
    if ((uint32_t)cp > ep_len(c, (i + 1) % c->n_ra)) return -1;
  }
  return 0;
}

uint64_t ref_cube_words(const ref_config* c) {
  return (1ull << c->r) * row_blocks(c) * slab_words(c);
}

/* ------------------------------------------------------------------ */
/* Mangling and hashing (reading R-hash)                                */
/* ------------------------------------------------------------------ */

/* MurmurHash3 fmix32 finalizer: xorshift-multiply chain, every step invertible. */
static uint32_t fmix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x85EBCA6Bu;
  x ^= x >> 13;
  x *= 0xC2B2AE35u;
  x ^= x >> 16;
  return x;
}

/* Inverse of fmix32: undo each step in reverse order.
 * x ^= x >> 16 is its own inverse on 32 bits; x ^= x >> 13 is undone by
 * y ^ (y >> 13) ^ (y >> 26); multiplication by an odd constant is undone by
 * its inverse mod 2^32. */
static uint32_t fmix32_inv(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7ED1B41Du;             /* 0xC2B2AE35^-1 mod 2^32 */
  x ^= (x >> 13) ^ (x >> 26);
  x *= 0xA5CB9243u;             /* 0x85EBCA6B^-1 mod 2^32 */
  x ^= x >> 16;
  return x;
}

/* lowbias32 (hash-prospector): same shape, different constants. */
static uint32_t lowbias32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7FEB352Du;
  x ^= x >> 15;
  x *= 0x846CA68Bu;
  x ^= x >> 16;
  return x;
}

/* Mangling of Sec. 3.1: a bijection on 32-bit IPs. */
uint32_t ref_mangle(const ref_config* c, uint32_t ip) { return fmix32(ip ^ c->seed_mangle); }

/* "use the mangling operation again to acquire the origin IP": the inverse. */
uint32_t ref_unmangle(const ref_config* c, uint32_t m) { return fmix32_inv(m) ^ c->seed_mangle; }

/* H_bv of Alg. 1: the bit of the column that an outer IP sets, in [0, g). */
uint32_t ref_hash_bv(const ref_config* c, uint32_t oip) {
  return lowbias32(oip ^ c->seed_bv) >> (32u - c->log2_g);
}

/* H_j of Sec. 3.2: VA j's column index from LP, in [0, c(|RA|+j)). */
uint32_t ref_hash_va(const ref_config* c, uint32_t j, uint32_t lp) {
  return lowbias32(lp ^ c->seed_va[j]) >> (32u - c->cbn[c->n_ra + j]);
}

/* Alg. 1's index computations for one inner IP: the sketch id (right r bits)
 * and the column of every array. RA columns are cbn(i) consecutive bits of the
 * mangled IP starting at CL_bs(i) (wrapping inside LP); VA columns are H_j(LP). */
void ref_host_columns(const ref_config* c, uint32_t iip, uint32_t* cs_out, uint32_t* cols) {
  uint32_t m = ref_mangle(c, iip);
  uint32_t cs = m & mask32(c->r);
  uint32_t lp = m >> c->r;
  for (uint32_t i = 0; i < c->n_ra; ++i)
    cols[i] = rotr_lp(c, lp, ra_offset(c, i)) & mask32(c->cbn[i]);
  for (uint32_t j = 0; j < c->n_va; ++j) cols[c->n_ra + j] = ref_hash_va(c, j, lp);
  *cs_out = cs;
}

/* ------------------------------------------------------------------ */
/* Cube access (reading R-layout)                                       */
/* ------------------------------------------------------------------ */

/* Layout constants of one configuration, computed once per call so the
 * per-bit address arithmetic below stays a few multiplies and adds. */
typedef struct layout {
  uint64_t R;                       /* row blocks per column = g/64 */
  uint64_t W;                       /* words per row block = sum of c(a) */
  uint64_t aoff[REF_MAX_ARRAYS];    /* A_off(a) */
} layout;

static layout layout_of(const ref_config* c) {
  layout l;
  l.R = row_blocks(c);
  l.W = slab_words(c);
  for (uint32_t a = 0; a < REF_MAX_ARRAYS; ++a) l.aoff[a] = a < n_arrays(c) ? array_offset(c, a) : 0;
  return l;
}

static uint64_t word_index(const layout* l, uint32_t cs, uint32_t a, uint32_t col, uint32_t b) {
  return ((uint64_t)cs * l->R + (b >> 6)) * l->W + l->aoff[a] + col;
}

static void set_bit(const layout* l, uint64_t* cube, uint32_t cs, uint32_t a, uint32_t col,
                    uint32_t b) {
  cube[word_index(l, cs, a, col, b)] |= 1ull << (b & 63u);
}

/* Copies one column (g bits) into out[0 .. g/64). */
static void read_column(const layout* l, const uint64_t* cube, uint32_t cs, uint32_t a,
                        uint32_t col, uint64_t* out) {
  for (uint64_t rb = 0; rb < l->R; ++rb) out[rb] = cube[word_index(l, cs, a, col, (uint32_t)(rb * 64u))];
}

static uint32_t column_zeros(const layout* l, const uint64_t* words) {
  uint32_t ones = 0;
  for (uint64_t rb = 0; rb < l->R; ++rb) ones += (uint32_t)__builtin_popcountll(words[rb]);
  return (uint32_t)(l->R * 64u) - ones;
}

/* ------------------------------------------------------------------ */
/* Update (Alg. 1) and merge (Sec. 3.3)                                 */
/* ------------------------------------------------------------------ */

/* One IP pair <iip, oip>: set bit H_bv(oip) in the iip's column of every array. */
static void update_one(const ref_config* c, const layout* l, uint64_t* cube, uint32_t iip,
                       uint32_t oip) {
  uint32_t cols[REF_MAX_ARRAYS];
  uint32_t cs;
  uint32_t bv = ref_hash_bv(c, oip);
  ref_host_columns(c, iip, &cs, cols);
  for (uint32_t a = 0; a < n_arrays(c); ++a) set_bit(l, cube, cs, a, cols[a], bv);
}

/* pairs[2k] = source IP, pairs[2k+1] = destination IP. side SRC keys the cube
 * by the source (inner = source), side DST by the destination. */
void ref_update(const ref_config* c, uint64_t* cube, const uint32_t* pairs, uint64_t n, int side) {
  layout l = layout_of(c);
  for (uint64_t k = 0; k < n; ++k) {
    uint32_t src = pairs[2 * k], dst = pairs[2 * k + 1];
    if (side == REF_SIDE_SRC)
      update_one(c, &l, cube, src, dst);
    else
      update_one(c, &l, cube, dst, src);
  }
}

/* Global server: bitwise OR of same-structure cubes (reading R-merge). dst may
 * be one of the sources. */
void ref_merge_or(const ref_config* c, uint64_t* dst, const uint64_t* const* srcs, int k) {
  uint64_t words = ref_cube_words(c);
  for (uint64_t w = 0; w < words; ++w) {
    uint64_t acc = 0;
    for (int s = 0; s < k; ++s) acc |= srcs[s][w];
    dst[w] = acc;
  }
}

/* Timing leg over all host cores (used only by the benchmark's CPU baseline
 * and the test that checks it against ref_update): the pairs are divided
 * among OpenMP threads and every bit is set with an atomic OR. The update
 * only ever sets bits (Sec. 3.2), so the cube is the same set union as
 * ref_update's whatever the interleaving. */
void ref_update_omp(const ref_config* c, uint64_t* cube, const uint32_t* pairs, uint64_t n,
                    int side) {
  layout l = layout_of(c);
  const uint32_t A = n_arrays(c);
#pragma omp parallel for schedule(static, 65536)
  for (int64_t k = 0; k < (int64_t)n; ++k) {
    uint32_t src = pairs[2 * k], dst = pairs[2 * k + 1];
    uint32_t iip = side == REF_SIDE_SRC ? src : dst;
    uint32_t oip = side == REF_SIDE_SRC ? dst : src;
    uint32_t cols[REF_MAX_ARRAYS];
    uint32_t cs;
    uint32_t bv = ref_hash_bv(c, oip);
    ref_host_columns(c, iip, &cs, cols);
    for (uint32_t a = 0; a < A; ++a)
      __atomic_fetch_or(&cube[word_index(&l, cs, a, cols[a], bv)], 1ull << (bv & 63u),
                        __ATOMIC_RELAXED);
  }
}

/* Threads an OpenMP region of the oracle runs with. */
int ref_omp_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------ */
/* Column statistics and thresholds (Alg. 2, Thm. 1, Thm. 2)            */
/* ------------------------------------------------------------------ */

/* zeros[cs * W + A_off(a) + col] = g - popcount(column); ones[cs * A + a] =
 * number of one bits in array a of sketch cs. */
void ref_column_zeros(const ref_config* c, const uint64_t* cube, uint16_t* zeros, uint32_t* ones) {
  uint64_t buf[512];
  uint32_t A = n_arrays(c);
  layout l = layout_of(c);
  for (uint32_t cs = 0; cs < (1u << c->r); ++cs) {
    for (uint32_t a = 0; a < A; ++a) {
      uint64_t total_ones = 0;
      for (uint32_t col = 0; col < n_cols(c, a); ++col) {
        read_column(&l, cube, cs, a, col, buf);
        uint32_t z = column_zeros(&l, buf);
        zeros[(uint64_t)cs * slab_words(c) + array_offset(c, a) + col] = (uint16_t)z;
        total_ones += g_bits(c) - z;
      }
      ones[cs * A + a] = (uint32_t)total_ones;
    }
  }
}

/* Thm. 1 with reading R-eps: eps = prod_a ones(a) / (c(a) * g), in array order.
 * Threshold on union-column zeros (reading R-thr, R-cmp). */
void ref_thresholds(const ref_config* c, const uint32_t* ones, double theta, int rule, double* eps,
                    int32_t* zmax) {
  uint32_t A = n_arrays(c);
  double g = (double)g_bits(c);
  double x = exp(-theta / g);
  for (uint32_t cs = 0; cs < (1u << c->r); ++cs) {
    double e = 1.0;
    for (uint32_t a = 0; a < A; ++a) e = e * ((double)ones[cs * A + a] / ((double)n_cols(c, a) * g));
    double zf;
    if (rule == REF_THR_PAPER)
      zf = (g + g * e) * x - g * e;
    else
      zf = (g - g * e) * x;
    eps[cs] = e;
    zmax[cs] = zf < 0.0 ? -1 : (int32_t)floor(zf);
  }
}

/* Thm. 2: est = -g * ln(Z / (g - g*eps)), with reading R-est. */
static double estimate(const ref_config* c, uint32_t z, double eps, uint8_t* flags) {
  double g = (double)g_bits(c);
  uint32_t zc = z;
  *flags = 0;
  if (zc == 0) {
    zc = 1;
    *flags |= REF_FLAG_SATURATED;
  }
  double est = -g * log((double)zc / (g - g * eps));
  return est < 0.0 ? 0.0 : est;
}

/* Union column (Def. 2) of a host given its columns; returns Z. */
static uint32_t union_zeros(const ref_config* c, const layout* l, const uint64_t* cube, uint32_t cs,
                            const uint32_t* cols) {
  uint64_t uc[512], col[512];
  for (uint64_t rb = 0; rb < l->R; ++rb) uc[rb] = ~0ull;
  for (uint32_t a = 0; a < n_arrays(c); ++a) {
    read_column(l, cube, cs, a, cols[a], col);
    for (uint64_t rb = 0; rb < l->R; ++rb) uc[rb] &= col[rb];
  }
  return column_zeros(l, uc);
}

/* Per-sketch eps and Zmax from the cube (helper shared by restore paths). */
static void sketch_thresholds(const ref_config* c, const uint64_t* cube, double theta, int rule,
                              double* eps, int32_t* zmax) {
  uint32_t S = 1u << c->r;
  uint64_t zn = (uint64_t)S * slab_words(c);
  uint16_t* zeros = (uint16_t*)malloc(zn * sizeof(uint16_t));
  uint32_t* ones = (uint32_t*)malloc((uint64_t)S * n_arrays(c) * sizeof(uint32_t));
  ref_column_zeros(c, cube, zeros, ones);
  ref_thresholds(c, ones, theta, rule, eps, zmax);
  free(zeros);
  free(ones);
}

/* ------------------------------------------------------------------ */
/* Restore (Alg. 2 + Alg. 3)                                             */
/* ------------------------------------------------------------------ */

static int cmp_host_ip(const void* a, const void* b) {
  uint32_t x = ((const ref_host*)a)->ip, y = ((const ref_host*)b)->ip;
  return x < y ? -1 : (x > y ? 1 : 0);
}

typedef struct out_buf {
  ref_host* out;
  uint64_t cap;
  uint64_t n;
} out_buf;

static void emit(out_buf* ob, const ref_config* c, uint32_t cs, uint32_t lp, uint32_t z, double eps) {
  if (ob->n < ob->cap) {
    ref_host h;
    memset(&h, 0, sizeof h);
    /* IP = LP || RP, RP = sketch id, then unmangle. */
    h.ip = ref_unmangle(c, (lp << c->r) | cs);
    h.zeros = (uint16_t)z;
    h.cs = (uint8_t)cs;
    h.est = estimate(c, z, eps, &h.flags);
    ob->out[ob->n] = h;
  }
  ob->n++;
}

/* Returns 0, or 1 if more than cap hosts were found (n_out then holds the
 * full count and out holds the first cap found, unsorted). */
int ref_restore(const ref_config* c, const uint64_t* cube, double theta, int rule, ref_host* out,
                uint64_t cap, uint64_t* n_out, ref_restore_stats* st) {
  uint32_t S = 1u << c->r;
  uint32_t nra = c->n_ra;
  double* eps = (double*)malloc(S * sizeof(double));
  int32_t* zmax = (int32_t*)malloc(S * sizeof(int32_t));
  sketch_thresholds(c, cube, theta, rule, eps, zmax);

  uint32_t* hc[REF_MAX_RA];
  uint32_t nhc[REF_MAX_RA];
  for (uint32_t i = 0; i < nra; ++i) hc[i] = (uint32_t*)malloc(n_cols(c, i) * sizeof(uint32_t));
  uint64_t colbuf[512];
  layout l = layout_of(c);
  out_buf ob = {out, cap, 0};
  ref_restore_stats s;
  memset(&s, 0, sizeof s);

  for (uint32_t cs = 0; cs < S; ++cs) {
    /* Alg. 2: hot columns of every RA, ascending (loop bound reads [0, c(i)-1]). */
    for (uint32_t i = 0; i < nra; ++i) {
      nhc[i] = 0;
      for (uint32_t j = 0; j < n_cols(c, i); ++j) {
        read_column(&l, cube, cs, i, j, colbuf);
        if ((int64_t)column_zeros(&l, colbuf) <= (int64_t)zmax[cs]) hc[i][nhc[i]++] = j;
      }
      s.hot_columns += nhc[i];
    }
    int any_empty = 0;
    for (uint32_t i = 0; i < nra; ++i) any_empty |= (nhc[i] == 0);
    if (any_empty) continue;

    /* Alg. 3 over every tuple of the cartesian product, lexicographic order. */
    uint32_t idx[REF_MAX_RA] = {0, 0, 0, 0};
    for (;;) {
      uint32_t t[REF_MAX_RA];
      for (uint32_t i = 0; i < nra; ++i) t[i] = hc[i][idx[i]];
      s.tuples++;

      int ok = 1;
      for (uint32_t i = 0; i < nra && ok; ++i) {
        uint32_t cp = (uint32_t)cp_len(c, i);
        uint32_t mine = t[i] >> ep_len(c, i);                 /* CP of hc_i */
        uint32_t next = t[(i + 1) % nra] & mask32(cp);        /* first |CP(i)| bits of hc_{i+1} */
        if (mine != next) ok = 0;
      }
      if (ok) {
        s.cp_valid++;
        /* LP = concatenation of every column's EP. */
        uint32_t lp = 0;
        for (uint32_t i = 0; i < nra; ++i)
          lp |= rotl_lp(c, t[i] & mask32(ep_len(c, i)), ra_offset(c, i));
        uint32_t cols[REF_MAX_ARRAYS];
        for (uint32_t i = 0; i < nra; ++i) cols[i] = t[i];
        for (uint32_t j = 0; j < c->n_va; ++j) cols[nra + j] = ref_hash_va(c, j, lp);
        uint32_t z = union_zeros(c, &l, cube, cs, cols);
        if ((int64_t)z <= (int64_t)zmax[cs]) {
          s.accepted++;
          emit(&ob, c, cs, lp, z, eps[cs]);
        }
      }

      /* odometer */
      int32_t k = (int32_t)nra - 1;
      while (k >= 0) {
        if (++idx[k] < nhc[k]) break;
        idx[k] = 0;
        --k;
      }
      if (k < 0) break;
    }
  }

  for (uint32_t i = 0; i < nra; ++i) free(hc[i]);
  free(eps);
  free(zmax);
  *n_out = ob.n;
  if (st) *st = s;
  if (ob.n > cap) return 1;
  qsort(out, ob.n, sizeof(ref_host), cmp_host_ip);
  return 0;
}

/* The plain definition the restore reaches: every IP whose union column has
 * at most Zmax[cs] zeros. Enumerates all 2^32 addresses (tiny g only); the
 * address space is cut into 256 ascending chunks spread over threads, each
 * chunk keeps its hits in order, and the chunks are concatenated, so the
 * output is ascending by construction. */
int ref_restore_bruteforce(const ref_config* c, const uint64_t* cube, double theta, int rule,
                           ref_host* out, uint64_t cap, uint64_t* n_out) {
  uint32_t S = 1u << c->r;
  double* eps = (double*)malloc(S * sizeof(double));
  int32_t* zmax = (int32_t*)malloc(S * sizeof(int32_t));
  sketch_thresholds(c, cube, theta, rule, eps, zmax);
  layout l = layout_of(c);
  enum { CHUNKS = 256 };
  ref_host* hits[CHUNKS];
  uint64_t counts[CHUNKS];
#pragma omp parallel for schedule(dynamic, 1)
  for (int k = 0; k < CHUNKS; ++k) {
    uint64_t lo = (uint64_t)k << 24, hi = (uint64_t)(k + 1) << 24;
    uint64_t cnt = 0, room = 1024;
    ref_host* buf = (ref_host*)malloc(room * sizeof(ref_host));
    for (uint64_t ip = lo; ip < hi; ++ip) {
      uint32_t cols[REF_MAX_ARRAYS], cs;
      ref_host_columns(c, (uint32_t)ip, &cs, cols);
      uint32_t z = union_zeros(c, &l, cube, cs, cols);
      if ((int64_t)z <= (int64_t)zmax[cs]) {
        if (cnt == room) {
          room *= 2;
          buf = (ref_host*)realloc(buf, room * sizeof(ref_host));
        }
        ref_host h;
        memset(&h, 0, sizeof h);
        h.ip = (uint32_t)ip;
        h.zeros = (uint16_t)z;
        h.cs = (uint8_t)cs;
        h.est = estimate(c, z, eps[cs], &h.flags);
        buf[cnt++] = h;
      }
    }
    hits[k] = buf;
    counts[k] = cnt;
  }
  uint64_t total = 0;
  for (int k = 0; k < CHUNKS; ++k) {
    for (uint64_t i = 0; i < counts[k]; ++i) {
      if (total < cap) out[total] = hits[k][i];
      total++;
    }
    free(hits[k]);
  }
  *n_out = total;
  free(eps);
  free(zmax);
  return total > cap ? 1 : 0;
}

/* Thm. 2 estimate for given inner IPs: Z of each union column and its estimate. */
void ref_estimate(const ref_config* c, const uint64_t* cube, const uint32_t* hosts, uint64_t n,
                  double* est, uint16_t* zeros, uint8_t* flags) {
  uint32_t S = 1u << c->r;
  double* eps = (double*)malloc(S * sizeof(double));
  int32_t* zmax = (int32_t*)malloc(S * sizeof(int32_t));
  sketch_thresholds(c, cube, 0.0, REF_THR_THM2, eps, zmax);
  layout l = layout_of(c);
  for (uint64_t k = 0; k < n; ++k) {
    uint32_t cols[REF_MAX_ARRAYS], cs;
    ref_host_columns(c, hosts[k], &cs, cols);
    uint32_t z = union_zeros(c, &l, cube, cs, cols);
    uint8_t f;
    double e = estimate(c, z, eps[cs], &f);
    if (est) est[k] = e;
    if (zeros) zeros[k] = (uint16_t)z;
    if (flags) flags[k] = f;
  }
  free(eps);
  free(zmax);
}

/* Per-array zero counts of a host's own columns (the per-layer popcount view
 * of one host: g - zeros of each of its |RA|+|VA| columns). */
void ref_host_layer_zeros(const ref_config* c, const uint64_t* cube, const uint32_t* hosts,
                          uint64_t n, uint16_t* layer_zeros) {
  uint64_t buf[512];
  uint32_t A = n_arrays(c);
  layout l = layout_of(c);
  for (uint64_t k = 0; k < n; ++k) {
    uint32_t cols[REF_MAX_ARRAYS], cs;
    ref_host_columns(c, hosts[k], &cs, cols);
    for (uint32_t a = 0; a < A; ++a) {
      read_column(&l, cube, cs, a, cols[a], buf);
      layer_zeros[k * A + a] = (uint16_t)column_zeros(&l, buf);
    }
  }
}

/* ------------------------------------------------------------------ */
/* Row fills (extension of Thm. 1 for the learned estimator)             */
/* ------------------------------------------------------------------ */

/* row_ones[(cs * A + a) * g + b] = number of columns of array a in sketch cs
 * whose bit b is set. Thm. 1 takes every row of an array to be set with the
 * same probability; these counts are what that probability is per row. */
void ref_row_ones(const ref_config* c, const uint64_t* cube, uint32_t* row_ones) {
  layout l = layout_of(c);
  uint32_t A = n_arrays(c);
  uint64_t g = g_bits(c);
  memset(row_ones, 0, sizeof(uint32_t) * (size_t)((1u << c->r) * A * g));
  for (uint32_t cs = 0; cs < (1u << c->r); ++cs)
    for (uint32_t a = 0; a < A; ++a)
      for (uint32_t col = 0; col < n_cols(c, a); ++col)
        for (uint32_t rb = 0; rb < l.R; ++rb) {
          /* each one bit of this word of the column is one row */
          uint64_t w = cube[word_index(&l, cs, a, col, rb * 64u)];
          while (w) {
            uint32_t bit = (uint32_t)__builtin_ctzll(w);
            row_ones[((uint64_t)cs * A + a) * g + rb * 64u + bit] += 1;
            w &= w - 1;
          }
        }
}

/* Row-aware shared-bit mass of each sketch: the sum over rows b of the
 * product over arrays (in array order) of row_ones / c(a). It is the
 * expected number of one bits in the union column of an inner IP the window
 * never saw when rows fill unevenly; with every row of an array equally full
 * it equals g * eps of Thm. 1. */
void ref_row_shared(const ref_config* c, const uint32_t* row_ones, double* shared) {
  uint32_t A = n_arrays(c);
  uint64_t g = g_bits(c);
  for (uint32_t cs = 0; cs < (1u << c->r); ++cs) {
    double s = 0.0;
    for (uint64_t b = 0; b < g; ++b) {
      double q = 1.0;
      for (uint32_t a = 0; a < A; ++a)
        q = q * ((double)row_ones[((uint64_t)cs * A + a) * g + b] / (double)n_cols(c, a));
      s += q;
    }
    shared[cs] = s;
  }
}

/* ------------------------------------------------------------------ */
/* Exact per-host distinct-peer counts (Sec. 3.1, Sec. 5.1 baseline)     */
/* ------------------------------------------------------------------ */

static int cmp_u64(const void* a, const void* b) {
  uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
  return x < y ? -1 : (x > y ? 1 : 0);
}

/* Sort-unique of (host << 32 | peer); hosts_out ascending with their number
 * of distinct peers |OP(host)|. Outputs must hold n entries. Returns the
 * number of distinct hosts. */
uint64_t ref_exact_counts(const uint32_t* pairs, uint64_t n, int side, uint32_t* hosts_out,
                          uint32_t* counts_out) {
  if (n == 0) return 0;
  uint64_t* keys = (uint64_t*)malloc(n * sizeof(uint64_t));
  for (uint64_t k = 0; k < n; ++k) {
    uint32_t src = pairs[2 * k], dst = pairs[2 * k + 1];
    uint32_t host = side == REF_SIDE_SRC ? src : dst;
    uint32_t peer = side == REF_SIDE_SRC ? dst : src;
    keys[k] = ((uint64_t)host << 32) | peer;
  }
  qsort(keys, n, sizeof(uint64_t), cmp_u64);
  uint64_t nh = 0;
  for (uint64_t k = 0; k < n; ++k) {
    if (k > 0 && keys[k] == keys[k - 1]) continue; /* duplicate flow */
    uint32_t host = (uint32_t)(keys[k] >> 32);
    if (nh > 0 && hosts_out[nh - 1] == host) {
      counts_out[nh - 1]++;
    } else {
      hosts_out[nh] = host;
      counts_out[nh] = 1;
      nh++;
    }
  }
  free(keys);
  return nh;
}

/* ref_exact_counts over all host cores (benchmark timing leg; tested
 * against ref_exact_counts): the (host, peer) keys are bucketed by the
 * host's top 8 bits, each bucket is sorted and counted by one thread, and the
 * buckets are concatenated in order, so the output is the same ascending
 * list. */
uint64_t ref_exact_counts_omp(const uint32_t* pairs, uint64_t n, int side, uint32_t* hosts_out,
                              uint32_t* counts_out) {
  enum { NB = 256 };
  if (n == 0) return 0;
  const int T = omp_get_max_threads();
  uint64_t* keys = (uint64_t*)malloc(n * sizeof(uint64_t));
  uint64_t* hist = (uint64_t*)calloc((size_t)T * NB, sizeof(uint64_t));
  uint64_t start[NB + 1];
  uint64_t nh_b[NB];
#pragma omp parallel num_threads(T)
  {
    const int t = omp_get_thread_num();
    const uint64_t lo = n * (uint64_t)t / (uint64_t)T, hi = n * (uint64_t)(t + 1) / (uint64_t)T;
    uint64_t* h = hist + (size_t)t * NB;
    for (uint64_t k = lo; k < hi; ++k) {
      uint32_t host = side == REF_SIDE_SRC ? pairs[2 * k] : pairs[2 * k + 1];
      h[host >> 24]++;
    }
#pragma omp barrier
#pragma omp single
    {
      uint64_t acc = 0;
      for (int b = 0; b < NB; ++b) {
        start[b] = acc;
        for (int u = 0; u < T; ++u) {
          uint64_t v = hist[(size_t)u * NB + b];
          hist[(size_t)u * NB + b] = acc;
          acc += v;
        }
      }
      start[NB] = acc;
    }
    for (uint64_t k = lo; k < hi; ++k) {
      uint32_t src = pairs[2 * k], dst = pairs[2 * k + 1];
      uint32_t host = side == REF_SIDE_SRC ? src : dst;
      uint32_t peer = side == REF_SIDE_SRC ? dst : src;
      keys[h[host >> 24]++] = ((uint64_t)host << 32) | peer;
    }
#pragma omp barrier
#pragma omp for schedule(dynamic, 1)
    for (int b = 0; b < NB; ++b) {
      uint64_t* kb = keys + start[b];
      const uint64_t m = start[b + 1] - start[b];
      qsort(kb, m, sizeof(uint64_t), cmp_u64);
      /* distinct hosts of the bucket with their distinct peers, written in
       * place at the front of the bucket's key range */
      uint64_t nh = 0, prev = 0;
      for (uint64_t k = 0; k < m; ++k) {
        const uint64_t key = kb[k];   /* read before slot nh <= k is rewritten */
        if (k > 0 && key == prev) continue;
        prev = key;
        uint32_t host = (uint32_t)(key >> 32);
        if (nh > 0 && (uint32_t)(kb[nh - 1] >> 32) == host) {
          kb[nh - 1]++;
        } else {
          kb[nh++] = ((uint64_t)host << 32) | 1u;
        }
      }
      nh_b[b] = nh;
    }
  }
  uint64_t out = 0;
  for (int b = 0; b < NB; ++b)
    for (uint64_t k = 0; k < nh_b[b]; ++k, ++out) {
      hosts_out[out] = (uint32_t)(keys[start[b] + k] >> 32);
      counts_out[out] = (uint32_t)keys[start[b] + k];
    }
  free(hist);
  free(keys);
  return out;
}

/* ------------------------------------------------------------------ */
/* Exhaustive self-checks used by the pins                               */
/* ------------------------------------------------------------------ */

/* Number of x in [0, 2^32) with unmangle(mangle(x)) != x. */
uint64_t ref_check_mangle_bijection(const ref_config* c) {
  uint64_t bad = 0;
#pragma omp parallel for reduction(+ : bad) schedule(static)
  for (int64_t hi = 0; hi < 65536; ++hi) {
    for (uint32_t lo = 0; lo < 65536; ++lo) {
      uint32_t x = ((uint32_t)hi << 16) | lo;
      if (ref_unmangle(c, ref_mangle(c, x)) != x) bad++;
    }
  }
  return bad;
}

/* For every LP in [0, 2^(32-r)): its RA columns form a CP-valid tuple and the
 * EP concatenation gives LP back. Returns the number of LPs that fail. */
uint64_t ref_check_lp_roundtrip(const ref_config* c) {
  uint64_t L = lp_bits(c);
  uint64_t bad = 0;
#pragma omp parallel for reduction(+ : bad) schedule(static)
  for (int64_t lp = 0; lp < (int64_t)(1ull << L); ++lp) {
    uint32_t t[REF_MAX_RA];
    for (uint32_t i = 0; i < c->n_ra; ++i)
      t[i] = rotr_lp(c, (uint32_t)lp, ra_offset(c, i)) & mask32(c->cbn[i]);
    int ok = 1;
    for (uint32_t i = 0; i < c->n_ra; ++i) {
      uint32_t cp = (uint32_t)cp_len(c, i);
      if ((t[i] >> ep_len(c, i)) != (t[(i + 1) % c->n_ra] & mask32(cp))) ok = 0;
    }
    uint32_t back = 0;
    for (uint32_t i = 0; i < c->n_ra; ++i)
      back |= rotl_lp(c, t[i] & mask32(ep_len(c, i)), ra_offset(c, i));
    if (!ok || back != (uint32_t)lp) bad++;
  }
  return bad;
}

/* Tuple check of Alg. 3 on an explicit tuple (for pins on random tuples):
 * returns 1 and writes the LP if every CP matches, else 0. */
int ref_tuple_check(const ref_config* c, const uint32_t* t, uint32_t* lp_out) {
  for (uint32_t i = 0; i < c->n_ra; ++i) {
    uint32_t cp = (uint32_t)cp_len(c, i);
    if ((t[i] >> ep_len(c, i)) != (t[(i + 1) % c->n_ra] & mask32(cp))) return 0;
  }
  uint32_t lp = 0;
  for (uint32_t i = 0; i < c->n_ra; ++i) lp |= rotl_lp(c, t[i] & mask32(ep_len(c, i)), ra_offset(c, i));
  *lp_out = lp;
  return 1;
}

/* |EP(i)| and |CP(i)| as the oracle reads them (for pins). */
void ref_ep_cp(const ref_config* c, uint32_t* ep, int32_t* cp) {
  for (uint32_t i = 0; i < c->n_ra; ++i) {
    ep[i] = ep_len(c, i);
    cp[i] = cp_len(c, i);
  }
}
