/*
 * cbaa.h -- C ABI of libcbaa, the gfx950 (MI355X) implementation of the CBAA
 * super-host detector of Xu, Ding and Hu, "GPU based Real-time Super Hosts
 * Detection at Distributed Edge Routers" (arXiv 1901.06207).
 *
 * A super host is an inner IP that exchanges packets with at least theta
 * distinct outer IPs in a time window (Def. 1). Local servers at edge routers
 * scan packets into a cube of bit arrays (Sec. 3.1-3.2, Alg. 1); a global
 * server ORs the local cubes and restores the super hosts from hot columns
 * (Sec. 3.3, Algs. 2-3, Thm. 2).
 *
 * Conventions shared by every call:
 *  - Pointers named d_* are device pointers on the current HIP device; h_*
 *    are host pointers. The caller owns every buffer. The library never
 *    allocates or frees device memory and keeps no pointer after a call.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Calls that take a stream only enqueue work and return before it runs;
 *    a kernel fault surfaces at the caller's next synchronisation.
 *  - Every call returns CBAA_OK (0) or a negative CBAA_E* code and has no
 *    other effect when it fails argument checks. cbaa_strerror() names a
 *    code; cbaa_last_error() gives the detail of this thread's last failure.
 *  - No C++ exception crosses this interface.
 */
#ifndef CBAA_H
#define CBAA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CBAA_ABI_VERSION 2u
#define CBAA_MAX_RA 4
#define CBAA_MAX_VA 2
#define CBAA_MAX_ARRAYS (CBAA_MAX_RA + CBAA_MAX_VA)
#define CBAA_MAX_BATCH 32

/* Return codes. */
#define CBAA_OK 0
#define CBAA_EINVAL (-1)    /* null pointer, bad size or enum value */
#define CBAA_ECONFIG (-2)   /* configuration fails cbaa_config_validate */
#define CBAA_ESCRATCH (-3)  /* scratch buffer smaller than the *_scratch_bytes query */
#define CBAA_EHIP (-4)      /* a HIP runtime call failed (detail in cbaa_last_error) */

/* Which address of a (source, destination) pair is the inner host whose
 * cardinality is recorded. The paper ignores direction (Sec. 3.1); a cube is
 * keyed by one side. */
#define CBAA_SIDE_SRC 0
#define CBAA_SIDE_DST 1

/* Threshold rule on union-column zeros Z (Sec. 3.3, Thm. 2):
 *  THM2  : Zmax = floor((g - g*eps) * exp(-theta/g)) -- est >= theta <=> Z <= Zmax
 *  PAPER : Zmax = floor((g + g*eps) * exp(-theta/g) - g*eps) -- the printed form
 * Both reduce to floor(g exp(-theta/g)) when eps = 0. */
#define CBAA_THR_THM2 0
#define CBAA_THR_PAPER 1

/* Restored host flag: the union column had no zero bit (estimate uses Z = 1). */
#define CBAA_FLAG_SATURATED 1u

/* Bits of cbaa_restore_stats.status. */
#define CBAA_STATUS_CONFIG 1u  /* a cube read had no valid header of this configuration:
                                  nothing was restored (n_hosts = 0) */
#define CBAA_STATUS_BUDGET 2u  /* the tuple check stopped at its work budget: the list
                                  holds the hosts found until then, not all of them */

/*
 * Configuration (Sec. 3.1-3.3). Arrays 0..n_ra-1 are restoring arrays (RA),
 * arrays n_ra..n_ra+n_va-1 validating arrays (VA).
 *
 *  r          2^r cardinality sketches; the sketch of an inner IP is the low r
 *             bits (RP) of its mangled address, LP = the other 32-r bits.
 *  log2_g     g = 2^log2_g bits per column (bits vector of Eq. 1).
 *  cbn[a]     array a has c(a) = 2^cbn[a] columns.
 *  cl_bs[i]   RA i's column index is cbn[i] consecutive bits of the mangled
 *             address starting at bit cl_bs[i] (bit 0 = least significant);
 *             a field that runs past bit 31 wraps inside LP, never into RP.
 *  seeds      mangle M(x) = fmix32(x ^ seed_mangle) (MurmurHash3 finalizer,
 *             inverted exactly at restore time); the outer IP sets bit
 *             H_bv(oip) = lowbias32(oip ^ seed_bv) >> (32 - log2_g); VA j's
 *             column is H_j(LP) = lowbias32(LP ^ seed_va[j]) >> (32 - cbn).
 *             lowbias32 is C. Wellons' hash-prospector mixer.
 *
 * Paper defaults (Sec. 5.3): r=4, |RA|=3, |VA|=1, g=c=2^12, a 128 MiB cube.
 */
typedef struct cbaa_config {
  uint32_t r;
  uint32_t n_ra;
  uint32_t n_va;
  uint32_t log2_g;
  uint32_t cbn[CBAA_MAX_ARRAYS];
  uint32_t cl_bs[CBAA_MAX_RA];
  uint32_t seed_mangle;
  uint32_t seed_bv;
  uint32_t seed_va[CBAA_MAX_VA];
} cbaa_config;

/* One restored super host (Sec. 3.3, last paragraph; est from Thm. 2). */
typedef struct cbaa_host {
  uint32_t ip;     /* original (unmangled) inner IPv4 address */
  uint16_t zeros;  /* Z: zero bits of its union column (Def. 2) */
  uint8_t cs;      /* cardinality sketch id (= RP) */
  uint8_t flags;   /* CBAA_FLAG_* */
  double est;      /* -g ln(max(Z,1) / (g - g*eps)), clamped at 0 */
} cbaa_host;

/* Device-side restore counters, written by cbaa_restore. */
typedef struct cbaa_restore_stats {
  uint64_t n_hosts;         /* super hosts found; > capacity means the output was cut */
  uint64_t hot_columns;     /* sum over sketches and RAs of |HC(i)| (Alg. 2) */
  uint64_t partial_checked; /* partial tuples whose AND-ed columns were counted */
  uint64_t tuples_checked;  /* complete CP-valid tuples whose union column was counted */
  uint64_t tuple_space;     /* sum over sketches of prod_i |HC(i)|: the tuples Alg. 3
                               enumerates before its CP check (saturates at 2^64 - 1) */
  uint64_t status;          /* CBAA_STATUS_* bits; 0 = complete */
} cbaa_restore_stats;

/* Cube memory layout. A cube is a 256-byte header followed by the bits.
 *
 * Header (Sec. 3.3: only arrays of the same structure are merged; the header
 * records the structure so that a merge or restore can tell):
 *   word 0  magic CBAA_CUBE_MAGIC
 *   word 1  config hash: cbaa_config_hash() of the configuration it was built with
 *   word 2  bytes of bits after the header
 *   word 3  low 32 bits CBAA_ABI_VERSION, high 32 bits state: CBAA_CUBE_VALID, or
 *           CBAA_CUBE_MIXED once bits of another configuration (or of a cube with
 *           no valid header) have been OR-ed into it
 *   words 4..31 zero
 * cbaa_cube_init and fresh batch streams write a valid header; updates and
 * merges mark their destination MIXED when a source or the destination itself
 * does not carry this configuration's valid header; restores report such a cube
 * in cbaa_restore_stats.status and restore nothing from it. These checks run on
 * the device inside the calls' own launches, so every call stays asynchronous
 * and capturable; cbaa_cube_check reads a header back synchronously.
 *
 * Bits (64-bit little-endian words after the header). Bit b of column `col` of
 * array a in sketch cs is bit (b & 63) of word
 *     ((cs * R + (b >> 6)) * W) + A_off(a) + col
 * where R = g/64, W = sum_a c(a) and A_off(a) = sum_{a' < a} c(a'). A run of
 * W words (one 64-bit row block of every column of one sketch) is contiguous. */
#define CBAA_HEADER_BYTES 256u
#define CBAA_CUBE_MAGIC 0x4542554341414243ull /* "CBAACUBE" in little-endian bytes */
#define CBAA_CUBE_VALID 0u
#define CBAA_CUBE_MIXED 1u

/* ---- configuration -------------------------------------------------- */

/* Writes the paper's evaluated dimensions (Sec. 5.3) with RA start bits
 * (4, 14, 23) (EP lengths 10, 9, 9; CP lengths 2, 3, 3) and fixed seeds. */
int cbaa_config_default(cbaa_config* h_out);

/* Checks a configuration: 1 <= r <= 8; 2 <= n_ra <= 4; n_va <= 2;
 * 6 <= log2_g <= 15; 1 <= cbn <= 16 and cbn[i] <= 32-r for RAs; r <= cl_bs[i]
 * <= 31 strictly increasing; with |EP(i)| = (o(i+1) - o(i)) mod (32-r),
 * o(i) = cl_bs[i] - r (Sec. 3.3): 0 <= |CP(i)| = cbn[i] - |EP(i)| <= |EP(i+1)|,
 * which makes LP recoverable and the pairwise CP check of Alg. 3 exact.
 * Returns CBAA_OK or CBAA_ECONFIG. */
int cbaa_config_validate(const cbaa_config* h_cfg);

/* Bytes of one cube: the 256-byte header plus 2^r * g/8 * sum_a c(a) bytes of
 * bits (2^27 at the defaults). 0 if the configuration is invalid. */
uint64_t cbaa_cube_bytes(const cbaa_config* h_cfg);

/* 64-bit FNV-1a hash of a valid configuration: the bytes of these 32-bit
 * little-endian fields in this order: r, n_ra, n_va, log2_g, cbn[0 .. n_ra+n_va),
 * cl_bs[0 .. n_ra), seed_mangle, seed_bv, seed_va[0 .. n_va). Fields beyond the
 * counts are not hashed. 0 if the configuration is invalid. */
uint64_t cbaa_config_hash(const cbaa_config* h_cfg);

/* Reads the cube's header back (synchronises `stream`): CBAA_OK if it is a
 * valid header of this configuration, CBAA_ECONFIG if it is missing, of
 * another configuration or marked CBAA_CUBE_MIXED. */
int cbaa_cube_check(const cbaa_config* h_cfg, const void* d_cube, void* stream);

/* Bytes of scratch the partitioned update path needs to take n_pairs packets
 * into n_cubes (1 or 2) cubes in one pass. Smaller (non-zero) scratch makes
 * cbaa_update split the batch; see cbaa_update. */
uint64_t cbaa_update_scratch_bytes(const cbaa_config* h_cfg, uint64_t n_pairs, int n_cubes);

/* Bytes of scratch cbaa_restore needs for `capacity` output hosts, and that
 * cbaa_estimate needs (capacity 0). */
uint64_t cbaa_restore_scratch_bytes(const cbaa_config* h_cfg, uint64_t capacity);

/* ---- local server ---------------------------------------------------- */

/* Starts a window: writes the header and zeroes the bits of a cube of
 * cbaa_cube_bytes bytes (Sec. 3.1: all bits vectors start at zero). d_cube
 * must be 16-byte aligned. */
int cbaa_cube_init(const cbaa_config* h_cfg, void* d_cube, void* stream);

/* Alg. 1 for a batch: for every pair k, with (host, peer) = (src, dst) for
 * CBAA_SIDE_SRC or (dst, src) for CBAA_SIDE_DST, sets bit H_bv(peer) in the
 * host's column of every array of its sketch. d_pairs holds n_pairs (source,
 * destination) uint32 pairs, interleaved, 8-byte aligned. The result is the
 * OR of every pair's bits: independent of order, duplicates, batching and of
 * concurrent updates of the same cube from other streams.
 * d_scratch/scratch_bytes: NULL/0 selects direct global atomics; otherwise
 * the batch is partitioned by (sketch, row block) and applied through LDS
 * tiles, in as many passes as the scratch requires (CBAA_ESCRATCH if it holds
 * less than one pass of the minimum size). A scratch buffer belongs to one
 * call at a time: calls that may overlap (other streams) need their own.
 * n_pairs = 0 is a no-op. */
int cbaa_update(const cbaa_config* h_cfg, void* d_cube, const uint32_t* d_pairs,
                uint64_t n_pairs, int side, void* d_scratch, uint64_t scratch_bytes,
                void* stream);

/* Both directions from one read of the batch: d_cube_src keyed by source,
 * d_cube_dst keyed by destination. Same semantics as two cbaa_update calls. */
int cbaa_update2(const cbaa_config* h_cfg, void* d_cube_src, void* d_cube_dst,
                 const uint32_t* d_pairs, uint64_t n_pairs, void* d_scratch,
                 uint64_t scratch_bytes, void* stream);

/* One edge router's batch inside cbaa_update_batch. */
typedef struct cbaa_stream_batch {
  const uint32_t* d_pairs;  /* n_pairs (source, destination) pairs, 8-byte aligned */
  uint64_t n_pairs;
  void* d_cube;             /* keyed by `side`; keyed by source when d_cube_dst is set */
  void* d_cube_dst;         /* NULL, or the destination-keyed cube (both sides per read) */
  int side;                 /* CBAA_SIDE_*; ignored when d_cube_dst is set */
  int flags;                /* 0 or CBAA_BATCH_FRESH */
} cbaa_stream_batch;

/* The stream's cube(s) start this call empty: whatever they held before is
 * overwritten, as if zeroed first (Alg. 1 starts every window from empty
 * arrays; folding that into the update saves a pass over the cube and lets
 * the update store whole row blocks instead of OR-ing them). A fresh
 * stream's cubes may not be named by any other stream of the batch. */
#define CBAA_BATCH_FRESH 1

/* Tile and partition shapes of the partitioned update (0 = library default):
 * chunk_pairs  pairs per piece of the sample that sizes the bins' regions
 *              (every 64th piece of a stream is counted; multiple of 1024,
 *              <= 2^22)
 * seg_records  records per apply work item (1024 .. 2^24)
 * apply_blocks persistent blocks of the apply step (1..65536) */
typedef struct cbaa_tuning {
  uint32_t chunk_pairs;
  uint32_t seg_records;
  uint32_t apply_blocks;
  uint32_t reserved;
} cbaa_tuning;

/* Scratch bytes cbaa_update_batch needs for these streams and shapes. */
uint64_t cbaa_update_batch_scratch_bytes(const cbaa_config* h_cfg,
                                         const cbaa_stream_batch* h_streams, int k,
                                         const cbaa_tuning* h_tuning);

/* Alg. 1 for the batches of k (1..CBAA_MAX_BATCH) edge routers at once, with
 * uneven sizes, through one sequence of launches of the partitioned path:
 * the same result as k cbaa_update (or cbaa_update2) calls (after zeroing
 * the cubes of streams flagged CBAA_BATCH_FRESH). Either every stream sets
 * d_cube_dst or none does. Streams without the flag may share cubes. The scratch
 * must hold the whole batch (CBAA_ESCRATCH otherwise); a stream may have up to
 * about 0.45 x 2^32 / cubes pairs (its records' regions and overflow list are
 * addressed with 32-bit offsets; CBAA_EINVAL beyond). Only enqueues device work, so the
 * call can be captured into a HIP graph and replayed. Configurations outside
 * the partitioned path's limits (cbaa_update_scratch_bytes returns 0) get
 * CBAA_ECONFIG. */
int cbaa_update_batch(const cbaa_config* h_cfg, const cbaa_stream_batch* h_streams, int k,
                      const cbaa_tuning* h_tuning, void* d_scratch, uint64_t scratch_bytes,
                      void* stream);

/* ---- global server --------------------------------------------------- */

/* Sec. 3.3: d_dst = bitwise OR of k cubes of one configuration. h_srcs is a
 * host array of k >= 1 device pointers; d_dst (not NULL) may equal any of
 * them. d_dst gets a valid header when every source has one of this
 * configuration, else a header marked CBAA_CUBE_MIXED. */
int cbaa_merge_or(const cbaa_config* h_cfg, void* d_dst, const void* const* h_srcs, int k,
                  void* stream);

/* Per-column zero counts (the quantity Alg. 2 thresholds) and per-array fill.
 * d_zeros: uint16[2^r * W], entry cs*W + A_off(a) + col = g - popcount;
 * d_ones : uint32[2^r * (n_ra+n_va)], entry cs*A + a = one bits of array a. */
int cbaa_column_zeros(const cbaa_config* h_cfg, const void* d_cube, uint16_t* d_zeros,
                      uint32_t* d_ones, void* stream);

/* Restores the super hosts of a merged cube (Sec. 3.3): per sketch eps =
 * product of array fills (Thm. 1 with each array's measured fill as P_1),
 * Zmax by `thr_rule` for `theta`, hot columns of every RA (Alg. 2), CP-valid
 * tuples (Alg. 3) whose union column has Z <= Zmax, IP = M^-1(LP || RP).
 * d_out receives min(n, capacity) cbaa_host entries sorted by ip ascending;
 * d_stats (device) receives the counters, n_hosts being the full count n
 * (when n > capacity the output holds an unspecified subset: call again
 * with more capacity). d_scratch holds cbaa_restore_scratch_bytes(capacity).
 * max_checks bounds the tuple check's work: once it has examined more than
 * max_checks tuples (partial tuples whose AND is counted, and complete
 * CP-valid tuples), it stops, every wave exits soon after (each overshoots
 * by at most a few hundred tuples) and d_stats->status gets
 * CBAA_STATUS_BUDGET (the list then holds the hosts found so far, n_hosts
 * counting them). 0 selects CBAA_DEFAULT_MAX_CHECKS. An
 * over-full window (every column hot) thus ends in bounded time instead of
 * enumerating up to 2^(32 - r) tuples per sketch.
 * A cube without this configuration's valid header gives status
 * CBAA_STATUS_CONFIG and no hosts.
 * Asynchronous: read d_stats after synchronising the stream. */
#define CBAA_DEFAULT_MAX_CHECKS (1ull << 28)
int cbaa_restore(const cbaa_config* h_cfg, const void* d_cube, double theta, int thr_rule,
                 uint64_t max_checks, void* d_scratch, uint64_t scratch_bytes, cbaa_host* d_out,
                 uint64_t capacity, cbaa_restore_stats* d_stats, void* stream);

/* The global server's window end in one call (Sec. 3.3): d_dst = bitwise OR
 * of the k router cubes (as cbaa_merge_or; d_dst may equal a source), then
 * the restore of d_dst exactly as cbaa_restore. For k <= 16 the OR and the
 * per-column zero counts the restore starts from are computed in one pass
 * over the sources, so the merged cube is written once and never re-read
 * for the counts; larger k merges first. Arguments and results as for
 * cbaa_merge_or and cbaa_restore; status CBAA_STATUS_CONFIG when any source
 * lacks this configuration's valid header.
 * d_dst may be NULL when k <= 16: the merged cube is then not stored, and
 * the restore reads each column it needs (hot columns, VA columns) as the OR
 * of the sources. The restored list and stats are those of the stored case.
 * NULL with k > 16 returns CBAA_EINVAL. */
int cbaa_merge_restore(const cbaa_config* h_cfg, void* d_dst, const void* const* h_srcs, int k,
                       double theta, int thr_rule, uint64_t max_checks, void* d_scratch,
                       uint64_t scratch_bytes, cbaa_host* d_out, uint64_t capacity,
                       cbaa_restore_stats* d_stats, void* stream);

/* cbaa_merge_restore in two calls, so that a caller can order the
 * bandwidth-bound half of one window end against other work: for instance
 * the two sides of a window on two streams, the second side's merge scan
 * waiting (on an event) for the first side's, so that it runs while the
 * first side's latency-bound tuple check does.
 * cbaa_merge_scan: the OR-merge of the k sources (stored in d_dst unless it
 * is NULL), the column scan, the thresholds (Thm. 1, Thm. 2) and the hot
 * column lists (Alg. 2), kept in d_scratch.
 * cbaa_restore_scanned: the rest of the restore (Alg. 3's tuple check and
 * the ordered list) from that scratch.
 * Both take exactly cbaa_merge_restore's arguments, and the pair gives its
 * result, provided that the second call names the same configuration,
 * destination, sources, scratch, capacity and stats as the first, runs after
 * it in stream order, and no call in between writes the sources, the
 * destination or the scratch. Each checks its arguments as cbaa_merge_restore
 * does; the scan leaves d_out untouched. */
int cbaa_merge_scan(const cbaa_config* h_cfg, void* d_dst, const void* const* h_srcs, int k,
                    double theta, int thr_rule, uint64_t max_checks, void* d_scratch,
                    uint64_t scratch_bytes, cbaa_host* d_out, uint64_t capacity,
                    cbaa_restore_stats* d_stats, void* stream);
int cbaa_restore_scanned(const cbaa_config* h_cfg, void* d_dst, const void* const* h_srcs, int k,
                         double theta, int thr_rule, uint64_t max_checks, void* d_scratch,
                         uint64_t scratch_bytes, cbaa_host* d_out, uint64_t capacity,
                         cbaa_restore_stats* d_stats, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * cbaa_merge_restore without a scratch argument. Its scratch is an array of
 * CBAA_NOALLOC_SCRATCH_BYTES inside the library, one copy per device, held
 * from the first call on that device until the process ends; the call itself
 * allocates nothing, host or device (at most 64 sources, kept on the stack).
 * The first call on a device resolves the array's address (make it outside
 * graph capture). Arguments, results and asynchrony are those of
 * cbaa_merge_restore. CBAA_ESCRATCH when cbaa_restore_scratch_bytes(cfg,
 * capacity) exceeds the array (at the paper's dimensions that is a capacity
 * above about 1.5 million hosts). Every call on a device shares that device's
 * array, which keeps the last call's contents: calls that overlap on one device
 * (other streams, other threads) race and must be serialised by the caller. */
#define CBAA_NOALLOC_SCRATCH_BYTES (64ull << 20)
int cbaa_merge_restore_noalloc(const cbaa_config* h_cfg, void* d_dst, const void* const* h_srcs,
                               int k, double theta, int thr_rule, uint64_t max_checks,
                               cbaa_host* d_out, uint64_t capacity, cbaa_restore_stats* d_stats,
                               void* stream);

/* Thm. 2 estimate for given inner IPs: d_est[k] (double), d_zeros[k] (Z of
 * the union column) and, if d_layer_zeros is not NULL, the zero count of each
 * of the host's n_ra+n_va columns at d_layer_zeros[k*A + a] (uint16). eps is
 * measured from the cube as in cbaa_restore. d_scratch holds
 * cbaa_restore_scratch_bytes(cfg, 0). The header is not checked (see
 * cbaa_cube_check). */
int cbaa_estimate(const cbaa_config* h_cfg, const void* d_cube, const uint32_t* d_hosts,
                  uint64_t n, double* d_est, uint16_t* d_zeros, uint16_t* d_layer_zeros,
                  void* d_scratch, uint64_t scratch_bytes, void* stream);

/* ---- errors ---------------------------------------------------------- */

const char* cbaa_strerror(int code);
const char* cbaa_last_error(void);
uint32_t cbaa_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CBAA_H */
