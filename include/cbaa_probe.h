/*
 * cbaa_probe.h -- measurement probes of libcbaa. They are not steps of the
 * method: they measure on the device the two ceilings the update kernels are
 * priced against, instead of taking them from a datasheet.
 *
 * Conventions are those of cbaa.h: d_* are device pointers on the current
 * device owned by the caller, `stream` is a hipStream_t, calls only enqueue
 * work, and return CBAA_OK or CBAA_EINVAL (bad argument, nothing launched) or
 * CBAA_EHIP.
 */
#ifndef CBAA_PROBE_H
#define CBAA_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* HBM streaming ceiling: copies `bytes` (a multiple of 16) from d_src to
 * d_dst, both 16-byte aligned and not overlapping, with `blocks` blocks of
 * 256 threads (0 = 2048; at most 2^20) that stride over the buffers in
 * 16-byte loads and stores, nontemporal ones with CBAA_PROBE_NONTEMPORAL in
 * `flags`. Time it with events on `stream`; bytes moved = 2 x bytes. */
#define CBAA_PROBE_NONTEMPORAL 1u
int cbaa_probe_copy(void* d_dst, const void* d_src, uint64_t bytes, uint32_t blocks,
                    uint32_t flags, void* stream);

/* Fills d_addr[0..n) with word indices drawn uniformly from [0, 2^log2_words)
 * (the top bits of a mixed counter, seeded), for cbaa_probe_atomic_or. */
int cbaa_probe_addresses(uint32_t* d_addr, uint64_t n, uint32_t log2_words, uint32_t seed,
                         void* stream);

/* Random-atomic ceiling of the paper's one-thread-per-packet update (Sec. 4.1,
 * Alg. 1: a pair sets |RA| + |VA| bits, 4 at the paper's dimensions): n (a
 * multiple of 4) device-scope 32-bit atomic ORs whose results are unused, into
 * d_buf of `words` uint32 words (a power of two up to 2^32; 2^25 words = one
 * 128 MiB cube). Thread t takes indices d_addr[4t .. 4t+4) (16-byte aligned)
 * masked to the buffer, so every access stays inside it. */
int cbaa_probe_atomic_or(uint32_t* d_buf, uint64_t words, const uint32_t* d_addr, uint64_t n,
                         void* stream);

#ifdef __cplusplus
}
#endif

#endif /* CBAA_PROBE_H */
