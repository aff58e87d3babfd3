/*
 * dsm_probe.h -- C ABI of libdsm_probe.so: plain streaming kernels that give
 * the benchmark a measured bandwidth ceiling on the same GPU, in the same
 * run, beside the fused lattice Boltzmann step of libdsm.so.  They are
 * measurement tools, not part of the method: the fused step is a read-write
 * stream (about half of its bytes read, half written), so the rate of a
 * plain device copy is the ceiling its own traffic mix can reach.
 *
 * Ownership: every pointer is a caller-owned device buffer; nothing is
 * allocated.  Work is enqueued on `stream` (hipStream_t; NULL = default
 * stream) and the call returns without synchronising.
 */
#ifndef DSM_PROBE_H
#define DSM_PROBE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* kinds of stream */
enum {
    DSM_PROBE_COPY = 0,     /* dst[i] = src[i], 16 bytes per lane, grid-stride        */
    DSM_PROBE_COPY_NT = 1,  /* the same with non-temporal stores                       */
    DSM_PROBE_READ = 2,     /* reads src; each lane writes one 16-byte sum to dst      */
    DSM_PROBE_WRITE = 3,    /* dst[i] = a constant, non-temporal stores                 */
    DSM_PROBE_COPY4 = 4     /* copy at 4 bytes per lane (the fused step's access size), */
                            /* non-temporal stores                                      */
};

/* Streams `bytes` (a multiple of 16; src and dst 16-byte aligned and not
 * overlapping; for DSM_PROBE_READ dst must hold 16 bytes per lane of the
 * grid, blocks * 256 lanes) with `blocks` workgroups of 256 lanes.
 * Returns 0, or -1 for invalid arguments (checked before any device work),
 * or -3 if the launch fails. */
int dsm_probe_stream(int kind, const void* src, void* dst, size_t bytes, int blocks, void* stream);

#ifdef __cplusplus
}
#endif
#endif
