/*
 * hbm_probe.h -- C ABI of libhbmprobe, a streaming-copy probe that measures
 * the practical HBM ceiling of a kernel moving the same bytes as one lattice
 * Boltzmann step (each population read once and written once, Eq. (1)).
 * A measurement tool beside liblbsoft, not part of the step.
 */
#ifndef LBSOFT_HBM_PROBE_H
#define LBSOFT_HBM_PROBE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Enqueue one copy of `bytes` bytes from device buffer src to device buffer
 * dst (both 16-byte aligned, not overlapping; bytes a multiple of 16) on the
 * HIP stream `stream` (NULL: null stream), as `blocks` workgroups of
 * `threads` lanes (64..256, a multiple of 64) moving 16-byte items in a
 * grid-stride loop with `unroll` (1, 2 or 4) items in flight per lane;
 * nt != 0 uses nontemporal stores.  Returns 0, -1 for invalid arguments
 * (nothing enqueued) or -3 if the launch failed.  Asynchronous; the caller
 * owns both buffers. */
int hbm_copy(const void* src, void* dst, size_t bytes, int blocks, int threads, int nt,
             int unroll, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* LBSOFT_HBM_PROBE_H */
