/*
 * bwprobe.h -- memory-bandwidth probes of the MI355X the solver runs on.
 *
 * Not part of the solver's C ABI: small measurement kernels that give the
 * ceilings the solver's HBM-bound kernels are compared with (a streaming
 * read, a streaming copy, and repeated reads of a buffer small enough to
 * stay in the memory-side Infinity Cache).  Each call runs its kernel
 * ``iters`` times on a private stream of default priority, after one
 * untimed run, and returns the average kernel time measured with HIP events
 * on that stream.  All pointers are device pointers owned by the caller;
 * nothing is allocated on the device.  Returns 0, or -1 for a bad argument
 * (bytes not a positive multiple of 32768, iters < 1, a null pointer) and
 * -2 when a HIP call fails.
 */
#ifndef ASSG_BWPROBE_H
#define ASSG_BWPROBE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Reads ``bytes`` of ``buf`` once per iteration with 16-byte loads, every
 * workgroup a contiguous 32 KiB piece, and writes one double per workgroup
 * into ``partial`` (device, at least bytes / 32768 doubles) so that the
 * loads are not removed.  ``nontemporal``: 1 streaming loads, 0 ordinary
 * loads (cached in L2 and the Infinity Cache). */
int assg_bw_read(const void* buf, size_t bytes, int nontemporal, int iters, double* partial,
                 float* ms_avg);

/* Copies ``bytes`` from src to dst (device, not overlapping) per iteration,
 * streaming loads and stores, 32 KiB per workgroup. */
int assg_bw_copy(const void* src, void* dst, size_t bytes, int iters, float* ms_avg);

#ifdef __cplusplus
}
#endif

#endif /* ASSG_BWPROBE_H */
