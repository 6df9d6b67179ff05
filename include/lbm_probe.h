/*
 * lbm_probe.h -- C ABI of the measurement library libprobe.so, built beside
 * the solver library but not part of it: plain streaming kernels that give
 * the practical HBM ceiling quoted next to the published peak in the
 * rooflines of the step kernels.  Nothing of the method runs here.
 */
#ifndef LBM_PROBE_H
#define LBM_PROBE_H

#include <stddef.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

/* The HBM rate that plain
 * streaming kernels reach on this device, the practical ceiling next to the
 * published peak in the rooflines of the step kernels.  kind 0 copies src to
 * dst with one 4-byte element per thread (the access width of the population
 * gathers), kind 1 copies with one 16-byte element per thread, kind 2 only
 * reads src, 16 bytes per thread, kind 3 copies eight 4-byte elements per
 * thread (each load coalesced over the block).  Kinds 4 and 5 move the
 * populations of the 3-D node update without its arithmetic: every node of a
 * 128 x 128 x nz box loads 19 populations of two components from its
 * neighbours' slots in 38 planes (pull streaming, as in eq. 2) and stores 38
 * values at its own slots, 16 nodes per thread along the slowest axis; kind 4
 * issues a node's loads after the previous node's stores, kind 5 before them;
 * kind 6 keeps both components of a population side by side in one 8-byte
 * slot (19 planes; 19 loads and 19 stores of 8 bytes per node).
 * They count 304 bytes per node of the largest box that fits in the buffers
 * (at most 2^31 - 1 bytes, and room for at least 20 planes).  bytes (a
 * multiple of 16, at least 16) is the size of src and of dst, both
 * caller-owned device buffers.  Runs one
 * warm-up and reps timed launches on hip_stream (NULL = default) with HIP
 * events, synchronises, and writes the rate in GB/s (bytes read plus bytes
 * written, per second) to *gbs.  LBM_EINVAL for bad arguments, LBM_EDEVICE
 * for HIP errors. */
lbm_status lbm_stream_probe(const void *src, void *dst, size_t bytes, int kind, int reps, void *hip_stream,
                            double *gbs);

#ifdef __cplusplus
}
#endif
#endif
