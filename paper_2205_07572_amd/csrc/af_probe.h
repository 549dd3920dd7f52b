/*
 * af_probe.h -- measurement helpers exported by libaf.so that are not part
 * of the method's interface (include/af.h).  They serve benchmarks only.
 */
#ifndef AF_PROBE_H
#define AF_PROBE_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#include "af.h"

#ifdef __cplusplus
extern "C" {
#endif

/* af_fma_probe -- nblocks blocks of 256 threads each run 8 independent
 * multiply-add chains of 16 x iters steps in `prec` (AF_FP32 or AF_FP64),
 * compiled like the library's kernels, and write one value per thread to out
 * (device, [nblocks * 256] elements of that precision).  2 * 8 * 16 * iters *
 * 256 * nblocks flops; timing it on `stream` gives the vector FMA rate the
 * kernels can reach on this device.  AF_ERR_ARG for a bad precision, a null
 * out or counts below 1; nothing is launched then. */
af_status af_fma_probe(int32_t prec, void* out, int32_t nblocks, int32_t iters, hipStream_t stream);

/* af_amr_coarse_step_timed -- af_amr_coarse_step (subcycled, eager) that
 * also records a pair of HIP events on `stream` around each launch of the
 * batched step kernel: events[2k] before and events[2k + 1] after the k-th,
 * for the first max_launches launches (events: caller-created hipEvent_t,
 * 2 * max_launches of them, created with timing enabled).  *nlaunch receives
 * the number of launches timed; cell_updates (host, max_launches entries, or
 * NULL) the interior leaf cell-updates of each.  Hierarchies stepped by the
 * one-level path or the per-level path (variable coefficients) record
 * nothing. */
af_status af_amr_coarse_step_timed(af_ctx* ctx, af_hier* h, af_state* bufs, uint32_t* level_buf_mask, double t0,
                                   double dt0, double* flux_reg, hipStream_t stream, void** events,
                                   int32_t max_launches, int32_t* nlaunch, double* cell_updates);

#ifdef __cplusplus
}
#endif
#endif /* AF_PROBE_H */
