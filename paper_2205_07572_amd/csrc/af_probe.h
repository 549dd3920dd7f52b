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

#ifdef __cplusplus
}
#endif
#endif /* AF_PROBE_H */
