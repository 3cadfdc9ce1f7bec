/*
 * nys_noalloc.h -- the allocation-free kernel product of libnys (see nys.h for the
 * conventions shared by every entry point).
 */
#ifndef NYS_NOALLOC_H
#define NYS_NOALLOC_H

#include "nys.h"

#ifdef __cplusplus
extern "C" {
#endif

/* ---- allocation-free kernel product ----------------------------------------
 * kernel_matvec_noalloc: kernel_matvec (same arguments, same result, same kernels)
 * for callers that cannot allocate device memory -- code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  It takes no workspace: its
 * scratch is a fixed array of nys_noalloc_scratch_bytes() bytes (256 MiB) that each
 * GPU the library runs on holds until the process ends, and it calls no hipMalloc,
 * hipFree or allocating library routine.  A product whose workspace
 * (nys_workspace_bytes(NYS_OP_KERNEL_MATVEC, ...)) exceeds that size returns
 * NYS_ENOMEM before any device work.  Every call on one GPU shares that GPU's array
 * and leaves its contents behind: calls that overlap on one GPU (concurrent streams
 * or threads) race and must be serialised by the caller.  Like kernel_matvec it
 * synchronises the stream once, after packing the points. */
int32_t kernel_matvec_noalloc(nys_kernel k, int32_t deriv, int32_t prec, const double *Xr, int64_t nr,
                              const double *Xc, int64_t nc, int32_t d, const void *V, int32_t m, void *Out,
                              double alpha, double beta, void *stream);
size_t nys_noalloc_scratch_bytes(void);

#ifdef __cplusplus
}
#endif

#endif /* NYS_NOALLOC_H */
