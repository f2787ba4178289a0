/*
 * qlra_noalloc.h -- the solve of qlra() without device allocation (MI355X /
 * gfx950 library for pass-efficient randomized low-rank approximation of
 * quaternion matrices, arXiv 2507.13731).  Declarations beside qlra.h.
 */
#ifndef QLRA_NOALLOC_H
#define QLRA_NOALLOC_H

#include "qlra.h"

#ifdef __cplusplus
extern "C" {
#endif

/* ---- a solve that allocates nothing ----
 *
 * For callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation.  qlra_noalloc() takes
 * the arguments of qlra() and computes exactly what qlra() computes (the same
 * kernels), but its workspace is a device array of qlra_noalloc_max_bytes()
 * bytes (128 MiB) inside the library, one per GPU, held from the library's
 * first use on that GPU until the process ends; opts->workspace and
 * opts->workspace_bytes are ignored.  It allocates no memory and creates no
 * stream, event or graph: opts->graph is ignored and the per-pass estimates
 * run on the caller's stream.  A solve whose qlra_workspace_size() exceeds
 * the maximum is rejected with QLRA_E_TOO_LARGE before anything is enqueued.
 * Every call on a GPU uses that GPU's one array: calls that may overlap on one
 * GPU (other streams, other threads) race and must be ordered by the caller;
 * each call clears what must start at zero itself.  qlra_noalloc_status()
 * reports the status word of the last such solve on the current GPU as
 * qlra_status() does for a workspace (it synchronises `stream`). */
size_t qlra_noalloc_max_bytes(void);
int qlra_noalloc(const float* A, int64_t m, int64_t n, int64_t lda, int64_t a_plane_stride,
                 int k, int p, int pass_budget, int scheme, uint64_t seed, const qlra_opts_t* opts,
                 float* U, int64_t ldu, int64_t u_plane_stride,
                 double* S,
                 float* V, int64_t ldv, int64_t v_plane_stride,
                 double* pass_err);
int qlra_noalloc_status(void* stream, int* status);

#ifdef __cplusplus
}
#endif
#endif /* QLRA_NOALLOC_H */
