// Host entry points of the HIP kernels (implemented in kernels.hip).
#pragma once
#include <hip/hip_runtime_api.h>

#include <cstdint>

#include "plan.h"

namespace dd {

// numeric factorisation (enqueue only); with a side stream the trailing
// updates' look-ahead part runs there, joined back before returning
hipError_t factor(const Plan &P, uint8_t *ws, const void *vals, hipStream_t st, KTimer *tm = nullptr,
                  const SideStream *side = nullptr);
// one launch of the factorisation kernels (the tile tuner's measurements)
hipError_t run_launch(const Plan &P, uint8_t *ws, const Launch &L, hipStream_t st);
// torn right-hand sides (interleaved complex FP64, ld ldf) -> internal vector
hipError_t rhs_in(const Plan &P, uint8_t *ws, const void *f, int64_t ldf, int nrhs, hipStream_t st);
// one DD solve of the internal right-hand side (with_c: constraint rhs in vc;
// subset: the backward substitution skips the domains whose byte in the
// workspace's domain mask is 0)
hipError_t solve_core(const Plan &P, uint8_t *ws, int nrhs, bool with_c, hipStream_t st, KTimer *tm = nullptr,
                      bool subset = false, const int *gate = nullptr);
// internal solution / multipliers -> interleaved complex FP64 (subset: only
// the rows of the domains selected in the domain mask)
hipError_t sol_out(const Plan &P, uint8_t *ws, void *u, int64_t ldu, void *lam, int64_t ldl, int nrhs,
                   hipStream_t st, bool subset = false);
hipError_t interface_inverse_out(const Plan &P, uint8_t *ws, int front, void *out, hipStream_t st);
// the rows listed in the workspace's selection region (nsel torn row ids) of
// the internal solution -> interleaved complex FP64 out (nsel x nrhs, ld ldo)
hipError_t sel_out(const Plan &P, uint8_t *ws, int64_t nsel, void *out, int64_t ldo, int nrhs, hipStream_t st);
// FP64 iterative refinement around the FP32 factorisation
// FP64 copy of the operator values (caller's CSR order) into the workspace's
// SELL-64 layout, read by the refinement residual
hipError_t operator_copy(const Plan &P, uint8_t *ws, const void *vals, hipStream_t st);
hipError_t refine_init(const Plan &P, uint8_t *ws, int nrhs, hipStream_t st);
// gate (device int, may be null): the launches return at once while it is
// nonzero (a converged refinement skips its remaining enqueued iterations)
hipError_t refine_update(const Plan &P, uint8_t *ws, int nrhs, hipStream_t st, const int *gate = nullptr);
hipError_t refine_resid(const Plan &P, uint8_t *ws, const void *f, int64_t ldf, int nrhs, bool fnorm,
                        hipStream_t st, const int *gate = nullptr);
// refinement control words in the workspace: [0] converged (or non-finite),
// [1] correction iterations that ran, [2] non-finite residual; and the last
// maxima of the torn and the assembled relative residual (2 doubles)
int *refine_ctl(const Plan &P, uint8_t *ws);
const double *refine_rel(const Plan &P, uint8_t *ws);
hipError_t refine_ctl_reset(const Plan &P, uint8_t *ws, hipStream_t st);
// convergence test of the last residual (count: a correction preceded it)
hipError_t refine_test(const Plan &P, uint8_t *ws, int nrhs, double tol, bool count, hipStream_t st);
hipError_t refine_out(const Plan &P, uint8_t *ws, void *u, int64_t ldu, void *lam, int64_t ldl, int nrhs,
                      hipStream_t st);

}  // namespace dd
