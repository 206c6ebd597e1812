// Launch wrappers of the HIP kernels (kernels.hip).  dtype: 0 = complex64,
// 1 = complex128.  All launches are asynchronous on stream s.
#pragma once
#include <hip/hip_runtime.h>

#include "fl_common.h"

namespace fl {

hipError_t launch_sweep(int dtype, const fl_geom& g, void* psi, const void* gates, const fl_pass& pd, hipStream_t s);
hipError_t launch_rdm(int dtype, const fl_geom& g, const void* psi, const fl_pass& pd, double* partials, int grid,
                      int nslot, hipStream_t s);
// complex64 bond reductions over full 13-bit tiles; pd from plan_cover_groups
// of geometry (L, 13, 5) (L >= 14)
hipError_t launch_rdm_groups(const fl_geom& g, const void* psi, const fl_pass& pd, double* partials, int grid,
                             int nslot, hipStream_t s);
hipError_t launch_finalize(const double* partials, int nblocks, int nvals, double* out, hipStream_t s);
// <H0> and the norm from finalized bond sums red[L*16] and FP64 bond terms h64[(L-1)*32]:
// out[0] = <H0>, out[1] = <psi|psi>; rdm (may be NULL) = [L-1][4][4] complex
hipError_t launch_energy_contract(const double* red, const double* h64, int L, double* out, double* rdm, hipStream_t s);
hipError_t launch_init(int dtype, void* psi, int L, const void* tabs, int a, int b, hipStream_t s);
hipError_t launch_overlap(int dta, const void* a, int dtb, const void* b, uint64_t n, double* partials, int grid,
                          hipStream_t s);
hipError_t launch_apply_h(int dtype, const fl_geom& g, const void* psi, void* lam, const void* hmat, const fl_pass& pd,
                          int first, hipStream_t s);
hipError_t launch_adjoint(int dtype, const fl_geom& g, void* psi, void* lam, const void* gates, const fl_pass& pd,
                          double* Mpart, int grid, hipStream_t s);
// reverse pass of the 4-qubit-window form (complex64, full 13-bit tiles) on
// the matrix cores: mats = the pass's window fragments (4 KiB per group, the
// transposes of the forward's), Qpart [grid][FL_WIN4_MAX_GROUPS][512]
// per-workgroup scratch, Qsum [pass groups][512] += the pass's window
// overlaps (Re, Im of 16x16)
hipError_t launch_adjoint_win4(const fl_geom& g, void* psi, void* lam, const void* mats, const fl_pass& pd,
                               double* Qpart, int grid, double* Qsum, hipStream_t s);
hipError_t launch_zero(double* p, uint64_t n, hipStream_t s);
// 4-qubit windows on FP32 MFMA; full tiles only (C + W = 13); mats: 4 KiB of fragments per window
hipError_t launch_dense4(const fl_geom& g, void* psi, const void* mats, const fl_pass& pd, hipStream_t s);
// mode 0: FP32 MFMA, 1: split-BF16x3 MFMA; mats: pre-arranged window matrices of the plan
hipError_t launch_dense6(int mode, const fl_geom& g, void* psi, const void* mats, const fl_pass& pd, hipStream_t s);

}  // namespace fl
