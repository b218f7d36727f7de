// Host-callable launchers of the step kernels (defined in kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "ep_device.h"

namespace ep {

// One launch over a block map: nblocks workgroups, workgroup b working on
// instance bmap[b].inst, node tile bmap[b].lblk.  single: the table holds one
// instance and workgroups map to its tiles without a block map read (xmap 0:
// each XCD sweeps a contiguous range of tiles; 1: workgroup b takes tile b).
// ionic_npt: nodes per thread of the ionic kernel (1, 2 or 4; TILE / npt
// threads per workgroup).  A batch launches the ionic kernel per (model,
// ionic scheme) group.
struct Launch {
  InstDesc* insts;
  const BlockMap* bmap;
  int nblocks;
  hipStream_t stream;
  bool single;
  int xmap = 0;
  int ionic_npt = 1;
  bool ionic_bdf = false;  // the instances use the semi-implicit BDF ionic scheme
  // matrix-free operator (single instance, FP64): degree of its hexahedra
  // (0: assembled) and element count; the SpMV and rhs launches then run
  // the element kernels first
  int mf_p = 0;
  int64_t mf_elems = 0;
  bool mf_cmp = false;     // compressed geometry factors (element constants)
  // pipelined CG of instances whose operators are all 14-diagonal symmetric
  // DIA with Jacobi preconditioning: the specialized kernels
  int pipe_op = 0;
};

void launch_ionic(int model, bool mixed, const Launch& L);
void launch_residual(bool mixed, bool with_rhs, const Launch& L);
void launch_cg_spmv(bool mixed, const Launch& L);
void launch_cg_update(bool mixed, const Launch& L);
// FP64: the update with the finalize's work (partial sums, convergence,
// step lengths) done by every workgroup; a round is SpMV then this kernel
void launch_cg_update64(const Launch& L);
// FP64 pipelined CG: the start (w_0 = A u_0, m_0, delta_0) after the
// residual, then one launch per iteration (instances without cg_pipe skip)
void launch_cg_pipe_start(const Launch& L);
void launch_cg_pipe(const Launch& L);
// mixed precision: the pipelined FP32 inner solve (start after each
// residual, then one launch per inner iteration)
void launch_cg_pipe32_start(const Launch& L);
void launch_cg_pipe32(const Launch& L);
// one workgroup per instance listed in ids (device array of n_ids indices);
// ids == nullptr with n_ids == 1: the single instance at insts[0]
void launch_cg_finalize(bool mixed, InstDesc* insts, const int32_t* ids, int n_ids, hipStream_t stream);
void launch_activation(const Launch& L);
// ids: device array of instance indices to advance by one step
void launch_end_step(InstDesc* insts, const int32_t* ids, int n_ids, hipStream_t stream);
void launch_fill(double* x, int64_t n, double v, hipStream_t stream);
// reg: per-node subdomain (NaN where < 0) or nullptr
void launch_to_mv(void* dst, const double* u, int64_t n, double a, double b, bool f32, hipStream_t stream,
                  const int32_t* reg = nullptr);
// several subdomains: the ionic step over all n_pts ionic points, then the
// interface correction of the load over its n_crow rows
// (model < 0: the subdomains run different models; bdf: the paper's
// semi-implicit BDF ionic scheme)
void launch_ionic_het(int model, bool mixed, bool bdf, InstDesc* insts, int64_t n_pts, hipStream_t st);
void launch_ici_correction(InstDesc* insts, int64_t n_crow, hipStream_t st);
// single-cell pacing (cell.hip): n_steps steps of nc cells from step index
// step0; uh [3][nc] potential history (u_n, u_{n-1}, u_{n-2}), w [n_vars][nc],
// params [nc][NPARAM]; stimulus amp (model units per ms) on steps whose
// index k+1 mod period (in steps) lies in [1, dur]
void launch_cell_pace(int model, double* uh, double* w, const double* params, int nc, double dt, int bdf,
                      int64_t step0, int64_t n_steps, int64_t period, int64_t dur, double amp, hipStream_t st);


// Allocation-free pacing (cell.hip).  The staging of up to PACE_MAX_CELLS
// cells (potential history [3][nc], state [18][nc], parameter rows
// [nc][NPARAM]) lives in a file-scope device array of PACE_SCRATCH_DOUBLES
// doubles, one copy per device, shared by every call on that device.
constexpr int PACE_MAX_CELLS = 16384;
constexpr int PACE_MAX_DEVICES = 64;
constexpr size_t PACE_SCRATCH_DOUBLES = (size_t)PACE_MAX_CELLS * (3 + 18 + NPARAM);
struct PaceDefaults {
  double mp[NPARAM];   // parameter row of the model and cell type
  double init[19];     // u, then the state (model initial conditions)
};
// device address of the current device's copy of the pacing scratch array
// (looked up once per device); `device` must be the current device
hipError_t pace_scratch(int device, double** ptr);
void launch_pace_stage(const PaceDefaults& def, const double* params, int n_params, const double* init, int nv,
                       int nc, double* uh, double* w, double* mp, hipStream_t st);
void launch_pace_unstage(const double* uh, const double* w, int nv, int nc, double* out, hipStream_t st);

}  // namespace ep
