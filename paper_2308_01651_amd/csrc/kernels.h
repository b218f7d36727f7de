// Host-callable launchers of the step kernels (defined in kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "ep_device.h"

namespace ep {

// One launch over a block map: nblocks workgroups of WG threads, workgroup b
// working on instance bmap[b].inst, node tile bmap[b].lblk.
struct Launch {
  const InstDesc* insts;
  const BlockMap* bmap;
  int nblocks;
  hipStream_t stream;
};

void launch_ionic(int model, bool mixed, const Launch& L);
void launch_residual(bool mixed, bool with_rhs, const Launch& L);
void launch_cg_spmv(bool mixed, const Launch& L);
void launch_cg_update(bool mixed, const Launch& L);
void launch_activation(const Launch& L);
// ids: device array of instance indices to advance by one step
void launch_end_step(const InstDesc* insts, const int32_t* ids, int n_ids, hipStream_t stream);
void launch_fill(double* x, int64_t n, double v, hipStream_t stream);
void launch_to_mv(void* dst, const double* u, int64_t n, double a, double b, bool f32, hipStream_t stream);

}  // namespace ep
