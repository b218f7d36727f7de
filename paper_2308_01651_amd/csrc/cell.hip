// Single-cell pacing on the GPU: many independent cells (one per thread),
// each the monodomain step without diffusion (paper, Section "Ventricular
// slab": the ionic state is initialized by long single-cell runs paced at the
// cardiac period).  With K 1 = 0 and a uniform state the linear system of a
// step reduces to alpha u_{n+1} = u_BDF + dt (I_app - I_ion(u_EXT, w_{n+1})),
// with the Rush-Larsen ionic step of the tissue kernels at u_EXT.  State and
// potential history stay in registers for a chunk of steps; the host
// launches chunks until the requested number of beats is done.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ep_device.h"
#include "ionic_models.h"
#include "kernels.h"

namespace ep {

template <int MODEL>
__global__ __launch_bounds__(256) void k_cell_pace(double* __restrict__ uh, double* __restrict__ w,
                                                   const double* __restrict__ params, int nc, double dt, int bdf,
                                                   int64_t step0, int64_t n_steps, int64_t period, int64_t dur,
                                                   double amp) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  const double* mp = params + (int64_t)c * NPARAM;
  double u0 = uh[c], u1 = uh[nc + c], u2 = uh[2 * nc + c];
  // state rows [var][cell]
  double x[18];
  const int nv = MODEL == M_AP ? 1 : (MODEL == M_BO ? 3 : (MODEL == M_TTP06 ? 18 : 0));
#pragma unroll
  for (int v = 0; v < 18; v++) x[v] = v < nv ? w[(int64_t)v * nc + c] : 0.0;
  for (int64_t k = 0; k < n_steps; k++) {
    const int64_t step = step0 + k;
    const int sig = (int)min((int64_t)bdf, step + 1);
    double ue, ub, alpha;
    if (sig == 1) {
      ue = u0; ub = u0; alpha = 1.0;
    } else if (sig == 2) {
      ue = 2.0 * u0 - u1; ub = 2.0 * u0 - 0.5 * u1; alpha = 1.5;
    } else {
      ue = 3.0 * u0 - 3.0 * u1 + u2; ub = 3.0 * u0 - 1.5 * u1 + u2 * (1.0 / 3.0); alpha = 11.0 / 6.0;
    }
    double iion = 0.0;
    if (MODEL == M_AP) {
      iion = ap_step<double>(ue, dt, mp, x[0]);
    } else if (MODEL == M_BO) {
      iion = bo_step<double>(ue, dt, mp, x[0], x[1], x[2]);
    } else if (MODEL == M_TTP06) {
      TtpState<double> S;
#pragma unroll
      for (int v = 0; v < 12; v++) S.g[v] = x[v];
      S.cai = x[12]; S.casr = x[13]; S.cass = x[14]; S.nai = x[15]; S.ki = x[16]; S.rr = x[17];
      iion = ttp06_step<double>(ue, dt, mp, S);
#pragma unroll
      for (int v = 0; v < 12; v++) x[v] = S.g[v];
      x[12] = S.cai; x[13] = S.casr; x[14] = S.cass; x[15] = S.nai; x[16] = S.ki; x[17] = S.rr;
    }
    // stimulus on step k+1 when (k+1) mod period lies in [1, dur] (period 0: one pulse)
    int64_t q = step + 1;
    if (period > 0) q = (q - 1) % period + 1;
    const double iapp = (q <= dur) ? amp : 0.0;
    const double un = (ub + dt * (iapp - iion)) / alpha;
    u2 = u1;
    u1 = u0;
    u0 = un;
  }
  uh[c] = u0;
  uh[nc + c] = u1;
  uh[2 * nc + c] = u2;
#pragma unroll
  for (int v = 0; v < 18; v++)
    if (v < nv) w[(int64_t)v * nc + c] = x[v];
}

// ---------------------------------------------------------------------------
// Allocation-free pacing: the staging of the cells' potential history, state
// and parameter rows lives in one file-scope device array.  Host code never
// uses the array's name as an address: each device's copy is looked up once
// with hipGetSymbolAddress and that pointer is what the kernels receive.
// ---------------------------------------------------------------------------

static __device__ __align__(256) double scratch[PACE_SCRATCH_DOUBLES];

namespace {
std::mutex g_scratch_mu;
double* g_scratch_ptr[PACE_MAX_DEVICES] = {};
}  // namespace

hipError_t pace_scratch(int device, double** ptr) {
  *ptr = nullptr;
  if (device < 0 || device >= PACE_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    // the caller has made `device` current
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = static_cast<double*>(p);
  }
  *ptr = g_scratch_ptr[device];
  return hipSuccess;
}

// Staging of nc cells into the scratch layout the pacing kernel reads:
// parameter rows (defaults, then the first n_params entries of the cell's
// row of params when params is given), the potential history (three copies
// of the starting u) and the state rows [var][cell].  init: [nc][1 + nv] or
// null (the model's initial conditions for every cell).
__global__ __launch_bounds__(256) void k_pace_stage(PaceDefaults def, const double* __restrict__ params,
                                                    int n_params, const double* __restrict__ init, int nv, int nc,
                                                    double* __restrict__ uh, double* __restrict__ w,
                                                    double* __restrict__ mp) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  for (int k = 0; k < NPARAM; k++)
    mp[(int64_t)c * NPARAM + k] = (params && k < n_params) ? params[(int64_t)c * n_params + k] : def.mp[k];
  const double u0 = init ? init[(int64_t)c * (1 + nv)] : def.init[0];
  for (int k = 0; k < 3; k++) uh[(int64_t)k * nc + c] = u0;
  for (int v = 0; v < nv; v++) w[(int64_t)v * nc + c] = init ? init[(int64_t)c * (1 + nv) + 1 + v] : def.init[1 + v];
}

// Paced cells back into rows [nc][1 + nv] (u, then the state).
__global__ __launch_bounds__(256) void k_pace_unstage(const double* __restrict__ uh, const double* __restrict__ w,
                                                      int nv, int nc, double* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  out[(int64_t)c * (1 + nv)] = uh[c];
  for (int v = 0; v < nv; v++) out[(int64_t)c * (1 + nv) + 1 + v] = w[(int64_t)v * nc + c];
}

void launch_pace_stage(const PaceDefaults& def, const double* params, int n_params, const double* init, int nv,
                       int nc, double* uh, double* w, double* mp, hipStream_t st) {
  if (nc <= 0) return;
  hipLaunchKernelGGL(k_pace_stage, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st, def, params, n_params,
                     init, nv, nc, uh, w, mp);
}

void launch_pace_unstage(const double* uh, const double* w, int nv, int nc, double* out, hipStream_t st) {
  if (nc <= 0) return;
  hipLaunchKernelGGL(k_pace_unstage, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st, uh, w, nv, nc, out);
}

void launch_cell_pace(int model, double* uh, double* w, const double* params, int nc, double dt, int bdf,
                      int64_t step0, int64_t n_steps, int64_t period, int64_t dur, double amp, hipStream_t st) {
  if (nc <= 0 || n_steps <= 0) return;
  const dim3 g((unsigned)((nc + 255) / 256)), b(256);
  switch (model) {
    case M_AP: hipLaunchKernelGGL(k_cell_pace<M_AP>, g, b, 0, st, uh, w, params, nc, dt, bdf, step0, n_steps, period, dur, amp); break;
    case M_BO: hipLaunchKernelGGL(k_cell_pace<M_BO>, g, b, 0, st, uh, w, params, nc, dt, bdf, step0, n_steps, period, dur, amp); break;
    case M_TTP06: hipLaunchKernelGGL(k_cell_pace<M_TTP06>, g, b, 0, st, uh, w, params, nc, dt, bdf, step0, n_steps, period, dur, amp); break;
    default: hipLaunchKernelGGL(k_cell_pace<M_PASSIVE>, g, b, 0, st, uh, w, params, nc, dt, bdf, step0, n_steps, period, dur, amp); break;
  }
}

}  // namespace ep
