// C-ABI implementation: simulation objects, one-time setup, the step loop
// and the batched pool.  All per-node arithmetic of a step runs in the HIP
// kernels of kernels.hip; this file only configures, uploads and sequences.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstddef>
#include <cmath>
#include <cstring>
#include <limits>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/ep.h"
#include "assembly.h"
#include "ep_device.h"
#include "kernels.h"

using namespace ep;

namespace {

thread_local std::string g_err;

ep_status fail(ep_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define EP_HIP(call)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) return fail(EP_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// ---- model tables (defaults from the original model publications) ----------

struct ModelInfo {
  int nvars;
  double mv_per_unit, mv_offset, threshold;
};

ModelInfo model_info(int model) {
  switch (model) {
    case EP_AP: return {1, 100.0, -80.0, 0.5};
    case EP_BO: return {3, 85.7, -84.0, 0.5};
    case EP_TTP06: return {18, 1.0, 0.0, -40.0};
    default: return {0, 1.0, 0.0, 0.5};
  }
}

void default_params(int model, int variant, double* mp) {
  for (int k = 0; k < NPARAM; k++) mp[k] = 0.0;
  if (model == EP_AP) {
    const double p[6] = {8.0, 0.15, 0.002, 0.2, 0.3, 12.9};
    std::copy(p, p + 6, mp);
  } else if (model == EP_BO) {
    // minimal model, EPI set
    const double p[28] = {0.0,    1.55,    0.3,     0.13,   0.006, 0.006,  60.0,   1150.0, 1.4506, 60.0,
                          15.0,   65.0,    0.03,    200.0,  0.11,  400.0,  6.0,    30.0181, 0.9957, 2.0458,
                          0.65,   2.7342,  16.0,    2.0994, 0.9087, 1.8875, 0.07,   0.94};
    std::copy(p, p + 28, mp);
  } else if (model == EP_TTP06) {
    const double p[16] = {14.838, 5.405, 0.294,  0.153, 0.392, 3.980e-5, 0.00029, 0.000592,
                          0.1238, 0.0146, 1000.0, 2.724, 0.102, 0.00036,  0.006375, 0.0038};
    std::copy(p, p + 16, mp);
    if (variant == EP_CELL_ENDO) mp[2] = 0.073;
    if (variant == EP_CELL_MID) mp[4] = 0.098;
    mp[16] = (variant == EP_CELL_ENDO) ? 1.0 : 0.0;
  }
}

int n_model_params(int model) {
  switch (model) {
    case EP_AP: return 6;
    case EP_BO: return 28;
    case EP_TTP06: return 16;
    default: return 0;
  }
}

// u, then the state in model order
std::vector<double> default_init(int model) {
  switch (model) {
    case EP_AP: return {0.0, 0.0};
    case EP_BO: return {0.0, 1.0, 1.0, 0.0};
    case EP_TTP06:
      return {-85.23, 0.00172, 0.7444, 0.7045, 0.00621, 0.4712, 0.00095, 0.999998, 2.42e-8, 3.373e-5,
              0.7888, 0.9755,  0.9953, 0.000126, 3.64,  0.00036, 8.604,  136.89,   0.9073};
    default: return {0.0};
  }
}

// ---- device allocation bookkeeping ------------------------------------------

struct DevMem {
  std::vector<void*> ptrs;
  std::vector<size_t> sizes;   // bytes of each allocation, as ptrs
  size_t bytes = 0;
  hipError_t alloc(void** p, size_t nbytes) {
    *p = nullptr;
    if (nbytes == 0) nbytes = 256;
    hipError_t e = hipMalloc(p, nbytes);
    if (e == hipSuccess) {
      ptrs.push_back(*p);
      sizes.push_back(nbytes);
      bytes += nbytes;
    }
    return e;
  }
  // [lo, lo + nbytes) lies inside one allocation of this set
  bool covers(const void* lo, size_t nbytes) const {
    const uintptr_t a = reinterpret_cast<uintptr_t>(lo);
    for (size_t k = 0; k < ptrs.size(); k++) {
      const uintptr_t b = reinterpret_cast<uintptr_t>(ptrs[k]);
      if (a >= b && a - b <= sizes[k] && nbytes <= sizes[k] - (a - b)) return true;
    }
    return false;
  }
  void release() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
    sizes.clear();
    bytes = 0;
  }
};

struct Stim {
  int shape;
  double c[3];
  double size, amp, t0, dur, period;
};

// Per-kernel event timers: kinds 0 ionic, 1 rhs residual, 2 cg spmv,
// 3 cg update, 4 activation, 5 refinement residual, 6 cg finalize,
// 7 pipelined cg iteration.
struct KernelTimers {
  static constexpr int K = EP_N_KERNEL_KINDS;
  int on = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[K];
  std::vector<hipEvent_t> spare;
  double ms[K] = {};
  int64_t count[K] = {};
  hipEvent_t get() {
    if (!spare.empty()) {
      hipEvent_t e = spare.back();
      spare.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  // launch fn bracketed by events when the timers are on
  template <typename F>
  void timed(hipStream_t st, int kind, F&& fn) {
    if (!on) {
      fn();
      return;
    }
    hipEvent_t a = get(), b = get();
    if (!a || !b) {
      fn();
      return;
    }
    (void)hipEventRecord(a, st);
    fn();
    (void)hipEventRecord(b, st);
    pending[kind].emplace_back(a, b);
  }
  // add up completed event pairs (after a stream synchronization)
  void harvest() {
    for (int k = 0; k < K; k++) {
      for (auto& pr : pending[k]) {
        float t = 0.0f;
        if (hipEventElapsedTime(&t, pr.first, pr.second) == hipSuccess) {
          ms[k] += t;
          count[k] += 1;
        }
        spare.push_back(pr.first);
        spare.push_back(pr.second);
      }
      pending[k].clear();
    }
  }
  void zero() {
    for (int k = 0; k < K; k++) {
      ms[k] = 0.0;
      count[k] = 0;
    }
  }
  double avg_us(int k) const { return count[k] ? 1e3 * ms[k] / (double)count[k] : 0.0; }
  void destroy() {
    harvest();
    for (auto e : spare) (void)hipEventDestroy(e);
    spare.clear();
  }
};

// The launch sequences of one step captured as HIP graphs and replayed: the
// step prologue (ionic, rhs residual, SpMV, finalize), one and two CG rounds
// (update, SpMV, finalize), a refinement sweep (residual, SpMV, finalize) and
// the epilogue (activation, end of step).  Every kernel reads its per-step
// control from device memory, so the graphs stay valid across steps; they
// are dropped when the launch configuration changes.
struct StepGraphs {
  hipGraphExec_t pro = nullptr, round1 = nullptr, round2 = nullptr, ir = nullptr, epi = nullptr;
  bool valid = false;
  void reset() {
    for (hipGraphExec_t* g : {&pro, &round1, &round2, &ir, &epi}) {
      if (*g) (void)hipGraphExecDestroy(*g);
      *g = nullptr;
    }
    valid = false;
  }
};

// Host-side launch policy of the mixed-precision solve.  Each step runs
// inner FP32 sweeps, each ended by an FP64 refinement residual; the host
// launches a predicted number of inner rounds, then the refinement kernels,
// then reads the control state.  Rounds launched after the inner solve has
// converged, and a refinement launched before it has, return at once but
// still cost a launch each, and a short prediction costs an extra read.  The
// prediction is kept per sweep index (the first sweep of a step is the
// longest) from the last step's counts, plus one round of slack.
struct SweepPredictor {
  int pred[3] = {8, 4, 3};
  int rounds(int sweep) const { return std::max(1, pred[std::min(sweep, 2)]); }
  void learn(int sweep, int its) { pred[std::min(sweep, 2)] = std::max(1, its + 1); }
};

template <typename F>
hipError_t capture_graph(hipStream_t st, F&& fn, hipGraphExec_t* out) {
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  fn();
  e = hipStreamEndCapture(st, &g);
  if (e != hipSuccess) return e;
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  return e;
}

}  // namespace

struct ep_sim {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // configuration
  int elem = 0;
  int64_t n = 0, n_elems = 0;
  std::vector<double> xyz, f0, s0, n0;
  std::vector<int32_t> conn;
  double sl = 0.17, st = 0.019, sn = 0.019, chi = 140.0, cm = 0.01;
  int model = -1, variant = 0;
  std::vector<double> params, init;
  std::vector<Stim> stims;
  double dt = 0.05, rtol = 1e-10, inner_rtol = 1e-4;
  int bdf = 1, prec = EP_FP64, precond = EP_JACOBI, block = 1, max_it = 1000, max_outer = 30;
  int ionic_scheme = 0;   // EP_IONIC_RUSH_LARSEN or EP_IONIC_BDF
  int ionic_fp64 = 0;     // mixed precision: ionic step in FP64 (EP_OPT_IONIC_FP64)
  int cg_variant = EP_CG_AUTO;   // FP64 CG formulation (EP_OPT_CG_VARIANT)
  int x0_extrap = 0;             // EP_OPT_INITIAL_GUESS
  int fmt_pref = EP_FMT_AUTO;
  // subdomains: element labels (empty: one subdomain) and per-label settings
  std::vector<int32_t> material;
  struct RegionCfg {
    int variant = -1;                 // -1: the sim's
    bool has_params = false;
    std::vector<double> params;
    double sig[3] = {-1.0, -1.0, -1.0};  // negative: the sim's
    int conductive = 1;
    int model = -1;                   // -1: the sim's ionic model
  } region_cfg[EP_MAX_REGIONS];
  int timers = 0;
  // products
  bool finalized = false;
  bool in_pool = false;
  DevMem mem;
  InstDesc desc{};
  InstDesc* d_desc = nullptr;
  BlockMap* d_bmap = nullptr;
  int nblocks = 0;
  InstState* d_st = nullptr;
  InstState* h_st = nullptr;  // pinned
  int64_t guard = 0;
  int64_t nnz = 0;
  int nvars = 0;
  ModelInfo mi{};
  double ms_setup = 0.0;
  double ms_phase[4] = {0, 0, 0, 0};
  hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  KernelTimers kt;
  // launch shapes (see Launch) and graph replay of the step
  int xmap = 0, ionic_npt = 1, use_graph = 0;
  StepGraphs graphs;
  int32_t* d_ids = nullptr;  // device list {0}: the instance advanced by k_end_step
  InstDesc* d_desc_own = nullptr;  // the sim's own descriptor (d_desc points into a pool table while pooled)
  hipStream_t stream_own = nullptr;
  int pool_slot = -1;
  ep_pool* pool = nullptr;   // the pool that steps this sim while in_pool
  int it_pred = 8;      // CG iterations launched before the first convergence check
  // several subdomains (finalized): ionic points and the per-node primary
  // subdomain (-1: node outside every conducting subdomain)
  bool het = false;
  int64_t n_pts = 0;
  int64_t n_crow = 0;
  std::vector<int32_t> node_reg;
  std::vector<int32_t> sec_node;
  std::vector<int32_t> pt_model;   // ionic model of every ionic point (several subdomains)
  int het_model = -1;              // the one model of all subdomains, or -1 when they differ
  int st_rows64 = 0, st_rows32 = 0;  // rows of the FP64 / FP32 state arrays
  int64_t sell_nnz = 0;   // stored entries of the SELL operator (slices padded to their widest row)
  int64_t n_cent = 0;     // entries of the interface correction
  SweepPredictor sweeps;  // inner rounds per refinement sweep (mixed)
  int sweeps_last = 1;    // refinement sweeps the last step needed (mixed)
  int sticky = EP_OK;
  double* tk_save = nullptr;   // saved solver state for timing the pipelined CG kernel
  // the ionic step runs in FP32 (state arrays and arithmetic)
  bool ionic_f32() const { return prec == EP_MIXED && !ionic_fp64; }
};

namespace {

int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

ep_status check_sim(ep_sim* s) {
  if (!s) return fail(EP_EINVAL, "null sim");
  return EP_OK;
}

// Read the device state into pinned host memory (synchronizes the stream).
// The CG formulation a sim runs: EP_CG_AUTO takes the pipelined one for
// linear elements (small condition numbers; its recurrences reach every
// tolerance tested there) whose iteration's data (operator and vectors, about
// 232 B per node in FP64, 124 B in the FP32 inner solve) fits in three
// quarters of the 256 MB last-level cache, and Chronopoulos-Gear otherwise:
// once the data streams from HBM, the fused iteration is no faster in FP64
// (C1 at h = 0.05 mm, 3.45M nodes: 6.64 against 6.68 ms per step) and much
// slower in FP32 (5.62 against 3.81 ms: the separate SpMV keeps its FP32
// operator in the cache).
int cg_resolved(const ep_sim* s) {
  if (s->cg_variant != EP_CG_AUTO) return s->cg_variant;
  if (s->elem != EP_HEX8 && s->elem != EP_TET4) return EP_CG_CHRONOPOULOS_GEAR;
  const double bytes = (double)s->n * (s->prec == EP_MIXED ? 124.0 : 232.0);
  return bytes <= 0.75 * 256e6 ? EP_CG_PIPELINED : EP_CG_CHRONOPOULOS_GEAR;
}

ep_status pull_state(ep_sim* s) {
  EP_HIP(hipMemcpyAsync(s->h_st, s->d_st, sizeof(InstState), hipMemcpyDeviceToHost, s->stream));
  EP_HIP(hipStreamSynchronize(s->stream));
  if (s->kt.on) s->kt.harvest();
  return EP_OK;
}

double stim_profile(const Stim& t, const double* x) {
  const double dx = x[0] - t.c[0], dy = x[1] - t.c[1], dz = x[2] - t.c[2];
  if (t.shape == EP_CUBE) {
    const double m = std::max(std::fabs(dx), std::max(std::fabs(dy), std::fabs(dz)));
    return m <= 0.5 * t.size + 1e-9 ? 1.0 : 0.0;
  }
  if (t.shape == EP_SPHERE) return std::sqrt(dx * dx + dy * dy + dz * dz) <= t.size + 1e-9 ? 1.0 : 0.0;
  return std::exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * t.size * t.size));
}

// ionic model of subdomain r
int region_model(const ep_sim* s, int r) { return s->region_cfg[r].model >= 0 ? s->region_cfg[r].model : s->model; }

// rows a model's state takes in the FP64 and FP32 state arrays (mixed
// precision keeps TTP06's Na_i and K_i in FP64, everything else in FP32)
void state_rows(int model, bool mixed, int* rows64, int* rows32) {
  const int nv = model_info(model).nvars;
  if (!mixed) {
    *rows64 = nv;
    *rows32 = 0;
  } else if (model == EP_TTP06) {
    *rows64 = 2;
    *rows32 = 16;
  } else {
    *rows64 = 0;
    *rows32 = nv;
  }
}

// one point's state (model order) into its column of the state arrays
void pack_state(int model, bool mixed, const double* w, double* s64, float* s32, int64_t stride) {
  const int nv = model_info(model).nvars;
  if (!mixed) {
    for (int v = 0; v < nv; v++) s64[(size_t)v * stride] = w[v];
  } else if (model == EP_TTP06) {
    for (int v = 0; v < 18; v++) {
      if (v < 15) s32[(size_t)v * stride] = (float)w[v];
      else if (v == 15) s64[0] = w[v];
      else if (v == 16) s64[(size_t)stride] = w[v];
      else s32[(size_t)15 * stride] = (float)w[v];
    }
  } else {
    for (int v = 0; v < nv; v++) s32[(size_t)v * stride] = (float)w[v];
  }
}

void unpack_state(int model, bool mixed, const double* s64, const float* s32, int64_t stride, double* w) {
  const int nv = model_info(model).nvars;
  if (!mixed) {
    for (int v = 0; v < nv; v++) w[v] = s64[(size_t)v * stride];
  } else if (model == EP_TTP06) {
    for (int v = 0; v < 18; v++) {
      if (v < 15) w[v] = s32[(size_t)v * stride];
      else if (v == 15) w[v] = s64[0];
      else if (v == 16) w[v] = s64[(size_t)stride];
      else w[v] = s32[(size_t)15 * stride];
    }
  } else {
    for (int v = 0; v < nv; v++) w[v] = s32[(size_t)v * stride];
  }
}

size_t estimate_bytes(const ep_sim* s) {
  const int64_t n = s->n;
  // a hexahedral lattice of degree p couples a node to (p + 2)^3 nodes on average
  const int hex_p = s->elem == EP_HEX8 ? 1 : s->elem == EP_HEX27 ? 2 : s->elem == EP_HEX64 ? 3
                  : s->elem == EP_HEX125 ? 4 : s->elem == EP_HEX216 ? 5 : s->elem == EP_HEX343 ? 6 : 0;
  const double nnz_row = hex_p ? std::pow(hex_p + 2.0, 3.0) : (s->elem == EP_TET10) ? 40.0 : 16.0;
  const bool mixed = s->prec == EP_MIXED;
  const ModelInfo mi = model_info(s->model);
  double per_node = 11 * 8.0 + 24.0;                            // FP64 vectors, activation
  per_node += (double)s->bdf * s->block * (mixed ? 12.0 : 8.0);  // preconditioner(s)
  per_node += mixed ? 5 * 4.0 : 0.0;
  per_node += (s->ionic_f32() ? (mi.nvars * 4.0 + 8.0) : mi.nvars * 8.0) * (s->ionic_scheme == EP_IONIC_BDF ? RING : 1);
  per_node += nnz_row * ((s->bdf + 1) * 8.0 + 4.0 + (mixed ? s->bdf * 4.0 : 0.0));
  per_node += 8.0 * std::min<size_t>(s->stims.size(), MAX_STIM);
  return (size_t)(per_node * n * 1.05) + (1u << 20);
}

template <typename T>
hipError_t upload(DevMem& m, T** d, const T* h, size_t count, hipStream_t st) {
  hipError_t e = m.alloc((void**)d, count * sizeof(T));
  if (e != hipSuccess) return e;
  return hipMemcpyAsync(*d, h, count * sizeof(T), hipMemcpyHostToDevice, st);
}

// Block-Jacobi preconditioner: for every run of bs consecutive rows (the
// last run may be shorter) the exact inverse of the diagonal block of the
// symmetrized operator (A + A^T)/2, by Cholesky factorization, stored
// column-wise: out[j * ld + i] = (B^-1)(i - i0, j).  False if a block is not
// positive definite.
bool block_inverses(const Csr& A, const std::vector<double>& val, int bs, int64_t ld, std::vector<double>& out) {
  const int64_t n = (int64_t)A.rowptr.size() - 1;
  const int64_t nb = (n + bs - 1) / bs;
  out.assign((size_t)bs * ld, 0.0);
  std::atomic<bool> ok{true};
  parallel_for(nb, [&](int64_t k) {
    thread_local std::vector<double> B, L, X;
    const int64_t i0 = k * bs;
    const int m = (int)std::min<int64_t>(bs, n - i0);
    B.assign((size_t)m * m, 0.0);
    L.assign((size_t)m * m, 0.0);
    X.assign((size_t)m * m, 0.0);
    for (int a = 0; a < m; a++) {
      const int64_t r = i0 + a;
      for (int64_t t = A.rowptr[r]; t < A.rowptr[r + 1]; t++) {
        const int64_t c = A.col[t] - i0;
        if (c < 0 || c >= m) continue;
        B[(size_t)a * m + c] += 0.5 * val[t];
        B[(size_t)c * m + a] += 0.5 * val[t];
      }
    }
    // B = L L^T
    for (int j = 0; j < m; j++) {
      double d = B[(size_t)j * m + j];
      for (int t = 0; t < j; t++) d -= L[(size_t)j * m + t] * L[(size_t)j * m + t];
      if (!(d > 0.0)) {
        ok = false;
        return;
      }
      const double ljj = std::sqrt(d);
      L[(size_t)j * m + j] = ljj;
      for (int a = j + 1; a < m; a++) {
        double v = B[(size_t)a * m + j];
        for (int t = 0; t < j; t++) v -= L[(size_t)a * m + t] * L[(size_t)j * m + t];
        L[(size_t)a * m + j] = v / ljj;
      }
    }
    // columns of B^-1: L y = e_c, then L^T x = y
    std::vector<double> y(m);
    for (int c = 0; c < m; c++) {
      for (int a = 0; a < m; a++) {
        double v = (a == c) ? 1.0 : 0.0;
        for (int t = 0; t < a; t++) v -= L[(size_t)a * m + t] * y[t];
        y[a] = v / L[(size_t)a * m + a];
      }
      for (int a = m - 1; a >= 0; a--) {
        double v = y[a];
        for (int t = a + 1; t < m; t++) v -= L[(size_t)t * m + a] * X[(size_t)t * m + c];
        X[(size_t)a * m + c] = v / L[(size_t)a * m + a];
      }
    }
    for (int a = 0; a < m; a++)
      for (int c = 0; c < m; c++)
        out[(size_t)c * ld + i0 + a] = 0.5 * (X[(size_t)a * m + c] + X[(size_t)c * m + a]);
  });
  return ok;
}

// Tile map 2 of a single instance on a hexahedral lattice (the 14-diagonal
// DIA of Q1 elements, offsets 0, 1, nx - 1 .. nx + 1 and P + {-nx, 0, nx} +
// {-1, 0, 1} with P = nx ny the plane): the tiles, ordered by the lattice
// line y of their middle row (then by index), are cut into N_XCD runs of
// ceil(tiles / N_XCD); workgroup b takes the (b / N_XCD)-th tile of run
// b mod N_XCD, in ascending tile order (workgroups go round-robin over the
// dies, so each die receives one run: one band of lines through every plane).
// Empty if the operator is not such a lattice.
std::vector<int32_t> lattice_tile_table(const InstDesc& D, int64_t n, int ntiles, int nblocks) {
  std::vector<int32_t> tab;
  if (D.fmt != FMT_DIA || D.nup != 14) return tab;
  const int64_t nx = D.off[3], P = D.off[9];
  if (nx < 3 || P < 3 * nx || P % nx != 0 || n <= 0) return tab;
  int k = 0;
  for (int64_t dz = 0; dz <= 1; dz++)
    for (int64_t dy = -1; dy <= 1; dy++)
      for (int64_t dx = -1; dx <= 1; dx++) {
        const int64_t o = dz * P + dy * nx + dx;
        if (o < 0) continue;
        if (k >= 14 || D.off[k] != o) return tab;
        k++;
      }
  std::vector<std::pair<int64_t, int32_t>> key((size_t)ntiles);
  for (int32_t t = 0; t < ntiles; t++) {
    const int64_t rm = std::min<int64_t>((int64_t)t * TILE + TILE / 2, n - 1);
    key[(size_t)t] = {(rm % P) / nx, t};
  }
  std::sort(key.begin(), key.end());
  const int per = (ntiles + N_XCD - 1) / N_XCD;
  if (nblocks != N_XCD * per) return tab;
  tab.assign((size_t)nblocks, -1);
  for (int x = 0; x < N_XCD; x++) {
    std::vector<int32_t> run;
    for (int j = x * per; j < std::min(ntiles, (x + 1) * per); j++) run.push_back(key[(size_t)j].second);
    std::sort(run.begin(), run.end());
    for (size_t j = 0; j < run.size(); j++) tab[j * N_XCD + (size_t)x] = run[j];
  }
  return tab;
}

ep_status finalize_impl(ep_sim* s) {
  auto t0 = std::chrono::steady_clock::now();
  if (s->finalized) return fail(EP_ESTATE, "sim already finalized");
  if (s->n <= 0) return fail(EP_ESTATE, "no mesh uploaded");
  if (s->model < 0) return fail(EP_ESTATE, "no ionic model set");
  EP_HIP(hipSetDevice(s->device));
  // ---- subdomain settings ----
  const bool het = !s->material.empty();
  std::vector<double> rsig(3 * EP_MAX_REGIONS);
  std::vector<unsigned char> ron(EP_MAX_REGIONS);
  for (int r = 0; r < EP_MAX_REGIONS; r++) {
    const ep_sim::RegionCfg& c = s->region_cfg[r];
    const double glob[3] = {s->sl, s->st, s->sn};
    for (int k = 0; k < 3; k++) rsig[3 * r + k] = c.sig[k] >= 0.0 ? c.sig[k] : glob[k];
    ron[r] = (unsigned char)c.conductive;
    if (c.has_params && (int)c.params.size() > n_model_params(region_model(s, r)))
      return fail(EP_EINVAL, "region parameters: more than the model has");
    if (!het && c.model >= 0 && c.model != s->model)
      return fail(EP_EINVAL, "a subdomain ionic model needs material ids");
  }
  // the matrix-free operator (hexahedra of degree 2 or 3, FP64, one
  // subdomain, Jacobi): the device applies it element by element; the host
  // still assembles once, for the Jacobi diagonal
  const bool mf = s->fmt_pref == EP_FMT_MF;
  if (mf) {
    if (s->elem != EP_HEX27 && s->elem != EP_HEX64)
      return fail(EP_EINVAL, "the matrix-free operator takes hexahedra of degree 2 or 3");
    if (s->prec != EP_FP64) return fail(EP_EINVAL, "the matrix-free operator runs in FP64");
    if (het) return fail(EP_EINVAL, "the matrix-free operator takes one subdomain");
    if (s->block != 1) return fail(EP_EINVAL, "the matrix-free operator uses the Jacobi preconditioner");
    if (s->in_pool) return fail(EP_EINVAL, "matrix-free sims are not admitted to pools");
  }
  // ---- assembly ----
  Csr A;
  std::vector<char> err;
  const double* fib0 = s->f0.empty() ? nullptr : s->f0.data();
  const double* fib1 = s->s0.empty() ? nullptr : s->s0.data();
  const double* fib2 = s->n0.empty() ? nullptr : s->n0.data();
  if (!assemble_csr(s->elem, s->n, s->xyz.data(), s->n_elems, s->conn.data(), fib0, fib1, fib2, s->sl, s->st,
                    s->sn, s->chi, s->cm, A, err, het ? s->material.data() : nullptr, rsig.data(), ron.data()))
    return fail(EP_EINVAL, std::string("assembly: ") + (err.empty() ? "failed" : err.data()));
  const int64_t n = s->n;
  // subdomains of each node: the lowest conducting one is the node's primary
  // subdomain (its state lives at point i = node), every further one adds an
  // ionic point; nodes of no conducting subdomain carry no unknown
  std::vector<int32_t> sec_reg;
  s->het = het;
  s->node_reg.assign(het ? n : 0, 0);
  s->sec_node.clear();
  if (het) {
    const int npe = s->elem;
    std::vector<uint8_t> mask(n, 0);
    for (int64_t e = 0; e < s->n_elems; e++) {
      const int r = s->material[e];
      if (!ron[r]) continue;
      for (int k = 0; k < npe; k++) mask[s->conn[e * npe + k]] |= (uint8_t)(1u << r);
    }
    for (int64_t i = 0; i < n; i++) {
      if (!mask[i]) {
        s->node_reg[i] = -1;
        continue;
      }
      const int prim = __builtin_ctz(mask[i]);
      s->node_reg[i] = prim;
      for (int r = prim + 1; r < EP_MAX_REGIONS; r++)
        if (mask[i] & (1u << r)) {
          s->sec_node.push_back((int32_t)i);
          sec_reg.push_back(r);
        }
    }
    if (s->node_reg.end() == std::find_if(s->node_reg.begin(), s->node_reg.end(), [](int32_t r) { return r >= 0; }))
      return fail(EP_EINVAL, "no conducting subdomain");
  }
  s->n_pts = n + (int64_t)s->sec_node.size();
  // ionic model of every point; the state arrays take the most rows any
  // model present needs
  s->pt_model.assign(het ? s->n_pts : 0, s->model);
  s->het_model = s->model;
  {
    int r64 = 0, r32 = 0;
    state_rows(s->model, s->ionic_f32(), &r64, &r32);
    if (het) {
      for (int64_t p = 0; p < s->n_pts; p++) {
        const int r = p < n ? s->node_reg[p] : sec_reg[p - n];
        const int m = r < 0 ? s->model : region_model(s, r);
        s->pt_model[p] = m;
        if (m != s->model) s->het_model = -1;
        int a = 0, b = 0;
        state_rows(m, s->ionic_f32(), &a, &b);
        r64 = std::max(r64, a);
        r32 = std::max(r32, b);
      }
    }
    s->st_rows64 = r64;
    s->st_rows32 = r32;
  }
  const int64_t nnz = A.nnz();
  s->nnz = nnz;
  const bool mixed = s->prec == EP_MIXED;
  const double alphas[3] = {1.0, 1.5, 11.0 / 6.0};
  const int nsig = s->bdf;
  // diagonal positions
  std::vector<int64_t> dpos(n);
  for (int64_t i = 0; i < n; i++) {
    const int32_t* c = &A.col[A.rowptr[i]];
    const int64_t len = A.rowptr[i + 1] - A.rowptr[i];
    dpos[i] = A.rowptr[i] + (std::lower_bound(c, c + len, (int32_t)i) - c);
  }
  // ---- format choice ----
  std::vector<int64_t> offs = distinct_offsets(A);
  const int64_t n_slices = (n + SLICE - 1) / SLICE;
  std::vector<int64_t> slice_ptr(n_slices + 1, 0);
  for (int64_t sl = 0; sl < n_slices; sl++) {
    int64_t w = 0;
    for (int64_t i = sl * SLICE; i < std::min(n, (sl + 1) * SLICE); i++)
      w = std::max(w, A.rowptr[i + 1] - A.rowptr[i]);
    slice_ptr[sl + 1] = slice_ptr[sl] + w * SLICE;
  }
  const int64_t sell_nnz = slice_ptr[n_slices];
  s->sell_nnz = sell_nnz;
  const int64_t stride = round_up(n, 64);
  const double vb = mixed ? 4.0 : 8.0;
  // symmetric DIA keeps the offsets >= 0; the pattern of an FE operator is
  // symmetric, so every stored offset o > 0 also stands for -o
  std::vector<int64_t> up;
  bool sym_pattern = true;
  for (int64_t o : offs)
    if (o >= 0) up.push_back(o);
  for (int64_t o : up)
    if (o > 0 && !std::binary_search(offs.begin(), offs.end(), -o)) sym_pattern = false;
  bool use_dia = false;
  if (mf) {
    // no assembled operator on the device
  } else if (sym_pattern && (int)offs.size() <= MAX_DIAG && (int)up.size() <= MAX_UP) {
    const double dia_bytes = (double)up.size() * stride * vb;
    const double sell_bytes = (double)sell_nnz * (vb + 4.0);
    use_dia = (s->fmt_pref == EP_FMT_DIA) || (s->fmt_pref == EP_FMT_AUTO && dia_bytes < sell_bytes);
  } else if (s->fmt_pref == EP_FMT_DIA) {
    return fail(EP_EINVAL, "pattern has more than 32 distinct offsets; DIA not possible");
  }
  InstDesc& D = s->desc;
  std::memset(&D, 0, sizeof(D));
  D.n = n;
  D.model = s->model;
  D.bdf = s->bdf;
  D.prec = s->prec;
  D.max_it = s->max_it;
  D.max_outer = s->max_outer;
  D.dt = s->dt;
  D.inv_dt = 1.0 / s->dt;
  D.rtol = s->rtol;
  D.inner_rtol = s->inner_rtol;
  s->mi = model_info(s->model);
  D.threshold = s->mi.threshold;
  s->nvars = s->mi.nvars;
  D.nvars = s->nvars;
  D.precond = s->precond;
  D.block = s->block;
  D.bld = round_up(n, 64);
  D.ionic_scheme = s->ionic_scheme;
  default_params(s->model, s->variant, D.mp);
  for (size_t k = 0; k < s->params.size(); k++) D.mp[k] = s->params[k];
  hipStream_t st = s->stream;
  DevMem& m = s->mem;
  // ---- matrix values for each BDF order, and Jacobi diagonals ----
  std::vector<std::vector<double>> valA(nsig, std::vector<double>(nnz));
  for (int q = 0; q < nsig; q++) {
    const double c = alphas[q] / s->dt;
    for (int64_t t = 0; t < nnz; t++) valA[q][t] = c * A.valM[t] + A.valK[t];
    // a node outside every conducting subdomain: identity row (its row and
    // column of M and K are zero), so it drops out of the solve
    if (het)
      for (int64_t i = 0; i < n; i++)
        if (s->node_reg[i] < 0) valA[q][dpos[i]] = 1.0;
  }
  auto to_dev_d = [&](const std::vector<double>& h, const double** d) -> hipError_t {
    double* p;
    hipError_t e = upload(m, &p, h.data(), h.size(), st);
    *d = p;
    return e;
  };
  auto to_dev_f = [&](const std::vector<double>& h, const float** d) -> hipError_t {
    std::vector<float> f(h.begin(), h.end());
    float* p;
    hipError_t e = upload(m, &p, f.data(), f.size(), st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);  // f is a temporary
    *d = p;
    return e;
  };
  std::vector<std::vector<double>> hostvals;  // keep alive until sync
  if (mf) {
    MfData mfd;
    std::vector<char> err_mf;
    if (!mf_setup(s->elem, n, s->xyz.data(), s->n_elems, s->conn.data(), fib0, fib1, fib2, s->sl, s->st, s->sn,
                  s->chi, s->cm, mfd, err_mf))
      return fail(EP_EINVAL, std::string("matrix-free setup: ") + (err_mf.empty() ? "failed" : err_mf.data()));
    D.fmt = FMT_MF;
    D.nup = 0;
    s->guard = 0;
    D.mf_p = mfd.p;
    D.n_elems = s->n_elems;
    D.mf_cmp = mfd.cmp ? 1 : 0;
    for (int k = 0; k < 4; k++) D.mfW[k] = mfd.W[k];
    const int n1 = mfd.p + 1;
    for (int k = 0; k < n1 * n1; k++) {
      D.mfV[k] = mfd.V[k];
      D.mfD[k] = mfd.Dv[k];
    }
    const double* geo;
    EP_HIP(to_dev_d(mfd.geo, &geo));
    D.geo = geo;
    int32_t* dconn;
    EP_HIP(upload(m, &dconn, s->conn.data(), s->conn.size(), st));
    D.econn = dconn;
    int64_t* dptr;
    EP_HIP(upload(m, &dptr, mfd.adj_ptr.data(), mfd.adj_ptr.size(), st));
    D.adj_ptr = dptr;
    int32_t* dadj;
    EP_HIP(upload(m, &dadj, mfd.adj.data(), mfd.adj.size(), st));
    D.adj = dadj;
    EP_HIP(m.alloc((void**)&D.yA, (size_t)s->n_elems * s->elem * sizeof(double)));
    EP_HIP(m.alloc((void**)&D.yM, (size_t)s->n_elems * s->elem * sizeof(double)));
    EP_HIP(hipStreamSynchronize(st));   // mfd is a temporary
  } else if (use_dia) {
    D.fmt = FMT_DIA;
    D.nup = (int)up.size();
    const int64_t g = up.back();
    for (size_t d = 0; d < up.size(); d++) D.off[d] = (int32_t)up[d];
    s->guard = round_up(std::max<int64_t>(g, 1), 64);
    const int64_t G = s->guard;
    const int64_t ld = stride + G;
    D.ld = ld;
    // value of (i, i + o) stored at row i; symmetrized (A + A^T)/2 so that
    // the last-bit asymmetry of the element integrals does not matter
    auto to_dia = [&](const std::vector<double>& v) {
      std::vector<double> out((size_t)D.nup * ld + G, 0.0);
      double* p = out.data() + G;
      parallel_for(n, [&](int64_t i) {
        const int32_t* c = &A.col[A.rowptr[i]];
        const int64_t len = A.rowptr[i + 1] - A.rowptr[i];
        for (int d = 0; d < D.nup; d++) {
          const int64_t j = i + up[d];
          if (j >= n) continue;
          const int32_t* f = std::lower_bound(c, c + len, (int32_t)j);
          if (f == c + len || *f != j) continue;
          const double aij = v[A.rowptr[i] + (f - c)];
          const int32_t* cj = &A.col[A.rowptr[j]];
          const int64_t lj = A.rowptr[j + 1] - A.rowptr[j];
          const int32_t* fj = std::lower_bound(cj, cj + lj, (int32_t)i);
          const double aji = (fj != cj + lj && *fj == i) ? v[A.rowptr[j] + (fj - cj)] : aij;
          p[(size_t)d * ld + i] = 0.5 * (aij + aji);
        }
      });
      return out;
    };
    auto dev_dia = [&](const std::vector<double>& h, const double** d) -> hipError_t {
      double* base;
      hipError_t e = upload(m, &base, h.data(), h.size(), st);
      *d = base + G;
      return e;
    };
    auto dev_dia_f = [&](const std::vector<double>& h, const float** d) -> hipError_t {
      std::vector<float> f(h.begin(), h.end());
      float* base;
      hipError_t e = upload(m, &base, f.data(), f.size(), st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      *d = base + G;
      return e;
    };
    hostvals.push_back(to_dia(A.valM));
    EP_HIP(dev_dia(hostvals.back(), &D.valM));
    for (int q = 0; q < nsig; q++) {
      hostvals.push_back(to_dia(valA[q]));
      EP_HIP(dev_dia(hostvals.back(), &D.valA[q]));
      if (mixed) EP_HIP(dev_dia_f(hostvals.back(), &D.valA32[q]));
    }
  } else {
    D.fmt = FMT_SELL;
    D.nup = 0;
    s->guard = 0;
    std::vector<int32_t> col(sell_nnz, 0);
    std::vector<int64_t> pos(nnz);
    for (int64_t sl = 0; sl < n_slices; sl++) {
      const int64_t w = (slice_ptr[sl + 1] - slice_ptr[sl]) / SLICE;
      for (int lane = 0; lane < SLICE; lane++) {
        const int64_t i = sl * SLICE + lane;
        for (int64_t k = 0; k < w; k++) {
          const int64_t p = slice_ptr[sl] + k * SLICE + lane;
          if (i < n && A.rowptr[i] + k < A.rowptr[i + 1]) {
            col[p] = A.col[A.rowptr[i] + k];
            pos[A.rowptr[i] + k] = p;
          } else {
            col[p] = (int32_t)std::min<int64_t>(i, n - 1);
          }
        }
      }
    }
    auto to_sell = [&](const std::vector<double>& v) {
      std::vector<double> out(sell_nnz, 0.0);
      for (int64_t t = 0; t < nnz; t++) out[pos[t]] = v[t];
      return out;
    };
    int32_t* dcol;
    EP_HIP(upload(m, &dcol, col.data(), col.size(), st));
    D.col = dcol;
    int64_t* dsp;
    EP_HIP(upload(m, &dsp, slice_ptr.data(), slice_ptr.size(), st));
    D.slice_ptr = dsp;
    hostvals.push_back(to_sell(A.valM));
    EP_HIP(to_dev_d(hostvals.back(), &D.valM));
    for (int q = 0; q < nsig; q++) {
      hostvals.push_back(to_sell(valA[q]));
      EP_HIP(to_dev_d(hostvals.back(), &D.valA[q]));
      if (mixed) EP_HIP(to_dev_f(hostvals.back(), &D.valA32[q]));
    }
    EP_HIP(hipStreamSynchronize(st));  // col lives on the host stack frame
  }
  for (int q = 0; q < nsig; q++) {
    if (s->block == 1) {
      // padded to whole 64-row groups: the solver kernels read rows in pairs
      std::vector<double> dinv(round_up(n, 64), 0.0);
      for (int64_t i = 0; i < n; i++) dinv[i] = 1.0 / valA[q][dpos[i]];
      hostvals.push_back(dinv);
    } else {
      std::vector<double> binv;
      if (!block_inverses(A, valA[q], s->block, D.bld, binv))
        return fail(EP_EINVAL, "a diagonal block of the system matrix is not positive definite");
      hostvals.push_back(std::move(binv));
    }
    EP_HIP(to_dev_d(hostvals.back(), &D.dinv[q]));
    if (mixed) EP_HIP(to_dev_f(hostvals.back(), &D.dinv32[q]));
  }
  // ---- vectors (guarded) ----
  const int64_t G = s->guard;
  // rows padded to whole 64-row groups (the solver kernels read rows in
  // pairs; the SELL format has no guard cells)
  const int64_t nv = round_up(n, 64) + 2 * G;
  auto vec_d = [&](double** p) -> hipError_t {
    double* raw;
    hipError_t e = m.alloc((void**)&raw, nv * sizeof(double));
    if (e != hipSuccess) return e;
    e = hipMemsetAsync(raw, 0, nv * sizeof(double), st);
    *p = raw + G;
    return e;
  };
  auto vec_f = [&](float** p) -> hipError_t {
    float* raw;
    hipError_t e = m.alloc((void**)&raw, nv * sizeof(float));
    if (e != hipSuccess) return e;
    e = hipMemsetAsync(raw, 0, nv * sizeof(float), st);
    *p = raw + G;
    return e;
  };
  for (int k = 0; k < RING; k++) EP_HIP(vec_d(&D.U[k]));
  EP_HIP(vec_d(&D.g));
  EP_HIP(vec_d(&D.b));
  EP_HIP(vec_d(&D.r));
  EP_HIP(vec_d(&D.z));
  EP_HIP(vec_d(&D.p));
  EP_HIP(vec_d(&D.s));
  EP_HIP(vec_d(&D.w));
  if (mixed) {
    EP_HIP(vec_f(&D.r32));
    EP_HIP(vec_f(&D.z32));
    EP_HIP(vec_f(&D.p32));
    EP_HIP(vec_f(&D.s32));
    EP_HIP(vec_f(&D.w32));
  }
  // ---- ionic state ----
  const int nvars = s->nvars;
  // one state array per time level under the BDF ionic scheme, one shared
  // by all four level slots under Rush-Larsen
  const int n_levels = s->ionic_scheme == EP_IONIC_BDF ? RING : 1;
  const int n32 = s->st_rows32;
  const int n64 = s->st_rows64;
  // stride n_pts: the nodes' states, then the extra interface points'
  const int64_t npts = s->n_pts;
  for (int k = 0; k < RING; k++) {
    if (k < n_levels) {
      EP_HIP(m.alloc((void**)&D.st32[k], std::max<int64_t>(1, (int64_t)n32 * npts) * sizeof(float)));
      EP_HIP(m.alloc((void**)&D.st64[k], std::max<int64_t>(1, (int64_t)n64 * npts) * sizeof(double)));
    } else {
      D.st32[k] = D.st32[0];
      D.st64[k] = D.st64[0];
    }
  }
  // ---- several subdomains: points, parameter rows, interface correction ----
  D.het = het ? 1 : 0;
  D.n_pts = npts;
  if (het) {
    const int64_t nsec = npts - n;
    std::vector<int32_t> pt_reg(s->node_reg);
    pt_reg.insert(pt_reg.end(), sec_reg.begin(), sec_reg.end());
    int32_t* d_reg;
    EP_HIP(upload(m, &d_reg, pt_reg.data(), pt_reg.size(), st));
    D.pt_reg = d_reg;
    std::vector<int32_t> secn(s->sec_node);
    if (secn.empty()) secn.push_back(0);
    int32_t* d_sec;
    EP_HIP(upload(m, &d_sec, secn.data(), secn.size(), st));
    D.sec_node = d_sec;
    // parameter row of each subdomain: its cell type's defaults, the sim's
    // overrides, then the subdomain's own
    std::vector<double> rtab((size_t)MAX_REGIONS * NPARAM, 0.0);
    const ModelInfo m0 = model_info(s->model);
    for (int r = 0; r < MAX_REGIONS; r++) {
      const ep_sim::RegionCfg& c = s->region_cfg[r];
      const int mr = region_model(s, r);
      double* row = &rtab[(size_t)r * NPARAM];
      default_params(mr, c.variant >= 0 ? c.variant : s->variant, row);
      if (mr == s->model)
        for (size_t k = 0; k < s->params.size(); k++) row[k] = s->params[k];
      if (c.has_params)
        for (size_t k = 0; k < c.params.size(); k++) row[k] = c.params[k];
      // the field is in the sim model's units u_mV = a0 u + b0; model r sees
      // u_r = (a0 u + b0 - br) / ar and contributes (ar / a0) I_r
      const ModelInfo mi_r = model_info(mr);
      D.rmodel[r] = mr;
      D.rconv[r][0] = m0.mv_per_unit / mi_r.mv_per_unit;
      D.rconv[r][1] = (m0.mv_offset - mi_r.mv_offset) / mi_r.mv_per_unit;
      D.rconv[r][2] = mi_r.mv_per_unit / m0.mv_per_unit;
    }
    D.multi_model = s->het_model < 0 ? 1 : 0;
    double* d_rtab;
    EP_HIP(upload(m, &d_rtab, rtab.data(), rtab.size(), st));
    D.rtab = d_rtab;
    EP_HIP(m.alloc((void**)&D.ipt, (size_t)npts * sizeof(double)));
    EP_HIP(hipMemsetAsync(D.ipt, 0, (size_t)npts * sizeof(double), st));
    EP_HIP(m.alloc((void**)&D.cvec, (size_t)n * sizeof(double)));
    EP_HIP(hipMemsetAsync(D.cvec, 0, (size_t)n * sizeof(double), st));
    // C(j, q) = M^r(j, node_q) for the extra point q = (node_q, r), from the
    // mass matrix of subdomain r alone
    struct Ent {
      int32_t row, q;
      double v;
    };
    std::vector<Ent> ents;
    const int npe = s->elem;
    for (int r = 0; r < MAX_REGIONS; r++) {
      std::vector<int64_t> qs;
      for (int64_t q = 0; q < nsec; q++)
        if (sec_reg[q] == r) qs.push_back(q);
      if (qs.empty()) continue;
      std::vector<int32_t> conn_r;
      for (int64_t e = 0; e < s->n_elems; e++)
        if (s->material[e] == r) conn_r.insert(conn_r.end(), &s->conn[e * npe], &s->conn[e * npe] + npe);
      Csr Mr;
      std::vector<char> err_r;
      if (!assemble_csr(s->elem, n, s->xyz.data(), (int64_t)conn_r.size() / npe, conn_r.data(), fib0, fib1, fib2,
                        rsig[3 * r], rsig[3 * r + 1], rsig[3 * r + 2], s->chi, s->cm, Mr, err_r))
        return fail(EP_EINVAL, std::string("subdomain assembly: ") + (err_r.empty() ? "failed" : err_r.data()));
      for (int64_t q : qs) {
        const int32_t k = s->sec_node[q];
        for (int64_t t = Mr.rowptr[k]; t < Mr.rowptr[k + 1]; t++) {
          const int32_t j = Mr.col[t];
          const int32_t* cj = &Mr.col[Mr.rowptr[j]];
          const int64_t lj = Mr.rowptr[j + 1] - Mr.rowptr[j];
          const int64_t pos = Mr.rowptr[j] + (std::lower_bound(cj, cj + lj, k) - cj);
          ents.push_back({j, (int32_t)q, Mr.valM[pos]});
        }
      }
    }
    std::sort(ents.begin(), ents.end(), [](const Ent& a, const Ent& b) { return a.row < b.row || (a.row == b.row && a.q < b.q); });
    std::vector<int32_t> crow, ccol;
    std::vector<int64_t> cptr(1, 0);
    std::vector<double> cval;
    for (size_t t = 0; t < ents.size(); t++) {
      if (t == 0 || ents[t].row != ents[t - 1].row) {
        if (t > 0) cptr.push_back((int64_t)t);
        crow.push_back(ents[t].row);
      }
      ccol.push_back(ents[t].q);
      cval.push_back(ents[t].v);
    }
    cptr.push_back((int64_t)ents.size());
    s->n_cent = (int64_t)ents.size();
    if (crow.empty()) cptr.assign(1, 0);
    s->n_crow = (int64_t)crow.size();
    D.n_crow = (int32_t)crow.size();
    if (!crow.empty()) {
      int32_t *d_crow, *d_ccol;
      int64_t* d_cptr;
      double* d_cval;
      EP_HIP(upload(m, &d_crow, crow.data(), crow.size(), st));
      EP_HIP(upload(m, &d_cptr, cptr.data(), cptr.size(), st));
      EP_HIP(upload(m, &d_ccol, ccol.data(), ccol.size(), st));
      EP_HIP(upload(m, &d_cval, cval.data(), cval.size(), st));
      D.crow = d_crow;
      D.cptr = d_cptr;
      D.ccol = d_ccol;
      D.cval = d_cval;
    }
    EP_HIP(hipStreamSynchronize(st));  // host vectors above are temporaries
  }
  EP_HIP(m.alloc((void**)&D.smax, n * sizeof(double)));
  EP_HIP(m.alloc((void**)&D.at, n * sizeof(double)));
  EP_HIP(m.alloc((void**)&D.tcross, n * sizeof(double)));
  // ---- stimuli, grouped by timing ----
  {
    std::map<std::tuple<int64_t, int64_t, int64_t>, std::vector<double>> groups;
    const double scale = 1.0 / (s->chi * s->cm * s->mi.mv_per_unit);
    for (const Stim& t : s->stims) {
      const int64_t s0 = llround(t.t0 / s->dt), du = llround(t.dur / s->dt);
      const int64_t pe = t.period > 0 ? llround(t.period / s->dt) : 0;
      auto& prof = groups[std::make_tuple(s0, du, pe)];
      if (prof.empty()) prof.assign(n, 0.0);
      for (int64_t i = 0; i < n; i++) prof[i] += t.amp * scale * stim_profile(t, &s->xyz[3 * i]);
    }
    if ((int)groups.size() > MAX_STIM) return fail(EP_EINVAL, "more than 8 distinct stimulus timings");
    int k = 0;
    for (auto& kv : groups) {
      StimGroup& sg = D.stim[k++];
      sg.amp = 1.0;
      sg.s0 = std::get<0>(kv.first);
      sg.dur = std::get<1>(kv.first);
      sg.period = std::get<2>(kv.first);
      hostvals.push_back(kv.second);
      double* p;
      EP_HIP(upload(m, &p, hostvals.back().data(), n, st));
      sg.prof = p;
    }
    D.n_stim = k;
  }
  // ---- control state, partials, block map ----
  const int ntiles = (int)((n + TILE - 1) / TILE);
  D.blk0 = 0;
  D.nblk = ntiles;
  // single-instance launches cover N_XCD * ceil(tiles / N_XCD) workgroups
  s->nblocks = N_XCD * ((ntiles + N_XCD - 1) / N_XCD);
  D.tile_tab = nullptr;
  {
    std::vector<int32_t> tab = lattice_tile_table(D, n, ntiles, s->nblocks);
    if (!tab.empty()) {
      int32_t* dt;
      EP_HIP(upload(m, &dt, tab.data(), tab.size(), st));
      D.tile_tab = dt;
    }
  }
  EP_HIP(m.alloc((void**)&D.partial, (size_t)ntiles * PART_DOUBLES * sizeof(double)));
  D.cg_pipe = cg_resolved(s) == EP_CG_PIPELINED ? 1 : 0;
  D.x0_extrap = s->x0_extrap;
  if (D.cg_pipe) {
    EP_HIP(m.alloc((void**)&D.pipe_rec, (size_t)ntiles * PIPE_REC * sizeof(double)));
    EP_HIP(hipMemsetAsync(D.pipe_rec, 0, (size_t)ntiles * PIPE_REC * sizeof(double), st));
    if (mixed) {
      EP_HIP(vec_f(&D.m32[0]));
      EP_HIP(vec_f(&D.m32[1]));
    }
  }
  {
    const int32_t zero = 0;
    EP_HIP(upload(m, &s->d_ids, &zero, 1, st));
    EP_HIP(hipStreamSynchronize(st));
  }
  EP_HIP(hipHostMalloc((void**)&s->h_st, sizeof(InstState), hipHostMallocDefault));
  std::memset(s->h_st, 0, sizeof(InstState));
  std::vector<BlockMap> bm(ntiles);
  for (int b = 0; b < ntiles; b++) bm[b] = {0, b};
  EP_HIP(upload(m, &s->d_bmap, bm.data(), bm.size(), st));
  EP_HIP(m.alloc((void**)&s->d_desc, sizeof(InstDesc)));
  s->d_desc_own = s->d_desc;
  // the state lives inside the device descriptor (its first member)
  s->d_st = reinterpret_cast<InstState*>(reinterpret_cast<char*>(s->d_desc) + offsetof(InstDesc, st));
  EP_HIP(hipStreamSynchronize(st));
  hostvals.clear();
  for (int k = 0; k < 5; k++) EP_HIP(hipEventCreate(&s->ev[k]));
  s->finalized = true;
  // ---- initial state ----
  std::vector<double> init = s->init.empty() ? default_init(s->model) : s->init;
  std::vector<double> u(n, init[0]);
  std::vector<double> w((size_t)nvars * n);
  for (int v = 0; v < nvars; v++)
    for (int64_t i = 0; i < n; i++) w[(size_t)v * n + i] = init[1 + v];
  ep_status rc = ep_sim_set_state(s, u.data(), w.data(), nullptr, 0);
  if (rc != EP_OK) return rc;
  s->ms_setup = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return EP_OK;
}

// Host-side consistency check of a descriptor before kernels use it: every
// array the configured path touches is present, lies with the whole range
// the kernels address (guard cells, padded rows, DIA diagonals, SELL slices,
// state rows, element arrays) inside one of the sim's allocations, and the
// DIA geometry keeps all shifted accesses inside the guard cells.  A
// failure is a library bug; it is reported instead of launching.
ep_status validate_desc(const ep_sim* s, const InstDesc& D) {
  const int64_t guard = s->guard;
  auto bad = [](const char* what) { return fail(EP_EHIP, std::string("internal descriptor check: ") + what); };
  if (D.n <= 0 || D.nblk != (int)((D.n + TILE - 1) / TILE)) return bad("tile count");
  if (D.bdf < 1 || D.bdf > 3) return bad("bdf");
  if (!D.partial || !D.g || !D.b || !D.r || !D.z || !D.p || !D.s || !D.w) return bad("vectors");
  for (int k = 0; k < RING; k++)
    if (!D.U[k]) return bad("history ring");
  if (!D.u_new || !D.u_cur || !D.u_prev1 || !D.u_prev2) return bad("history slots");
  if ((!D.valM && D.fmt != FMT_MF) || !D.smax || !D.at || !D.tcross) return bad("arrays");
  if (D.het) {
    if (D.n_pts < D.n || !D.pt_reg || !D.sec_node || !D.rtab || !D.ipt || !D.cvec) return bad("subdomain arrays");
    if (D.n_crow > 0 && (!D.crow || !D.cptr || !D.ccol || !D.cval)) return bad("interface correction");
  } else if (D.n_pts != D.n) {
    return bad("ionic points");
  }
  for (int q = 0; q < D.bdf; q++) {
    if ((!D.valA[q] && D.fmt != FMT_MF) || !D.dinv[q]) return bad("operator values");
    if (D.prec == P_MIXED && (!D.valA32[q] || !D.dinv32[q])) return bad("FP32 operator values");
  }
  if (D.prec == P_MIXED && (!D.r32 || !D.z32 || !D.p32 || !D.s32 || !D.w32)) return bad("FP32 vectors");
  for (int k = 0; k < RING; k++)
    if (!D.st64[k] || !D.st32[k]) return bad("ionic state levels");
  if (D.ionic_scheme != 0 && D.ionic_scheme != 1) return bad("ionic scheme");
  if (D.block < 1 || D.block > 64 || (D.block & (D.block - 1)) != 0 || D.bld < ((D.n + 63) / 64) * 64)
    return bad("preconditioner blocks");
  if (D.fmt == FMT_DIA) {
    if (D.nup < 1 || D.nup > MAX_UP || D.off[0] != 0) return bad("DIA diagonals");
    for (int d = 1; d < D.nup; d++)
      if (D.off[d] <= D.off[d - 1] || D.off[d] > guard) return bad("DIA offsets exceed the guard");
    if (D.ld < ((D.n + 63) / 64) * 64 + guard) return bad("DIA leading dimension");
  } else if (D.fmt == FMT_SELL) {
    if (!D.col || !D.slice_ptr) return bad("SELL arrays");
  } else if (D.fmt == FMT_MF) {
    if ((D.mf_p != 2 && D.mf_p != 3) || D.n_elems <= 0 || !D.geo || !D.econn || !D.yA || !D.yM || !D.adj_ptr ||
        !D.adj || D.prec != P_FP64 || D.het)
      return bad("matrix-free operator arrays");
  } else {
    return bad("matrix format");
  }
  if (D.n_stim < 0 || D.n_stim > MAX_STIM) return bad("stimuli");
  for (int k = 0; k < D.n_stim; k++)
    if (!D.stim[k].prof) return bad("stimulus profile");
  // ---- address ranges ----
  const DevMem& m = s->mem;
  const int64_t n = D.n, n64 = ((n + 63) / 64) * 64, G = guard, npts = D.n_pts;
  auto in = [&](const void* p, int64_t lo_elems, int64_t elems, size_t esz) {
    return m.covers(static_cast<const char*>(p) - (size_t)lo_elems * esz, (size_t)elems * esz);
  };
  // vectors: rows up to the 64-row padding, with G guard cells on each side
  const double* v64[] = {D.g, D.b, D.r, D.z, D.p, D.s, D.w, D.U[0], D.U[1], D.U[2], D.U[3]};
  for (const double* v : v64)
    if (!in(v, G, n64 + 2 * G, 8)) return bad("vector range");
  if (D.prec == P_MIXED) {
    const float* v32[] = {D.r32, D.z32, D.p32, D.s32, D.w32};
    for (const float* v : v32)
      if (!in(v, G, n64 + 2 * G, 4)) return bad("FP32 vector range");
  }
  const int nsig = D.bdf;
  for (int q = 0; q < nsig; q++) {
    if (!in(D.dinv[q], 0, D.block == 1 ? n64 : D.bld * D.block, 8)) return bad("preconditioner range");
    if (D.prec == P_MIXED && !in(D.dinv32[q], 0, D.block == 1 ? n64 : D.bld * D.block, 4))
      return bad("FP32 preconditioner range");
  }
  if (D.fmt == FMT_DIA) {
    const int64_t span = (int64_t)D.nup * D.ld;
    for (int q = 0; q <= nsig; q++) {
      const double* v = q < nsig ? D.valA[q] : D.valM;
      if (!in(v, G, span + G, 8)) return bad("DIA value range");
      if (q < nsig && D.prec == P_MIXED && !in(D.valA32[q], G, span + G, 4)) return bad("FP32 DIA value range");
    }
  } else if (D.fmt == FMT_SELL) {
    const int64_t ns = (n + SLICE - 1) / SLICE;
    if (!in(D.slice_ptr, 0, ns + 1, 8) || !in(D.col, 0, s->sell_nnz, 4)) return bad("SELL index range");
    for (int q = 0; q <= nsig; q++) {
      const double* v = q < nsig ? D.valA[q] : D.valM;
      if (!in(v, 0, s->sell_nnz, 8)) return bad("SELL value range");
      if (q < nsig && D.prec == P_MIXED && !in(D.valA32[q], 0, s->sell_nnz, 4)) return bad("FP32 SELL value range");
    }
  } else {
    const int64_t npe = s->elem, ent = D.n_elems * npe, Q = npe;
    if (D.n_elems != s->n_elems || !in(D.econn, 0, ent, 4) || !in(D.geo, 0, D.n_elems * 7 * (D.mf_cmp ? 1 : Q), 8) ||
        !in(D.yA, 0, ent, 8) || !in(D.yM, 0, ent, 8) || !in(D.adj_ptr, 0, n + 1, 8) || !in(D.adj, 0, ent, 4))
      return bad("matrix-free array range");
  }
  for (int k = 0; k < RING; k++)
    if (!in(D.st64[k], 0, std::max<int64_t>(1, (int64_t)s->st_rows64 * npts), 8) ||
        !in(D.st32[k], 0, std::max<int64_t>(1, (int64_t)s->st_rows32 * npts), 4))
      return bad("ionic state range");
  if (!in(D.smax, 0, n, 8) || !in(D.at, 0, n, 8) || !in(D.tcross, 0, n, 8)) return bad("activation range");
  if (!in(D.partial, 0, (int64_t)D.nblk * PART_DOUBLES, 8)) return bad("partial sums range");
  if (D.cg_pipe && !in(D.pipe_rec, 0, (int64_t)D.nblk * PIPE_REC, 8)) return bad("pipelined CG records");
  if (D.tile_tab && !in(D.tile_tab, 0, s->nblocks, 4)) return bad("tile table range");
  if (D.cg_pipe && D.prec == P_MIXED && (!in(D.m32[0], G, n64 + 2 * G, 4) || !in(D.m32[1], G, n64 + 2 * G, 4)))
    return bad("pipelined FP32 vector range");
  for (int k = 0; k < D.n_stim; k++)
    if (!in(D.stim[k].prof, 0, n, 8)) return bad("stimulus profile range");
  if (D.het) {
    if (!in(D.pt_reg, 0, npts, 4) || !in(D.sec_node, 0, std::max<int64_t>(1, npts - n), 4) ||
        !in(D.rtab, 0, (int64_t)MAX_REGIONS * NPARAM, 8) || !in(D.ipt, 0, npts, 8) || !in(D.cvec, 0, n, 8))
      return bad("subdomain array range");
    if (D.n_crow > 0 && (!in(D.crow, 0, D.n_crow, 4) || !in(D.cptr, 0, D.n_crow + 1, 8) ||
                         !in(D.ccol, 0, s->n_cent, 4) || !in(D.cval, 0, s->n_cent, 8)))
      return bad("interface correction range");
  }
  return EP_OK;
}

Launch launch_of(ep_sim* s) {
  Launch L{s->d_desc, s->d_bmap, s->nblocks, s->stream, true};
  if (s->desc.fmt == FMT_MF) {
    L.mf_p = s->desc.mf_p;
    L.mf_elems = s->n_elems;
    L.mf_cmp = s->desc.mf_cmp != 0;
  }
  L.xmap = (s->xmap == 2 && !s->desc.tile_tab) ? 0 : s->xmap;   // map 2 needs a lattice
  L.ionic_npt = s->ionic_npt;
  L.ionic_bdf = s->ionic_scheme == EP_IONIC_BDF;
  L.pipe_op = (s->desc.fmt == FMT_DIA && s->desc.nup == 14 && s->desc.block == 1) ? 1 : 0;
  return L;
}

// One time step of one sim (host sequencing; all arithmetic on the device).
// Kernel order: ionic, residual(+rhs), then the solve.  FP64 pipelined CG:
// the start kernel, then rounds of one iteration kernel; FP64
// Chronopoulos-Gear: rounds of {SpMV, update}; mixed: SpMV, finalize, then
// rounds of {update, SpMV, finalize}, with an FP64 refinement residual
// (+ SpMV, finalize) after each inner sweep.  The kernels decide convergence
// on the device; the host reads that flag after a chunk of rounds.  With
// graphs on (and no timers), the same sequences are replayed from captured
// graphs.
ep_status step_once(ep_sim* s) {
  const Launch L = launch_of(s);
  const bool mixed = s->prec == EP_MIXED;
  KernelTimers& kt = s->kt;
  hipStream_t st = s->stream;
  auto fin = [&] { kt.timed(st, 6, [&] { launch_cg_finalize(mixed, s->d_desc, nullptr, 1, st); }); };
  // FP64: a round is SpMV then the update (which adds the partial sums
  // itself); mixed: update, SpMV, finalize
  const bool pipe = s->desc.cg_pipe;
  auto round = [&] {
    if (pipe) {
      kt.timed(st, 7, [&] { mixed ? launch_cg_pipe32(L) : launch_cg_pipe(L); });
      return;
    }
    if (!mixed) {
      kt.timed(st, 2, [&] { launch_cg_spmv(false, L); });
      kt.timed(st, 3, [&] { launch_cg_update64(L); });
      return;
    }
    kt.timed(st, 3, [&] { launch_cg_update(mixed, L); });
    kt.timed(st, 2, [&] { launch_cg_spmv(mixed, L); });
    fin();
  };
  auto pro = [&] {
    if (s->timers) (void)hipEventRecord(s->ev[0], st);
    kt.timed(st, 0, [&] {
      if (s->het) {
        launch_ionic_het(s->het_model, s->ionic_f32(), s->ionic_scheme == EP_IONIC_BDF, s->d_desc, s->n_pts, st);
        launch_ici_correction(s->d_desc, s->n_crow, st);
      } else {
        launch_ionic(s->model, s->ionic_f32(), L);
      }
    });
    if (s->timers) (void)hipEventRecord(s->ev[1], st);
    kt.timed(st, 1, [&] { launch_residual(mixed, true, L); });
    if (s->timers) (void)hipEventRecord(s->ev[2], st);
    if (pipe) {
      kt.timed(st, 2, [&] { mixed ? launch_cg_pipe32_start(L) : launch_cg_pipe_start(L); });
    } else if (mixed) {
      kt.timed(st, 2, [&] { launch_cg_spmv(mixed, L); });
      fin();
    }
  };
  auto ir = [&] {
    kt.timed(st, 5, [&] { launch_residual(true, false, L); });
    if (pipe) {
      // the start and the sweep's first iteration, which takes the outer
      // decision, so the host's next read sees it
      kt.timed(st, 2, [&] { launch_cg_pipe32_start(L); });
      kt.timed(st, 7, [&] { launch_cg_pipe32(L); });
      return;
    }
    kt.timed(st, 2, [&] { launch_cg_spmv(true, L); });
    fin();
  };
  auto epi = [&] {
    if (s->timers) (void)hipEventRecord(s->ev[3], st);
    kt.timed(st, 4, [&] { launch_activation(L); });
    launch_end_step(s->d_desc, s->d_ids, 1, st);
  };
  const bool graph = s->use_graph && !kt.on && !s->timers;
  StepGraphs& G = s->graphs;
  if (graph && !G.valid) {
    G.reset();
    EP_HIP(capture_graph(st, pro, &G.pro));
    EP_HIP(capture_graph(st, round, &G.round1));
    EP_HIP(capture_graph(st, [&] { round(); round(); }, &G.round2));
    if (mixed) EP_HIP(capture_graph(st, ir, &G.ir));
    EP_HIP(capture_graph(st, epi, &G.epi));
    G.valid = true;
  }
  auto rounds = [&](int c) -> hipError_t {
    if (!graph) {
      for (int k = 0; k < c; k++) round();
      return hipGetLastError();
    }
    for (; c >= 2; c -= 2) {
      hipError_t e = hipGraphLaunch(G.round2, st);
      if (e != hipSuccess) return e;
    }
    return c ? hipGraphLaunch(G.round1, st) : hipSuccess;
  };
  if (graph) EP_HIP(hipGraphLaunch(G.pro, st));
  else pro();
  if (!mixed) {
    // K updates take K + 1 rounds: the last one finds the residual converged
    int chunk = std::max(1, s->it_pred) + 1;
    for (int n_rounds = 0;; n_rounds++) {
      EP_HIP(rounds(chunk));
      ep_status rc = pull_state(s);
      if (rc != EP_OK) return rc;
      if (s->h_st->conv) break;
      if (n_rounds > s->max_it + 2) return fail(EP_EHIP, "solver control lost (no convergence flag)");
      chunk = 2;
    }
    s->it_pred = std::max(1, s->h_st->it_step);
  } else {
    // sweep = refinement residuals evaluated so far in this step; a sweep
    // that has not converged after its predicted rounds continues by 2.
    // Pipelined inner solve: the sweeps the last step needed are enqueued
    // before the first read (a sweep's launches do nothing once the step
    // has converged, and a refinement residual does nothing before its
    // sweep's inner solve is done), and each sweep's inner iteration count
    // comes from the device state.
    int sweep = 0, sweep_start = 0, learned = 0;
    bool fresh = true;
    const int ahead = pipe ? std::max(1, std::min(s->sweeps_last, 3)) : 1;
    for (int reads = 0;; reads++) {
      const int nsw = reads == 0 ? ahead : 1;
      for (int j = 0; j < nsw; j++) {
        EP_HIP(rounds(fresh ? s->sweeps.rounds(sweep + j) : 2));
        if (graph) EP_HIP(hipGraphLaunch(G.ir, st));
        else ir();
      }
      ep_status rc = pull_state(s);
      if (rc != EP_OK) return rc;
      const int outer = s->h_st->outer, it_now = s->h_st->it_step;
      fresh = outer > sweep;
      if (pipe) {
        // sweep j's inner solve stopped at iteration sw_its[j]; its rounds
        // were that many plus the first (sweep 0) or without it (the first
        // iteration of later sweeps runs with their refinement residual)
        for (; learned < outer; learned++) {
          const int k_stop = s->h_st->sw_its[std::min(learned, 2)];
          s->sweeps.learn(learned, learned == 0 ? k_stop : k_stop - 1);
        }
        sweep = outer;
      } else if (fresh) {
        s->sweeps.learn(sweep, it_now - sweep_start);
        sweep = outer;
        sweep_start = it_now;
      }
      if (s->h_st->conv) break;
      if (reads > s->max_it + s->max_outer + 2) return fail(EP_EHIP, "solver control lost (no convergence flag)");
    }
    s->sweeps_last = s->h_st->outer;
  }
  if (graph) EP_HIP(hipGraphLaunch(G.epi, st));
  else epi();
  if (s->timers) {
    EP_HIP(hipEventRecord(s->ev[4], st));
    EP_HIP(hipEventSynchronize(s->ev[4]));
    for (int k = 0; k < 4; k++) {
      float ms = 0;
      EP_HIP(hipEventElapsedTime(&ms, s->ev[k], s->ev[k + 1]));
      s->ms_phase[k] += ms;
    }
  }
  const int flags = s->h_st->flags;
  if (flags & F_NAN) return EP_ENAN;
  if (flags & (F_NOCONV | F_BREAKDOWN)) return EP_ENOCONV;
  return EP_OK;
}

// Kernel-timer totals of one tuner candidate.
struct TimerSums {
  double ms[KernelTimers::K] = {};
  int64_t count[KernelTimers::K] = {};
  double avg_us(int k) const { return count[k] ? 1e3 * ms[k] / (double)count[k] : 0.0; }
};

// Tile-map score: the mean durations of the kernels that work on tiles (rhs
// and refinement residuals, SpMV or pipelined start, updates, pipelined
// iterations), each weighted by how often that kind ran over all candidates'
// trial steps (the same weights for every candidate).
static double tile_kernels_us(const TimerSums& a, const TimerSums& all) {
  double t = 0.0;
  for (int k : {1, 2, 3, 5, 7}) t += a.avg_us(k) * (double)all.count[k];
  return t;
}

// Tuner core: `trial` steps per candidate of one launch-shape setting with
// kernel timers on, in up to three rounds that visit the candidates in
// alternating order (A B C, C B A, A B C), so that the drift of the
// simulation's work from step to step (iteration counts follow the
// propagation phase) weighs on every candidate alike; each candidate is
// scored on the mean durations, over its rounds, of the kernels it affects
// (weighted, where several kinds count, by the launches of each kind over
// all candidates); the best is kept.  The steps are real steps of the simulation; every
// candidate computes bitwise the same results.
template <typename Step, typename Set, typename Score>
ep_status tune_one(KernelTimers& kt, hipStream_t st, int trial, const std::vector<int>& cands, Set&& set,
                   Step&& step, Score&& score, int* best_out) {
  const int nc = (int)cands.size();
  std::vector<TimerSums> acc((size_t)nc);
  const int rounds = std::min(trial, 3);
  for (int r = 0; r < rounds; r++) {
    const int steps = trial / rounds + (r < trial % rounds ? 1 : 0);
    for (int j = 0; j < nc; j++) {
      const int ci = (r & 1) ? nc - 1 - j : j;
      set(cands[(size_t)ci]);
      EP_HIP(hipStreamSynchronize(st));
      kt.harvest();
      kt.zero();
      for (int k = 0; k < steps; k++) {
        ep_status rc = step();
        if (rc != EP_OK && rc != EP_ENOCONV) return rc;
      }
      EP_HIP(hipStreamSynchronize(st));
      kt.harvest();
      for (int k = 0; k < KernelTimers::K; k++) {
        acc[(size_t)ci].ms[k] += kt.ms[k];
        acc[(size_t)ci].count[k] += kt.count[k];
      }
    }
  }
  TimerSums all;
  for (const TimerSums& a : acc)
    for (int k = 0; k < KernelTimers::K; k++) {
      all.ms[k] += a.ms[k];
      all.count[k] += a.count[k];
    }
  double best = std::numeric_limits<double>::infinity();
  int best_c = cands.front();
  for (int ci = 0; ci < nc; ci++) {
    const double t = score(acc[(size_t)ci], all);
    if (t < best) {
      best = t;
      best_c = cands[(size_t)ci];
    }
  }
  set(best_c);
  *best_out = best_c;
  return EP_OK;
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================

extern "C" {

const char* ep_last_error(void) { return g_err.c_str(); }
const char* ep_version(void) { return "ep_mi355x 0.1 (gfx950)"; }

ep_status ep_sim_create(int device, void* hip_stream, ep_sim** out) {
  if (!out) return fail(EP_EINVAL, "out is null");
  *out = nullptr;
  int count = 0;
  EP_HIP(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) return fail(EP_EINVAL, "no such device");
  EP_HIP(hipSetDevice(device));
  ep_sim* s = new ep_sim();
  s->device = device;
  if (hip_stream) {
    s->stream = (hipStream_t)hip_stream;
  } else {
    hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete s;
      return fail(EP_EHIP, std::string("hipStreamCreate: ") + hipGetErrorString(e));
    }
    s->own_stream = true;
  }
  *out = s;
  return EP_OK;
}

ep_status ep_sim_upload_mesh(ep_sim* s, int elem, int64_t n_nodes, const double* xyz, int64_t n_elems,
                             const int32_t* conn, const int32_t* material_id) {
  if (check_sim(s)) return EP_EINVAL;
  if (s->finalized) return fail(EP_ESTATE, "sim already finalized");
  if (elem != EP_HEX8 && elem != EP_TET4 && elem != EP_HEX27 && elem != EP_HEX64 && elem != EP_HEX125 &&
      elem != EP_HEX216 && elem != EP_HEX343 && elem != EP_TET10)
    return fail(EP_EINVAL, "elem must be EP_TET4, EP_TET10 or EP_HEX8 .. EP_HEX343");
  if (n_nodes <= 0 || n_elems <= 0 || !xyz || !conn) return fail(EP_EINVAL, "empty mesh");
  if (n_nodes >= (int64_t)INT32_MAX) return fail(EP_EINVAL, "too many nodes");
  if (material_id)
    for (int64_t e = 0; e < n_elems; e++)
      if (material_id[e] < 0 || material_id[e] >= EP_MAX_REGIONS)
        return fail(EP_EINVAL, "material id outside 0 .. EP_MAX_REGIONS - 1");
  for (int64_t k = 0; k < n_elems * elem; k++)
    if (conn[k] < 0 || conn[k] >= n_nodes) return fail(EP_EINVAL, "connectivity index out of range");
  s->elem = elem;
  s->n = n_nodes;
  s->n_elems = n_elems;
  s->xyz.assign(xyz, xyz + 3 * n_nodes);
  s->conn.assign(conn, conn + elem * n_elems);
  if (material_id) s->material.assign(material_id, material_id + n_elems);
  else s->material.clear();
  s->f0.clear();
  s->s0.clear();
  s->n0.clear();
  return EP_OK;
}

ep_status ep_sim_set_region(ep_sim* s, int region, int variant, const double* params, int n_params,
                            double sigma_l, double sigma_t, double sigma_n, int conductive) {
  if (check_sim(s)) return EP_EINVAL;
  if (s->finalized) return fail(EP_ESTATE, "sim already finalized");
  if (region < 0 || region >= EP_MAX_REGIONS) return fail(EP_EINVAL, "region outside 0 .. EP_MAX_REGIONS - 1");
  if (variant < -1 || variant > EP_CELL_MID) return fail(EP_EINVAL, "bad cell type");
  if (n_params < 0 || n_params > NPARAM || (n_params > 0 && !params)) return fail(EP_EINVAL, "bad parameter count");
  ep_sim::RegionCfg& r = s->region_cfg[region];
  r.variant = variant;
  r.has_params = params != nullptr && n_params > 0;
  r.params.assign(params ? params : nullptr, params ? params + n_params : nullptr);
  r.sig[0] = sigma_l;
  r.sig[1] = sigma_t;
  r.sig[2] = sigma_n;
  r.conductive = conductive != 0;
  return EP_OK;
}

ep_status ep_sim_set_region_model(ep_sim* s, int region, int model) {
  if (check_sim(s)) return EP_EINVAL;
  if (s->finalized) return fail(EP_ESTATE, "sim already finalized");
  if (region < 0 || region >= EP_MAX_REGIONS) return fail(EP_EINVAL, "region outside 0 .. EP_MAX_REGIONS - 1");
  if (model != -1 && (model < EP_PASSIVE || model > EP_TTP06)) return fail(EP_EINVAL, "unknown ionic model");
  s->region_cfg[region].model = model;
  return EP_OK;
}

ep_status ep_sim_upload_fibers(ep_sim* s, const double* f0, const double* s0, const double* n0) {
  if (check_sim(s)) return EP_EINVAL;
  if (s->finalized) return fail(EP_ESTATE, "sim already finalized");
  if (s->n <= 0) return fail(EP_ESTATE, "upload the mesh first");
  if (!f0 || !s0 || !n0) return fail(EP_EINVAL, "null fiber array");
  s->f0.assign(f0, f0 + 3 * s->n);
  s->s0.assign(s0, s0 + 3 * s->n);
  s->n0.assign(n0, n0 + 3 * s->n);
  return EP_OK;
}

ep_status ep_sim_set_conductivity(ep_sim* s, double sl, double st, double sn, double chi, double cm) {
  if (check_sim(s)) return EP_EINVAL;
  if (s->finalized) return fail(EP_ESTATE, "sim already finalized");
  if (!(sl >= 0 && st >= 0 && sn >= 0 && chi > 0 && cm > 0)) return fail(EP_EINVAL, "bad conductivity");
  s->sl = sl; s->st = st; s->sn = sn; s->chi = chi; s->cm = cm;
  return EP_OK;
}

ep_status ep_sim_set_ionic_model(ep_sim* s, int model, int variant, const double* params, int n_params,
                                 const double* init_state) {
  if (check_sim(s)) return EP_EINVAL;
  if (s->finalized) return fail(EP_ESTATE, "sim already finalized");
  if (model < EP_PASSIVE || model > EP_TTP06) return fail(EP_EINVAL, "unknown ionic model");
  if (model == EP_TTP06 && (variant < 0 || variant > 2)) return fail(EP_EINVAL, "bad TTP06 cell type");
  if (n_params < 0 || n_params > n_model_params(model) || (n_params > 0 && !params))
    return fail(EP_EINVAL, "bad parameter count");
  s->model = model;
  s->variant = variant;
  s->params.assign(params ? params : nullptr, params ? params + n_params : nullptr);
  if (init_state) s->init.assign(init_state, init_state + 1 + model_info(model).nvars);
  else s->init.clear();
  return EP_OK;
}

ep_status ep_sim_add_stimulus(ep_sim* s, int shape, const double c[3], double size, double amp, double t0,
                              double dur, double period) {
  if (check_sim(s)) return EP_EINVAL;
  if (s->finalized) return fail(EP_ESTATE, "sim already finalized");
  if (shape < EP_CUBE || shape > EP_GAUSS || !c || !(size > 0) || !(dur >= 0) || !(period >= 0))
    return fail(EP_EINVAL, "bad stimulus");
  s->stims.push_back(Stim{shape, {c[0], c[1], c[2]}, size, amp, t0, dur, period});
  return EP_OK;
}

ep_status ep_sim_set_solver(ep_sim* s, double dt, int bdf, int precision, int precond, int block, double rtol,
                            int max_it) {
  if (check_sim(s)) return EP_EINVAL;
  if (s->finalized) return fail(EP_ESTATE, "sim already finalized");
  if (!(dt > 0) || bdf < 1 || bdf > 3 || (precision != EP_FP64 && precision != EP_MIXED) ||
      (precond != EP_JACOBI && precond != EP_BJACOBI) || !(rtol > 0) || max_it < 1)
    return fail(EP_EINVAL, "bad solver settings");
  const bool pow2 = block >= 1 && block <= 64 && (block & (block - 1)) == 0;
  if ((precond == EP_JACOBI && block != 1) || (precond == EP_BJACOBI && !pow2))
    return fail(EP_EINVAL, "block must be 1 for Jacobi and one of 1, 2, 4, ..., 64 for block Jacobi");
  s->dt = dt; s->bdf = bdf; s->prec = precision; s->precond = precond; s->block = block;
  s->rtol = rtol; s->max_it = max_it;
  return EP_OK;
}

ep_status ep_sim_set_option(ep_sim* s, int key, double value) {
  if (check_sim(s)) return EP_EINVAL;
  if (key == EP_OPT_PHASE_TIMERS) {
    s->timers = value != 0.0;
    return EP_OK;
  }
  if (key == EP_OPT_KERNEL_TIMERS) {
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    s->kt.harvest();
    s->kt.on = value != 0.0;
    s->kt.zero();
    return EP_OK;
  }
  if (key == EP_OPT_IONIC_NPT || key == EP_OPT_TILE_MAP || key == EP_OPT_GRAPH) {
    const int v = (int)value;
    if ((double)v != value) return fail(EP_EINVAL, "launch option values are integers");
    if (key == EP_OPT_IONIC_NPT && v != 1 && v != 2 && v != 4) return fail(EP_EINVAL, "ionic nodes per thread: 1, 2 or 4");
    if (key == EP_OPT_TILE_MAP && v != 0 && v != 1 && v != 2) return fail(EP_EINVAL, "tile map: 0, 1 or 2");
    if (key == EP_OPT_GRAPH && v != 0 && v != 1) return fail(EP_EINVAL, "graph: 0 or 1");
    if (s->stream) EP_HIP(hipStreamSynchronize(s->stream));
    if (key == EP_OPT_IONIC_NPT) s->ionic_npt = v;
    if (key == EP_OPT_TILE_MAP) s->xmap = v;
    if (key == EP_OPT_GRAPH) s->use_graph = v;
    s->graphs.reset();
    return EP_OK;
  }
  if (s->finalized) return fail(EP_ESTATE, "sim already finalized");
  switch (key) {
    case EP_OPT_MATRIX_FORMAT:
      if (value != EP_FMT_AUTO && value != EP_FMT_SELL && value != EP_FMT_DIA && value != EP_FMT_MF)
        return fail(EP_EINVAL, "format");
      s->fmt_pref = (int)value;
      return EP_OK;
    case EP_OPT_INNER_RTOL:
      if (!(value > 0 && value < 1)) return fail(EP_EINVAL, "inner rtol");
      s->inner_rtol = value;
      return EP_OK;
    case EP_OPT_MAX_OUTER:
      if (!(value >= 1)) return fail(EP_EINVAL, "max outer");
      s->max_outer = (int)value;
      return EP_OK;
    case EP_OPT_IONIC_SCHEME:
      if (value != EP_IONIC_RUSH_LARSEN && value != EP_IONIC_BDF) return fail(EP_EINVAL, "ionic scheme");
      s->ionic_scheme = (int)value;
      return EP_OK;
    case EP_OPT_IONIC_FP64:
      if (value != 0.0 && value != 1.0) return fail(EP_EINVAL, "ionic FP64: 0 or 1");
      s->ionic_fp64 = (int)value;
      return EP_OK;
    case EP_OPT_INITIAL_GUESS:
      if (value != EP_X0_EXT && value != EP_X0_EXTRAP3) return fail(EP_EINVAL, "initial guess");
      s->x0_extrap = value == EP_X0_EXTRAP3 ? 1 : 0;
      return EP_OK;
    case EP_OPT_CG_VARIANT:
      if (value != EP_CG_AUTO && value != EP_CG_PIPELINED && value != EP_CG_CHRONOPOULOS_GEAR)
        return fail(EP_EINVAL, "CG variant");
      s->cg_variant = (int)value;
      return EP_OK;
    default: return fail(EP_EINVAL, "unknown option");
  }
}

ep_status ep_sim_finalize(ep_sim* s) {
  if (check_sim(s)) return EP_EINVAL;
  if (s->in_pool) return fail(EP_ESTATE, "sim belongs to a pool");
  ep_status rc = finalize_impl(s);
  if (rc != EP_OK && !s->finalized) s->mem.release();
  return rc;
}

ep_status ep_sim_device_bytes_estimate(ep_sim* s, size_t* bytes) {
  if (check_sim(s) || !bytes) return fail(EP_EINVAL, "null argument");
  *bytes = estimate_bytes(s);
  return EP_OK;
}

ep_status ep_sim_step(ep_sim* s, int n_steps) {
  if (check_sim(s)) return EP_EINVAL;
  if (!s->finalized) return fail(EP_ESTATE, "finalize first");
  if (s->in_pool) return fail(EP_ESTATE, "sim is stepped by its pool");
  if (n_steps < 0) return fail(EP_EINVAL, "negative step count");
  EP_HIP(hipSetDevice(s->device));
  ep_status worst = EP_OK;
  for (int k = 0; k < n_steps; k++) {
    ep_status rc = step_once(s);
    if (rc == EP_ENAN || rc == EP_EHIP) {
      if (rc == EP_ENAN) g_err = "NaN in the solution";
      return rc;
    }
    if (rc == EP_ENOCONV) {
      worst = rc;
      g_err = "linear solve did not converge within max_it";
    }
  }
  return worst;
}

ep_status ep_sim_autotune(ep_sim* s, int trial_steps, int* ionic_npt, int* tile_map) {
  if (check_sim(s)) return EP_EINVAL;
  if (!s->finalized) return fail(EP_ESTATE, "finalize first");
  if (s->in_pool) return fail(EP_ESTATE, "sim is stepped by its pool");
  if (trial_steps < 1) return fail(EP_EINVAL, "trial_steps must be >= 1");
  EP_HIP(hipSetDevice(s->device));
  KernelTimers& kt = s->kt;
  EP_HIP(hipStreamSynchronize(s->stream));
  kt.harvest();
  const int was_on = kt.on;
  kt.on = 1;
  auto step = [&] { return step_once(s); };
  int npt = s->ionic_npt, xm = s->xmap;
  ep_status rc = tune_one(
      kt, s->stream, trial_steps, {1, 2, 4}, [&](int c) { s->ionic_npt = c; }, step,
      [](const TimerSums& a, const TimerSums&) { return a.avg_us(0); }, &npt);
  if (rc == EP_OK)
    rc = tune_one(
        kt, s->stream, trial_steps, s->desc.tile_tab ? std::vector<int>{0, 2} : std::vector<int>{0, 1},
        [&](int c) { s->xmap = c; }, step,
        [](const TimerSums& a, const TimerSums& all) { return tile_kernels_us(a, all); }, &xm);
  kt.zero();
  kt.on = was_on;
  s->graphs.reset();
  if (rc != EP_OK) return rc;
  if (ionic_npt) *ionic_npt = npt;
  if (tile_map) *tile_map = xm;
  return EP_OK;
}

ep_status ep_sim_sync(ep_sim* s) {
  if (check_sim(s)) return EP_EINVAL;
  EP_HIP(hipStreamSynchronize(s->stream));
  return EP_OK;
}

ep_status ep_sim_set_state(ep_sim* s, const double* u, const double* w, const double* u_prev,
                           int64_t step_index) {
  if (check_sim(s)) return EP_EINVAL;
  if (!s->finalized) return fail(EP_ESTATE, "finalize first");
  if (!u || (s->nvars > 0 && !w) || step_index < 0) return fail(EP_EINVAL, "null state");
  const int64_t n = s->n;
  InstDesc& D = s->desc;
  hipStream_t st = s->stream;
  EP_HIP(hipSetDevice(s->device));
  EP_HIP(hipStreamSynchronize(st));
  EP_HIP(hipMemcpyAsync(D.U[step_index & 3], u, n * sizeof(double), hipMemcpyHostToDevice, st));
  for (int k = 1; k < 3; k++) {
    const double* src = (u_prev && k < s->bdf) ? u_prev + (size_t)(k - 1) * n : u;
    EP_HIP(hipMemcpyAsync(D.U[(step_index - k) & 3], src, n * sizeof(double), hipMemcpyHostToDevice, st));
  }
  // state arrays have one column per ionic point (stride np), rows in each
  // point's model layout; an extra interface point starts from its node's
  // state, a point whose subdomain runs another model from that model's
  // initial conditions
  const int64_t np = s->n_pts;
  const bool f32 = s->ionic_f32();
  const int r64 = s->st_rows64, r32 = s->st_rows32;
  if (r64 + r32 > 0) {
    std::vector<double> h64((size_t)r64 * np, 0.0);
    std::vector<float> h32((size_t)r32 * np, 0.0f);
    std::vector<double> col(18), ic_other;
    for (int64_t p = 0; p < np; p++) {
      const int m = s->het ? s->pt_model[p] : s->model;
      const int64_t node = p < n ? p : s->sec_node[p - n];
      const int nvm = model_info(m).nvars;
      if (m == s->model) {
        for (int v = 0; v < nvm; v++) col[v] = w[(size_t)v * n + node];
      } else {
        ic_other = default_init(m);
        for (int v = 0; v < nvm; v++) col[v] = ic_other[1 + v];
      }
      pack_state(m, f32, col.data(), h64.data() + p, h32.data() + p, np);
    }
    // level n and, for the BDF ionic scheme, levels n-1 and n-2 (copies)
    for (int k = 0; k < 3; k++) {
      const int slot = (int)((step_index - k) & 3);
      if (k > 0 && D.st64[slot] == D.st64[step_index & 3]) break;
      if (r64 > 0) EP_HIP(hipMemcpyAsync(D.st64[slot], h64.data(), h64.size() * 8, hipMemcpyHostToDevice, st));
      if (r32 > 0) EP_HIP(hipMemcpyAsync(D.st32[slot], h32.data(), h32.size() * 4, hipMemcpyHostToDevice, st));
    }
    EP_HIP(hipStreamSynchronize(st));   // h64 / h32 are temporaries
  }
  launch_fill(D.smax, n, -std::numeric_limits<double>::infinity(), st);
  launch_fill(D.at, n, std::numeric_limits<double>::quiet_NaN(), st);
  launch_fill(D.tcross, n, std::numeric_limits<double>::quiet_NaN(), st);
  EP_HIP(hipGetLastError());
  std::memset(s->h_st, 0, sizeof(InstState));
  s->h_st->step = step_index;
  // earlier levels not given are copies of u: a constant history, consistent
  // at every order; given ones are consistent up to the BDF order
  s->h_st->hist = u_prev ? s->bdf : 3;
  // descriptor with a fresh control state and the history slots of step n
  D.st = *s->h_st;
  D.u_new = D.U[(step_index + 1) & 3];
  D.u_cur = D.U[step_index & 3];
  D.u_prev1 = D.U[(step_index - 1) & 3];
  D.u_prev2 = D.U[(step_index - 2) & 3];
  {
    ep_status vr = validate_desc(s, D);
    if (vr != EP_OK) return vr;
  }
  EP_HIP(hipMemcpyAsync(s->d_desc, &D, sizeof(InstDesc), hipMemcpyHostToDevice, st));
  EP_HIP(hipStreamSynchronize(st));
  return EP_OK;
}

ep_status ep_sim_get_state(ep_sim* s, double* u, double* w, double* u_prev) {
  if (check_sim(s)) return EP_EINVAL;
  if (!s->finalized) return fail(EP_ESTATE, "finalize first");
  ep_status rc = pull_state(s);
  if (rc) return rc;
  const int64_t n = s->n;
  const int64_t step = s->h_st->step;
  InstDesc& D = s->desc;
  hipStream_t st = s->stream;
  if (u) EP_HIP(hipMemcpyAsync(u, D.U[step & 3], n * 8, hipMemcpyDeviceToHost, st));
  if (u_prev)
    for (int k = 1; k < s->bdf; k++)
      EP_HIP(hipMemcpyAsync(u_prev + (size_t)(k - 1) * n, D.U[(step - k) & 3], n * 8, hipMemcpyDeviceToHost, st));
  const int nv = s->nvars;
  if (w && nv > 0) {
    // the nodes' columns of the state (stride n_pts; extra points dropped);
    // a node whose primary subdomain runs another model reports the first
    // nv variables of that model's state (zeros past its own count)
    const int64_t np = s->n_pts;
    const bool f32 = s->ionic_f32();
    const int r64 = s->st_rows64, r32 = s->st_rows32;
    if (!f32 && !s->het) {
      EP_HIP(hipMemcpyAsync(w, D.st64[step & 3], (size_t)nv * n * 8, hipMemcpyDeviceToHost, st));
    } else {
      std::vector<double> h64((size_t)std::max(r64, 1) * np);
      std::vector<float> h32((size_t)std::max(r32, 1) * np);
      if (r64 > 0) EP_HIP(hipMemcpyAsync(h64.data(), D.st64[step & 3], (size_t)r64 * np * 8, hipMemcpyDeviceToHost, st));
      if (r32 > 0) EP_HIP(hipMemcpyAsync(h32.data(), D.st32[step & 3], (size_t)r32 * np * 4, hipMemcpyDeviceToHost, st));
      EP_HIP(hipStreamSynchronize(st));
      double col[18];
      for (int64_t i = 0; i < n; i++) {
        const int m = s->het ? s->pt_model[i] : s->model;
        for (int v = 0; v < 18; v++) col[v] = 0.0;
        unpack_state(m, f32, h64.data() + i, h32.data() + i, np, col);
        for (int v = 0; v < nv; v++) w[(size_t)v * n + i] = col[v];
      }
    }
  }
  EP_HIP(hipStreamSynchronize(st));
  if (s->het) {
    const double nan = std::numeric_limits<double>::quiet_NaN();
    for (int64_t i = 0; i < n; i++)
      if (s->node_reg[i] < 0) {
        if (u) u[i] = nan;
        if (u_prev)
          for (int k = 1; k < s->bdf; k++) u_prev[(size_t)(k - 1) * n + i] = nan;
        if (w)
          for (int v = 0; v < nv; v++) w[(size_t)v * n + i] = nan;
      }
  }
  return EP_OK;
}

int ep_sim_n_vars(const ep_sim* s) { return s ? model_info(s->model).nvars : -1; }

ep_status ep_sim_get_potential(ep_sim* s, double* out) {
  if (check_sim(s) || !out) return fail(EP_EINVAL, "null argument");
  ep_status rc = ep_sim_get_state(s, out, nullptr, nullptr);
  if (rc) return rc;
  const double a = s->mi.mv_per_unit, b = s->mi.mv_offset;
  if (a != 1.0 || b != 0.0)
    for (int64_t i = 0; i < s->n; i++) out[i] = a * out[i] + b;
  return EP_OK;
}

ep_status ep_sim_get_potential_device(ep_sim* s, void* dst, int dtype) {
  if (check_sim(s) || !dst) return fail(EP_EINVAL, "null argument");
  if (!s->finalized) return fail(EP_ESTATE, "finalize first");
  if (dtype != EP_DTYPE_F64 && dtype != EP_DTYPE_F32) return fail(EP_EINVAL, "dtype");
  ep_status rc = pull_state(s);
  if (rc) return rc;
  const double* src = s->desc.U[s->h_st->step & 3];
  launch_to_mv(dst, src, s->n, s->mi.mv_per_unit, s->mi.mv_offset, dtype == EP_DTYPE_F32, s->stream,
               s->het ? s->desc.pt_reg : nullptr);
  EP_HIP(hipGetLastError());
  EP_HIP(hipStreamSynchronize(s->stream));
  return EP_OK;
}

static ep_status get_times(ep_sim* s, double* out, bool maxslope) {
  if (check_sim(s) || !out) return fail(EP_EINVAL, "null argument");
  if (!s->finalized) return fail(EP_ESTATE, "finalize first");
  const int64_t n = s->n;
  std::vector<double> tc(n);
  EP_HIP(hipStreamSynchronize(s->stream));
  EP_HIP(hipMemcpyAsync(tc.data(), s->desc.tcross, n * 8, hipMemcpyDeviceToHost, s->stream));
  if (maxslope) EP_HIP(hipMemcpyAsync(out, s->desc.at, n * 8, hipMemcpyDeviceToHost, s->stream));
  EP_HIP(hipStreamSynchronize(s->stream));
  for (int64_t i = 0; i < n; i++) {
    if (!maxslope) out[i] = tc[i];
    else if (std::isnan(tc[i])) out[i] = std::numeric_limits<double>::quiet_NaN();
    if (s->het && s->node_reg[i] < 0) out[i] = std::numeric_limits<double>::quiet_NaN();
  }
  return EP_OK;
}

ep_status ep_sim_get_activation_times(ep_sim* s, double* out) { return get_times(s, out, true); }
ep_status ep_sim_get_threshold_times(ep_sim* s, double* out) { return get_times(s, out, false); }

ep_status ep_sim_get_stats(ep_sim* s, ep_stats* o) {
  if (check_sim(s) || !o) return fail(EP_EINVAL, "null argument");
  std::memset(o, 0, sizeof(*o));
  o->n_nodes = s->n;
  if (!s->finalized) return EP_OK;
  ep_status rc = pull_state(s);
  if (rc) return rc;
  const InstState& S = *s->h_st;
  o->nnz = s->nnz;
  o->steps = S.step;
  o->cg_iters_total = S.it_total;
  o->cg_iters_last = S.it_last;
  o->cg_iters_max = S.it_max;
  o->ir_sweeps_total = S.outer_total;
  o->rel_residual_last = S.bb > 0 ? std::sqrt(S.rr_outer / S.bb) : 0.0;
  if (s->prec != EP_MIXED && S.bb > 0) o->rel_residual_last = std::sqrt(S.rr / S.bb);
  if (s->prec != EP_MIXED && S.bb == 0) o->rel_residual_last = 0.0;
  o->matrix_format = s->desc.fmt == FMT_DIA ? EP_FMT_DIA : (s->desc.fmt == FMT_MF ? EP_FMT_MF : EP_FMT_SELL);
  o->n_diag = s->desc.fmt == FMT_DIA ? 2 * s->desc.nup - 1 : 0;
  o->mf_compressed = s->desc.fmt == FMT_MF && s->desc.mf_cmp ? 1 : 0;
  o->device_bytes = (int64_t)s->mem.bytes;
  o->ms_ionic = s->ms_phase[0];
  o->ms_rhs = s->ms_phase[1];
  o->ms_solve = s->ms_phase[2];
  o->ms_activation = s->ms_phase[3];
  o->ms_setup = s->ms_setup;
  return EP_OK;
}

ep_status ep_sim_get_kernel_times(ep_sim* s, double* ms, int64_t* launches) {
  if (check_sim(s) || !ms || !launches) return fail(EP_EINVAL, "null argument");
  if (s->stream) EP_HIP(hipStreamSynchronize(s->stream));
  s->kt.harvest();
  for (int k = 0; k < KernelTimers::K; k++) {
    ms[k] = s->kt.ms[k];
    launches[k] = s->kt.count[k];
  }
  return EP_OK;
}

ep_status ep_sim_timer_overhead(ep_sim* s, int reps, double* us_per_pair) {
  if (check_sim(s) || reps < 1 || !us_per_pair) return fail(EP_EINVAL, "bad timer-overhead arguments");
  EP_HIP(hipSetDevice(s->device));
  hipStream_t st = s->stream;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev((size_t)reps);
  for (auto& e : ev) {
    EP_HIP(hipEventCreate(&e.first));
    EP_HIP(hipEventCreate(&e.second));
  }
  EP_HIP(hipStreamSynchronize(st));
  for (auto& e : ev) {
    EP_HIP(hipEventRecord(e.first, st));
    EP_HIP(hipEventRecord(e.second, st));
  }
  EP_HIP(hipStreamSynchronize(st));
  double sum = 0.0;
  for (auto& e : ev) {
    float ms = 0.0f;
    EP_HIP(hipEventElapsedTime(&ms, e.first, e.second));
    sum += ms;
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  *us_per_pair = 1e3 * sum / reps;
  return EP_OK;
}

// Back-to-back launches of the pipelined CG iteration on a copy of a
// mid-solve state: the vectors, partial sums, tile records and control state
// the kernel touches are saved, then, in batches, restored, the stopping
// test disabled (tol2 = 0) and the iteration launched `batch` times under
// HIP events; afterwards everything is restored.  The state between steps
// is that of the last step's final iteration, which found the residual
// converged: past that test the recurrences continue as in a longer solve.
ep_status time_pipe(ep_sim* s, int reps, double* us_per_launch) {
  const InstDesc& D = s->desc;
  if (!D.cg_pipe || D.prec != P_FP64) return fail(EP_EINVAL, "the sim does not use the FP64 pipelined CG");
  hipStream_t st = s->stream;
  const int64_t G = s->guard, nv = ((s->n + 63) / 64) * 64 + 2 * G;
  const int64_t step = s->h_st->step;
  double* vec[8] = {D.z, D.w, D.p, D.s, D.U[(step + 1) & 3], D.r, D.g, D.b};
  const int64_t npart = (int64_t)D.nblk * PART_DOUBLES, nrec = (int64_t)D.nblk * PIPE_REC;
  const int64_t total = 8 * nv + npart + nrec;
  if (!s->tk_save) EP_HIP(s->mem.alloc((void**)&s->tk_save, (size_t)total * sizeof(double)));
  double* sv = s->tk_save;
  auto copy = [&](bool save) -> hipError_t {
    for (int k = 0; k < 8; k++) {
      double* a = vec[k] - G;
      double* b = sv + k * nv;
      hipError_t e = hipMemcpyAsync(save ? b : a, save ? a : b, nv * 8, hipMemcpyDeviceToDevice, st);
      if (e != hipSuccess) return e;
    }
    hipError_t e = hipMemcpyAsync(save ? sv + 8 * nv : D.partial, save ? D.partial : sv + 8 * nv, npart * 8,
                                  hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(save ? sv + 8 * nv + npart : D.pipe_rec, save ? D.pipe_rec : sv + 8 * nv + npart, nrec * 8,
                         hipMemcpyDeviceToDevice, st);
    return e;
  };
  const InstState saved = *s->h_st;
  InstState armed = saved;
  armed.tol2 = 0.0;
  armed.conv = 0;
  std::vector<double> rec((size_t)nrec);
  EP_HIP(hipMemcpyAsync(rec.data(), D.pipe_rec, nrec * 8, hipMemcpyDeviceToHost, st));
  EP_HIP(hipStreamSynchronize(st));
  const int batch = std::min(reps, 16);
  if ((int)rec[0] + 1 + batch >= s->max_it) return fail(EP_ESTATE, "too few iterations left below max_it");
  EP_HIP(copy(true));
  const Launch L = launch_of(s);
  hipEvent_t a = nullptr, b = nullptr;
  EP_HIP(hipEventCreate(&a));
  EP_HIP(hipEventCreate(&b));
  double ms_total = 0.0;
  int done = 0;
  bool short_run = false;
  hipError_t err = hipSuccess;
  while (done < reps && err == hipSuccess) {
    const int nb = std::min(batch, reps - done);
    err = copy(false);
    if (err == hipSuccess) err = hipMemcpyAsync(s->d_st, &armed, sizeof(InstState), hipMemcpyHostToDevice, st);
    if (err == hipSuccess) err = hipEventRecord(a, st);
    for (int k = 0; k < nb && err == hipSuccess; k++) launch_cg_pipe(L);
    if (err == hipSuccess) err = hipGetLastError();
    if (err == hipSuccess) err = hipEventRecord(b, st);
    if (err == hipSuccess) err = hipMemcpyAsync(s->h_st, s->d_st, sizeof(InstState), hipMemcpyDeviceToHost, st);
    if (err == hipSuccess) err = hipStreamSynchronize(st);
    if (err != hipSuccess) break;
    float ms = 0.0f;
    err = hipEventElapsedTime(&ms, a, b);
    ms_total += ms;
    if (s->h_st->it_step != armed.it_step + nb || s->h_st->conv) short_run = true;
    done += nb;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  // restore the state whatever happened above
  EP_HIP(copy(false));
  *s->h_st = saved;
  EP_HIP(hipMemcpyAsync(s->d_st, &saved, sizeof(InstState), hipMemcpyHostToDevice, st));
  EP_HIP(hipStreamSynchronize(st));
  EP_HIP(err);
  if (short_run) return fail(EP_ESTATE, "a timed iteration stopped early (breakdown)");
  *us_per_launch = 1e3 * ms_total / reps;
  return EP_OK;
}

ep_status ep_sim_time_kernel(ep_sim* s, int kind, int reps, double* us_per_launch) {
  if (check_sim(s) || reps < 1 || !us_per_launch) return fail(EP_EINVAL, "bad time-kernel arguments");
  if (kind != EP_K_RHS && kind != EP_K_CG_SPMV && kind != EP_K_CG_PIPE)
    return fail(EP_EINVAL, "only the rhs, SpMV and pipelined CG kernels can be timed");
  if (!s->finalized) return fail(EP_ESTATE, "finalize first");
  if (s->in_pool) return fail(EP_ESTATE, "sim is stepped by its pool");
  EP_HIP(hipSetDevice(s->device));
  hipStream_t st = s->stream;
  EP_HIP(hipStreamSynchronize(st));
  EP_HIP(hipMemcpyAsync(s->h_st, s->d_st, sizeof(InstState), hipMemcpyDeviceToHost, st));
  EP_HIP(hipStreamSynchronize(st));
  // between steps the solve-control flags are clear, so both kernels do their
  // full work; everything they write is recomputed by the next step
  if (s->h_st->conv || s->h_st->conv_in || s->h_st->restart) return fail(EP_ESTATE, "a step is in progress");
  if (kind == EP_K_CG_PIPE) return time_pipe(s, reps, us_per_launch);
  const Launch L = launch_of(s);
  const bool mixed = s->prec == EP_MIXED;
  hipEvent_t a = nullptr, b = nullptr;
  EP_HIP(hipEventCreate(&a));
  EP_HIP(hipEventCreate(&b));
  EP_HIP(hipEventRecord(a, st));
  for (int k = 0; k < reps; k++) {
    if (kind == EP_K_CG_SPMV) launch_cg_spmv(mixed, L);
    else launch_residual(mixed, true, L);
  }
  EP_HIP(hipGetLastError());
  EP_HIP(hipEventRecord(b, st));
  EP_HIP(hipEventSynchronize(b));
  float ms = 0.0f;
  EP_HIP(hipEventElapsedTime(&ms, a, b));
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  *us_per_launch = 1e3 * (double)ms / reps;
  return EP_OK;
}

void ep_sim_destroy(ep_sim* s) {
  if (!s) return;
  // a pooled sim leaves its pool first, so that the pool's table never
  // points at freed memory
  if (s->in_pool && s->pool) (void)ep_pool_release(s->pool, s->pool_slot, nullptr);
  (void)hipSetDevice(s->device);
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  s->kt.destroy();
  s->graphs.reset();
  for (auto& e : s->ev)
    if (e) (void)hipEventDestroy(e);
  s->mem.release();
  if (s->h_st) (void)hipHostFree(s->h_st);
  if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
  delete s;
}

ep_status ep_cell_pace(int device, int model, int variant, int n_cells, const double* params, int n_params,
                       const double* init, double dt_ms, int bdf_order, double period_ms, double stim_mV_per_ms,
                       double stim_dur_ms, int n_beats, double* out) {
  if (model < EP_PASSIVE || model > EP_TTP06) return fail(EP_EINVAL, "unknown ionic model");
  if (model == EP_TTP06 && (variant < 0 || variant > 2)) return fail(EP_EINVAL, "bad TTP06 cell type");
  if (n_cells < 1 || !out || !(dt_ms > 0) || bdf_order < 1 || bdf_order > 3 || !(period_ms > 0) ||
      !(stim_dur_ms >= 0) || n_beats < 0 || n_params < 0 || n_params > n_model_params(model) ||
      (n_params > 0 && !params))
    return fail(EP_EINVAL, "bad pacing arguments");
  int count = 0;
  EP_HIP(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) return fail(EP_EINVAL, "no such device");
  EP_HIP(hipSetDevice(device));
  const ModelInfo mi = model_info(model);
  const int nv = mi.nvars, nc = n_cells;
  // per-cell parameters: defaults of (model, variant), then the caller's overrides
  std::vector<double> mp((size_t)nc * NPARAM);
  for (int c = 0; c < nc; c++) {
    default_params(model, variant, &mp[(size_t)c * NPARAM]);
    for (int k = 0; k < n_params; k++) mp[(size_t)c * NPARAM + k] = params[(size_t)c * n_params + k];
  }
  const std::vector<double> ic = default_init(model);
  std::vector<double> uh((size_t)3 * nc), w((size_t)std::max(nv, 1) * nc, 0.0);
  for (int c = 0; c < nc; c++) {
    const double* row = init ? init + (size_t)c * (1 + nv) : ic.data();
    for (int k = 0; k < 3; k++) uh[(size_t)k * nc + c] = row[0];
    for (int v = 0; v < nv; v++) w[(size_t)v * nc + c] = row[1 + v];
  }
  DevMem m;
  struct Guard {
    DevMem& m;
    hipStream_t s = nullptr;
    ~Guard() {
      if (s) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
      }
      m.release();
    }
  } guard{m};
  EP_HIP(hipStreamCreateWithFlags(&guard.s, hipStreamNonBlocking));
  hipStream_t st = guard.s;
  double *d_uh, *d_w, *d_mp;
  EP_HIP(upload(m, &d_uh, uh.data(), uh.size(), st));
  EP_HIP(upload(m, &d_w, w.data(), w.size(), st));
  EP_HIP(upload(m, &d_mp, mp.data(), mp.size(), st));
  const int64_t period = std::max<int64_t>(1, (int64_t)std::llround(period_ms / dt_ms));
  const int64_t dur = (int64_t)std::llround(stim_dur_ms / dt_ms);
  const int64_t total = (int64_t)n_beats * period;
  const int64_t chunk = 20000;  // bounds each launch's duration
  for (int64_t s0 = 0; s0 < total; s0 += chunk) {
    launch_cell_pace(model, d_uh, d_w, d_mp, nc, dt_ms, bdf_order, s0, std::min(chunk, total - s0), period, dur,
                     stim_mV_per_ms / mi.mv_per_unit, st);
    EP_HIP(hipGetLastError());
  }
  EP_HIP(hipMemcpyAsync(uh.data(), d_uh, uh.size() * 8, hipMemcpyDeviceToHost, st));
  EP_HIP(hipMemcpyAsync(w.data(), d_w, w.size() * 8, hipMemcpyDeviceToHost, st));
  EP_HIP(hipStreamSynchronize(st));
  bool nan = false;
  for (int c = 0; c < nc; c++) {
    out[(size_t)c * (1 + nv)] = uh[c];
    nan |= !(uh[c] == uh[c]);
    for (int v = 0; v < nv; v++) out[(size_t)c * (1 + nv) + 1 + v] = w[(size_t)v * nc + c];
  }
  if (nan) return fail(EP_ENAN, "a paced cell produced NaN");
  return EP_OK;
}

ep_status ep_cell_pace_device(int device, void* hip_stream, int model, int variant, int n_cells, const double* params,
                              int n_params, const double* init, double dt_ms, int bdf_order, double period_ms,
                              double stim_mV_per_ms, double stim_dur_ms, int n_beats, double* out) {
  if (model < EP_PASSIVE || model > EP_TTP06) return fail(EP_EINVAL, "unknown ionic model");
  if (model == EP_TTP06 && (variant < 0 || variant > 2)) return fail(EP_EINVAL, "bad TTP06 cell type");
  if (n_cells < 1 || !out || !(dt_ms > 0) || bdf_order < 1 || bdf_order > 3 || !(period_ms > 0) ||
      !(stim_dur_ms >= 0) || n_beats < 0 || n_params < 0 || n_params > n_model_params(model) ||
      (n_params > 0 && !params))
    return fail(EP_EINVAL, "bad pacing arguments");
  if (n_cells > PACE_MAX_CELLS)
    return fail(EP_EINVAL, "ep_cell_pace_device: more than " + std::to_string(PACE_MAX_CELLS) +
                               " cells (the size of its fixed device scratch); use ep_cell_pace");
  int count = 0;
  EP_HIP(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) return fail(EP_EINVAL, "no such device");
  EP_HIP(hipSetDevice(device));
  double* base = nullptr;
  EP_HIP(pace_scratch(device, &base));
  const ModelInfo mi = model_info(model);
  const int nv = mi.nvars, nc = n_cells;
  PaceDefaults def{};
  default_params(model, variant, def.mp);
  const std::vector<double> ic = default_init(model);
  for (size_t k = 0; k < ic.size() && k < 19; k++) def.init[k] = ic[k];
  // scratch layout: uh [3][nc], w [18][nc], parameter rows [nc][NPARAM]
  double* d_uh = base;
  double* d_w = d_uh + (size_t)3 * nc;
  double* d_mp = d_w + (size_t)18 * nc;
  hipStream_t st = (hipStream_t)hip_stream;
  launch_pace_stage(def, n_params > 0 ? params : nullptr, n_params, init, nv, nc, d_uh, d_w, d_mp, st);
  EP_HIP(hipGetLastError());
  const int64_t period = std::max<int64_t>(1, (int64_t)std::llround(period_ms / dt_ms));
  const int64_t dur = (int64_t)std::llround(stim_dur_ms / dt_ms);
  const int64_t total = (int64_t)n_beats * period;
  const int64_t chunk = 20000;  // bounds each launch's duration
  for (int64_t s0 = 0; s0 < total; s0 += chunk) {
    launch_cell_pace(model, d_uh, d_w, d_mp, nc, dt_ms, bdf_order, s0, std::min(chunk, total - s0), period, dur,
                     stim_mV_per_ms / mi.mv_per_unit, st);
    EP_HIP(hipGetLastError());
  }
  launch_pace_unstage(d_uh, d_w, nv, nc, out, st);
  EP_HIP(hipGetLastError());
  return EP_OK;
}

ep_status ep_assemble_csr(int elem, int64_t n_nodes, const double* xyz, int64_t n_elems, const int32_t* conn,
                          const double* f0, const double* s0, const double* n0, double sl, double st, double sn,
                          double chi, double cm, int64_t* nnz_out, int64_t* rowptr, int32_t* col, double* valM,
                          double* valK) {
  if (!xyz || !conn || !nnz_out) return fail(EP_EINVAL, "null argument");
  Csr A;
  std::vector<char> err;
  if (!assemble_csr(elem, n_nodes, xyz, n_elems, conn, f0, s0, n0, sl, st, sn, chi, cm, A, err))
    return fail(EP_EINVAL, std::string("assembly: ") + (err.empty() ? "failed" : err.data()));
  *nnz_out = A.nnz();
  if (!rowptr) return EP_OK;
  if (!col || !valM || !valK) return fail(EP_EINVAL, "null output array");
  std::copy(A.rowptr.begin(), A.rowptr.end(), rowptr);
  std::copy(A.col.begin(), A.col.end(), col);
  std::copy(A.valM.begin(), A.valM.end(), valM);
  std::copy(A.valK.begin(), A.valK.end(), valK);
  return EP_OK;
}


}  // extern "C"

// ============================================================================
// Batched / serving pool.  Resident simulations share one descriptor table;
// every phase of a step is one launch over all active instances (per ionic
// model for the ionic kernel), each instance converging on its own.
// ============================================================================

struct ep_pool {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  size_t budget = 0, in_use = 0;
  int max_slots = 0;
  int prec = EP_FP64;
  struct Slot {
    ep_sim* sim = nullptr;
    int64_t target = 0;
    int64_t done_steps = 0;
    bool done = false;
    int status = EP_OK;
  };
  std::vector<Slot> slots;
  InstDesc* d_table = nullptr;
  InstState* h_states = nullptr;  // pinned, one per slot
  DevMem mem;                     // table
  DevMem maps;                    // launch tables, rebuilt on membership change
  bool dirty = true;
  std::vector<int> active;
  BlockMap* d_all = nullptr;
  int nb_all = 0;
  // ionic launches per (model, ionic precision, ionic scheme): index
  // 4 * model + 2 * (FP32 ionic) + scheme
  BlockMap* d_model[16] = {};
  int nb_model[16] = {};
  int32_t* d_ids = nullptr;
  // instances with several subdomains: their ionic step runs per instance
  // (ionic points, interface correction) instead of in the model groups
  std::vector<int> het_slots;
  int it_pred = 8;
  SweepPredictor sweeps;  // mixed: rounds per sweep (largest over the instances)
  KernelTimers kt;
  int ionic_npt = 1, list_order = 0, use_graph = 0;  // launch shapes (EP_OPT_*)
  StepGraphs graphs;
  // CG formulations among the active members: the pool launches the kernels
  // of each one present (the kernels of one form skip the other's members)
  bool has_pipe = false, has_cgg = false;
  bool all_dia14 = false;   // every active member: 14-diagonal DIA, Jacobi (specialized kernels)
};

namespace {

// Workgroup -> (instance, tile) list in XCD order: each die receives a
// contiguous run of the list; padding entries carry lblk = -1.
std::vector<BlockMap> xcd_order(const std::vector<BlockMap>& items) {
  const int T = (int)items.size();
  const int per = (T + N_XCD - 1) / N_XCD;
  std::vector<BlockMap> out((size_t)per * N_XCD, BlockMap{items.empty() ? 0 : items[0].inst, -1});
  for (int b = 0; b < per * N_XCD; b++) {
    const int t = (b % N_XCD) * per + b / N_XCD;
    if (t < T) out[b] = items[t];
  }
  return out;
}

ep_status pool_rebuild(ep_pool* P) {
  // kernels of the previous step may still read the old tables
  EP_HIP(hipStreamSynchronize(P->stream));
  P->graphs.reset();
  P->maps.release();
  P->active.clear();
  for (int k = 0; k < P->max_slots; k++)
    if (P->slots[k].sim && !P->slots[k].done) P->active.push_back(k);
  P->has_pipe = P->has_cgg = false;
  P->all_dia14 = !P->active.empty();
  for (int k : P->active) {
    const InstDesc& D = P->slots[k].sim->desc;
    (D.cg_pipe ? P->has_pipe : P->has_cgg) = true;
    if (!(D.fmt == FMT_DIA && D.nup == 14 && D.block == 1)) P->all_dia14 = false;
  }
  std::vector<BlockMap> all, per_model[16];
  P->het_slots.clear();
  for (int k : P->active) {
    const ep_sim* s = P->slots[k].sim;
    const int nt = s->desc.nblk;
    if (s->het) P->het_slots.push_back(k);
    for (int t = 0; t < nt; t++) {
      all.push_back(BlockMap{k, t});
      if (!s->het) per_model[4 * s->model + 2 * (s->ionic_f32() ? 1 : 0) + s->ionic_scheme].push_back(BlockMap{k, t});
    }
  }
  auto put = [&](const std::vector<BlockMap>& v, BlockMap** d, int* nb) -> hipError_t {
    *nb = 0;
    *d = nullptr;
    if (v.empty()) return hipSuccess;
    std::vector<BlockMap> o = P->list_order ? v : xcd_order(v);
    *nb = (int)o.size();
    hipError_t e = P->maps.alloc((void**)d, o.size() * sizeof(BlockMap));
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(*d, o.data(), o.size() * sizeof(BlockMap), hipMemcpyHostToDevice, P->stream);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(P->stream);
  };
  EP_HIP(put(all, &P->d_all, &P->nb_all));
  for (int m = 0; m < 16; m++) EP_HIP(put(per_model[m], &P->d_model[m], &P->nb_model[m]));
  std::vector<int32_t> ids(P->active.begin(), P->active.end());
  if (!ids.empty()) {
    EP_HIP(P->maps.alloc((void**)&P->d_ids, ids.size() * sizeof(int32_t)));
    EP_HIP(hipMemcpyAsync(P->d_ids, ids.data(), ids.size() * sizeof(int32_t), hipMemcpyHostToDevice, P->stream));
    EP_HIP(hipStreamSynchronize(P->stream));
  }
  P->dirty = false;
  return EP_OK;
}

ep_status pool_pull(ep_pool* P) {
  EP_HIP(hipMemcpy2DAsync(P->h_states, sizeof(InstState), P->d_table, sizeof(InstDesc), sizeof(InstState),
                          (size_t)P->max_slots, hipMemcpyDeviceToHost, P->stream));
  EP_HIP(hipStreamSynchronize(P->stream));
  return EP_OK;
}

bool pool_all_conv(ep_pool* P) {
  for (int k : P->active)
    if (!P->h_states[k].conv) return false;
  return true;
}

int pool_iters(ep_pool* P) {
  int m = 0;
  for (int k : P->active) m = std::max(m, P->h_states[k].it_step);
  return m;
}

ep_status pool_step_once(ep_pool* P) {
  const bool mixed = P->prec == EP_MIXED;
  const bool pipe = P->has_pipe, cgg = P->has_cgg;
  const int ni = (int)P->active.size();
  Launch L{P->d_table, P->d_all, P->nb_all, P->stream, false};
  L.ionic_npt = P->ionic_npt;
  L.pipe_op = P->all_dia14 ? 1 : 0;
  KernelTimers& kt = P->kt;
  hipStream_t st = P->stream;
  auto fin = [&] { kt.timed(st, 6, [&] { launch_cg_finalize(mixed, P->d_table, P->d_ids, ni, st); }); };
  auto round = [&] {
    if (pipe) kt.timed(st, 7, [&] { mixed ? launch_cg_pipe32(L) : launch_cg_pipe(L); });
    if (!cgg) return;
    if (!mixed) {
      kt.timed(st, 2, [&] { launch_cg_spmv(false, L); });
      kt.timed(st, 3, [&] { launch_cg_update64(L); });
      return;
    }
    kt.timed(st, 3, [&] { launch_cg_update(mixed, L); });
    kt.timed(st, 2, [&] { launch_cg_spmv(mixed, L); });
    fin();
  };
  auto pro = [&] {
    kt.timed(st, 0, [&] {
      for (int m = 0; m < 16; m++)
        if (P->nb_model[m] > 0) {
          Launch Lm{P->d_table, P->d_model[m], P->nb_model[m], st, false};
          Lm.ionic_npt = P->ionic_npt;
          Lm.ionic_bdf = (m & 1) != 0;
          launch_ionic(m / 4, (m & 2) != 0, Lm);
        }
      for (int k : P->het_slots) {
        const ep_sim* s = P->slots[k].sim;
        launch_ionic_het(s->het_model, s->ionic_f32(), s->ionic_scheme == EP_IONIC_BDF, P->d_table + k, s->n_pts, st);
        launch_ici_correction(P->d_table + k, s->n_crow, st);
      }
    });
    kt.timed(st, 1, [&] { launch_residual(mixed, true, L); });
    if (pipe) kt.timed(st, 2, [&] { mixed ? launch_cg_pipe32_start(L) : launch_cg_pipe_start(L); });
    if (cgg && mixed) {
      kt.timed(st, 2, [&] { launch_cg_spmv(mixed, L); });
      fin();
    }
  };
  auto ir = [&] {
    kt.timed(st, 5, [&] { launch_residual(true, false, L); });
    if (pipe) {
      // the start and the sweep's first iteration, which takes the outer
      // decision, so the host's next read sees it
      kt.timed(st, 2, [&] { launch_cg_pipe32_start(L); });
      kt.timed(st, 7, [&] { launch_cg_pipe32(L); });
    }
    if (cgg) {
      kt.timed(st, 2, [&] { launch_cg_spmv(true, L); });
      fin();
    }
  };
  auto epi = [&] {
    kt.timed(st, 4, [&] { launch_activation(L); });
    launch_end_step(P->d_table, P->d_ids, ni, st);
  };
  const bool graph = P->use_graph && !kt.on;
  StepGraphs& G = P->graphs;
  if (graph && !G.valid) {
    G.reset();
    EP_HIP(capture_graph(st, pro, &G.pro));
    EP_HIP(capture_graph(st, round, &G.round1));
    EP_HIP(capture_graph(st, [&] { round(); round(); }, &G.round2));
    if (mixed) EP_HIP(capture_graph(st, ir, &G.ir));
    EP_HIP(capture_graph(st, epi, &G.epi));
    G.valid = true;
  }
  auto rounds = [&](int c) -> hipError_t {
    if (!graph) {
      for (int k = 0; k < c; k++) round();
      return hipGetLastError();
    }
    for (; c >= 2; c -= 2) {
      hipError_t e = hipGraphLaunch(G.round2, st);
      if (e != hipSuccess) return e;
    }
    return c ? hipGraphLaunch(G.round1, st) : hipSuccess;
  };
  if (graph) EP_HIP(hipGraphLaunch(G.pro, st));
  else pro();
  // mixed: sweep index = the smallest refinement count over the instances not
  // yet converged; its rounds are predicted from the slowest instance
  int chunk = std::max(1, mixed ? P->sweeps.rounds(0) : P->it_pred + 1);
  int sweep = 0, sweep_start = 0;
  for (int n_rounds = 0;; n_rounds++) {
    EP_HIP(rounds(chunk));
    if (mixed) {
      if (graph) EP_HIP(hipGraphLaunch(G.ir, st));
      else ir();
    }
    ep_status rc = pool_pull(P);
    if (rc != EP_OK) return rc;
    if (P->kt.on) P->kt.harvest();
    if (mixed) {
      int outer = 1 << 30, it_now = 0;
      for (int k : P->active) {
        const InstState& S = P->h_states[k];
        if (!S.conv) outer = std::min(outer, S.outer);
        it_now = std::max(it_now, S.it_step);
      }
      const bool all = pool_all_conv(P);
      if (all || outer > sweep) {
        P->sweeps.learn(sweep, it_now - sweep_start);
        sweep = all ? sweep + 1 : outer;
        sweep_start = it_now;
        chunk = P->sweeps.rounds(sweep);
      } else {
        chunk = 2;
      }
    }
    if (pool_all_conv(P)) break;
    if (n_rounds > 20000) return fail(EP_EHIP, "pool solver control lost (no convergence flag)");
    if (!mixed) chunk = 2;
  }
  if (!mixed) P->it_pred = std::max(1, pool_iters(P));
  if (graph) EP_HIP(hipGraphLaunch(G.epi, st));
  else epi();
  EP_HIP(hipGetLastError());
  bool changed = false;
  for (int k : P->active) {
    ep_pool::Slot& sl = P->slots[k];
    sl.done_steps += 1;
    const int fl = P->h_states[k].flags;
    if (fl & F_NAN) {
      sl.status = EP_ENAN;
      sl.done = true;
      changed = true;
    } else if (fl & (F_NOCONV | F_BREAKDOWN)) {
      sl.status = EP_ENOCONV;
    }
    if (sl.done_steps >= sl.target && !sl.done) {
      sl.done = true;
      changed = true;
    }
  }
  if (changed) P->dirty = true;
  return EP_OK;
}

}  // namespace

extern "C" {

ep_status ep_pool_create(int device, void* hip_stream, size_t hbm_budget_bytes, int max_slots, int precision,
                         ep_pool** out) {
  if (!out || max_slots < 1 || max_slots > 4096 || (precision != EP_FP64 && precision != EP_MIXED))
    return fail(EP_EINVAL, "bad pool arguments");
  *out = nullptr;
  int count = 0;
  EP_HIP(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) return fail(EP_EINVAL, "no such device");
  EP_HIP(hipSetDevice(device));
  ep_pool* P = new ep_pool();
  P->device = device;
  P->budget = hbm_budget_bytes;
  P->max_slots = max_slots;
  P->prec = precision;
  P->slots.resize(max_slots);
  if (hip_stream) {
    P->stream = (hipStream_t)hip_stream;
  } else if (hipStreamCreateWithFlags(&P->stream, hipStreamNonBlocking) != hipSuccess) {
    delete P;
    return fail(EP_EHIP, "hipStreamCreate failed");
  } else {
    P->own_stream = true;
  }
  if (P->mem.alloc((void**)&P->d_table, (size_t)max_slots * sizeof(InstDesc)) != hipSuccess ||
      hipHostMalloc((void**)&P->h_states, (size_t)max_slots * sizeof(InstState), hipHostMallocDefault) != hipSuccess) {
    P->mem.release();
    if (P->own_stream) (void)hipStreamDestroy(P->stream);
    delete P;
    return fail(EP_ENOMEM, "pool table allocation failed");
  }
  std::memset(P->h_states, 0, (size_t)max_slots * sizeof(InstState));
  *out = P;
  return EP_OK;
}

ep_status ep_pool_admit(ep_pool* P, ep_sim* s, int64_t n_steps_total, int* slot) {
  if (!P || !s || !slot || n_steps_total < 1) return fail(EP_EINVAL, "bad admit arguments");
  if (s->in_pool) return fail(EP_ESTATE, "sim already belongs to a pool");
  if (s->prec != P->prec) return fail(EP_EINVAL, "sim precision differs from the pool's");
  if (s->fmt_pref == EP_FMT_MF || (s->finalized && s->desc.fmt == FMT_MF))
    return fail(EP_EINVAL, "matrix-free sims are not admitted to pools");
  if (s->device != P->device) return fail(EP_EINVAL, "sim device differs from the pool's");
  int free_slot = -1;
  for (int k = 0; k < P->max_slots; k++)
    if (!P->slots[k].sim) {
      free_slot = k;
      break;
    }
  // a sim finalized beforehand (set up on its own stream, e.g. by another
  // thread while the pool steps) is only linked into the table
  const size_t need = s->finalized ? s->mem.bytes : estimate_bytes(s);
  if (free_slot < 0 || P->in_use + need > P->budget) return fail(EP_EAGAIN, "pool full (slots or HBM budget)");
  EP_HIP(hipSetDevice(P->device));
  if (s->finalized) EP_HIP(hipStreamSynchronize(s->stream));   // its setup copies are done
  // the sim runs on the pool's stream while pooled
  s->stream_own = s->stream;
  s->stream = P->stream;
  if (!s->finalized) {
    ep_status rc = finalize_impl(s);
    if (rc != EP_OK) {
      if (!s->finalized) s->mem.release();
      s->stream = s->stream_own;
      return rc;
    }
  }
  InstDesc* dst = P->d_table + free_slot;
  EP_HIP(hipMemcpyAsync(dst, s->d_desc_own, sizeof(InstDesc), hipMemcpyDeviceToDevice, P->stream));
  EP_HIP(hipStreamSynchronize(P->stream));
  s->d_desc = dst;
  s->d_st = reinterpret_cast<InstState*>(reinterpret_cast<char*>(dst) + offsetof(InstDesc, st));
  s->graphs.reset();
  s->in_pool = true;
  s->pool_slot = free_slot;
  s->pool = P;
  ep_pool::Slot& sl = P->slots[free_slot];
  sl.sim = s;
  sl.target = n_steps_total;
  sl.done_steps = 0;
  sl.done = false;
  sl.status = EP_OK;
  P->in_use += std::max(need, s->mem.bytes);
  P->dirty = true;
  *slot = free_slot;
  return EP_OK;
}

ep_status ep_pool_step(ep_pool* P, int n_steps) {
  if (!P || n_steps < 0) return fail(EP_EINVAL, "bad pool step arguments");
  EP_HIP(hipSetDevice(P->device));
  for (int k = 0; k < n_steps; k++) {
    if (P->dirty) {
      ep_status rc = pool_rebuild(P);
      if (rc != EP_OK) return rc;
    }
    if (P->active.empty()) break;
    ep_status rc = pool_step_once(P);
    if (rc != EP_OK) return rc;
  }
  return EP_OK;
}

ep_status ep_pool_poll(ep_pool* P, int* done_slots, int cap, int* n_done) {
  if (!P || !n_done || (cap > 0 && !done_slots)) return fail(EP_EINVAL, "bad poll arguments");
  int c = 0;
  for (int k = 0; k < P->max_slots; k++)
    if (P->slots[k].sim && P->slots[k].done) {
      if (c < cap) done_slots[c] = k;
      c++;
    }
  *n_done = std::min(c, std::max(cap, 0));
  return EP_OK;
}

ep_status ep_pool_release(ep_pool* P, int slot, ep_sim** sim_out) {
  if (!P || slot < 0 || slot >= P->max_slots || !P->slots[slot].sim) return fail(EP_EINVAL, "no sim in that slot");
  ep_sim* s = P->slots[slot].sim;
  EP_HIP(hipStreamSynchronize(P->stream));
  EP_HIP(hipMemcpyAsync(s->d_desc_own, P->d_table + slot, sizeof(InstDesc), hipMemcpyDeviceToDevice, P->stream));
  EP_HIP(hipStreamSynchronize(P->stream));
  s->d_desc = s->d_desc_own;
  s->d_st = reinterpret_cast<InstState*>(reinterpret_cast<char*>(s->d_desc) + offsetof(InstDesc, st));
  s->graphs.reset();
  s->stream = s->stream_own;
  s->in_pool = false;
  s->pool_slot = -1;
  s->pool = nullptr;
  const size_t need = estimate_bytes(s);
  P->in_use -= std::min(P->in_use, std::max(need, s->mem.bytes));
  const int status = P->slots[slot].status;
  P->slots[slot] = ep_pool::Slot{};
  P->dirty = true;
  if (sim_out) *sim_out = s;
  if (status != EP_OK) {
    g_err = status == EP_ENAN ? "the simulation produced NaN" : "a linear solve did not converge";
    return (ep_status)status;
  }
  return EP_OK;
}

ep_status ep_pool_get_info(ep_pool* P, int* n_active, size_t* bytes_in_use) {
  if (!P) return fail(EP_EINVAL, "null pool");
  int a = 0;
  for (auto& sl : P->slots)
    if (sl.sim && !sl.done) a++;
  if (n_active) *n_active = a;
  if (bytes_in_use) *bytes_in_use = P->in_use;
  return EP_OK;
}

ep_status ep_pool_set_option(ep_pool* P, int key, double value) {
  if (!P) return fail(EP_EINVAL, "null pool");
  const int v = (int)value;
  if ((double)v != value) return fail(EP_EINVAL, "launch option values are integers");
  if (key == EP_OPT_IONIC_NPT) {
    if (v != 1 && v != 2 && v != 4) return fail(EP_EINVAL, "ionic nodes per thread: 1, 2 or 4");
  } else if (key == EP_OPT_TILE_MAP || key == EP_OPT_GRAPH) {
    if (v != 0 && v != 1) return fail(EP_EINVAL, "option value: 0 or 1");
  } else {
    return fail(EP_EINVAL, "unknown pool option");
  }
  EP_HIP(hipSetDevice(P->device));
  EP_HIP(hipStreamSynchronize(P->stream));
  if (key == EP_OPT_IONIC_NPT) P->ionic_npt = v;
  if (key == EP_OPT_GRAPH) P->use_graph = v;
  if (key == EP_OPT_TILE_MAP && P->list_order != v) {
    P->list_order = v;
    P->dirty = true;
  }
  P->graphs.reset();
  return EP_OK;
}

ep_status ep_pool_autotune(ep_pool* P, int trial_steps, int* ionic_npt, int* tile_map) {
  if (!P || trial_steps < 1) return fail(EP_EINVAL, "bad autotune arguments");
  EP_HIP(hipSetDevice(P->device));
  EP_HIP(hipStreamSynchronize(P->stream));
  KernelTimers& kt = P->kt;
  kt.harvest();
  kt.on = 1;
  auto step = [&]() -> ep_status {
    if (P->dirty) {
      ep_status rc = pool_rebuild(P);
      if (rc != EP_OK) return rc;
    }
    if (P->active.empty()) return EP_OK;
    return pool_step_once(P);
  };
  int npt = P->ionic_npt, lo = P->list_order;
  ep_status rc = tune_one(
      kt, P->stream, trial_steps, {1, 2, 4}, [&](int c) { P->ionic_npt = c; }, step,
      [](const TimerSums& a, const TimerSums&) { return a.avg_us(0); }, &npt);
  if (rc == EP_OK)
    rc = tune_one(
        kt, P->stream, trial_steps, {0, 1},
        [&](int c) {
          if (P->list_order != c) {
            P->list_order = c;
            P->dirty = true;
          }
        },
        step, [](const TimerSums& a, const TimerSums& all) { return tile_kernels_us(a, all); }, &lo);
  kt.zero();
  kt.on = 0;
  P->graphs.reset();
  if (rc != EP_OK) return rc;
  if (ionic_npt) *ionic_npt = npt;
  if (tile_map) *tile_map = lo;
  return EP_OK;
}

void ep_pool_destroy(ep_pool* P) {
  if (!P) return;
  (void)hipSetDevice(P->device);
  (void)hipStreamSynchronize(P->stream);
  for (int k = 0; k < P->max_slots; k++)
    if (P->slots[k].sim) (void)ep_pool_release(P, k, nullptr);
  P->graphs.reset();
  P->kt.destroy();
  P->maps.release();
  P->mem.release();
  if (P->h_states) (void)hipHostFree(P->h_states);
  if (P->own_stream) (void)hipStreamDestroy(P->stream);
  delete P;
}

}  // extern "C"
