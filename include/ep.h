/*
 * ep.h -- C ABI of the MI355X monodomain time-step library (libep_mi355x.so).
 *
 * What it computes (Africa et al., "lifex-ep", Section "Cardiac
 * electrophysiology: numerical discretization"): the monodomain equation
 * (eq. of the monodomain model, one subdomain, homogeneous Neumann boundary)
 * discretized in space by linear finite elements (Q1 hexahedra or P1
 * tetrahedra) and in time by the BDF/IMEX scheme of the same section:
 *   1. ionic step at every node, evaluated at the extrapolated potential
 *      u_EXT (eq. of the time-discrete ionic model): gating variables by
 *      Rush-Larsen, other variables by one explicit step;
 *   2. linear monodomain step (eq. of the time-discrete monodomain equation
 *      and the algebraic linear system that follows it):
 *        (alpha/dt M + K) u_{n+1} = M (u_BDF/dt + I_app - I_ion),
 *      with the ionic current interpolated from nodal values (ICI), solved by
 *      Jacobi-preconditioned CG in FP64, or by FP32 CG inside FP64 iterative
 *      refinement (mixed precision);
 *   3. activation time = time of the largest du/dt at each node (Section
 *      "Slab benchmark").
 * Units: mm, ms, mV, mS/mm, 1/mm, uF/mm^2, uA/mm^3.
 *
 * Conventions
 *   - Every call returns ep_status; ep_last_error() gives a message for the
 *     last non-OK status on the calling thread.  No C++ exception crosses
 *     this interface.
 *   - Host input arrays are borrowed for the duration of the call and copied.
 *     Host output arrays are caller-allocated with the sizes stated.
 *   - All device memory is owned by the library, except the `dst` of
 *     ep_sim_get_potential_device, which the caller owns (e.g. a torch tensor).
 *   - An ep_sim is not thread-safe; different sims may be used from
 *     different threads.
 *   - Work is enqueued on the sim's HIP stream.  Errors raised on the device
 *     (non-convergence, NaN) are reported by the next call that synchronizes.
 */
#ifndef EP_MI355X_H
#define EP_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ep_sim ep_sim;
typedef struct ep_pool ep_pool;

typedef enum {
  EP_OK = 0,
  EP_EINVAL = -1,   /* invalid argument or call order                        */
  EP_ENOMEM = -2,   /* device or host allocation failed                      */
  EP_EHIP = -3,     /* HIP runtime error (no device, launch failure, ...)    */
  EP_ENOCONV = -4,  /* a linear solve hit max_it; the step kept its iterate  */
  EP_ENAN = -5,     /* NaN in the solution; stepping stopped                 */
  EP_EAGAIN = -6,   /* pool full (HBM budget or slots); retry after release  */
  EP_ESTATE = -7    /* call not valid in the object's current state          */
} ep_status;

/* element types: tetrahedra of degree 1, 2; hexahedra of degree p = 1..6
 * ((p + 1)^3 nodes) */
enum { EP_TET4 = 4, EP_TET10 = 10, EP_HEX8 = 8, EP_HEX27 = 27, EP_HEX64 = 64, EP_HEX125 = 125,
       EP_HEX216 = 216, EP_HEX343 = 343 };
enum { EP_PASSIVE = 0, EP_AP = 1, EP_BO = 2, EP_TTP06 = 3 };          /* ionic models    */
enum { EP_CELL_EPI = 0, EP_CELL_ENDO = 1, EP_CELL_MID = 2 };          /* TTP06 variants  */
enum { EP_CUBE = 0, EP_SPHERE = 1, EP_GAUSS = 2 };                    /* stimulus shapes */
enum { EP_FP64 = 0, EP_MIXED = 1 };                                   /* precision       */
enum { EP_JACOBI = 0, EP_BJACOBI = 1 };                               /* preconditioner  */
enum { EP_DTYPE_F64 = 0, EP_DTYPE_F32 = 1 };
enum { EP_FMT_AUTO = 0, EP_FMT_SELL = 1, EP_FMT_DIA = 2, EP_FMT_MF = 3 };  /* operator format */

/* Options for ep_sim_set_option (before finalize unless stated). */
enum {
  EP_OPT_MATRIX_FORMAT = 1, /* EP_FMT_*; AUTO picks DIA when it moves fewer bytes than
                             * SELL.  EP_FMT_MF: no assembled operator on the device;
                             * hexahedra of degree 2 or 3 (EP_HEX27, EP_HEX64), FP64,
                             * one subdomain, Jacobi, not in pools (EP_EINVAL at
                             * finalize otherwise): the operator is applied element by
                             * element by sum factorization on the Gauss points of the
                             * assembly (paper: matrix-free high-order solvers on GPUs) */
  EP_OPT_INNER_RTOL = 2,    /* mixed precision: inner FP32 CG relative tolerance (1e-4)  */
  EP_OPT_MAX_OUTER = 3,     /* mixed precision: max refinement sweeps per step (30)      */
  EP_OPT_PHASE_TIMERS = 4,  /* 1: time ionic / rhs / solve / activation phases (any time) */
  EP_OPT_KERNEL_TIMERS = 5, /* 1: bracket every kernel launch with HIP events and sum
                               their durations per kernel (any time; resets the sums) */
  /* Launch shapes (any time; also ep_pool_set_option).  They change which
   * thread or workgroup computes a node, never the arithmetic: results are
   * bitwise the same for every setting. */
  EP_OPT_IONIC_NPT = 6,     /* nodes per thread of the ionic kernel: 1 (512-thread
                               workgroups, default), 2 (256) or 4 (128)               */
  EP_OPT_TILE_MAP = 7,      /* 0: each XCD sweeps a contiguous range of 512-row tiles
                               (default); 1: workgroup b takes tile b; 2: on the
                               14-diagonal DIA of a Q1 hexahedral lattice, each XCD
                               takes the tiles of one band of lattice lines through
                               every plane (other operators run map 0)             */
  EP_OPT_GRAPH = 8,         /* 1: replay the step's launch sequences from captured
                               HIP graphs (ignored while timers are on).  The stream
                               must allow capture (not the legacy null stream).      */
  EP_OPT_IONIC_SCHEME = 9,  /* EP_IONIC_* (before finalize)                           */
  EP_OPT_IONIC_FP64 = 10,   /* mixed precision: 1 steps the ionic model (state and
                             * arithmetic) in FP64 while the inner CG stays FP32;
                             * 0 (default) FP32 (before finalize)                  */
  EP_OPT_CG_VARIANT = 11,   /* CG formulation, EP_CG_* (before finalize): of the FP64
                             * solve, or of the FP32 inner solve of each mixed-
                             * precision refinement sweep.  Both formulations are
                             * PCG with the same preconditioner; results agree to
                             * the solver tolerance, not bitwise.                 */
  EP_OPT_INITIAL_GUESS = 12 /* initial guess of each step's solve (before finalize):
                             * EP_X0_EXT (default; u_EXT, the reading the oracle
                             * uses) or EP_X0_EXTRAP3 (third-order extrapolation of
                             * the potential once three consistent levels exist:
                             * about 4 % fewer CG iterations on C1; not in the
                             * paper).  Changes results within the solver
                             * tolerance only.                                    */
};

/* FP64 CG formulations (EP_OPT_CG_VARIANT).  EP_CG_PIPELINED: one kernel per
 * iteration (the SpMV of m = P^-1 w, the global sums and all vector updates
 * of the pipelined recurrences; a reformulation of CG not in the paper, which
 * names the preconditioned CG solve).  Its extra recurrences (w = A u,
 * z = A q) carry rounding from iteration to iteration, which limits the
 * attainable residual on ill-conditioned systems: a degree-5 hexahedral
 * operator stalled above rtol 1e-13.  EP_CG_CHRONOPOULOS_GEAR: two kernels
 * per iteration (SpMV, then the fused update).  EP_CG_AUTO (default):
 * pipelined for linear elements (EP_HEX8, EP_TET4) when the iteration's data
 * (about 232 B per node in FP64, 124 B per node in the FP32 inner solve)
 * fits in 192 MB, three quarters of the GPU's 256 MB last-level cache;
 * Chronopoulos-Gear for larger meshes and higher degrees.  A pool may hold
 * members of both formulations: it launches the kernels of each one
 * present, and each kernel skips the other's members. */
enum { EP_CG_AUTO = 0, EP_CG_PIPELINED = 1, EP_CG_CHRONOPOULOS_GEAR = 2 };

/* Initial guesses (EP_OPT_INITIAL_GUESS). */
enum { EP_X0_EXT = 0, EP_X0_EXTRAP3 = 1 };

/* Ionic integrators (EP_OPT_IONIC_SCHEME).  EP_IONIC_RUSH_LARSEN (default):
 * gates by the exponential at u_EXT, other variables one explicit step.
 * EP_IONIC_BDF: the paper's time-discrete ionic model, (alpha w_{n+1} -
 * w_BDF)/dt = H(u_EXT, w_EXT, w_{n+1}) with the potential's BDF order, gates
 * implicit, other variables explicit (Aliev-Panfilov v implicit in its -v
 * term); it keeps three earlier levels of the ionic state (4x its memory).
 * ep_sim_set_state fills the earlier levels with copies of w. */
enum { EP_IONIC_RUSH_LARSEN = 0, EP_IONIC_BDF = 1 };

/* Kernel kinds reported by ep_sim_get_kernel_times. */
enum {
  EP_K_IONIC = 0,      /* ionic step + nodal right-hand side               */
  EP_K_RHS = 1,        /* b = M g and r0 = b - A x0 (dual SpMV)            */
  EP_K_CG_SPMV = 2,    /* w = A z with <w, z>                              */
  EP_K_CG_UPDATE = 3,  /* fused CG vector update with <r, z>, <r, r>       */
  EP_K_ACTIVATION = 4, /* activation-time tracking, end of step            */
  EP_K_IR_RESIDUAL = 5,/* FP64 refinement residual (mixed precision)       */
  EP_K_CG_FINALIZE = 6,/* per-instance reduction, convergence, step lengths */
  EP_K_CG_PIPE = 7     /* pipelined CG iteration (FP64; its start kernel,    */
                       /* w_0 = A u_0, counts as EP_K_CG_SPMV)               */
};
#define EP_N_KERNEL_KINDS 8

typedef struct ep_stats {
  int64_t n_nodes;
  int64_t nnz;              /* nonzeros of the assembled operator                   */
  int64_t steps;            /* completed time steps                                 */
  int64_t cg_iters_total;   /* CG iterations (inner iterations when mixed)         */
  int32_t cg_iters_last;    /* CG iterations of the last step                       */
  int32_t cg_iters_max;     /* largest per-step count                               */
  int64_t ir_sweeps_total;  /* mixed precision: FP64 refinement sweeps              */
  double rel_residual_last; /* ||b - A u||_2 / ||b||_2 at the end of the last solve */
  int32_t matrix_format;    /* EP_FMT_SELL, EP_FMT_DIA or EP_FMT_MF                  */
  int32_t n_diag;           /* DIA diagonals (0 for SELL)                           */
  int64_t device_bytes;     /* device memory held by the sim                        */
  double ms_ionic, ms_rhs, ms_solve, ms_activation; /* phase times (if enabled)     */
  double ms_setup;          /* host assembly + upload in ep_sim_finalize            */
  int32_t mf_compressed;    /* EP_FMT_MF: 1 if every element keeps 7 geometry
                               constants (affine elements with one diffusion
                               tensor), 0 if 7 factors per quadrature point      */
} ep_stats;

/* ---- simulation lifecycle -------------------------------------------------- */

/* Create a simulation on HIP device `device`.  hip_stream: a hipStream_t to
 * enqueue on (e.g. torch.cuda.current_stream().cuda_stream), or NULL for a
 * library-owned stream.  EP_EHIP if the device is not usable. */
ep_status ep_sim_create(int device, void* hip_stream, ep_sim** out);

/* Mesh (paper: tetrahedral or hexahedral conforming mesh).  xyz: [n_nodes][3]
 * coordinates in mm; conn: [n_elems][elem] node indices, hexahedra in
 * lexicographic corner order (corner a + 2b + 4c at reference (a, b, c)).
 * EP_HEX27 .. EP_HEX343: hexahedra of degree p = 2 .. 6 (paper: the
 * higher-order hexahedral Q_p spaces), node a + (p+1) b + (p+1)^2 c at
 * reference (a/p, b/p, c/p), e.g. a + 3b + 9c at (a/2, b/2, c/2) for p = 2.
 * EP_TET10: quadratic tetrahedra (paper: P2), vertices 0-3 then the nodes of
 * the edges 01, 02, 03, 12, 13, 23.  All higher-order elements are
 * isoparametric: edge nodes off the edge midpoints make a curved element;
 * finalize rejects (EP_EINVAL) an element whose map folds over.
 * Higher-order elements' operators are stored in the sliced-ELL format.
 * material_id: NULL (one subdomain) or [n_elems] subdomain labels 0 ..
 * EP_MAX_REGIONS - 1 (paper: Material IDs of the mesh's volumes; see
 * ep_sim_set_region).  EP_EINVAL on bad sizes or out-of-range indices or
 * labels (element geometry is checked in finalize). */
ep_status ep_sim_upload_mesh(ep_sim* sim, int elem, int64_t n_nodes, const double* xyz,
                             int64_t n_elems, const int32_t* conn, const int32_t* material_id);

#define EP_MAX_REGIONS 8

/* Settings of subdomain `region` (paper: the monodomain problem on several
 * subdomains with one ionic model each, eq. (2); per-subdomain parameter
 * overrides; "disable conduction" for scar).  Applies to the elements whose
 * material id is `region`; a region never set takes the sim's settings.
 *   variant: EP_CELL_* (TTP06 cell type) or -1 for the sim's;
 *   params / n_params: overrides of the model's first parameters as in
 *     ep_sim_set_ionic_model (NULL: the sim's parameters);
 *   sigma_l, sigma_t, sigma_n: conductivities in mS/mm (negative: the sim's);
 *   conductive: 0 removes the region from the problem (its elements do not
 *     enter M and K; nodes no other element uses drop out of the solve and
 *     report NaN; they count in n_nodes but carry no unknown).
 * The ionic state of a node on the interface of several subdomains is kept
 * once per subdomain and the ionic load is sum_i M^i I_ion^i exactly.  Both
 * ionic schemes (EP_OPT_IONIC_SCHEME) apply.  Call before finalize;
 * EP_EINVAL on a bad region, variant or parameter count. */
ep_status ep_sim_set_region(ep_sim* sim, int region, int variant, const double* params, int n_params,
                            double sigma_l, double sigma_t, double sigma_n, int conductive);

/* Ionic model of subdomain `region` (paper: eq. (2) gives every subdomain
 * Omega_i its own ionic model), EP_AP / EP_BO / EP_TTP06 / EP_PASSIVE, or -1
 * for the sim's model (the default).  The potential stays one field in the
 * sim model's units (u_mV = a u + b: TTP06 a = 1, b = 0; BO 85.7, -84; AP
 * 100, -80); a subdomain of another model is stepped at u_i = (a u + b -
 * b_i) / a_i and its current enters the load as (a_i / a) I_i.  The
 * subdomain's variant and parameter overrides (ep_sim_set_region) apply to
 * its model; the sim's parameter overrides apply only to subdomains of the
 * sim's model.  Its points start from that model's initial conditions
 * (ep_sim_set_state sets only points of the sim's model); ep_sim_get_state
 * reports, for a node whose lowest conducting subdomain runs another model,
 * the first n_vars variables of that model's state (zeros past its own
 * count).  Needs material ids (EP_EINVAL at finalize otherwise).  Call
 * before finalize; EP_EINVAL on a bad region or model. */
ep_status ep_sim_set_region_model(ep_sim* sim, int region, int model);

/* Fiber, sheet and normal directions per node (paper: the orthonormal triplet
 * f0, s0, n0 of the diffusion tensor), each [n_nodes][3].  Default if never
 * called: f0 = e_x, s0 = e_y, n0 = e_z. */
ep_status ep_sim_upload_fibers(ep_sim* sim, const double* f0, const double* s0, const double* n0);

/* Conductivities (mS/mm), membrane surface-to-volume ratio chi (1/mm) and
 * capacitance C_m (uF/mm^2); the diffusion tensor is
 * D = (sigma_l f f^T + sigma_t s s^T + sigma_n n n^T)/(chi C_m)
 * (paper: eq. of the diffusion tensor and the rescaling below the dimensional
 * monodomain equation).  Defaults 0.17, 0.019, 0.019, 140, 0.01. */
ep_status ep_sim_set_conductivity(ep_sim* sim, double sigma_l, double sigma_t, double sigma_n,
                                  double chi, double cm);

/* Ionic model (paper: the ionic models it ships).  variant: EP_CELL_* for
 * TTP06, 0 otherwise.  params: NULL for the published defaults, else
 * n_params values overriding the first slots of the model's parameter list:
 *   EP_AP:    k, a, eps0, mu1, mu2, T_ms
 *   EP_BO:    the 28 constants of the minimal model in the order u_o, u_u,
 *             theta_v, theta_w, theta_v-, theta_o, tau_v1-, tau_v2-, tau_v+,
 *             tau_w1-, tau_w2-, k_w-, u_w-, tau_w+, tau_fi, tau_o1, tau_o2,
 *             tau_so1, tau_so2, k_so, u_so, tau_s1, tau_s2, k_s, u_s, tau_si,
 *             tau_winf, w_inf*
 *   EP_TTP06: GNa, GK1, Gto, GKr, GKs, GCaL, GbNa, GbCa, GpCa, GpK, kNaCa,
 *             PNaK, Vrel, Vleak, Vmaxup, Vxfer
 * init_state: NULL for the model's initial conditions, else 1 + n_vars values
 * (u in model units, then the state in the order of ep_sim_set_state),
 * applied uniformly. */
ep_status ep_sim_set_ionic_model(ep_sim* sim, int model, int variant, const double* params,
                                 int n_params, const double* init_state);

/* Applied current (paper: "Applied current" impulses).  shape EP_CUBE (size =
 * edge, closed cube), EP_SPHERE (size = radius, closed ball), EP_GAUSS (size =
 * standard deviation, untruncated).  amp in uA/mm^3 (divided by chi C_m to give
 * mV/ms).  Active on steps n+1 whose time t_{n+1} lies in
 * (t0 + k period, t0 + k period + dur]; period 0 = one pulse.  Times are
 * rounded to whole steps.  At most 8 distinct timings. */
ep_status ep_sim_add_stimulus(ep_sim* sim, int shape, const double center_mm[3], double size_mm,
                              double amp_uA_per_mm3, double t0_ms, double dur_ms,
                              double period_ms);

/* Time step, BDF order (1..3; paper: BDF of order sigma with start-up at
 * lower orders), precision (EP_FP64 or EP_MIXED), preconditioner and block
 * size, relative residual tolerance ||b - A u|| <= rtol ||b||, and max CG
 * iterations per solve (inner solve when mixed).  Preconditioners (paper:
 * the software overview names block Jacobi among the preconditioners of its
 * CG solver): EP_JACOBI (block must be 1) or EP_BJACOBI, the
 * exact inverse of each diagonal block of `block` consecutive rows of the
 * system matrix (block 1, 2, 4, 8, 16, 32 or 64; 1 is Jacobi; the last
 * block may be shorter).  The inverses take block x 8 bytes per node per
 * BDF order (plus block x 4 in mixed precision).  EP_EINVAL otherwise. */
ep_status ep_sim_set_solver(ep_sim* sim, double dt_ms, int bdf_order, int precision, int precond,
                            int block, double rtol, int max_it);

ep_status ep_sim_set_option(ep_sim* sim, int key, double value);

/* Assemble M and K on the host, build the device operator and upload
 * everything.  The configuration is immutable afterwards. */
ep_status ep_sim_finalize(ep_sim* sim);

/* Enqueue and run n_steps time steps.  Blocks until the last step's solve
 * has converged.  EP_ENOCONV (the step kept its last iterate and stepping
 * went on) or EP_ENAN (stepping stopped) are sticky until the next step call. */
ep_status ep_sim_step(ep_sim* sim, int n_steps);
ep_status ep_sim_sync(ep_sim* sim);

/* Potential u_n in mV ([n_nodes], caller-allocated host array); dimensionless
 * models are mapped by u_mV = 100 u - 80 (AP) and 85.7 u - 84 (BO). */
ep_status ep_sim_get_potential(ep_sim* sim, double* out_mV);

/* Same into device memory owned by the caller: dtype EP_DTYPE_F64 or _F32,
 * [n_nodes] elements; enqueued on the sim's stream. */
ep_status ep_sim_get_potential_device(ep_sim* sim, void* dst, int dtype);

/* Activation times in ms ([n_nodes]): time t_{n+1} of the first strictly
 * largest forward difference (u_{n+1} - u_n)/dt; NaN where u never exceeded
 * the activation threshold (-40 mV for TTP06, 0.5 for AP / BO). */
ep_status ep_sim_get_activation_times(ep_sim* sim, double* out_ms);

/* Time (ms) of the first step whose u_{n+1} exceeded the activation
 * threshold, NaN if none ([n_nodes]). */
ep_status ep_sim_get_threshold_times(ep_sim* sim, double* out_ms);

ep_status ep_sim_get_stats(ep_sim* sim, ep_stats* out);

/* Summed durations (ms, from HIP events on the sim's stream) and launch
 * counts per kernel kind (EP_K_*), both arrays [EP_N_KERNEL_KINDS], since
 * EP_OPT_KERNEL_TIMERS was last set.  Launches that found their solve already
 * converged return at once and are counted too. */
ep_status ep_sim_get_kernel_times(ep_sim* sim, double* ms, int64_t* launches);

/* Mean elapsed time (us) of `reps` empty HIP event pairs recorded back to
 * back on the sim's stream: the part of an EP_OPT_KERNEL_TIMERS duration
 * that is the timer's own cost rather than the kernel's. */
ep_status ep_sim_timer_overhead(ep_sim* sim, int reps, double* us_per_pair);

/* Mean duration (us) of `reps` back-to-back launches of one kernel of the
 * step, between steps, on the sim's stream with the sim's launch shapes:
 * EP_K_CG_SPMV (w = A z) or EP_K_RHS (b = M g, r0 = b - A x0), the kernels
 * whose outputs the next step recomputes before reading them, or
 * EP_K_CG_PIPE (pipelined FP64 sims): the solver state is saved to a device
 * buffer (allocated on first use, about 9 vectors), the iteration is
 * launched `reps` times past the last step's solution with the stopping test
 * disabled, and the state is restored; EP_ESTATE if a launch stopped early
 * (breakdown).  For measurement; the simulation state is unchanged (bitwise).
 * EP_ESTATE before finalize, while pooled or during a step. */
ep_status ep_sim_time_kernel(ep_sim* sim, int kind, int reps, double* us_per_launch);

/* Launch-shape tuner (a growth direction, not in the paper): runs
 * trial_steps steps per candidate with kernel timers on, first for the
 * ionic nodes per thread (1, 2, 4; scored by the ionic kernel's mean time),
 * then for the tile map (0 and 2 on the Q1 lattice DIA, 0 and 1 otherwise;
 * scored by the mean durations of the residual, SpMV, update and pipelined
 * iteration kernels, each weighted by its launch count), and keeps the
 * fastest of each.  Each candidate's
 * trial_steps are split over up to three rounds that visit the candidates
 * in alternating order, so that the simulation's drift in work from step to
 * step weighs on all of them alike.  The 5 * trial_steps steps advance the
 * simulation like ep_sim_step (results do not depend on the shapes).
 * Writes the chosen EP_OPT_IONIC_NPT and EP_OPT_TILE_MAP values to the
 * non-NULL outputs.  EP_ESTATE before finalize or while pooled. */
ep_status ep_sim_autotune(ep_sim* sim, int trial_steps, int* ionic_npt, int* tile_map);

/* Raw state in model units (after finalize).  u: [n_nodes]; w: [n_vars][n_nodes]
 * in the model's state order (AP: v; BO: v, w, s; TTP06: m h j xr1 xr2 xs s r
 * d f f2 fcass cai casr cass nai ki rr); u_prev: [bdf-1][n_nodes] holding
 * u_{n-1}, u_{n-2} (NULL: copies of u).  set_state sets the step counter to
 * step_index and clears the activation-time tracking.  get_state fills any
 * non-NULL argument. */
ep_status ep_sim_set_state(ep_sim* sim, const double* u, const double* w, const double* u_prev,
                           int64_t step_index);
ep_status ep_sim_get_state(ep_sim* sim, double* u, double* w, double* u_prev);
int ep_sim_n_vars(const ep_sim* sim);

/* Free the sim and its device memory.  A sim that is still admitted to a
 * pool is released from it first (its slot frees; the pool keeps stepping
 * its other slots). */
void ep_sim_destroy(ep_sim* sim);

/* ---- batched / serving pool (many uneven simulations, one launch per phase) */

/* Pool on `device` with an HBM budget in bytes and at most max_slots
 * resident simulations, all of one precision. */
ep_status ep_pool_create(int device, void* hip_stream, size_t hbm_budget_bytes, int max_slots,
                         int precision, ep_pool** out);

/* Admit a sim.  A configured, not yet finalized sim is finalized by the pool
 * (host assembly and upload on the pool's stream) if its estimated device
 * footprint fits the remaining budget and a slot is free, else EP_EAGAIN
 * without allocating.  A sim finalized beforehand (on its own stream, for
 * instance by another thread while the pool steps) is only linked into the
 * pool's table if its allocated bytes fit the budget (else EP_EAGAIN; it
 * stays usable alone); admission then waits for its stream and costs no
 * assembly.  While pooled the sim runs on the pool's stream.  n_steps_total:
 * steps to run before the slot counts as done.  The pool does not take
 * ownership: destroy the sim after releasing it. */
ep_status ep_pool_admit(ep_pool* pool, ep_sim* sim, int64_t n_steps_total, int* slot);

/* Advance every active, unfinished slot by up to n_steps steps together. */
ep_status ep_pool_step(ep_pool* pool, int n_steps);

/* Slots that reached their step count: writes up to cap slot ids. */
ep_status ep_pool_poll(ep_pool* pool, int* done_slots, int cap, int* n_done);

/* Remove a slot from the pool and return its sim (results stay readable). */
ep_status ep_pool_release(ep_pool* pool, int slot, ep_sim** sim_out);
/* (returns the slot's final status: EP_OK, EP_ENAN or EP_ENOCONV; the sim is
 * released either way) */

ep_status ep_pool_get_info(ep_pool* pool, int* n_active, size_t* bytes_in_use);

/* EP_OPT_IONIC_NPT, EP_OPT_TILE_MAP (0: the workgroup list of each launch is
 * ordered so that each XCD receives a contiguous run; 1: list order) and
 * EP_OPT_GRAPH for the pool's own launches.  EP_EINVAL for other keys. */
ep_status ep_pool_set_option(ep_pool* pool, int key, double value);

/* ep_sim_autotune for the pool's launches: trial_steps pool steps per
 * candidate; the steps advance every active slot. */
ep_status ep_pool_autotune(ep_pool* pool, int trial_steps, int* ionic_npt, int* tile_map);
void ep_pool_destroy(ep_pool* pool);

/* Estimated device bytes ep_sim_finalize would allocate (sim configured, not
 * finalized); used for admission control. */
ep_status ep_sim_device_bytes_estimate(ep_sim* sim, size_t* bytes);

/* ---- single-cell pacing ------------------------------------------------------ */

/* Pace n_cells independent cells on the GPU (paper, Section "Ventricular
 * slab": ionic states initialized by long single-cell runs at the cardiac
 * period).  Each cell is the monodomain step without diffusion, with the
 * tissue's Rush-Larsen ionic step and BDF order: alpha u_{n+1} = u_BDF +
 * dt (I_app - I_ion(u_EXT, w_{n+1})).  params: [n_cells][n_params]
 * overrides of the model's first n_params parameters (NULL: defaults of
 * model/variant); init: [n_cells][1 + n_vars] starting u and state in model
 * units and state order (NULL: the model's initial conditions).  The
 * stimulus of stim_mV_per_ms (divided by the model's mV per unit for AP/BO)
 * is on during the first stim_dur_ms of every period_ms (times rounded to
 * whole steps, as in the tissue); n_beats periods are run, all from t = 0.
 * out: [n_cells][1 + n_vars], a row per cell in the layout
 * ep_sim_set_ionic_model takes as init_state.  EP_ENAN if a cell produced
 * NaN (out is still written). */
ep_status ep_cell_pace(int device, int model, int variant, int n_cells, const double* params, int n_params,
                       const double* init, double dt_ms, int bdf_order, double period_ms, double stim_mV_per_ms,
                       double stim_dur_ms, int n_beats, double* out);

/* ep_cell_pace for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same pacing and arithmetic, enqueued on hip_stream (NULL: the null
 * stream) of `device`, calling no hipMalloc, hipFree or stream creation and
 * not synchronizing.  params [n_cells][n_params] (or NULL), init
 * [n_cells][1 + n_vars] (or NULL) and out [n_cells][1 + n_vars] are DEVICE
 * pointers owned by the caller, laid out as in ep_cell_pace; out is valid once
 * the stream has reached the call (a cell that produced NaN shows NaN in out;
 * no status reports it).  The cells' potential history, state and parameter
 * rows are staged in a fixed device array of the library (about 6.9 MB per
 * device, held until the process ends), so n_cells is limited to 16384
 * (EP_EINVAL beyond).  Every call on a device uses that device's one array:
 * calls that overlap on one device (different streams, or threads without
 * ordering) race and give undefined results.  EP_EINVAL for bad arguments,
 * EP_EHIP if a launch fails. */
ep_status ep_cell_pace_device(int device, void* hip_stream, int model, int variant, int n_cells,
                              const double* params, int n_params, const double* init, double dt_ms,
                              int bdf_order, double period_ms, double stim_mV_per_ms, double stim_dur_ms,
                              int n_beats, double* out);

/* ---- host-only entry points (no GPU needed) -------------------------------- */

/* The library's finite-element assembly, for inspection: CSR of M and K
 * (see ep_sim_set_conductivity for D).  Call with rowptr == NULL to get
 * *nnz_out, then again with rowptr [n_nodes+1] (int64), col [nnz] (int32),
 * valM and valK [nnz] (double).  f0/s0/n0 may be NULL (axis-aligned). */
ep_status ep_assemble_csr(int elem, int64_t n_nodes, const double* xyz, int64_t n_elems,
                          const int32_t* conn, const double* f0, const double* s0,
                          const double* n0, double sigma_l, double sigma_t, double sigma_n,
                          double chi, double cm, int64_t* nnz_out, int64_t* rowptr, int32_t* col,
                          double* valM, double* valK);

const char* ep_last_error(void);
const char* ep_version(void);

#ifdef __cplusplus
}
#endif
#endif /* EP_MI355X_H */
