// Device-side data structures shared by the host runtime and the HIP kernels.
//
// Every kernel of the time step works on a table of simulation instances
// (InstDesc) and a block map that assigns each workgroup of the launch to one
// instance and one tile of its nodes.  A single simulation is a table of one;
// a batch of uneven simulations is a longer table and the same kernels.
// All per-step control (BDF start-up order, history ring slot, stimulus
// activity, CG scalars, convergence) lives in device memory (InstState), so a
// step needs no per-step kernel arguments from the host.
#pragma once
#include <stdint.h>

namespace ep {

constexpr int WG = 256;        // threads per workgroup of node-parallel kernels
constexpr int RPT = 2;         // rows (nodes) per thread in the solver kernels
// One row per thread (RPT = 1) made a GPU memory fault in a DIA test whose
// cause has not been found; that configuration is switched off.
static_assert(RPT == 2, "only RPT == 2 has been validated on the GPU");
constexpr int TILE = WG * RPT; // nodes per workgroup; thread t owns rows t and t + WG
constexpr int FIN_WG = 1024;   // threads of the one-workgroup-per-instance finalize
constexpr int SLICE = 64;      // SELL slice height = one wavefront
constexpr int MAX_DIAG = 32;   // largest diagonal count of a DIA-stored pattern
constexpr int MAX_UP = (MAX_DIAG + 1) / 2;  // stored (upper) diagonals of a symmetric DIA
constexpr int N_XCD = 8;       // accelerator complex dies; workgroups go round-robin
constexpr int MAX_STIM = 8;    // stimulus groups per instance
constexpr int NPARAM = 32;     // model parameter slots
constexpr int MAX_REGIONS = 8; // subdomains of one simulation
constexpr int RING = 4;        // potential history ring (u_{n+1}, u_n, u_{n-1}, u_{n-2})

enum Fmt : int32_t { FMT_SELL = 1, FMT_DIA = 2, FMT_MF = 3 };
enum Model : int32_t { M_PASSIVE = 0, M_AP = 1, M_BO = 2, M_TTP06 = 3 };
enum Prec : int32_t { P_FP64 = 0, P_MIXED = 1 };
enum Flag : int32_t { F_NAN = 1, F_NOCONV = 2, F_BREAKDOWN = 4 };

// One group of stimuli that share their timing: I_app(i) = amp * prof[i]
// while the step index k = n+1 satisfies (k - s0) mod period in [1, dur]
// (period 0: single pulse, k - s0 in [1, dur]).
struct StimGroup {
  const double* prof;
  double amp;
  int64_t s0, dur, period;
};

// Mutable per-instance state.  The CG scalars are owned by the one-workgroup
// finalize kernel; the wide kernels only read them (and workgroup 0 of the
// update kernel advances the iteration counters, which no workgroup of that
// kernel reads).  Kernel boundaries make the writes visible.
struct InstState {
  int64_t step;        // completed steps n (advanced by k_end_step only)
  int32_t it;          // CG iterations done in the current (inner) solve
  int32_t it_f;        // iteration index whose step lengths the finalize set
  // solve-control flags, adjacent so that a kernel reads them in one load;
  // no kernel writes a flag that another workgroup of the same kernel reads
  int32_t conv;        // 1: the step's solve is done
  int32_t conv_in;     // 1: the inner FP32 solve of this sweep is done
  int32_t restart;     // 1: a refinement residual restarted the inner solve
  int32_t flags;       // Flag bits, sticky until cleared by the host
  int32_t outer;       // refinement sweeps in this step
  int32_t it_step;     // CG iterations in the current step (all sweeps)
  int32_t it_last;     // CG iterations of the last finished step
  int32_t it_max;      // largest per-step CG count so far
  int64_t it_total;    // CG iterations over all steps
  int64_t outer_total;
  int32_t hist;        // potential levels u_n, u_{n-1}, ... that form a consistent history (1..3)
  int32_t sw_its[3];   // pipelined mixed: inner iteration at which sweep 0, 1, 2+ of this step stopped
  // step lengths of the current iteration (finalize) and of the previous
  // one (shifted by the update kernel), so that the finalize is idempotent
  double gamma_cur, alpha_cur, beta, gamma_prev, alpha_prev;
  double rr, bb, tol2, rr_in0, rr_outer;
  // FP64 solve without a finalize kernel: gamma_k and alpha_k of iteration k
  // in slot k & 1, written by the update kernel of iteration k and read by
  // that of iteration k + 1
  double gam[2], alp[2];
};
// Per-instance descriptor.  The mutable state sits inside it (first member),
// so kernels reach it without another pointer hop; the potential history
// slots are rotated on the device at the end of every step, so kernels do not
// need the step counter to find them: u_new = U[(n+1)&3], u_cur = U[n&3],
// u_prev1 = U[(n-1)&3], u_prev2 = U[(n-2)&3].
struct InstDesc {
  InstState st;
  double *u_new, *u_cur, *u_prev1, *u_prev2;
  int64_t n;               // nodes
  int64_t ld;              // DIA: leading dimension of one stored diagonal
  int32_t blk0, nblk;      // this instance's workgroups in node-parallel launches
  int32_t model, bdf, prec, fmt;
  int32_t nup, max_it, max_outer, n_stim;   // nup: stored (upper) DIA diagonals
  int32_t nvars, precond, block;         // block: rows per preconditioner block (1: Jacobi)
  int32_t ionic_scheme;    // 0: Rush-Larsen, 1: the paper's semi-implicit BDF
  int64_t bld;             // block Jacobi: leading dimension of the inverse-block columns
  double dt, inv_dt, rtol, inner_rtol, threshold;
  double mp[NPARAM];       // ionic model parameters
  int32_t off[MAX_UP];     // DIA: offsets >= 0 of the stored diagonals, off[0] = 0
  // matrix, one shared pattern; values of A_sigma = (alpha_sigma/dt) M + K.
  // DIA (symmetric): value of row i, stored diagonal d at val[d * ld + i] for
  // i in [-guard, n); A(i, i + off[d]) = A(i + off[d], i) = val[d*ld + i], so
  // the mirrored entry A(i, i - off[d]) is val[d*ld + i - off[d]].
  const int32_t* col;      // SELL column indices
  const int64_t* slice_ptr;// SELL slice offsets (elements), n_slices + 1
  const double* valA[3];
  const double* valM;
  const float* valA32[3];
  // preconditioner of A_sigma.  Jacobi: dinv[i] = 1/A(i, i).  Block Jacobi
  // over consecutive runs of `block` rows (block divides 64, so a run never
  // leaves a wavefront): dinv[j * bld + i] = (B^-1)(i - i0, j), B the
  // diagonal block of A_sigma whose first row is i0 = i - i % block
  // (columns past a ragged last block hold 0).
  const double* dinv[3];
  const float* dinv32[3];
  // FP64 vectors (padded by `guard` zero entries on both sides)
  double* U[RING];
  double *g, *b, *r, *z, *p, *s, *w;
  // FP32 inner-solve vectors (mixed precision)
  float *r32, *z32, *p32, *s32, *w32;
  // ionic state, structure of arrays [var][n], one array per time level: the
  // state of level m lives in st64[m & 3] / st32[m & 3] (the BDF scheme keeps
  // w_{n+1}, w_n, w_{n-1}, w_{n-2}; under Rush-Larsen all four alias one array)
  double* st64[RING];      // FP64 state (all variables in FP64 mode; nai, ki in mixed)
  float* st32[RING];       // FP32 state (mixed mode)
  // activation tracking
  double *smax, *at, *tcross;
  StimGroup stim[MAX_STIM];
  double* partial;         // per-workgroup partial sums, PART_DOUBLES * nblk
  // several subdomains (het != 0).  Ionic points: point i < n is node i with
  // its primary subdomain; points n .. n_pts-1 are the extra (node,
  // subdomain) pairs of interface nodes.  The ionic state arrays have stride
  // n_pts.  The load is M g minus the interface correction cvec = C Delta,
  // C(j, q) = M^r(j, node_q) for q = (node_q, r), Delta_q = I_q - I_node_q.
  int32_t het;
  int32_t n_crow;          // rows with an interface correction
  int64_t n_pts;           // ionic points (n when het == 0)
  const int32_t* pt_reg;   // [n_pts] subdomain of each point; -1: node outside every conducting one
  const int32_t* sec_node; // [n_pts - n] node of each extra point
  const double* rtab;      // [MAX_REGIONS][NPARAM] ionic parameters per subdomain
  double* ipt;             // [n_pts] I_ion of each point
  double* cvec;            // [n] interface correction, zero off its rows
  const int32_t* crow;     // [n_crow] row of each correction row
  const int64_t* cptr;     // [n_crow + 1] entries of each correction row
  const int32_t* ccol;     // extra point (counted from 0) of each entry
  const double* cval;      // C value of each entry
  // several ionic models (multi_model != 0): model of each subdomain and the
  // conversion of the potential field into that model's units and of its
  // current back: u_model = rconv[r][0] u + rconv[r][1], I_field =
  // rconv[r][2] I_model (identity for subdomains of the simulation's model)
  int32_t multi_model;
  int32_t rmodel[MAX_REGIONS];
  double rconv[MAX_REGIONS][3];
  // matrix-free operator (fmt == FMT_MF, FP64): hexahedra of degree mf_p,
  // applied element by element by sum factorization into element results,
  // which the row kernels add up per node (A z: yA; the rhs's M g: yM)
  int32_t mf_p;
  int64_t n_elems;
  const int32_t* econn;    // [n_elems][(mf_p + 1)^3] element nodes
  const double* geo;       // [n_elems][7][(mf_p + 1)^3] quadrature-point factors ([n_elems][7] if mf_cmp)
  double* yA;              // [n_elems][(mf_p + 1)^3]
  double* yM;              // [n_elems][(mf_p + 1)^3]
  const int64_t* adj_ptr;  // [n + 1] element entries of each node
  const int32_t* adj;      // entry e * npe + k, ascending
  double mfV[16], mfD[16]; // 1-D basis factor j and derivative at Gauss point q: [q * (p + 1) + j]
  int32_t mf_cmp;          // geo compressed to [n_elems][7] element constants x Gauss weights mfW
  double mfW[4];
  // Pipelined CG (cg_pipe != 0; the FP64 solve, or the FP32 inner solve of
  // mixed precision): one kernel per iteration.  Its iteration index, the
  // previous step lengths and the inner-solve state live in one record per
  // tile, pipe_rec[PIPE_REC * lblk + {0: k, 1: gamma_k, 2: alpha_k, 3: this
  // sweep's inner solve done, 4: the sweep's initial inner residual}], read
  // and written only by the workgroup of that tile, so no workgroup of a
  // launch can see another's update of the same launch.  m = P^-1 w
  // alternates: FP64 between b (even k) and g (odd k), both free during the
  // FP64 solve; FP32 between m32[0] and m32[1].
  int32_t cg_pipe;
  int32_t x0_extrap;       // 1: initial guess by third-order extrapolation (else u_EXT)
  double* pipe_rec;        // [nblk][PIPE_REC]
  float* m32[2];
  // tile of each workgroup of a single-instance launch under tile map 2
  // (lattice operators: each XCD takes the tiles of a band of lattice lines
  // across all planes; -1 past the last tile of a band), or null
  const int32_t* tile_tab;
};
constexpr int PIPE_REC = 8;

// Partial-sum layout inside InstDesc::partial, in units of nblk doubles:
// residual kernel [4][nblk], SpMV [1][nblk], update [2][nblk]; the FP64
// update kernel that reduces its predecessors' partials itself writes
// iteration k's partials to [2][nblk] at PART_UPD + 2 (k & 1), so that no
// workgroup overwrites partials another workgroup of the same launch reads.
// The pipelined CG kernel writes iteration k's three partials
// (<r, P^-1 r>, <w, P^-1 r>, <r, r>) to [3][nblk] at PART_PIPE + 3 (k & 1).
constexpr int PART_RES = 0, PART_SPMV = 4, PART_UPD = 5, PART_PIPE = 5, PART_DOUBLES = 11;

struct BlockMap {
  int32_t inst;
  int32_t lblk;            // workgroup index inside the instance
};

}  // namespace ep
