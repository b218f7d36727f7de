// HIP kernels (gfx950) of one monodomain time step.
//
// Step pipeline per instance (paper: IMEX staggering of the numerical section;
// the time-discrete ionic model, then the linear monodomain system):
//   k_ionic      BDF history combination, Rush-Larsen / explicit ionic step at
//                u_EXT, I_ion(u_EXT, w_{n+1}), stimulus, nodal RHS vector
//                g = u_BDF/dt + I_app - I_ion, initial guess x0 = u_EXT
//   k_residual   b = M g (ionic current interpolation: the load is the mass
//                matrix applied to nodal values) fused with r0 = b - A x0 and
//                the preconditioner; FP64.  Re-used, without M g, as the FP64
//                residual of each mixed-precision refinement sweep.
//   k_cg_spmv    w = A z and <w, z>       (Chronopoulos-Gear PCG: one SpMV and
//   k_cg_update  p, s, x, r, z updates    one fused vector sweep per iteration)
//   k_activation running argmax of (u_{n+1} - u_n)/dt, threshold crossing
//
// Memory layout: structure-of-arrays, one thread per node, 256-thread
// workgroups (4 wavefronts of 64).  Matrix formats: DIA (column offsets shared
// by all rows, no index traffic; values [diag][stride]) when the pattern has
// few distinct offsets, else SELL with 64-row slices (one wavefront per slice,
// column-major inside the slice).  Vectors that SpMV gathers from carry zero
// guard cells so DIA rows near the ends stay in bounds.
//
// Reductions are deterministic and need no synchronization between
// workgroups inside a kernel: each workgroup writes its partial sum, and a
// one-workgroup-per-instance finalize kernel adds the instance's partials in
// a fixed order, decides convergence and forms the CG step lengths.  A batch
// of instances reduces per instance, so each instance's result does not
// depend on the batch.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "ep_device.h"
#include "ionic_models.h"
#include "kernels.h"

namespace ep {

// Device arrays are global memory, but a pointer read from the instance
// descriptor is generic, and generic accesses compile to flat instructions.
// Flat loads also count against the scalar-load counter, so every scalar load
// of a descriptor field (a diagonal offset, a state flag) would wait for all
// vector loads in flight.  gmem() re-types such a pointer as global.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> gmem(T* p) {
  return (gptr<T>)p;
}

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Workgroup sum of v[], stored by thread 0 at P[c * nblk + lblk].
// Every thread of the workgroup must call it.
template <int NV>
__device__ __forceinline__ void write_partials(double (&v)[NV], double* __restrict__ P, int nblk, int lblk) {
  __shared__ double sh[WG / 64][NV];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < NV; c++) v[c] = wave_sum(v[c]);
  if (lane == 0) {
#pragma unroll
    for (int c = 0; c < NV; c++) sh[wv][c] = v[c];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int c = 0; c < NV; c++) gmem(P)[(int64_t)c * nblk + lblk] = (sh[0][c] + sh[1][c]) + (sh[2][c] + sh[3][c]);
  }
}

// Sum of the partials P[c * nblk + b], b < nblk, in a fixed order; every
// thread of the (NT-thread) workgroup obtains bitwise the same totals.
template <int NT, int NV>
__device__ __forceinline__ void reduce_partials(const double* __restrict__ P, int nblk, double (&out)[NV]) {
  __shared__ double sh[NT / 64][NV];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double acc[NV];
#pragma unroll
  for (int c = 0; c < NV; c++) acc[c] = 0.0;
  for (int b = threadIdx.x; b < nblk; b += NT) {
#pragma unroll
    for (int c = 0; c < NV; c++) acc[c] += gmem(P)[(int64_t)c * nblk + b];
  }
#pragma unroll
  for (int c = 0; c < NV; c++) acc[c] = wave_sum(acc[c]);
  if (lane == 0) {
#pragma unroll
    for (int c = 0; c < NV; c++) sh[wv][c] = acc[c];
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < NV; c++) {
    double a = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; w++) a += sh[w][c];
    out[c] = a;
  }
}

// Sum of the partial streams P[c[j] * nblk + b], b < nblk, for NV stream
// indices c[j], in a fixed order (that of reduce_partials); every thread of
// the NT-thread workgroup obtains bitwise the same totals.
template <int NT, int NV>
__device__ __forceinline__ void reduce_streams(const double* __restrict__ P, const int (&c)[NV], int nblk,
                                               double (&out)[NV]) {
  __shared__ double sh[NT / 64][NV];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double acc[NV];
#pragma unroll
  for (int j = 0; j < NV; j++) acc[j] = 0.0;
  for (int b = threadIdx.x; b < nblk; b += NT) {
#pragma unroll
    for (int j = 0; j < NV; j++) acc[j] += gmem(P)[(int64_t)c[j] * nblk + b];
  }
#pragma unroll
  for (int j = 0; j < NV; j++) acc[j] = wave_sum(acc[j]);
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < NV; j++) sh[wv][j] = acc[j];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < NV; j++) {
    double a = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; w++) a += sh[w][j];
    out[j] = a;
  }
}

// Solve-control flags written by earlier kernels (kernel boundaries make them
// visible).  Plain loads of the three adjacent words, issued together.
struct Ctl {
  int conv, conv_in, restart;
};
__device__ __forceinline__ Ctl ld_ctl(const InstState& S) {
  return Ctl{S.conv, S.conv_in, S.restart};
}
// true when the CG kernels of this instance have nothing to do: the step is
// solved, or the inner solve of this sweep is done and no refinement
// residual has restarted it
__device__ __forceinline__ bool cg_idle(const InstState& S) {
  const Ctl c = ld_ctl(S);
  return c.conv != 0 || (c.conv_in != 0 && c.restart == 0);
}


// ---------------------------------------------------------------------------
// matrix-free operator of hexahedra of degree P (2 or 3): element results by
// sum factorization on the (P + 1)^3 Gauss points (the paper lists
// matrix-free high-order solvers as the route to GPUs).  y_e = sum_q
// [N m_q u(q) + dN^T C_q grad_ref u(q)] with u = x_e interpolated; the
// 1-D factors (V, Dv) act one direction at a time: n1^4 operations per
// contraction instead of n1^6 for the element matrix.  n1^2 threads per
// element, each holding one column of n1 values in registers; the x and y
// directions go through LDS.  One wavefront per workgroup carries
// 64 / n1^2 elements.  The node sums are taken by the row kernels
// (mf_row), in ascending entry order.
// ---------------------------------------------------------------------------

template <int P>
struct MfShape {
  static constexpr int N1 = P + 1, T = N1 * N1, NPE = N1 * N1 * N1, EPW = 64 / T;
};

// WHICH 0: yA = (c M + K) z; 1: yM = M g; 2: yA = (c M + K) x0 (rhs residual);
// 3: yA = (c M + K) m_k of the pipelined CG (k from tile 0's record)
// CMP: every element's factors are an element constant times the point's
// Gauss weight (affine elements with one D): 7 loads per element.
template <int P, int WHICH, bool CMP>
__global__ __launch_bounds__(64) void k_mf_apply(InstDesc* __restrict__ insts) {
  using S_ = MfShape<P>;
  constexpr int N1 = S_::N1, T = S_::T, NPE = S_::NPE, EPW = S_::EPW;
  constexpr bool STIFF = WHICH != 1;
  const InstDesc& I = insts[0];
  const InstState& St = I.st;
  if ((WHICH == 0 || WHICH == 3) && cg_idle(St)) return;
  __shared__ double buf[EPW > 0 ? EPW : 1][5][NPE];
  const int slot = threadIdx.x / T, t = threadIdx.x % T;
  const int64_t e = (int64_t)blockIdx.x * EPW + slot;
  const bool live = slot < EPW && e < I.n_elems;
  const int ts = live ? slot : 0;          // idle threads keep in-range LDS indices
  double (*B)[NPE] = buf[ts];
  const int i1 = t % N1, i2 = t / N1;      // the thread's two in-plane indices
  auto L = [](int x, int y, int z) { return x + N1 * (y + N1 * z); };
  const double* __restrict__ V = I.mfV;
  const double* __restrict__ Dv = I.mfD;
  const double* xin = WHICH == 0 ? I.z : (WHICH == 1 ? I.g : (WHICH == 2 ? I.u_new : nullptr));
  if (WHICH == 3) xin = (((int)gmem(I.pipe_rec)[0] + 1) & 1) ? I.g : I.b;
  const int sig = min(I.bdf, (int)St.step + 1);
  const double cmass = (sig == 1 ? 1.0 : (sig == 2 ? 1.5 : 11.0 / 6.0)) * I.inv_dt;
  // ---- forward: column (a, b) = (i1, i2) ----
  double X[N1], Y[N1], Yd[N1];
  if (live) {
#pragma unroll
    for (int c = 0; c < N1; c++) X[c] = gmem(xin)[gmem(I.econn)[e * NPE + L(i1, i2, c)]];
  } else {
#pragma unroll
    for (int c = 0; c < N1; c++) X[c] = 0.0;
  }
#pragma unroll
  for (int q = 0; q < N1; q++) {
    double y = 0.0, yd = 0.0;
#pragma unroll
    for (int c = 0; c < N1; c++) {
      y += V[q * N1 + c] * X[c];
      if (STIFF) yd += Dv[q * N1 + c] * X[c];
    }
    Y[q] = y;
    Yd[q] = yd;
  }
  if (live) {
#pragma unroll
    for (int q = 0; q < N1; q++) {
      B[0][L(i1, i2, q)] = Y[q];
      if (STIFF) B[1][L(i1, i2, q)] = Yd[q];
    }
  }
  __syncthreads();
  // y direction: thread (a, qy) = (i1, i2)
  if (live) {
#pragma unroll
    for (int qz = 0; qz < N1; qz++) {
      double w = 0.0, wy = 0.0, wz = 0.0;
#pragma unroll
      for (int b = 0; b < N1; b++) {
        const double y0 = B[0][L(i1, b, qz)];
        w += V[i2 * N1 + b] * y0;
        if (STIFF) {
          wy += Dv[i2 * N1 + b] * y0;
          wz += V[i2 * N1 + b] * B[1][L(i1, b, qz)];
        }
      }
      B[2][L(i1, i2, qz)] = w;
      if (STIFF) {
        B[3][L(i1, i2, qz)] = wy;
        B[4][L(i1, i2, qz)] = wz;
      }
    }
  }
  __syncthreads();
  // x direction and the quadrature point: thread (qx, qy) = (i1, i2)
  double Mq[N1], F0[N1], F1[N1], F2[N1];
  const gptr<const double> geo = gmem(I.geo) + (live ? e : 0) * 7 * (CMP ? 1 : NPE);
  double ge[7];
  if (CMP) {
#pragma unroll
    for (int c = 0; c < 7; c++) ge[c] = live ? geo[c] : 0.0;
  }
#pragma unroll
  for (int qz = 0; qz < N1; qz++) {
    double u = 0.0, ux = 0.0, uy = 0.0, uz = 0.0;
    if (live) {
#pragma unroll
      for (int a = 0; a < N1; a++) {
        const double w = B[2][L(a, i2, qz)];
        u += V[i1 * N1 + a] * w;
        if (STIFF) {
          ux += Dv[i1 * N1 + a] * w;
          uy += V[i1 * N1 + a] * B[3][L(a, i2, qz)];
          uz += V[i1 * N1 + a] * B[4][L(a, i2, qz)];
        }
      }
    }
    const int q = L(i1, i2, qz);
    const double wq = CMP ? I.mfW[i1] * I.mfW[i2] * I.mfW[qz] : 0.0;
    const double m = !live ? 0.0 : (CMP ? ge[6] * wq : geo[6 * NPE + q]);
    Mq[qz] = (STIFF ? cmass : 1.0) * m * u;
    if (STIFF) {
      double c0 = 0, c1 = 0, c2 = 0, c3 = 0, c4 = 0, c5 = 0;
      if (live && CMP) {
        c0 = ge[0] * wq; c1 = ge[1] * wq; c2 = ge[2] * wq;
        c3 = ge[3] * wq; c4 = ge[4] * wq; c5 = ge[5] * wq;
      } else if (live) {
        c0 = geo[q]; c1 = geo[NPE + q]; c2 = geo[2 * NPE + q];
        c3 = geo[3 * NPE + q]; c4 = geo[4 * NPE + q]; c5 = geo[5 * NPE + q];
      }
      F0[qz] = c0 * ux + c1 * uy + c2 * uz;
      F1[qz] = c1 * ux + c3 * uy + c4 * uz;
      F2[qz] = c2 * ux + c4 * uy + c5 * uz;
    }
  }
  __syncthreads();   // every read of the forward buffers is done
  if (live) {
#pragma unroll
    for (int qz = 0; qz < N1; qz++) {
      B[0][L(i1, i2, qz)] = Mq[qz];
      if (STIFF) {
        B[1][L(i1, i2, qz)] = F0[qz];
        B[2][L(i1, i2, qz)] = F1[qz];
        B[3][L(i1, i2, qz)] = F2[qz];
      }
    }
  }
  __syncthreads();
  // ---- backward (transposes) ----
  // x: thread (a, qy) = (i1, i2)
  double G0[N1], G1[N1], G2[N1];
#pragma unroll
  for (int qz = 0; qz < N1; qz++) {
    double g0 = 0.0, g1 = 0.0, g2 = 0.0;
    if (live) {
#pragma unroll
      for (int qx = 0; qx < N1; qx++) {
        g0 += V[qx * N1 + i1] * B[0][L(qx, i2, qz)];
        if (STIFF) {
          g0 += Dv[qx * N1 + i1] * B[1][L(qx, i2, qz)];
          g1 += V[qx * N1 + i1] * B[2][L(qx, i2, qz)];
          g2 += V[qx * N1 + i1] * B[3][L(qx, i2, qz)];
        }
      }
    }
    G0[qz] = g0;
    G1[qz] = g1;
    G2[qz] = g2;
  }
  __syncthreads();
  if (live) {
#pragma unroll
    for (int qz = 0; qz < N1; qz++) {
      B[0][L(i1, i2, qz)] = G0[qz];
      if (STIFF) {
        B[1][L(i1, i2, qz)] = G1[qz];
        B[4][L(i1, i2, qz)] = G2[qz];
      }
    }
  }
  __syncthreads();
  // y: thread (a, b) = (i1, i2); then z in registers
  if (!live) return;
  double H0[N1], H2[N1];
#pragma unroll
  for (int qz = 0; qz < N1; qz++) {
    double h0 = 0.0, h2 = 0.0;
#pragma unroll
    for (int qy = 0; qy < N1; qy++) {
      h0 += V[qy * N1 + i2] * B[0][L(i1, qy, qz)];
      if (STIFF) {
        h0 += Dv[qy * N1 + i2] * B[1][L(i1, qy, qz)];
        h2 += V[qy * N1 + i2] * B[4][L(i1, qy, qz)];
      }
    }
    H0[qz] = h0;
    H2[qz] = h2;
  }
  const gptr<double> yout = gmem(WHICH == 1 ? I.yM : I.yA) + e * NPE;
#pragma unroll
  for (int c = 0; c < N1; c++) {
    double y = 0.0;
#pragma unroll
    for (int qz = 0; qz < N1; qz++) {
      y += V[qz * N1 + c] * H0[qz];
      if (STIFF) y += Dv[qz * N1 + c] * H2[qz];
    }
    yout[L(i1, i2, c)] = y;
  }
}

// Node sum of element results: the value of row i of the operator product.
__device__ __forceinline__ double mf_row(const InstDesc& I, const double* __restrict__ y, int64_t i) {
  const gptr<const int64_t> ap = gmem(I.adj_ptr);
  const gptr<const int32_t> ad = gmem(I.adj);
  const gptr<const double> yv = gmem(y);
  double acc = 0.0;
  for (int64_t j = ap[i]; j < ap[i + 1]; j++) acc += yv[ad[j]];
  return acc;
}

// z = P^{-1} r for the row i this lane owns.  Jacobi (block 1): one scaling.
// Block Jacobi: a block of `bs` consecutive rows lies inside one wavefront
// (bs divides 64 and tiles start at multiples of 64), so the block's
// residual entries are gathered by lane shuffles and the row of the inverse
// block is read column by column (coalesced across the wavefront).  Every
// lane of the wavefront must call this (r = 0 on lanes without a row).
template <typename T>
__device__ __forceinline__ T precond_apply(const T* __restrict__ pinv, int64_t bld, int bs, int64_t i, bool valid,
                                           T r) {
  const gptr<const T> pv = gmem(pinv);
  if (bs == 1) return valid ? pv[i] * r : T(0);
  const int base = (int)(threadIdx.x & 63) & ~(bs - 1);
  T acc = T(0);
  for (int j = 0; j < bs; j++) {
    const T rj = __shfl(r, base + j, 64);
    if (valid) acc += pv[(int64_t)j * bld + i] * rj;
  }
  return acc;
}

// ---------------------------------------------------------------------------
// sparse row products
// ---------------------------------------------------------------------------

// Rounded product and fused multiply-add, spelled out so that the result
// does not depend on how the compiler contracts the code around an inlined
// row product (kernels that share a row product give the same bits).
__device__ __forceinline__ double mul_rn(double a, double b) { return __dmul_rn(a, b); }
__device__ __forceinline__ float mul_rn(float a, float b) { return __fmul_rn(a, b); }
__device__ __forceinline__ double fmad(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float fmad(float a, float b, float c) { return fmaf(a, b, c); }

// Symmetric DIA: diagonal 0 plus, for each stored offset o > 0, the entry at
// +o (stored at row i) and its mirror at -o (stored at row i - o).
template <int NU, typename V, typename X, typename A>
__device__ __forceinline__ A dia_row(const InstDesc& I, const V* __restrict__ val, const X* __restrict__ x,
                                     int64_t i, int nu) {
  const int64_t ld = I.ld;
  const gptr<const V> va = gmem(val);
  const gptr<const X> xa = gmem(x);
  A acc = mul_rn((A)va[i], (A)xa[i]);
  const int n_up = NU > 0 ? NU : nu;
#pragma unroll
  for (int d = 1; d < (NU > 0 ? NU : MAX_UP); d++) {
    if (NU == 0 && d >= n_up) break;
    const int o = I.off[d];
    acc = fmad((A)va[d * ld + i], (A)xa[i + o], acc);
    acc = fmad((A)va[d * ld + i - o], (A)xa[i - o], acc);
  }
  return acc;
}

template <typename V, typename X, typename A>
__device__ __forceinline__ A spmv_row(const InstDesc& I, const V* __restrict__ val, const X* __restrict__ x,
                                      int64_t i) {
  if (I.fmt == FMT_DIA) {
    if (I.nup == 14) return dia_row<14, V, X, A>(I, val, x, i, 14);   // 27-point (Q1 lattice)
    if (I.nup == 8) return dia_row<8, V, X, A>(I, val, x, i, 8);      // 15-point (P1 Kuhn lattice)
    return dia_row<0, V, X, A>(I, val, x, i, I.nup);
  }
  const int64_t slice = i >> 6;
  const int lane = (int)(i & 63);
  const int64_t o0 = gmem(I.slice_ptr)[slice], o1 = gmem(I.slice_ptr)[slice + 1];
  A acc = A(0);
  const gptr<const int32_t> col = gmem(I.col);
  const gptr<const V> va = gmem(val);
  const gptr<const X> xa = gmem(x);
  int64_t o = o0 + lane;
  for (; o + 3 * 64 < o1; o += 4 * 64) {
    const V v0 = va[o], v1 = va[o + 64], v2 = va[o + 128], v3 = va[o + 192];
    const int32_t c0 = col[o], c1 = col[o + 64], c2 = col[o + 128], c3 = col[o + 192];
    acc += (A)v0 * (A)xa[c0];
    acc += (A)v1 * (A)xa[c1];
    acc += (A)v2 * (A)xa[c2];
    acc += (A)v3 * (A)xa[c3];
  }
  for (; o < o1; o += 64) acc += (A)va[o] * (A)xa[col[o]];
  return acc;
}

// ---------------------------------------------------------------------------
// instance lookup: a single instance (no block map) or a batch
// ---------------------------------------------------------------------------

// Single instance: workgroups are dispatched round-robin over the N_XCD dies;
// tile = (b mod N_XCD) * per + b / N_XCD gives each die a contiguous range of
// tiles, so stencil neighbours of a tile mostly sit in the same die's L2.
// The launch has N_XCD * per workgroups; those past the last tile get
// lblk = -1 and must leave at once.
// XMAP = 1 maps workgroup b to tile b (dispatch order), for comparison by the
// tuner.  XMAP = 2 (lattice operators) reads the tile from a table in which
// each die holds the tiles of one band of lattice lines (y) across all
// planes (z): the far stencil neighbours of a row, one plane away, then lie
// in the same die's L2 except at the band's two edge lines, where the
// contiguous ranges of XMAP 0 cross dies once every plane's worth of rows.
template <bool SINGLE, int XMAP = 0>
__device__ __forceinline__ InstDesc& instance(InstDesc* __restrict__ insts, const BlockMap* __restrict__ bmap,
                                              int& lblk) {
  if (SINGLE) {
    InstDesc& I = insts[0];
    if (XMAP == 1) {
      lblk = (int)blockIdx.x < I.nblk ? (int)blockIdx.x : -1;
      return I;
    }
    if (XMAP == 2) {
      lblk = gmem(I.tile_tab)[blockIdx.x];
      return I;
    }
    const int per = (I.nblk + N_XCD - 1) / N_XCD;
    const int t = (int)(blockIdx.x % N_XCD) * per + (int)(blockIdx.x / N_XCD);
    lblk = t < I.nblk ? t : -1;
    return I;
  }
  const BlockMap bm = bmap[blockIdx.x];
  lblk = bm.lblk;
  return insts[bm.inst];
}

// ---------------------------------------------------------------------------
// ionic step + nodal RHS vector (one node per thread, TILE threads)
// ---------------------------------------------------------------------------

__device__ __forceinline__ double stimulus_at(const InstDesc& I, int64_t k, int64_t i) {
  double iapp = 0.0;
  for (int gi = 0; gi < I.n_stim; gi++) {
    const StimGroup& sg = I.stim[gi];
    int64_t q = k - sg.s0;
    if (q < 1) continue;
    if (sg.period > 0) q = (q - 1) % sg.period + 1;
    if (q <= sg.dur) iapp += sg.amp * gmem(sg.prof)[i];
  }
  return iapp;
}

// BDF / extrapolation weights over the history levels n, n-1, n-2 of order
// sig (the potential's coefficients; the paper applies the same BDF to the
// ionic model).
struct BdfW {
  double alpha, b[3], e[3];
};
__device__ __forceinline__ BdfW bdf_weights(int sig) {
  if (sig == 1) return BdfW{1.0, {1.0, 0.0, 0.0}, {1.0, 0.0, 0.0}};
  if (sig == 2) return BdfW{1.5, {2.0, -0.5, 0.0}, {2.0, -1.0, 0.0}};
  return BdfW{11.0 / 6.0, {3.0, -1.5, 1.0 / 3.0}, {3.0, -3.0, 1.0}};
}

// BDF combination and extrapolation of one state variable over `sig` levels
// (arrays a[0..sig-1] = levels n, n-1, n-2 of that variable at node i).
template <typename T>
__device__ __forceinline__ void combine(const BdfW& W, int sig, const T* const* lv, int64_t off, T& xb, T& xe) {
  T b = T(0), e = T(0);
  for (int k = 0; k < sig; k++) {
    const T x = gmem(lv[k])[off];
    b += T(W.b[k]) * x;
    e += T(W.e[k]) * x;
  }
  xb = b;
  xe = e;
}

// Ionic step of one ionic point: state index i (arrays [var][n], stride n),
// potential of node `node`, parameters mp.  With RHS the point also writes its
// node's load g = u_BDF/dt + I_app - I_ion and initial guess u_EXT; with
// KEEP_I it stores I_ion(point) for the interface correction.  CONV: the
// point's model works in other units than the potential field; it is stepped
// at u_model = cv[0] u_EXT + cv[1] and its current enters as cv[2] I_model.
template <int MODEL, bool MIXED, bool BDFS, bool RHS = true, bool KEEP_I = false, bool CONV = false>
__device__ __forceinline__ void ionic_point(const InstDesc& I, int64_t n, int64_t step, int64_t i, int64_t node,
                                            const double* __restrict__ mp, const double* cv = nullptr) {
  const int sig = min(I.bdf, (int)step + 1);
  const double u0 = gmem(I.u_cur)[node];
  double u_ext, u_bdf;
  if (sig == 1) {
    u_ext = u0;
    u_bdf = u0;
  } else if (sig == 2) {
    const double u1 = gmem(I.u_prev1)[node];
    u_ext = 2.0 * u0 - u1;
    u_bdf = 2.0 * u0 - 0.5 * u1;
  } else {
    const double u1 = gmem(I.u_prev1)[node], u2 = gmem(I.u_prev2)[node];
    u_ext = 3.0 * u0 - 3.0 * u1 + u2;
    u_bdf = 3.0 * u0 - 1.5 * u1 + u2 * (1.0 / 3.0);
  }
  // the potential the model sees (its own units)
  const double u_field = u_ext;
  if (CONV) u_ext = cv[0] * u_field + cv[1];
  // state levels: new w_{n+1}, then w_n, w_{n-1}, w_{n-2}
  const gptr<double> s64 = gmem(I.st64[(step + 1) & 3]);
  const gptr<float> s32 = gmem(I.st32[(step + 1) & 3]);
  const double* l64[3] = {I.st64[step & 3], I.st64[(step - 1) & 3], I.st64[(step - 2) & 3]};
  const float* l32[3] = {I.st32[step & 3], I.st32[(step - 1) & 3], I.st32[(step - 2) & 3]};
  // Rush-Larsen reads level n alone (weights 1)
  const BdfW W = bdf_weights(BDFS ? sig : 1);
  const int lev = BDFS ? sig : 1;
  double iion = 0.0;
  if (MODEL == M_AP) {
    if (MIXED) {
      float vb, ve;
      combine<float>(W, lev, l32, i, vb, ve);
      float v = vb;
      iion = BDFS ? (double)ap_step_bdf<float>((float)u_ext, (float)I.dt, (float)W.alpha, mp, vb, ve, v)
                  : (double)ap_step<float>((float)u_ext, (float)I.dt, mp, v);
      s32[i] = v;
    } else {
      double vb, ve;
      combine<double>(W, lev, l64, i, vb, ve);
      double v = vb;
      iion = BDFS ? ap_step_bdf<double>(u_ext, I.dt, W.alpha, mp, vb, ve, v)
                  : ap_step<double>(u_ext, I.dt, mp, v);
      s64[i] = v;
    }
  } else if (MODEL == M_BO) {
    if (MIXED) {
      float yb[3], ye[3];
      for (int k = 0; k < 3; k++) combine<float>(W, lev, l32, (int64_t)k * n + i, yb[k], ye[k]);
      float v = yb[0], w = yb[1], s = yb[2];
      iion = (double)bo_step<float, BDFS>((float)u_ext, (float)I.dt, mp, v, w, s, (float)W.alpha, yb);
      s32[i] = v; s32[n + i] = w; s32[2 * n + i] = s;
    } else {
      double yb[3], ye[3];
      for (int k = 0; k < 3; k++) combine<double>(W, lev, l64, (int64_t)k * n + i, yb[k], ye[k]);
      double v = yb[0], w = yb[1], s = yb[2];
      iion = bo_step<double, BDFS>(u_ext, I.dt, mp, v, w, s, W.alpha, yb);
      s64[i] = v; s64[n + i] = w; s64[2 * n + i] = s;
    }
  } else if (MODEL == M_TTP06) {
    // FP64 rows in state order: 12 gates, cai, casr, cass, nai, ki, rr.
    // Mixed: st32 rows 12 gates, cai, casr, cass, rr; st64 rows nai, ki.
    using R = typename std::conditional<MIXED, float, double>::type;
    TtpState<R> S, Sb, Se;
    R tb[3] = {R(0), R(0), R(0)};
    auto row = [&](int v) -> int64_t { return (int64_t)v * n + i; };
    const R* const* lr = reinterpret_cast<const R* const*>(MIXED ? (const void*)l32 : (const void*)l64);
#pragma unroll
    for (int k = 0; k < 12; k++) combine<R>(W, lev, lr, row(k), Sb.g[k], Se.g[k]);
    combine<R>(W, lev, lr, row(12), Sb.cai, Se.cai);
    combine<R>(W, lev, lr, row(13), Sb.casr, Se.casr);
    combine<R>(W, lev, lr, row(14), Sb.cass, Se.cass);
    combine<R>(W, lev, lr, row(MIXED ? 15 : 17), Sb.rr, Se.rr);
    combine<double>(W, lev, l64, MIXED ? i : row(15), Sb.nai, Se.nai);
    combine<double>(W, lev, l64, MIXED ? row(1) : row(16), Sb.ki, Se.ki);
    if (BDFS) {
      // BDF combination of the buffered calcium totals of each level
      for (int k = 0; k < lev; k++) {
        tb[0] += R(W.b[k]) * buffered_total<R>(gmem(lr[k])[row(12)], R(ttp::Bufc), R(ttp::Kbufc));
        tb[1] += R(W.b[k]) * buffered_total<R>(gmem(lr[k])[row(13)], R(ttp::Bufsr), R(ttp::Kbufsr));
        tb[2] += R(W.b[k]) * buffered_total<R>(gmem(lr[k])[row(14)], R(ttp::Bufss), R(ttp::Kbufss));
      }
    }
    S = Sb;   // Rush-Larsen (one level): Sb holds w_n
    iion = (double)ttp06_step<R, BDFS>((R)u_ext, (R)I.dt, mp, S, (R)W.alpha, &Sb, &Se, tb);
    const gptr<R> sr = gmem(reinterpret_cast<R*>(MIXED ? (void*)I.st32[(step + 1) & 3] : (void*)I.st64[(step + 1) & 3]));
#pragma unroll
    for (int k = 0; k < 12; k++) sr[row(k)] = S.g[k];
    sr[row(12)] = S.cai; sr[row(13)] = S.casr; sr[row(14)] = S.cass;
    sr[row(MIXED ? 15 : 17)] = S.rr;
    s64[MIXED ? i : row(15)] = S.nai;
    s64[MIXED ? row(1) : row(16)] = S.ki;
  }
  if (CONV) iion *= cv[2];
  if (KEEP_I) gmem(I.ipt)[i] = iion;
  if (RHS) {
    const double iapp = stimulus_at(I, step + 1, node);
    gmem(I.g)[node] = u_bdf * I.inv_dt + iapp - iion;
    // initial guess of the linear solve: u_EXT, or (option) the potential
    // extrapolated from the last three solutions once they form a
    // consistent history (one order above u_EXT for BDF2; only the
    // iteration count depends on it)
    double x0 = u_field;
    if (I.x0_extrap && I.st.hist >= 3) {
      const double a1 = gmem(I.u_prev1)[node], a2 = gmem(I.u_prev2)[node];
      x0 = 3.0 * u0 - 3.0 * a1 + a2;
    }
    gmem(I.u_new)[node] = x0;
  }
}

// One tile of TILE nodes per workgroup of TILE / NPT threads, NPT nodes per
// thread (node p * TILE / NPT + t of the tile).  NPT > 1 also asks the
// compiler for at least 4 (NPT 2) or 5 (NPT 4) waves per SIMD, trading
// registers (and, for the FP64 TTP06 model, some spills) for occupancy; the
// tuner measures which shape is fastest for a model and precision.
template <int MODEL, bool MIXED, bool SINGLE, int NPT, bool BDFS>
__global__ __launch_bounds__(TILE / NPT) __attribute__((amdgpu_waves_per_eu(NPT == 1 ? 1 : (NPT == 2 ? 4 : 5)))) void k_ionic(InstDesc* __restrict__ insts,
                                                      const BlockMap* __restrict__ bmap) {
  int lblk;
  const InstDesc& I = instance<SINGLE>(insts, bmap, lblk);
  if (lblk < 0) return;
  const int64_t step = I.st.step;
  for (int p = 0; p < NPT; p++) {
    const int64_t i = (int64_t)lblk * TILE + p * (TILE / NPT) + threadIdx.x;
    if (i < I.n) ionic_point<MODEL, MIXED, BDFS>(I, I.n, step, i, i, I.mp);
  }
}

// ---------------------------------------------------------------------------
// several subdomains (paper: monodomain on subdomains Omega_i, one ionic model
// each; the ionic load sum_i M^i I_ion^i)
// ---------------------------------------------------------------------------

// One thread per ionic point.  Points i < n are the nodes, each with its
// primary subdomain's parameters; they write the node's load and initial
// guess.  Points i >= n are the interface nodes' extra subdomains; they only
// keep I_ion.  A node outside every conducting subdomain (pt_reg < 0) is no
// unknown: load and guess 0, no ionic work.
// MODEL < 0: the subdomains run different ionic models; each point takes its
// subdomain's model (a switch per point) and unit conversion.
template <int MODEL, bool MIXED, bool BDFS, bool RHS>
__device__ __forceinline__ void het_point(const InstDesc& I, int64_t step, int64_t i, int64_t node, int r) {
  const double* mp = I.rtab + (int64_t)r * NPARAM;
  if (MODEL >= 0) {
    ionic_point<MODEL, MIXED, BDFS, RHS, true>(I, I.n_pts, step, i, node, mp);
    return;
  }
  const double* cv = I.rconv[r];
  switch (I.rmodel[r]) {
    case M_AP: ionic_point<M_AP, MIXED, BDFS, RHS, true, true>(I, I.n_pts, step, i, node, mp, cv); break;
    case M_BO: ionic_point<M_BO, MIXED, BDFS, RHS, true, true>(I, I.n_pts, step, i, node, mp, cv); break;
    case M_TTP06: ionic_point<M_TTP06, MIXED, BDFS, RHS, true, true>(I, I.n_pts, step, i, node, mp, cv); break;
    default: ionic_point<M_PASSIVE, MIXED, BDFS, RHS, true, true>(I, I.n_pts, step, i, node, mp, cv); break;
  }
}

template <int MODEL, bool MIXED, bool BDFS>
__global__ __launch_bounds__(WG) void k_ionic_het(InstDesc* __restrict__ insts) {
  const InstDesc& I = insts[0];
  const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (i >= I.n_pts) return;
  const int64_t step = I.st.step;
  const int r = gmem(I.pt_reg)[i];
  if (i < I.n) {
    if (r < 0) {
      gmem(I.g)[i] = 0.0;
      gmem(I.u_new)[i] = 0.0;
      gmem(I.ipt)[i] = 0.0;
      return;
    }
    het_point<MODEL, MIXED, BDFS, true>(I, step, i, i, r);
  } else {
    const int64_t node = gmem(I.sec_node)[i - I.n];
    het_point<MODEL, MIXED, BDFS, false>(I, step, i, node, r);
  }
}

// Interface correction of the load: cvec(j) = sum_q C(j, q) (I_q - I_node_q)
// over the extra points q coupled to row j; one thread per correction row.
__global__ __launch_bounds__(WG) void k_ici_correction(InstDesc* __restrict__ insts) {
  const InstDesc& I = insts[0];
  const int64_t t = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (t >= I.n_crow) return;
  const gptr<const double> ipt = gmem((const double*)I.ipt);
  const int64_t e0 = gmem(I.cptr)[t], e1 = gmem(I.cptr)[t + 1];
  double acc = 0.0;
  for (int64_t e = e0; e < e1; e++) {
    const int32_t q = gmem(I.ccol)[e];
    acc += gmem(I.cval)[e] * (ipt[I.n + q] - ipt[gmem(I.sec_node)[q]]);
  }
  gmem(I.cvec)[gmem(I.crow)[t]] = acc;
}

// ---------------------------------------------------------------------------
// residual r = b - A x (FP64), optionally with b = M g; preconditioner; start
// of a (inner) CG solve.  Partials: <r,z>, <r,r>, <b,b>, <r32,r32>.
// ---------------------------------------------------------------------------

template <bool MIXED, bool WITH_RHS, bool SINGLE, int XMAP>
__global__ __launch_bounds__(WG) void k_residual(InstDesc* __restrict__ insts, const BlockMap* __restrict__ bmap) {
  int lblk;
  InstDesc& I = instance<SINGLE, XMAP>(insts, bmap, lblk);
  if (lblk < 0) return;
  InstState& S = I.st;
  // a refinement sweep only restarts an instance whose inner solve is done
  const gptr<double> rec = gmem(I.pipe_rec) + PIPE_REC * (int64_t)lblk;
  if (!WITH_RHS) {
    // a refinement residual runs once the sweep's inner solve is done (the
    // pipelined inner solve records that per tile)
    if (MIXED && I.cg_pipe) {
      if (S.conv != 0 || rec[3] == 0.0) return;
    } else {
      const Ctl c = ld_ctl(S);
      if (c.conv != 0 || c.conv_in == 0) return;
    }
  }
  const int sig = min(I.bdf, (int)S.step + 1);
  const double* __restrict__ x = I.u_new;
  const gptr<double> b = gmem(I.b), r = gmem(I.r), z = gmem(I.z);
  const gptr<float> r32 = gmem(I.r32), z32 = gmem(I.z32);
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  const int64_t i0 = (int64_t)lblk * TILE + threadIdx.x;
#pragma unroll
  for (int rw = 0; rw < RPT; rw++) {
    const int64_t i = i0 + rw * WG;
    const bool valid = i < I.n;
    double bi = 0.0, ri = 0.0;
    if (valid) {
      const bool mf = !MIXED && I.fmt == FMT_MF;
      if (WITH_RHS) {
        bi = mf ? mf_row(I, I.yM, i) : spmv_row<double, double, double>(I, I.valM, I.g, i);
        if (I.het) bi -= gmem((const double*)I.cvec)[i];
        b[i] = bi;
      } else {
        bi = b[i];
      }
      ri = bi - (mf ? mf_row(I, I.yA, i) : spmv_row<double, double, double>(I, I.valA[sig - 1], x, i));
    }
    if (!MIXED) {
      const double zi = precond_apply<double>(I.dinv[sig - 1], I.bld, I.block, i, valid, ri);
      if (valid) {
        r[i] = ri;
        z[i] = zi;
        v[0] += ri * zi;
        v[1] += ri * ri;
      }
    } else {
      const float rf = (float)ri;
      const float zf = precond_apply<float>(I.dinv32[sig - 1], I.bld, I.block, i, valid, rf);
      if (valid) {
        r32[i] = rf;
        z32[i] = zf;
        v[0] += (double)rf * (double)zf;
        v[1] += ri * ri;
        v[3] += (double)rf * (double)rf;
      }
    }
    if (WITH_RHS) v[2] += bi * bi;
  }
  write_partials<4>(v, I.partial + (int64_t)PART_RES * I.nblk, I.nblk, lblk);
  if ((MIXED || WITH_RHS) && I.cg_pipe && threadIdx.x == 0) {
    // pipelined CG: this tile's record restarts at iteration -1 of a
    // (inner) solve that is not done
    rec[0] = -1.0;
    rec[1] = 1.0;
    rec[2] = 1.0;
    rec[3] = 0.0;
  }
  if (lblk == 0 && threadIdx.x == 0) {
    // a new (inner) solve starts at iteration 0; fields read by no workgroup
    // of this kernel (conv_in is cleared by the finalize that follows).  The
    // FP64 solve counts its iterations in the SpMV kernel, which advances
    // the counter before each update: it starts from -1.
    S.it = (MIXED || !WITH_RHS) ? 0 : -1;
    if (WITH_RHS) {
      S.conv = 0;
      S.conv_in = 0;
      S.outer = 0;
      S.restart = 0;
    } else {
      S.outer += 1;
      S.restart = 1;
    }
  }
}

// ---------------------------------------------------------------------------
// CG iteration, part 1: w = A z and the partials of <w, z>.
// ---------------------------------------------------------------------------

template <bool MIXED, bool SINGLE, int XMAP>
__global__ __launch_bounds__(WG) void k_cg_spmv(InstDesc* __restrict__ insts, const BlockMap* __restrict__ bmap) {
  int lblk;
  InstDesc& I = instance<SINGLE, XMAP>(insts, bmap, lblk);
  if (lblk < 0) return;
  InstState& S = I.st;
  // a pool may hold instances of the pipelined form, which skip this kernel
  if (cg_idle(S) || (!SINGLE && I.cg_pipe)) return;
  // FP64: the iteration index the following update kernel works on (no
  // workgroup of this kernel reads it)
  if (!MIXED && lblk == 0 && threadIdx.x == 0) S.it = S.it + 1;
  const int sig = min(I.bdf, (int)S.step + 1);
  const int64_t i0 = (int64_t)lblk * TILE + threadIdx.x;
  double v[1] = {0.0};
#pragma unroll
  for (int rw = 0; rw < RPT; rw++) {
    const int64_t i = i0 + rw * WG;
    if (i >= I.n) break;
    if (MIXED) {
      const float wi = spmv_row<float, float, float>(I, I.valA32[sig - 1], I.z32, i);
      gmem(I.w32)[i] = wi;
      v[0] += (double)wi * (double)gmem(I.z32)[i];
    } else {
      const double wi = I.fmt == FMT_MF ? mf_row(I, I.yA, i)
                                         : spmv_row<double, double, double>(I, I.valA[sig - 1], I.z, i);
      gmem(I.w)[i] = wi;
      v[0] += wi * gmem(I.z)[i];
    }
  }
  write_partials<1>(v, I.partial + (int64_t)PART_SPMV * I.nblk, I.nblk, lblk);
}

// ---------------------------------------------------------------------------
// CG iteration, part 2: one workgroup per instance.  Adds the partials of the
// kernels since the last finalize (residual or update, then SpMV), decides
// convergence of iteration k's residual and forms the Chronopoulos-Gear step
// lengths beta_k = gamma_k / gamma_{k-1},
// alpha_k = gamma_k / (delta_k - beta_k gamma_k / alpha_{k-1}).
// ---------------------------------------------------------------------------

// The kernel is latency bound: the descriptor and state fields it needs are
// loaded as one batch before any branch, and the partial sums (ordinary
// memory) are read before the idle test, so the chain of dependent loads is
// descriptor -> partials -> reduction.  A single instance (SINGLE) needs no
// instance-list lookup.
template <bool MIXED, bool SINGLE>
__global__ __launch_bounds__(FIN_WG) void k_cg_finalize(InstDesc* __restrict__ insts,
                                                        const int32_t* __restrict__ ids) {
  InstDesc& I = SINGLE ? insts[0] : insts[ids[blockIdx.x]];
  InstState& S = I.st;
  const Ctl ctl = ld_ctl(S);
  const int nblk = I.nblk;
  const int k = S.it;
  const double* __restrict__ P = I.partial;
  double t[4];
  double dl[1];
  // one pass over adjacent partial streams: residual [4] + SpMV [1] at the
  // start of a solve, SpMV [1] + update [2] afterwards
  static_assert(PART_SPMV == PART_RES + 4 && PART_UPD == PART_SPMV + 1, "partial stream layout");
  if (k == 0) {
    double a[5];
    reduce_partials<FIN_WG, 5>(P + (int64_t)PART_RES * nblk, nblk, a);
    t[0] = a[0]; t[1] = a[1]; t[2] = a[2]; t[3] = a[3];
    dl[0] = a[4];
  } else {
    double a[3];
    reduce_partials<FIN_WG, 3>(P + (int64_t)PART_SPMV * nblk, nblk, a);
    dl[0] = a[0];
    t[0] = a[1];
    t[1] = a[2];
    t[2] = t[3] = 0.0;
  }
  if (ctl.conv != 0 || (ctl.conv_in != 0 && ctl.restart == 0) || (!SINGLE && I.cg_pipe)) return;
  if (threadIdx.x != 0) return;
  S.restart = 0;
  S.conv_in = 0;
  const double delta = dl[0];
  const double gamma = t[0];
  bool done = false, stop_in = false;
  int flag = 0;
  double rr;
  if (k == 0) {
    const bool first = MIXED ? (S.outer == 0) : true;
    if (first) {
      S.bb = t[2];
      S.tol2 = I.rtol * I.rtol * t[2];
    }
    const double rr_outer = t[1];
    rr = MIXED ? t[3] : t[1];
    S.rr_outer = rr_outer;
    S.rr_in0 = rr;
    if (!(rr_outer == rr_outer) || !(gamma == gamma)) {
      done = true;
      flag = F_NAN;
    } else if (rr_outer <= S.tol2) {
      done = true;
    } else if (MIXED && S.outer > I.max_outer) {
      done = true;
      flag = F_NOCONV;
    }
  } else {
    rr = t[1];
    if (!(rr == rr)) {
      done = true;
      flag = F_NAN;
    } else if (MIXED) {
      stop_in = rr <= I.inner_rtol * I.inner_rtol * S.rr_in0 || k >= I.max_it;
    } else if (rr <= S.tol2) {
      done = true;
    } else if (k >= I.max_it) {
      done = true;
      flag = F_NOCONV;
    }
  }
  S.rr = rr;
  if (!done && !stop_in) {
    double beta, denom;
    if (k == 0) {
      beta = 0.0;
      denom = delta;
    } else {
      beta = gamma / S.gamma_prev;
      denom = delta - beta * gamma / S.alpha_prev;
    }
    const double alpha = gamma / denom;
    if (!(denom > 0.0) || !(alpha == alpha)) {
      if (delta == delta) {
        flag |= F_BREAKDOWN;
        if (MIXED) stop_in = true;
        else done = true;
      } else {
        flag |= F_NAN;
        done = true;
      }
    } else {
      S.gamma_cur = gamma;
      S.alpha_cur = alpha;
      S.beta = beta;
      S.it_f = k;
    }
  }
  if (flag) S.flags |= flag;
  if (done) S.conv = 1;
  if (stop_in) S.conv_in = 1;
}

// ---------------------------------------------------------------------------
// CG iteration, part 3: p = z + beta p, s = w + beta s, x += alpha p,
// r -= alpha s, z = P^{-1} r; partials <r, z>, <r, r>.
// ---------------------------------------------------------------------------

template <bool MIXED, bool SINGLE, int XMAP>
__global__ __launch_bounds__(WG) void k_cg_update(InstDesc* __restrict__ insts, const BlockMap* __restrict__ bmap) {
  int lblk;
  InstDesc& I = instance<SINGLE, XMAP>(insts, bmap, lblk);
  if (lblk < 0) return;
  InstState& S = I.st;
  if (cg_idle(S) || (!SINGLE && I.cg_pipe)) return;
  const int k = S.it_f;
  const double alpha = S.alpha_cur, beta = S.beta;
  const int sig = min(I.bdf, (int)S.step + 1);
  const gptr<double> x = gmem(I.u_new);
  const int64_t i0 = (int64_t)lblk * TILE + threadIdx.x;
  double v[2] = {0.0, 0.0};
#pragma unroll
  for (int rw = 0; rw < RPT; rw++) {
    const int64_t i = i0 + rw * WG;
    const bool valid = i < I.n;
    if (MIXED) {
      const float fb = (float)beta, fa = (float)alpha;
      float rn = 0.0f;
      if (valid) {
        const float z = gmem(I.z32)[i], w = gmem(I.w32)[i];
        const float pn = (k == 0) ? z : z + fb * gmem(I.p32)[i];
        const float sn = (k == 0) ? w : w + fb * gmem(I.s32)[i];
        x[i] += alpha * (double)pn;
        rn = gmem(I.r32)[i] - fa * sn;
        gmem(I.p32)[i] = pn; gmem(I.s32)[i] = sn; gmem(I.r32)[i] = rn;
      }
      const float zn = precond_apply<float>(I.dinv32[sig - 1], I.bld, I.block, i, valid, rn);
      if (valid) {
        gmem(I.z32)[i] = zn;
        v[0] += (double)rn * (double)zn;
        v[1] += (double)rn * (double)rn;
      }
    } else {
      double rn = 0.0;
      if (valid) {
        const double z = gmem(I.z)[i], w = gmem(I.w)[i];
        const double pn = (k == 0) ? z : z + beta * gmem(I.p)[i];
        const double sn = (k == 0) ? w : w + beta * gmem(I.s)[i];
        x[i] += alpha * pn;
        rn = gmem(I.r)[i] - alpha * sn;
        gmem(I.p)[i] = pn; gmem(I.s)[i] = sn; gmem(I.r)[i] = rn;
      }
      const double zn = precond_apply<double>(I.dinv[sig - 1], I.bld, I.block, i, valid, rn);
      if (valid) {
        gmem(I.z)[i] = zn;
        v[0] += rn * zn;
        v[1] += rn * rn;
      }
    }
  }
  write_partials<2>(v, I.partial + (int64_t)PART_UPD * I.nblk, I.nblk, lblk);
  if (lblk == 0 && threadIdx.x == 0) {
    // read by the next finalize only
    S.gamma_prev = S.gamma_cur;
    S.alpha_prev = S.alpha_cur;
    S.it = k + 1;
    S.it_step += 1;
  }
}

// ---------------------------------------------------------------------------
// FP64 CG iteration, part 2 without a finalize kernel: every workgroup adds
// the partial sums of the kernels before it (the residual or the previous
// update, and the SpMV) in the same fixed order, so all of them take the
// same convergence decision and the same step lengths bitwise; workgroup 0
// records them for the next iteration.  Iteration k (advanced by the SpMV
// kernel) keeps gamma_k, alpha_k in slot k & 1 and writes its partials to
// the stream pair k & 1, so no workgroup writes what another workgroup of
// the same launch reads.  The control flag `conv` is only ever set here
// once convergence is decided, and every workgroup reaching this launch
// takes that decision itself, so reading it early or late is equivalent.
// ---------------------------------------------------------------------------

template <bool SINGLE, int XMAP>
__global__ __launch_bounds__(WG) void k_cg_update64(InstDesc* __restrict__ insts, const BlockMap* __restrict__ bmap) {
  int lblk;
  InstDesc& I = instance<SINGLE, XMAP>(insts, bmap, lblk);
  if (lblk < 0) return;
  InstState& S = I.st;
  if (S.conv != 0 || (!SINGLE && I.cg_pipe)) return;
  const int k = S.it;
  const int nblk = I.nblk;
  const int sig = min(I.bdf, (int)S.step + 1);
  const int64_t i0 = (int64_t)lblk * TILE + threadIdx.x;
  // this thread's rows, loaded before the reduction so that they are in
  // flight while the partial sums are added
  double zv[RPT], wv[RPT], pv[RPT], sv[RPT], xv[RPT], rv[RPT];
#pragma unroll
  for (int rw = 0; rw < RPT; rw++) {
    const int64_t i = i0 + rw * WG;
    zv[rw] = wv[rw] = pv[rw] = sv[rw] = xv[rw] = rv[rw] = 0.0;
    if (i < I.n) {
      zv[rw] = gmem(I.z)[i];
      wv[rw] = gmem(I.w)[i];
      pv[rw] = gmem(I.p)[i];
      sv[rw] = gmem(I.s)[i];
      xv[rw] = gmem(I.u_new)[i];
      rv[rw] = gmem(I.r)[i];
    }
  }
  const double* __restrict__ P = I.partial;
  double gamma, rr, delta, bb = 0.0;
  if (k == 0) {
    double a[5];
    const int c[5] = {PART_RES, PART_RES + 1, PART_RES + 2, PART_RES + 3, PART_SPMV};
    reduce_streams<WG, 5>(P, c, nblk, a);
    gamma = a[0];
    rr = a[1];
    bb = a[2];
    delta = a[4];
  } else {
    double a[3];
    const int u = PART_UPD + 2 * ((k - 1) & 1);
    const int c[3] = {PART_SPMV, u, u + 1};
    reduce_streams<WG, 3>(P, c, nblk, a);
    delta = a[0];
    gamma = a[1];
    rr = a[2];
  }
  const double tol2 = (k == 0) ? I.rtol * I.rtol * bb : S.tol2;
  int flag = 0;
  bool done = false;
  double alpha = 0.0, beta = 0.0;
  if (!(rr == rr) || !(gamma == gamma)) {
    done = true;
    flag = F_NAN;
  } else if (rr <= tol2) {
    done = true;
  } else if (k >= I.max_it) {
    done = true;
    flag = F_NOCONV;
  } else {
    double denom;
    if (k == 0) {
      denom = delta;
    } else {
      beta = gamma / S.gam[(k - 1) & 1];
      denom = delta - beta * gamma / S.alp[(k - 1) & 1];
    }
    alpha = gamma / denom;
    if (!(denom > 0.0) || !(alpha == alpha)) {
      done = true;
      flag = (delta == delta) ? F_BREAKDOWN : F_NAN;
    }
  }
  if (lblk == 0 && threadIdx.x == 0) {
    // read by later kernels only
    S.rr = rr;
    if (k == 0) {
      S.bb = bb;
      S.tol2 = tol2;
    }
    if (done) {
      if (flag) S.flags |= flag;
      S.conv = 1;
    } else {
      S.gam[k & 1] = gamma;
      S.alp[k & 1] = alpha;
      S.it_step += 1;
    }
  }
  if (done) return;
  double v[2] = {0.0, 0.0};
#pragma unroll
  for (int rw = 0; rw < RPT; rw++) {
    const int64_t i = i0 + rw * WG;
    const bool valid = i < I.n;
    double rn = 0.0;
    if (valid) {
      const double pn = (k == 0) ? zv[rw] : zv[rw] + beta * pv[rw];
      const double sn = (k == 0) ? wv[rw] : wv[rw] + beta * sv[rw];
      gmem(I.u_new)[i] = xv[rw] + alpha * pn;
      rn = rv[rw] - alpha * sn;
      gmem(I.p)[i] = pn;
      gmem(I.s)[i] = sn;
      gmem(I.r)[i] = rn;
    }
    const double zn = precond_apply<double>(I.dinv[sig - 1], I.bld, I.block, i, valid, rn);
    if (valid) {
      gmem(I.z)[i] = zn;
      v[0] += rn * zn;
      v[1] += rn * rn;
    }
  }
  write_partials<2>(v, I.partial + (int64_t)(PART_UPD + 2 * (k & 1)) * nblk, nblk, lblk);
}

// ---------------------------------------------------------------------------
// FP64 pipelined PCG (Ghysels and Vanroose's reformulation of CG, in which
// the SpMV of an iteration acts on a vector the previous launch finished, so
// that the SpMV, the global sums and the vector updates share one launch).
// With P the (block) Jacobi preconditioner, u = P^-1 r and m = P^-1 w are
// formed on the fly (q = P^-1 s is never needed: z = A q is carried by its
// own recurrence).  Iteration k, given gamma_k = <r_k, u_k>, delta_k =
// <w_k, u_k> and <r_k, r_k> from the partials of the previous launch:
//   beta_k = gamma_k / gamma_{k-1}, alpha_k = gamma_k / (delta_k - beta_k gamma_k / alpha_{k-1})
//   z = A m_k + beta z,  s = w + beta s,  p = u + beta p
//   x += alpha p,  r -= alpha s,  w -= alpha z,  m_{k+1} = P^-1 w
// In exact arithmetic this is the same iteration as the Chronopoulos-Gear
// CG above; rounding differs, so results agree to the solver tolerance, not
// bitwise.  Start (after the residual kernel, whose z is u_0):
// k_cg_pipe_start forms w_0 = A u_0, m_0 = P^-1 w_0 and delta_0.
// ---------------------------------------------------------------------------

template <bool SINGLE, int XMAP>
__global__ __launch_bounds__(WG) void k_cg_pipe_start(InstDesc* __restrict__ insts,
                                                      const BlockMap* __restrict__ bmap) {
  int lblk;
  InstDesc& I = instance<SINGLE, XMAP>(insts, bmap, lblk);
  if (lblk < 0) return;
  const InstState& S = I.st;
  if (!I.cg_pipe || S.conv != 0) return;
  const int sig = min(I.bdf, (int)S.step + 1);
  const int64_t i0 = (int64_t)lblk * TILE + threadIdx.x;
  double v[1] = {0.0};
#pragma unroll
  for (int rw = 0; rw < RPT; rw++) {
    const int64_t i = i0 + rw * WG;
    const bool valid = i < I.n;
    double wi = 0.0;
    if (valid) {
      wi = I.fmt == FMT_MF ? mf_row(I, I.yA, i) : spmv_row<double, double, double>(I, I.valA[sig - 1], I.z, i);
      gmem(I.w)[i] = wi;
      v[0] += wi * gmem(I.z)[i];
    }
    // every lane takes part (block Jacobi shuffles across the wavefront)
    const double mi = precond_apply<double>(I.dinv[sig - 1], I.bld, I.block, i, valid, wi);
    if (valid) gmem(I.b)[i] = mi;
  }
  write_partials<1>(v, I.partial + (int64_t)PART_SPMV * I.nblk, I.nblk, lblk);
}

// OP 1: the operator is the 14-diagonal symmetric DIA of the Q1 lattice and
// the preconditioner Jacobi (the row product and the inverse diagonal are
// then fixed at compile time); OP 0: any format and preconditioner.
template <bool SINGLE, int XMAP, int OP>
__global__ __launch_bounds__(WG) void k_cg_pipe(InstDesc* __restrict__ insts, const BlockMap* __restrict__ bmap) {
  int lblk;
  InstDesc& I = instance<SINGLE, XMAP>(insts, bmap, lblk);
  if (lblk < 0) return;
  InstState& S = I.st;
  if (!I.cg_pipe || S.conv != 0) return;
  const int nblk = I.nblk;
  const int sig = min(I.bdf, (int)S.step + 1);
  const gptr<double> rec = gmem(I.pipe_rec) + PIPE_REC * (int64_t)lblk;
  const int k = (int)rec[0] + 1;
  const double gam_prev = rec[1], alp_prev = rec[2];
  const int64_t i0 = (int64_t)lblk * TILE + threadIdx.x;
  // this thread's rows, loaded before the reduction so that they are in
  // flight while the partial sums are added
  const double* dinv = I.dinv[sig - 1];
  double zv[RPT], wv[RPT], pv[RPT], sv[RPT], xv[RPT], rv[RPT], dv[RPT];
#pragma unroll
  for (int rw = 0; rw < RPT; rw++) {
    const int64_t i = i0 + rw * WG;
    zv[rw] = wv[rw] = pv[rw] = sv[rw] = xv[rw] = rv[rw] = dv[rw] = 0.0;
    if (i < I.n) {
      zv[rw] = gmem(I.z)[i];
      wv[rw] = gmem(I.w)[i];
      pv[rw] = gmem(I.p)[i];
      sv[rw] = gmem(I.s)[i];
      xv[rw] = gmem(I.u_new)[i];
      rv[rw] = gmem(I.r)[i];
      if (OP == 1) dv[rw] = gmem(dinv)[i];
    }
  }
  const double* __restrict__ P = I.partial;
  double gamma, delta, rr, bb = 0.0;
  if (k == 0) {
    double a[4];
    const int c[4] = {PART_RES, PART_SPMV, PART_RES + 1, PART_RES + 2};
    reduce_streams<WG, 4>(P, c, nblk, a);
    gamma = a[0];
    delta = a[1];
    rr = a[2];
    bb = a[3];
  } else {
    double a[3];
    const int u = PART_PIPE + 3 * ((k - 1) & 1);
    const int c[3] = {u, u + 1, u + 2};
    reduce_streams<WG, 3>(P, c, nblk, a);
    gamma = a[0];
    delta = a[1];
    rr = a[2];
  }
  const double tol2 = (k == 0) ? I.rtol * I.rtol * bb : S.tol2;
  int flag = 0;
  bool done = false;
  double alpha = 0.0, beta = 0.0;
  if (!(rr == rr) || !(gamma == gamma)) {
    done = true;
    flag = F_NAN;
  } else if (rr <= tol2) {
    done = true;
  } else if (k >= I.max_it) {
    done = true;
    flag = F_NOCONV;
  } else {
    double denom = delta;
    if (k > 0) {
      beta = gamma / gam_prev;
      denom = delta - beta * gamma / alp_prev;
    }
    alpha = gamma / denom;
    if (!(denom > 0.0) || !(alpha == alpha)) {
      done = true;
      flag = (delta == delta) ? F_BREAKDOWN : F_NAN;
    }
  }
  if (lblk == 0 && threadIdx.x == 0) {
    S.rr = rr;
    if (k == 0) {
      S.bb = bb;
      S.tol2 = tol2;
    }
    if (done) {
      if (flag) S.flags |= flag;
      S.conv = 1;
    } else {
      S.it_step += 1;
    }
  }
  if (done) return;
  // every thread has read the record (before the reduction's barrier)
  if (threadIdx.x == 0) {
    rec[0] = (double)k;
    rec[1] = gamma;
    rec[2] = alpha;
  }
  const double* m_in = (k & 1) ? I.g : I.b;
  const gptr<double> m_out = gmem((k & 1) ? I.b : I.g);
  const bool jacobi = OP == 1 || I.block == 1;
  double v[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int rw = 0; rw < RPT; rw++) {
    const int64_t i = i0 + rw * WG;
    const bool valid = i < I.n;
    double ni = 0.0, di = dv[rw];
    if (valid) {
      if (OP == 1) {
        ni = dia_row<14, double, double, double>(I, I.valA[sig - 1], m_in, i, 14);
      } else {
        ni = I.fmt == FMT_MF ? mf_row(I, I.yA, i) : spmv_row<double, double, double>(I, I.valA[sig - 1], m_in, i);
        if (jacobi) di = gmem(dinv)[i];
      }
    }
    // u = P^-1 r (every lane takes part in the block-Jacobi shuffles)
    // Every rounding step is written out (products by __dmul_rn, fused
    // multiply-adds by fma), so the compiler cannot contract differently in
    // the specialized and the generic instantiation: both give the same bits.
    const double ui = jacobi ? __dmul_rn(di, rv[rw]) : precond_apply<double>(dinv, I.bld, I.block, i, valid, rv[rw]);
    double wn = 0.0, rn = 0.0;
    if (valid) {
      const double zn = fma(beta, zv[rw], ni);
      const double sn = fma(beta, sv[rw], wv[rw]);
      const double pn = fma(beta, pv[rw], ui);
      gmem(I.u_new)[i] = fma(alpha, pn, xv[rw]);
      rn = fma(-alpha, sn, rv[rw]);
      wn = fma(-alpha, zn, wv[rw]);
      gmem(I.z)[i] = zn;
      gmem(I.s)[i] = sn;
      gmem(I.p)[i] = pn;
      gmem(I.r)[i] = rn;
      gmem(I.w)[i] = wn;
    }
    const double mn = jacobi ? __dmul_rn(di, wn) : precond_apply<double>(dinv, I.bld, I.block, i, valid, wn);
    const double un = jacobi ? __dmul_rn(di, rn) : precond_apply<double>(dinv, I.bld, I.block, i, valid, rn);
    if (valid) {
      m_out[i] = mn;
      v[0] = fma(rn, un, v[0]);
      v[1] = fma(wn, un, v[1]);
      v[2] = fma(rn, rn, v[2]);
    }
  }
  write_partials<3>(v, I.partial + (int64_t)(PART_PIPE + 3 * (k & 1)) * nblk, nblk, lblk);
}

// ---------------------------------------------------------------------------
// Mixed precision: the FP32 inner solve of each refinement sweep in the
// pipelined form (the same recurrences as k_cg_pipe in FP32 with FP64
// partial sums; the solution accumulates in FP64).  The start kernel runs
// right after a residual (the tile's record at iteration -1): w = A z,
// m = P^-1 w, delta.  The iteration kernel takes, at k = 0, the outer
// decisions of the sweep (FP64 residual against the tolerance, sweep limit)
// and afterwards stops the inner solve at inner_rtol relative to the
// sweep's first inner residual, recording that in the tile's record, which
// the next refinement residual reads.
// ---------------------------------------------------------------------------

// Relative inner residual below which an FP32 solve stops gaining accuracy
// on the FP64 residual (the FP32 operator differs from the FP64 one by about
// 6e-8 relative).
constexpr double INNER_FLOOR = 1e-5;

template <bool SINGLE, int XMAP>
__global__ __launch_bounds__(WG) void k_cg_pipe32_start(InstDesc* __restrict__ insts,
                                                        const BlockMap* __restrict__ bmap) {
  int lblk;
  InstDesc& I = instance<SINGLE, XMAP>(insts, bmap, lblk);
  if (lblk < 0) return;
  const InstState& S = I.st;
  if (!I.cg_pipe || S.conv != 0) return;
  if (gmem(I.pipe_rec)[PIPE_REC * (int64_t)lblk] != -1.0) return;   // not right after a residual
  const int sig = min(I.bdf, (int)S.step + 1);
  const int64_t i0 = (int64_t)lblk * TILE + threadIdx.x;
  double v[1] = {0.0};
#pragma unroll
  for (int rw = 0; rw < RPT; rw++) {
    const int64_t i = i0 + rw * WG;
    const bool valid = i < I.n;
    float wi = 0.0f;
    if (valid) {
      wi = spmv_row<float, float, float>(I, I.valA32[sig - 1], I.z32, i);
      gmem(I.w32)[i] = wi;
      v[0] += (double)wi * (double)gmem(I.z32)[i];
    }
    const float mi = precond_apply<float>(I.dinv32[sig - 1], I.bld, I.block, i, valid, wi);
    if (valid) gmem(I.m32[0])[i] = mi;
  }
  write_partials<1>(v, I.partial + (int64_t)PART_SPMV * I.nblk, I.nblk, lblk);
}

// OP as for k_cg_pipe: 1 = the 14-diagonal symmetric DIA with Jacobi.
template <bool SINGLE, int XMAP, int OP>
__global__ __launch_bounds__(WG) void k_cg_pipe32(InstDesc* __restrict__ insts, const BlockMap* __restrict__ bmap) {
  int lblk;
  InstDesc& I = instance<SINGLE, XMAP>(insts, bmap, lblk);
  if (lblk < 0) return;
  InstState& S = I.st;
  if (!I.cg_pipe || S.conv != 0) return;
  const gptr<double> rec = gmem(I.pipe_rec) + PIPE_REC * (int64_t)lblk;
  if (rec[3] != 0.0) return;   // this sweep's inner solve is done
  const int nblk = I.nblk;
  const int sig = min(I.bdf, (int)S.step + 1);
  const int k = (int)rec[0] + 1;
  const double gam_prev = rec[1], alp_prev = rec[2], rr_in0_rec = rec[4], f2_rec = rec[5];
  const int64_t i0 = (int64_t)lblk * TILE + threadIdx.x;
  const float* dinv = I.dinv32[sig - 1];
  float zv[RPT], wv[RPT], pv[RPT], sv[RPT], rv[RPT], dv[RPT];
  double xv[RPT];
#pragma unroll
  for (int rw = 0; rw < RPT; rw++) {
    const int64_t i = i0 + rw * WG;
    zv[rw] = wv[rw] = pv[rw] = sv[rw] = rv[rw] = dv[rw] = 0.0f;
    xv[rw] = 0.0;
    if (i < I.n) {
      zv[rw] = gmem(I.z32)[i];
      wv[rw] = gmem(I.w32)[i];
      pv[rw] = gmem(I.p32)[i];
      sv[rw] = gmem(I.s32)[i];
      rv[rw] = gmem(I.r32)[i];
      xv[rw] = gmem(I.u_new)[i];
      if (OP == 1) dv[rw] = gmem(dinv)[i];
    }
  }
  const double* __restrict__ P = I.partial;
  double gamma, delta, rr, rr_outer = 0.0, bb = 0.0;
  if (k == 0) {
    double a[5];
    const int c[5] = {PART_RES, PART_SPMV, PART_RES + 3, PART_RES + 1, PART_RES + 2};
    reduce_streams<WG, 5>(P, c, nblk, a);
    gamma = a[0];
    delta = a[1];
    rr = a[2];
    rr_outer = a[3];
    bb = a[4];
  } else {
    double a[3];
    const int u = PART_PIPE + 3 * ((k - 1) & 1);
    const int c[3] = {u, u + 1, u + 2};
    reduce_streams<WG, 3>(P, c, nblk, a);
    gamma = a[0];
    delta = a[1];
    rr = a[2];
  }
  const bool first = k == 0 && S.outer == 0;
  const double tol2 = first ? I.rtol * I.rtol * bb : S.tol2;
  const double rr_in0 = k == 0 ? rr : rr_in0_rec;
  // the sweep's inner target (squared reduction of the inner residual):
  // inner_rtol, or tighter when that finishes the step in this sweep: the
  // reduction that brings the FP64 residual to half the tolerance, if an
  // FP32 solve can reach it (not below INNER_FLOOR; otherwise another sweep
  // follows anyway and inner_rtol is the cheaper target)
  double f2 = f2_rec;
  if (k == 0) {
    const double want = 0.25 * tol2 / rr_outer, hi = I.inner_rtol * I.inner_rtol;
    f2 = (want >= INNER_FLOOR * INNER_FLOOR && want < hi) ? want : hi;
  }
  int flag = 0;
  bool done = false, stop_in = false;
  if (k == 0) {
    if (!(rr_outer == rr_outer) || !(gamma == gamma)) {
      done = true;
      flag = F_NAN;
    } else if (rr_outer <= tol2) {
      done = true;
    } else if (S.outer > I.max_outer) {
      done = true;
      flag = F_NOCONV;
    }
  } else if (!(rr == rr)) {
    done = true;
    flag = F_NAN;
  } else {
    stop_in = rr <= f2 * rr_in0 || k >= I.max_it;
  }
  double alpha = 0.0, beta = 0.0;
  if (!done && !stop_in) {
    double denom = delta;
    if (k > 0) {
      beta = gamma / gam_prev;
      denom = delta - beta * gamma / alp_prev;
    }
    alpha = gamma / denom;
    if (!(denom > 0.0) || !(alpha == alpha)) {
      if (delta == delta) {
        flag |= F_BREAKDOWN;
        stop_in = true;
      } else {
        flag |= F_NAN;
        done = true;
      }
    }
  }
  if (lblk == 0 && threadIdx.x == 0) {
    S.rr = rr;
    if (k == 0) {
      S.rr_outer = rr_outer;
      S.rr_in0 = rr;
    }
    if (first) {
      S.bb = bb;
      S.tol2 = tol2;
    }
    if (flag) S.flags |= flag;
    if (done) {
      S.conv = 1;
    } else if (stop_in) {
      S.conv_in = 1;
      S.sw_its[S.outer < 2 ? S.outer : 2] = k;
    } else {
      S.it_step += 1;
    }
  }
  // every thread has read the record (before the reduction's barrier)
  if (threadIdx.x == 0) {
    if (k == 0) {
      rec[4] = rr;
      rec[5] = f2;
    }
    if (stop_in && !done) rec[3] = 1.0;
  }
  if (done || stop_in) return;
  if (threadIdx.x == 0) {
    rec[0] = (double)k;
    rec[1] = gamma;
    rec[2] = alpha;
  }
  const float* m_in = I.m32[k & 1];
  const gptr<float> m_out = gmem(I.m32[(k + 1) & 1]);
  const bool jacobi = OP == 1 || I.block == 1;
  const float fa = (float)alpha, fb = (float)beta;
  double v[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int rw = 0; rw < RPT; rw++) {
    const int64_t i = i0 + rw * WG;
    const bool valid = i < I.n;
    float ni = 0.0f, di = dv[rw];
    if (valid) {
      if (OP == 1) {
        ni = dia_row<14, float, float, float>(I, I.valA32[sig - 1], m_in, i, 14);
      } else {
        ni = spmv_row<float, float, float>(I, I.valA32[sig - 1], m_in, i);
        if (jacobi) di = gmem(dinv)[i];
      }
    }
    const float ui = jacobi ? __fmul_rn(di, rv[rw]) : precond_apply<float>(dinv, I.bld, I.block, i, valid, rv[rw]);
    float wn = 0.0f, rn = 0.0f;
    if (valid) {
      const float zn = fmaf(fb, zv[rw], ni);
      const float sn = fmaf(fb, sv[rw], wv[rw]);
      const float pn = fmaf(fb, pv[rw], ui);
      gmem(I.u_new)[i] = fma(alpha, (double)pn, xv[rw]);
      rn = fmaf(-fa, sn, rv[rw]);
      wn = fmaf(-fa, zn, wv[rw]);
      gmem(I.z32)[i] = zn;
      gmem(I.s32)[i] = sn;
      gmem(I.p32)[i] = pn;
      gmem(I.r32)[i] = rn;
      gmem(I.w32)[i] = wn;
    }
    const float mn = jacobi ? __fmul_rn(di, wn) : precond_apply<float>(dinv, I.bld, I.block, i, valid, wn);
    const float un = jacobi ? __fmul_rn(di, rn) : precond_apply<float>(dinv, I.bld, I.block, i, valid, rn);
    if (valid) {
      m_out[i] = mn;
      v[0] = fma((double)rn, (double)un, v[0]);
      v[1] = fma((double)wn, (double)un, v[1]);
      v[2] = fma((double)rn, (double)rn, v[2]);
    }
  }
  write_partials<3>(v, I.partial + (int64_t)(PART_PIPE + 3 * (k & 1)) * nblk, nblk, lblk);
}

// ---------------------------------------------------------------------------
// activation time; end of step
// ---------------------------------------------------------------------------

template <bool SINGLE>
__global__ __launch_bounds__(TILE) void k_activation(InstDesc* __restrict__ insts, const BlockMap* __restrict__ bmap) {
  int lblk;
  const InstDesc& I = instance<SINGLE>(insts, bmap, lblk);
  if (lblk < 0) return;
  const int64_t i = (int64_t)lblk * TILE + threadIdx.x;
  if (i >= I.n) return;
  const double t = (double)(I.st.step + 1) * I.dt;
  const double un = gmem(I.u_new)[i];
  const double slope = (un - gmem(I.u_cur)[i]) * I.inv_dt;
  if (slope > gmem(I.smax)[i]) {
    gmem(I.smax)[i] = slope;
    gmem(I.at)[i] = t;
  }
  if (un > I.threshold) {
    const double tc = gmem(I.tcross)[i];
    if (tc != tc) gmem(I.tcross)[i] = t;
  }
}

// One thread per instance: advance the step counter, rotate the potential
// history slots and update the statistics.
__global__ void k_end_step(InstDesc* __restrict__ insts, const int32_t* __restrict__ ids, int n_ids) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_ids) return;
  InstDesc& I = insts[ids[t]];
  InstState& S = I.st;
  double* freed = I.u_prev2;
  I.u_prev2 = I.u_prev1;
  I.u_prev1 = I.u_cur;
  I.u_cur = I.u_new;
  I.u_new = freed;
  S.step += 1;
  S.hist = S.hist < 3 ? S.hist + 1 : 3;
  S.it_last = S.it_step;
  if (S.it_step > S.it_max) S.it_max = S.it_step;
  S.it_total += S.it_step;
  S.outer_total += S.outer;
  S.it_step = 0;
  S.it = 0;
  S.conv = 0;
  S.conv_in = 0;
  S.restart = 0;
}

// Potential in mV into a caller-owned device buffer: dst = a u + b (NaN at
// nodes outside every conducting subdomain, reg[i] < 0, when reg is given).
__global__ void k_to_mv(void* __restrict__ dst, const double* __restrict__ u, int64_t n, double a, double b,
                        int f32, const int32_t* __restrict__ reg) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = (reg && reg[i] < 0) ? __builtin_nan("") : a * u[i] + b;
  if (f32) static_cast<float*>(dst)[i] = (float)v;
  else static_cast<double*>(dst)[i] = v;
}

// Fill a device vector (used for initialisation; graph-safe, unlike memset nodes).
__global__ void k_fill(double* __restrict__ x, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

#define EP_LAUNCH2(KER, GRID, BLOCK, L)                                                     \
  do {                                                                                    \
    if ((L).single) hipLaunchKernelGGL((KER<true>), GRID, BLOCK, 0, (L).stream, (L).insts, (L).bmap); \
    else hipLaunchKernelGGL((KER<false>), GRID, BLOCK, 0, (L).stream, (L).insts, (L).bmap);        \
  } while (0)

template <int M, bool MX, int NPT>
static void ionic_dispatch_npt(const Launch& L) {
  const dim3 g(L.nblocks), b(TILE / NPT);
  if (L.ionic_bdf) {
    if (L.single) hipLaunchKernelGGL((k_ionic<M, MX, true, NPT, true>), g, b, 0, L.stream, L.insts, L.bmap);
    else hipLaunchKernelGGL((k_ionic<M, MX, false, NPT, true>), g, b, 0, L.stream, L.insts, L.bmap);
  } else {
    if (L.single) hipLaunchKernelGGL((k_ionic<M, MX, true, NPT, false>), g, b, 0, L.stream, L.insts, L.bmap);
    else hipLaunchKernelGGL((k_ionic<M, MX, false, NPT, false>), g, b, 0, L.stream, L.insts, L.bmap);
  }
}

template <int M, bool MX>
static void ionic_het_dispatch(InstDesc* d, int64_t n_pts, bool bdf, hipStream_t st) {
  const unsigned grid = (unsigned)((n_pts + WG - 1) / WG);
  if (bdf) hipLaunchKernelGGL((k_ionic_het<M, MX, true>), dim3(grid), dim3(WG), 0, st, d);
  else hipLaunchKernelGGL((k_ionic_het<M, MX, false>), dim3(grid), dim3(WG), 0, st, d);
}

template <int M, bool MX>
static void ionic_dispatch(const Launch& L) {
  if (L.ionic_npt == 4) ionic_dispatch_npt<M, MX, 4>(L);
  else if (L.ionic_npt == 2) ionic_dispatch_npt<M, MX, 2>(L);
  else ionic_dispatch_npt<M, MX, 1>(L);
}

void launch_ionic(int model, bool mixed, const Launch& L) {
  if (L.nblocks <= 0) return;
  switch (model) {
    case M_AP: mixed ? ionic_dispatch<M_AP, true>(L) : ionic_dispatch<M_AP, false>(L); break;
    case M_BO: mixed ? ionic_dispatch<M_BO, true>(L) : ionic_dispatch<M_BO, false>(L); break;
    case M_TTP06: mixed ? ionic_dispatch<M_TTP06, true>(L) : ionic_dispatch<M_TTP06, false>(L); break;
    default: mixed ? ionic_dispatch<M_PASSIVE, true>(L) : ionic_dispatch<M_PASSIVE, false>(L); break;
  }
}

void launch_ionic_het(int model, bool mixed, bool bdf, InstDesc* insts, int64_t n_pts, hipStream_t st) {
  if (n_pts <= 0) return;
  switch (model) {
    case M_AP:
      mixed ? ionic_het_dispatch<M_AP, true>(insts, n_pts, bdf, st) : ionic_het_dispatch<M_AP, false>(insts, n_pts, bdf, st);
      break;
    case M_BO:
      mixed ? ionic_het_dispatch<M_BO, true>(insts, n_pts, bdf, st) : ionic_het_dispatch<M_BO, false>(insts, n_pts, bdf, st);
      break;
    case M_TTP06:
      mixed ? ionic_het_dispatch<M_TTP06, true>(insts, n_pts, bdf, st)
            : ionic_het_dispatch<M_TTP06, false>(insts, n_pts, bdf, st);
      break;
    case M_PASSIVE:
      mixed ? ionic_het_dispatch<M_PASSIVE, true>(insts, n_pts, bdf, st)
            : ionic_het_dispatch<M_PASSIVE, false>(insts, n_pts, bdf, st);
      break;
    default:   // several ionic models
      mixed ? ionic_het_dispatch<-1, true>(insts, n_pts, bdf, st) : ionic_het_dispatch<-1, false>(insts, n_pts, bdf, st);
      break;
  }
}

void launch_ici_correction(InstDesc* insts, int64_t n_crow, hipStream_t st) {
  if (n_crow <= 0) return;
  hipLaunchKernelGGL(k_ici_correction, dim3((unsigned)((n_crow + WG - 1) / WG)), dim3(WG), 0, st, insts);
}

// CG-kernel launches: a single instance with the XCD-ordered (xmap 0), the
// dispatch-order (xmap 1) or the lattice-band (xmap 2) tile map, or a batch
// over its block map.
template <bool MX, bool RHS>
static void residual_dispatch(const Launch& L) {
  const dim3 g(L.nblocks), b(WG);
  if (!L.single) hipLaunchKernelGGL((k_residual<MX, RHS, false, 0>), g, b, 0, L.stream, L.insts, L.bmap);
  else if (L.xmap == 1) hipLaunchKernelGGL((k_residual<MX, RHS, true, 1>), g, b, 0, L.stream, L.insts, L.bmap);
  else if (L.xmap == 2) hipLaunchKernelGGL((k_residual<MX, RHS, true, 2>), g, b, 0, L.stream, L.insts, L.bmap);
  else hipLaunchKernelGGL((k_residual<MX, RHS, true, 0>), g, b, 0, L.stream, L.insts, L.bmap);
}

template <bool MX>
static void spmv_dispatch(const Launch& L) {
  const dim3 g(L.nblocks), b(WG);
  if (!L.single) hipLaunchKernelGGL((k_cg_spmv<MX, false, 0>), g, b, 0, L.stream, L.insts, L.bmap);
  else if (L.xmap == 1) hipLaunchKernelGGL((k_cg_spmv<MX, true, 1>), g, b, 0, L.stream, L.insts, L.bmap);
  else if (L.xmap == 2) hipLaunchKernelGGL((k_cg_spmv<MX, true, 2>), g, b, 0, L.stream, L.insts, L.bmap);
  else hipLaunchKernelGGL((k_cg_spmv<MX, true, 0>), g, b, 0, L.stream, L.insts, L.bmap);
}

template <bool MX>
static void update_dispatch(const Launch& L) {
  const dim3 g(L.nblocks), b(WG);
  if (!L.single) hipLaunchKernelGGL((k_cg_update<MX, false, 0>), g, b, 0, L.stream, L.insts, L.bmap);
  else if (L.xmap == 1) hipLaunchKernelGGL((k_cg_update<MX, true, 1>), g, b, 0, L.stream, L.insts, L.bmap);
  else if (L.xmap == 2) hipLaunchKernelGGL((k_cg_update<MX, true, 2>), g, b, 0, L.stream, L.insts, L.bmap);
  else hipLaunchKernelGGL((k_cg_update<MX, true, 0>), g, b, 0, L.stream, L.insts, L.bmap);
}

template <int P, bool CMP>
static void mf_apply(int which, const Launch& L) {
  constexpr int EPW = MfShape<P>::EPW;
  const unsigned grid = (unsigned)((L.mf_elems + EPW - 1) / EPW);
  if (grid == 0) return;
  if (which == 0) hipLaunchKernelGGL((k_mf_apply<P, 0, CMP>), dim3(grid), dim3(64), 0, L.stream, L.insts);
  else if (which == 1) hipLaunchKernelGGL((k_mf_apply<P, 1, CMP>), dim3(grid), dim3(64), 0, L.stream, L.insts);
  else if (which == 2) hipLaunchKernelGGL((k_mf_apply<P, 2, CMP>), dim3(grid), dim3(64), 0, L.stream, L.insts);
  else hipLaunchKernelGGL((k_mf_apply<P, 3, CMP>), dim3(grid), dim3(64), 0, L.stream, L.insts);
}

static void launch_mf_apply(int which, const Launch& L) {
  if (L.mf_p == 2) L.mf_cmp ? mf_apply<2, true>(which, L) : mf_apply<2, false>(which, L);
  else if (L.mf_p == 3) L.mf_cmp ? mf_apply<3, true>(which, L) : mf_apply<3, false>(which, L);
}

void launch_residual(bool mixed, bool with_rhs, const Launch& L) {
  if (L.nblocks <= 0) return;
  if (L.mf_p && with_rhs) {
    launch_mf_apply(1, L);   // M g
    launch_mf_apply(2, L);   // A x0
  }
  if (mixed) with_rhs ? residual_dispatch<true, true>(L) : residual_dispatch<true, false>(L);
  else with_rhs ? residual_dispatch<false, true>(L) : residual_dispatch<false, false>(L);
}

void launch_cg_spmv(bool mixed, const Launch& L) {
  if (L.nblocks <= 0) return;
  if (L.mf_p) launch_mf_apply(0, L);
  mixed ? spmv_dispatch<true>(L) : spmv_dispatch<false>(L);
}

void launch_cg_pipe32_start(const Launch& L) {
  if (L.nblocks <= 0) return;
  const dim3 g(L.nblocks), b(WG);
  if (!L.single) hipLaunchKernelGGL((k_cg_pipe32_start<false, 0>), g, b, 0, L.stream, L.insts, L.bmap);
  else if (L.xmap == 1) hipLaunchKernelGGL((k_cg_pipe32_start<true, 1>), g, b, 0, L.stream, L.insts, L.bmap);
  else if (L.xmap == 2) hipLaunchKernelGGL((k_cg_pipe32_start<true, 2>), g, b, 0, L.stream, L.insts, L.bmap);
  else hipLaunchKernelGGL((k_cg_pipe32_start<true, 0>), g, b, 0, L.stream, L.insts, L.bmap);
}

void launch_cg_pipe32(const Launch& L) {
  if (L.nblocks <= 0) return;
  const dim3 g(L.nblocks), b(WG);
  if (!L.single && L.pipe_op == 1) hipLaunchKernelGGL((k_cg_pipe32<false, 0, 1>), g, b, 0, L.stream, L.insts, L.bmap);
  else if (!L.single) hipLaunchKernelGGL((k_cg_pipe32<false, 0, 0>), g, b, 0, L.stream, L.insts, L.bmap);
  else if (L.pipe_op == 1 && L.xmap == 1) hipLaunchKernelGGL((k_cg_pipe32<true, 1, 1>), g, b, 0, L.stream, L.insts, L.bmap);
  else if (L.pipe_op == 1 && L.xmap == 2) hipLaunchKernelGGL((k_cg_pipe32<true, 2, 1>), g, b, 0, L.stream, L.insts, L.bmap);
  else if (L.pipe_op == 1) hipLaunchKernelGGL((k_cg_pipe32<true, 0, 1>), g, b, 0, L.stream, L.insts, L.bmap);
  else if (L.xmap == 1) hipLaunchKernelGGL((k_cg_pipe32<true, 1, 0>), g, b, 0, L.stream, L.insts, L.bmap);
  else if (L.xmap == 2) hipLaunchKernelGGL((k_cg_pipe32<true, 2, 0>), g, b, 0, L.stream, L.insts, L.bmap);
  else hipLaunchKernelGGL((k_cg_pipe32<true, 0, 0>), g, b, 0, L.stream, L.insts, L.bmap);
}

void launch_cg_pipe_start(const Launch& L) {
  if (L.nblocks <= 0) return;
  if (L.mf_p) launch_mf_apply(0, L);   // A u_0
  const dim3 g(L.nblocks), b(WG);
  if (!L.single) hipLaunchKernelGGL((k_cg_pipe_start<false, 0>), g, b, 0, L.stream, L.insts, L.bmap);
  else if (L.xmap == 1) hipLaunchKernelGGL((k_cg_pipe_start<true, 1>), g, b, 0, L.stream, L.insts, L.bmap);
  else if (L.xmap == 2) hipLaunchKernelGGL((k_cg_pipe_start<true, 2>), g, b, 0, L.stream, L.insts, L.bmap);
  else hipLaunchKernelGGL((k_cg_pipe_start<true, 0>), g, b, 0, L.stream, L.insts, L.bmap);
}

void launch_cg_pipe(const Launch& L) {
  if (L.nblocks <= 0) return;
  if (L.mf_p) launch_mf_apply(3, L);   // A m_k
  const dim3 g(L.nblocks), b(WG);
  if (!L.single && L.pipe_op == 1) hipLaunchKernelGGL((k_cg_pipe<false, 0, 1>), g, b, 0, L.stream, L.insts, L.bmap);
  else if (!L.single) hipLaunchKernelGGL((k_cg_pipe<false, 0, 0>), g, b, 0, L.stream, L.insts, L.bmap);
  else if (L.pipe_op == 1 && L.xmap == 1) hipLaunchKernelGGL((k_cg_pipe<true, 1, 1>), g, b, 0, L.stream, L.insts, L.bmap);
  else if (L.pipe_op == 1 && L.xmap == 2) hipLaunchKernelGGL((k_cg_pipe<true, 2, 1>), g, b, 0, L.stream, L.insts, L.bmap);
  else if (L.pipe_op == 1) hipLaunchKernelGGL((k_cg_pipe<true, 0, 1>), g, b, 0, L.stream, L.insts, L.bmap);
  else if (L.xmap == 1) hipLaunchKernelGGL((k_cg_pipe<true, 1, 0>), g, b, 0, L.stream, L.insts, L.bmap);
  else if (L.xmap == 2) hipLaunchKernelGGL((k_cg_pipe<true, 2, 0>), g, b, 0, L.stream, L.insts, L.bmap);
  else hipLaunchKernelGGL((k_cg_pipe<true, 0, 0>), g, b, 0, L.stream, L.insts, L.bmap);
}

void launch_cg_finalize(bool mixed, InstDesc* insts, const int32_t* ids, int n_ids, hipStream_t stream) {
  if (n_ids == 1 && ids == nullptr) {
    // single instance at insts[0]
    if (mixed) hipLaunchKernelGGL((k_cg_finalize<true, true>), dim3(1), dim3(FIN_WG), 0, stream, insts, ids);
    else hipLaunchKernelGGL((k_cg_finalize<false, true>), dim3(1), dim3(FIN_WG), 0, stream, insts, ids);
    return;
  }
  if (n_ids <= 0) return;
  if (mixed) hipLaunchKernelGGL((k_cg_finalize<true, false>), dim3(n_ids), dim3(FIN_WG), 0, stream, insts, ids);
  else hipLaunchKernelGGL((k_cg_finalize<false, false>), dim3(n_ids), dim3(FIN_WG), 0, stream, insts, ids);
}

void launch_cg_update(bool mixed, const Launch& L) {
  if (L.nblocks <= 0) return;
  mixed ? update_dispatch<true>(L) : update_dispatch<false>(L);
}

void launch_cg_update64(const Launch& L) {
  if (L.nblocks <= 0) return;
  const dim3 g(L.nblocks), b(WG);
  if (!L.single) hipLaunchKernelGGL((k_cg_update64<false, 0>), g, b, 0, L.stream, L.insts, L.bmap);
  else if (L.xmap == 1) hipLaunchKernelGGL((k_cg_update64<true, 1>), g, b, 0, L.stream, L.insts, L.bmap);
  else if (L.xmap == 2) hipLaunchKernelGGL((k_cg_update64<true, 2>), g, b, 0, L.stream, L.insts, L.bmap);
  else hipLaunchKernelGGL((k_cg_update64<true, 0>), g, b, 0, L.stream, L.insts, L.bmap);
}

void launch_activation(const Launch& L) {
  if (L.nblocks <= 0) return;
  EP_LAUNCH2(k_activation, dim3(L.nblocks), dim3(TILE), L);
}

void launch_end_step(InstDesc* insts, const int32_t* ids, int n_ids, hipStream_t stream) {
  if (n_ids <= 0) return;
  hipLaunchKernelGGL(k_end_step, dim3((unsigned)((n_ids + 63) / 64)), dim3(64), 0, stream, insts, ids, n_ids);
}

void launch_to_mv(void* dst, const double* u, int64_t n, double a, double b, bool f32, hipStream_t stream,
                  const int32_t* reg) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_to_mv, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, dst, u, n, a, b,
                     f32 ? 1 : 0, reg);
}

void launch_fill(double* x, int64_t n, double v, hipStream_t stream) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, x, n, v);
}

}  // namespace ep
