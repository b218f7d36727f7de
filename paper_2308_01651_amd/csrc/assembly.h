// Host-side one-time setup of the monodomain operator: finite-element mass
// and stiffness assembly, the sparsity pattern, and the device matrix formats.
#pragma once
#include <stdint.h>

#include <vector>

namespace ep {

struct Csr {
  int64_t n = 0;
  std::vector<int64_t> rowptr;   // n + 1
  std::vector<int32_t> col;      // nnz, sorted within each row
  std::vector<double> valM, valK;
  int64_t nnz() const { return (int64_t)col.size(); }
};

// Assemble M_jk = int phi_k phi_j and K_jk = int D grad phi_k . grad phi_j with
// D = (sigma_l f f^T + sigma_t s s^T + sigma_n n n^T)/(chi C_m) given at the
// nodes and interpolated with the FE basis.  elem = 8 (trilinear hexahedra,
// 2x2x2 Gauss points), 27 (triquadratic hexahedra, 3x3x3), 64 (tricubic
// hexahedra, 4x4x4), 4 (linear tetrahedra, closed form) or 10 (quadratic
// tetrahedra, 64-point conical product rule).
// fibers may be null (then f = e_x, s = e_y, n = e_z everywhere).
// Several subdomains: region (per element, nullable) selects the element's
// conductivities region_sigma[3 r .. 3 r + 2]; an element of a region with
// region_on[r] == 0 keeps its place in the sparsity pattern with zero values.
// Returns false and fills `err` on invalid input (bad index, inverted element).
bool assemble_csr(int elem, int64_t n_nodes, const double* xyz, int64_t n_elems,
                  const int32_t* conn, const double* f0, const double* s0, const double* n0,
                  double sigma_l, double sigma_t, double sigma_n, double chi, double cm,
                  Csr& out, std::vector<char>& err, const int32_t* region = nullptr,
                  const double* region_sigma = nullptr, const unsigned char* region_on = nullptr);

// Data of the matrix-free operator of hexahedra of degree p = 2 or 3
// (sum factorization on the (p + 1)^3 Gauss points the assembly uses).
// Per element and quadrature point q (x fastest), stored component-major
// per element, geo[(e * 7 + c) * Q + q]:
//   c = 0..5: the symmetric C = w det(J) J^-1 D J^-T (in the reference
//   frame: xx, xy, xz, yy, yz, zz), so that K_e x = sum_q dN^T C dN x;
//   c = 6: m = w det(J), so that M_e x = sum_q N m N^T x.
// V[q * n1 + j], Dv[q * n1 + j]: 1-D Lagrange factor j (equispaced nodes)
// and its derivative at Gauss point q.  Node adjacency for the gather:
// entries (e * npe + k) of node i, ascending, in adj_ptr[i] .. adj_ptr[i+1].
struct MfData {
  int p = 0;
  int64_t n_elems = 0;
  // per element and quadrature point: [e][7][Q] (xx, xy, xz, yy, yz, zz of
  // w det J J^-1 D J^-T, then w det J); compressed (every element affine
  // with one D, so each factor is the product of the point's Gauss weights
  // and an element constant): [e][7] with W the 1-D Gauss weights
  bool cmp = false;
  std::vector<double> geo;
  double W[4] = {0, 0, 0, 0};
  std::vector<double> V, Dv;
  std::vector<int64_t> adj_ptr;
  std::vector<int32_t> adj;
};
bool mf_setup(int elem, int64_t n_nodes, const double* xyz, int64_t n_elems, const int32_t* conn,
              const double* f0, const double* s0, const double* n0, double sigma_l, double sigma_t,
              double sigma_n, double chi, double cm, MfData& out, std::vector<char>& err);

// Distinct column offsets j - i over the pattern, ascending.
std::vector<int64_t> distinct_offsets(const Csr& A);

// Parallel loop helper over [0, n).
template <typename F>
void parallel_for(int64_t n, F&& f);

}  // namespace ep

#include <algorithm>
#include <thread>

namespace ep {
template <typename F>
void parallel_for(int64_t n, F&& f) {
  unsigned hw = std::thread::hardware_concurrency();
  int64_t nt = std::max<int64_t>(1, std::min<int64_t>(hw ? hw : 4, 32));
  if (n < 4096) nt = 1;
  if (nt == 1) {
    for (int64_t i = 0; i < n; i++) f(i);
    return;
  }
  std::vector<std::thread> th;
  const int64_t chunk = (n + nt - 1) / nt;
  for (int64_t t = 0; t < nt; t++) {
    const int64_t a = t * chunk, b = std::min(n, a + chunk);
    if (a >= b) break;
    th.emplace_back([a, b, &f]() {
      for (int64_t i = a; i < b; i++) f(i);
    });
  }
  for (auto& x : th) x.join();
}
}  // namespace ep
