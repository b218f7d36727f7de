// Finite-element assembly of the monodomain operator on the host (one-time
// setup; the per-step work runs in the HIP kernels).
//
// Space discretization as in the paper's numerical section: M_jk is the
// integral of phi_k phi_j, K_jk the integral of D grad phi_k . grad phi_j,
// with the fewest Gauss points that integrate M exactly.  The diffusion
// tensor is the paper's D = sigma_l f f^T + sigma_t s s^T + sigma_n n n^T
// divided by chi C_m (the rescaling of the dimensional monodomain equation),
// given per node and interpolated with the FE basis.
#include "assembly.h"

#include <atomic>
#include <cfloat>
#include <cmath>
#include <cstdio>
#include <cstring>

namespace ep {

namespace {

void set_err(std::vector<char>& err, const char* msg) {
  err.assign(msg, msg + std::strlen(msg) + 1);
}

// Nodal diffusion tensor (row-major 3x3) in mm^2/ms.
inline void nodal_tensor(const double* f, const double* s, const double* nn, double sl, double st,
                         double sn, double scale, double D[9]) {
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++)
      D[3 * a + b] = scale * (sl * f[a] * f[b] + st * s[a] * s[b] + sn * nn[a] * nn[b]);
}

// Positive semi-definiteness of a symmetric 3x3 tensor (row-major): every
// principal minor nonnegative, up to rounding relative to the trace.  The
// basis of an element of degree p >= 2 has negative lobes, so interpolating
// nodal tensors that change abruptly from node to node can leave the cone of
// such tensors; K is then no longer positive semi-definite.
bool psd3(const double D[9]) {
  const double tr = std::fabs(D[0]) + std::fabs(D[4]) + std::fabs(D[8]);
  const double tol = 1e-12;
  if (D[0] < -tol * tr || D[4] < -tol * tr || D[8] < -tol * tr) return false;
  const double t2 = tol * tr * tr;
  if (D[0] * D[4] - D[1] * D[3] < -t2 || D[0] * D[8] - D[2] * D[6] < -t2 || D[4] * D[8] - D[5] * D[7] < -t2)
    return false;
  const double det = D[0] * (D[4] * D[8] - D[5] * D[7]) - D[1] * (D[3] * D[8] - D[5] * D[6]) +
                     D[2] * (D[3] * D[7] - D[4] * D[6]);
  return det >= -tol * tr * tr * tr;
}

// Trilinear hexahedron, local corner k = a + 2b + 4c at reference (2a-1, 2b-1, 2c-1).
// Element matrices by 2x2x2 Gauss-Legendre quadrature.
int hex_element(const double X[8][3], const double Dn[8][9], double Me[64], double Ke[64]) {
  static const double g = 0.57735026918962576451;  // 1/sqrt(3)
  std::memset(Me, 0, 64 * sizeof(double));
  std::memset(Ke, 0, 64 * sizeof(double));
  for (int qz = 0; qz < 2; qz++)
    for (int qy = 0; qy < 2; qy++)
      for (int qx = 0; qx < 2; qx++) {
        const double xi[3] = {qx ? g : -g, qy ? g : -g, qz ? g : -g};
        double N[8], dN[8][3];
        for (int k = 0; k < 8; k++) {
          const double sg[3] = {(k & 1) ? 1.0 : -1.0, (k & 2) ? 1.0 : -1.0, (k & 4) ? 1.0 : -1.0};
          const double f0 = 1.0 + sg[0] * xi[0], f1 = 1.0 + sg[1] * xi[1], f2 = 1.0 + sg[2] * xi[2];
          N[k] = 0.125 * f0 * f1 * f2;
          dN[k][0] = 0.125 * sg[0] * f1 * f2;
          dN[k][1] = 0.125 * sg[1] * f0 * f2;
          dN[k][2] = 0.125 * sg[2] * f0 * f1;
        }
        // Jacobian J[r][c] = d x_c / d xi_r
        double J[3][3] = {{0}};
        for (int k = 0; k < 8; k++)
          for (int r = 0; r < 3; r++)
            for (int c = 0; c < 3; c++) J[r][c] += dN[k][r] * X[k][c];
        const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                           J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                           J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        if (!(det > 0.0)) return 1;
        double Ji[3][3];
        Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
        Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
        Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
        Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
        Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
        Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
        Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
        Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
        Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
        // physical gradient grad_x phi_k = J^{-1} grad_xi phi_k
        double G[8][3];
        for (int k = 0; k < 8; k++)
          for (int r = 0; r < 3; r++)
            G[k][r] = Ji[r][0] * dN[k][0] + Ji[r][1] * dN[k][1] + Ji[r][2] * dN[k][2];
        double Dq[9] = {0};
        for (int k = 0; k < 8; k++)
          for (int e = 0; e < 9; e++) Dq[e] += N[k] * Dn[k][e];
        double DG[8][3];
        for (int k = 0; k < 8; k++)
          for (int r = 0; r < 3; r++)
            DG[k][r] = Dq[3 * r] * G[k][0] + Dq[3 * r + 1] * G[k][1] + Dq[3 * r + 2] * G[k][2];
        for (int a = 0; a < 8; a++)
          for (int b = 0; b < 8; b++) {
            Me[8 * a + b] += det * N[a] * N[b];
            Ke[8 * a + b] += det * (G[a][0] * DG[b][0] + G[a][1] * DG[b][1] + G[a][2] * DG[b][2]);
          }
      }
  return 0;
}

// Triquadratic hexahedron (27 nodes), local node k = a + 3b + 9c at the
// reference point (a - 1, b - 1, c - 1); isoparametric map; 3x3x3
// Gauss-Legendre quadrature (exact for the mass matrix of an affine element).
int hex27_element(const double X[27][3], const double Dn[27][9], double* Me, double* Ke) {
  static const double gp[3] = {-0.77459666924148337704, 0.0, 0.77459666924148337704};  // -sqrt(3/5), 0, sqrt(3/5)
  static const double gw[3] = {5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0};
  std::memset(Me, 0, 27 * 27 * sizeof(double));
  std::memset(Ke, 0, 27 * 27 * sizeof(double));
  // 1-D quadratic Lagrange factors at the nodes -1, 0, 1 and their derivatives
  auto lag = [](double t, double v[3], double d[3]) {
    v[0] = 0.5 * t * (t - 1.0);
    v[1] = (1.0 - t) * (1.0 + t);
    v[2] = 0.5 * t * (t + 1.0);
    d[0] = t - 0.5;
    d[1] = -2.0 * t;
    d[2] = t + 0.5;
  };
  for (int qz = 0; qz < 3; qz++)
    for (int qy = 0; qy < 3; qy++)
      for (int qx = 0; qx < 3; qx++) {
        double vx[3], dx[3], vy[3], dy[3], vz[3], dz[3];
        lag(gp[qx], vx, dx);
        lag(gp[qy], vy, dy);
        lag(gp[qz], vz, dz);
        double N[27], dN[27][3];
        for (int c = 0; c < 3; c++)
          for (int b = 0; b < 3; b++)
            for (int a = 0; a < 3; a++) {
              const int k = a + 3 * b + 9 * c;
              N[k] = vx[a] * vy[b] * vz[c];
              dN[k][0] = dx[a] * vy[b] * vz[c];
              dN[k][1] = vx[a] * dy[b] * vz[c];
              dN[k][2] = vx[a] * vy[b] * dz[c];
            }
        double J[3][3] = {{0}};
        for (int k = 0; k < 27; k++)
          for (int r = 0; r < 3; r++)
            for (int c = 0; c < 3; c++) J[r][c] += dN[k][r] * X[k][c];
        const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                           J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                           J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        if (!(det > 0.0)) return 1;
        double Ji[3][3];
        Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
        Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
        Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
        Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
        Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
        Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
        Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
        Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
        Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
        double G[27][3];
        for (int k = 0; k < 27; k++)
          for (int r = 0; r < 3; r++)
            G[k][r] = Ji[r][0] * dN[k][0] + Ji[r][1] * dN[k][1] + Ji[r][2] * dN[k][2];
        double Dq[9] = {0};
        for (int k = 0; k < 27; k++)
          for (int e = 0; e < 9; e++) Dq[e] += N[k] * Dn[k][e];
        if (!psd3(Dq)) return 2;
        double DG[27][3];
        for (int k = 0; k < 27; k++)
          for (int r = 0; r < 3; r++)
            DG[k][r] = Dq[3 * r] * G[k][0] + Dq[3 * r + 1] * G[k][1] + Dq[3 * r + 2] * G[k][2];
        const double w = gw[qx] * gw[qy] * gw[qz] * det;
        for (int a = 0; a < 27; a++)
          for (int b = 0; b < 27; b++) {
            Me[27 * a + b] += w * N[a] * N[b];
            Ke[27 * a + b] += w * (G[a][0] * DG[b][0] + G[a][1] * DG[b][1] + G[a][2] * DG[b][2]);
          }
      }
  return 0;
}

// Tricubic hexahedron (64 nodes), local node k = a + 4b + 16c at the
// reference point (2a/3 - 1, 2b/3 - 1, 2c/3 - 1); isoparametric map; 4x4x4
// Gauss-Legendre quadrature (exact for the mass matrix of an affine element).
int hex64_element(const double X[64][3], const double Dn[64][9], double* Me, double* Ke) {
  static const double gp[4] = {-0.86113631159405257522, -0.33998104358485626480, 0.33998104358485626480,
                               0.86113631159405257522};
  static const double gw[4] = {0.34785484513745385737, 0.65214515486254614263, 0.65214515486254614263,
                               0.34785484513745385737};
  std::memset(Me, 0, 64 * 64 * sizeof(double));
  std::memset(Ke, 0, 64 * 64 * sizeof(double));
  // 1-D cubic Lagrange factors at the nodes -1, -1/3, 1/3, 1 (product form;
  // the derivative accumulates by the product rule)
  auto lag = [](double t, double v[4], double d[4]) {
    static const double z[4] = {-1.0, -1.0 / 3.0, 1.0 / 3.0, 1.0};
    for (int j = 0; j < 4; j++) {
      double val = 1.0, der = 0.0;
      for (int m = 0; m < 4; m++) {
        if (m == j) continue;
        const double f = (t - z[m]) / (z[j] - z[m]);
        der = der * f + val / (z[j] - z[m]);
        val *= f;
      }
      v[j] = val;
      d[j] = der;
    }
  };
  for (int qz = 0; qz < 4; qz++)
    for (int qy = 0; qy < 4; qy++)
      for (int qx = 0; qx < 4; qx++) {
        double vx[4], dx[4], vy[4], dy[4], vz[4], dz[4];
        lag(gp[qx], vx, dx);
        lag(gp[qy], vy, dy);
        lag(gp[qz], vz, dz);
        double N[64], dN[64][3];
        for (int c = 0; c < 4; c++)
          for (int b = 0; b < 4; b++)
            for (int a = 0; a < 4; a++) {
              const int k = a + 4 * b + 16 * c;
              N[k] = vx[a] * vy[b] * vz[c];
              dN[k][0] = dx[a] * vy[b] * vz[c];
              dN[k][1] = vx[a] * dy[b] * vz[c];
              dN[k][2] = vx[a] * vy[b] * dz[c];
            }
        double J[3][3] = {{0}};
        for (int k = 0; k < 64; k++)
          for (int r = 0; r < 3; r++)
            for (int c = 0; c < 3; c++) J[r][c] += dN[k][r] * X[k][c];
        const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                           J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                           J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        if (!(det > 0.0)) return 1;
        double Ji[3][3];
        Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
        Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
        Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
        Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
        Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
        Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
        Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
        Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
        Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
        double G[64][3];
        for (int k = 0; k < 64; k++)
          for (int r = 0; r < 3; r++)
            G[k][r] = Ji[r][0] * dN[k][0] + Ji[r][1] * dN[k][1] + Ji[r][2] * dN[k][2];
        double Dq[9] = {0};
        for (int k = 0; k < 64; k++)
          for (int e = 0; e < 9; e++) Dq[e] += N[k] * Dn[k][e];
        if (!psd3(Dq)) return 2;
        double DG[64][3];
        for (int k = 0; k < 64; k++)
          for (int r = 0; r < 3; r++)
            DG[k][r] = Dq[3 * r] * G[k][0] + Dq[3 * r + 1] * G[k][1] + Dq[3 * r + 2] * G[k][2];
        const double w = gw[qx] * gw[qy] * gw[qz] * det;
        for (int a = 0; a < 64; a++)
          for (int b = 0; b < 64; b++) {
            Me[64 * a + b] += w * N[a] * N[b];
            Ke[64 * a + b] += w * (G[a][0] * DG[b][0] + G[a][1] * DG[b][1] + G[a][2] * DG[b][2]);
          }
      }
  return 0;
}

// Gauss-Legendre points and weights of order n on [-1, 1]: Newton's method on
// the Legendre polynomial P_n (three-term recurrence), started from the
// asymptotic estimate cos(pi (i + 3/4) / (n + 1/2)) of the i-th root;
// w_i = 2 / ((1 - x_i^2) P_n'(x_i)^2).
static void gauss_legendre(int n, double* x, double* w) {
  for (int i = 0; i < n; i++) {
    double t = std::cos(std::acos(-1.0) * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; it++) {
      double p0 = 1.0, p1 = t;
      for (int j = 1; j < n; j++) {
        const double p2 = ((2.0 * j + 1.0) * t * p1 - j * p0) / (j + 1.0);
        p0 = p1;
        p1 = p2;
      }
      dp = n * (t * p1 - p0) / (t * t - 1.0);
      const double step = p1 / dp;
      t -= step;
      if (std::fabs(step) < 1e-16) break;
    }
    x[n - 1 - i] = t;
    w[n - 1 - i] = 2.0 / ((1.0 - t * t) * dp * dp);
  }
}

// Hexahedron of degree p = 4..6 ((p + 1)^3 nodes), local node
// k = a + (p + 1) b + (p + 1)^2 c at the reference point
// (2a/p - 1, 2b/p - 1, 2c/p - 1); isoparametric map; (p + 1)^3 Gauss-Legendre
// points (exact for the mass matrix of an affine element).
int hexp_element(int p, const double (*X)[3], const double (*Dn)[9], double* Me, double* Ke) {
  if (p < 4 || p > 6) return 1;
  const int n1 = p + 1, npe = n1 * n1 * n1;
  double gp[7], gw[7], z[7];
  gauss_legendre(n1, gp, gw);
  for (int j = 0; j < n1; j++) z[j] = -1.0 + 2.0 * j / p;
  // 1-D Lagrange factors at the equispaced nodes and their derivatives at
  // every Gauss point (product form, derivative by the product rule)
  double V[7][7], Dv[7][7];
  for (int q = 0; q < n1; q++)
    for (int j = 0; j < n1; j++) {
      double val = 1.0, der = 0.0;
      for (int m = 0; m < n1; m++) {
        if (m == j) continue;
        const double f = (gp[q] - z[m]) / (z[j] - z[m]);
        der = der * f + val / (z[j] - z[m]);
        val *= f;
      }
      V[q][j] = val;
      Dv[q][j] = der;
    }
  std::memset(Me, 0, (size_t)npe * npe * sizeof(double));
  std::memset(Ke, 0, (size_t)npe * npe * sizeof(double));
  std::vector<double> N(npe), dN(3 * npe), G(3 * npe), DG(3 * npe);
  for (int qz = 0; qz < n1; qz++)
    for (int qy = 0; qy < n1; qy++)
      for (int qx = 0; qx < n1; qx++) {
        for (int c = 0; c < n1; c++)
          for (int b = 0; b < n1; b++)
            for (int a = 0; a < n1; a++) {
              const int k = a + n1 * (b + n1 * c);
              N[k] = V[qx][a] * V[qy][b] * V[qz][c];
              dN[3 * k] = Dv[qx][a] * V[qy][b] * V[qz][c];
              dN[3 * k + 1] = V[qx][a] * Dv[qy][b] * V[qz][c];
              dN[3 * k + 2] = V[qx][a] * V[qy][b] * Dv[qz][c];
            }
        double J[3][3] = {{0}};
        for (int k = 0; k < npe; k++)
          for (int r = 0; r < 3; r++)
            for (int c = 0; c < 3; c++) J[r][c] += dN[3 * k + r] * X[k][c];
        const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                           J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                           J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        if (!(det > 0.0)) return 1;
        double Ji[3][3];
        Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
        Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
        Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
        Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
        Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
        Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
        Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
        Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
        Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
        for (int k = 0; k < npe; k++)
          for (int r = 0; r < 3; r++)
            G[3 * k + r] = Ji[r][0] * dN[3 * k] + Ji[r][1] * dN[3 * k + 1] + Ji[r][2] * dN[3 * k + 2];
        double Dq[9] = {0};
        for (int k = 0; k < npe; k++)
          for (int e = 0; e < 9; e++) Dq[e] += N[k] * Dn[k][e];
        if (!psd3(Dq)) return 2;
        for (int k = 0; k < npe; k++)
          for (int r = 0; r < 3; r++)
            DG[3 * k + r] = Dq[3 * r] * G[3 * k] + Dq[3 * r + 1] * G[3 * k + 1] + Dq[3 * r + 2] * G[3 * k + 2];
        const double w = gw[qx] * gw[qy] * gw[qz] * det;
        for (int a = 0; a < npe; a++) {
          const double wn = w * N[a];
          const double g0 = w * G[3 * a], g1 = w * G[3 * a + 1], g2 = w * G[3 * a + 2];
          double* mrow = Me + (size_t)npe * a;
          double* krow = Ke + (size_t)npe * a;
          for (int b = 0; b < npe; b++) {
            mrow[b] += wn * N[b];
            krow[b] += g0 * DG[3 * b] + g1 * DG[3 * b + 1] + g2 * DG[3 * b + 2];
          }
        }
      }
  return 0;
}

// Quadratic tetrahedron (10 nodes: vertices 0-3, then the nodes of the edges
// 01, 02, 03, 12, 13, 23), isoparametric: the map from the reference
// tetrahedron uses all ten nodes, so an element whose edge nodes sit off the
// edge midpoints is curved (straight-sided elements give an affine map).
// Quadrature: the conical product of 4-point Gauss-Legendre rules on the
// unit cube collapsed onto the tetrahedron (64 points, exact to degree 5 in
// the barycentric coordinates).  The Jacobian determinant must keep the
// sign of the vertex orientation at every point (no folded element).
int tet10_element(const double X[10][3], const double Dn[10][9], double* Me, double* Ke) {
  static const double gx[4] = {0.06943184420297371, 0.33000947820757187, 0.66999052179242813,
                               0.93056815579702629};  // Gauss-Legendre nodes on [0, 1]
  static const double gw[4] = {0.17392742256872693, 0.32607257743127307, 0.32607257743127307,
                               0.17392742256872693};
  static const int edge[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
  // d L_a / d l_r for the independent reference coordinates l_1, l_2, l_3
  static const double dl[4][3] = {{-1, -1, -1}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  double E[3][3];
  for (int r = 0; r < 3; r++)
    for (int c = 0; c < 3; c++) E[r][c] = X[r + 1][c] - X[0][c];
  const double det0 = E[0][0] * (E[1][1] * E[2][2] - E[1][2] * E[2][1]) -
                      E[0][1] * (E[1][0] * E[2][2] - E[1][2] * E[2][0]) +
                      E[0][2] * (E[1][0] * E[2][1] - E[1][1] * E[2][0]);
  if (det0 == 0.0 || !std::isfinite(det0)) return 1;
  const double orient = det0 > 0.0 ? 1.0 : -1.0;
  std::memset(Me, 0, 100 * sizeof(double));
  std::memset(Ke, 0, 100 * sizeof(double));
  for (int i = 0; i < 4; i++)
    for (int j = 0; j < 4; j++)
      for (int k = 0; k < 4; k++) {
        const double u = gx[i], v = gx[j], w = gx[k];
        double L[4];
        L[1] = u;
        L[2] = v * (1.0 - u);
        L[3] = w * (1.0 - u) * (1.0 - v);
        L[0] = 1.0 - L[1] - L[2] - L[3];
        double N[10], dN[10][3];
        for (int a = 0; a < 4; a++) {
          N[a] = L[a] * (2.0 * L[a] - 1.0);
          for (int r = 0; r < 3; r++) dN[a][r] = (4.0 * L[a] - 1.0) * dl[a][r];
        }
        for (int e = 0; e < 6; e++) {
          const int a = edge[e][0], b = edge[e][1];
          N[4 + e] = 4.0 * L[a] * L[b];
          for (int r = 0; r < 3; r++) dN[4 + e][r] = 4.0 * (L[b] * dl[a][r] + L[a] * dl[b][r]);
        }
        double J[3][3] = {{0}};
        for (int a = 0; a < 10; a++)
          for (int r = 0; r < 3; r++)
            for (int c = 0; c < 3; c++) J[r][c] += dN[a][r] * X[a][c];
        const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                           J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                           J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        if (!(orient * det > 0.0)) return 1;
        double Ji[3][3];
        Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
        Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
        Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
        Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
        Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
        Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
        Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
        Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
        Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
        double G[10][3];
        for (int a = 0; a < 10; a++)
          for (int c = 0; c < 3; c++) G[a][c] = Ji[c][0] * dN[a][0] + Ji[c][1] * dN[a][1] + Ji[c][2] * dN[a][2];
        // collapsed-cube weight times |det J| (the reference tetrahedron's
        // volume 1/6 cancels the factor 6 of the collapse)
        const double wq = gw[i] * gw[j] * gw[k] * (1.0 - u) * (1.0 - u) * (1.0 - v) * orient * det;
        double Dq[9] = {0};
        for (int a = 0; a < 10; a++)
          for (int t = 0; t < 9; t++) Dq[t] += N[a] * Dn[a][t];
        if (!psd3(Dq)) return 2;
        double DG[10][3];
        for (int a = 0; a < 10; a++)
          for (int r = 0; r < 3; r++)
            DG[a][r] = Dq[3 * r] * G[a][0] + Dq[3 * r + 1] * G[a][1] + Dq[3 * r + 2] * G[a][2];
        for (int a = 0; a < 10; a++)
          for (int b = 0; b < 10; b++) {
            Me[10 * a + b] += wq * N[a] * N[b];
            Ke[10 * a + b] += wq * (G[a][0] * DG[b][0] + G[a][1] * DG[b][1] + G[a][2] * DG[b][2]);
          }
      }
  return 0;
}

// Linear tetrahedron.  Gradients of the barycentric coordinates are constant;
// with D interpolated linearly, the degree-2 rule reduces exactly to
// K = V G^T mean(D) G, and M = V (1 + delta_ab)/20.
int tet_element(const double X[4][3], const double Dn[4][9], double Me[16], double Ke[16]) {
  double E[3][3];
  for (int r = 0; r < 3; r++)
    for (int c = 0; c < 3; c++) E[r][c] = X[r + 1][c] - X[0][c];
  const double det = E[0][0] * (E[1][1] * E[2][2] - E[1][2] * E[2][1]) -
                     E[0][1] * (E[1][0] * E[2][2] - E[1][2] * E[2][0]) +
                     E[0][2] * (E[1][0] * E[2][1] - E[1][1] * E[2][0]);
  if (det == 0.0 || !std::isfinite(det)) return 1;
  const double vol = std::fabs(det) / 6.0;
  // rows of E^{-T} ... gradient of L_{r+1} is column r of E^{-1}
  double Ei[3][3];
  Ei[0][0] = (E[1][1] * E[2][2] - E[1][2] * E[2][1]) / det;
  Ei[0][1] = (E[0][2] * E[2][1] - E[0][1] * E[2][2]) / det;
  Ei[0][2] = (E[0][1] * E[1][2] - E[0][2] * E[1][1]) / det;
  Ei[1][0] = (E[1][2] * E[2][0] - E[1][0] * E[2][2]) / det;
  Ei[1][1] = (E[0][0] * E[2][2] - E[0][2] * E[2][0]) / det;
  Ei[1][2] = (E[0][2] * E[1][0] - E[0][0] * E[1][2]) / det;
  Ei[2][0] = (E[1][0] * E[2][1] - E[1][1] * E[2][0]) / det;
  Ei[2][1] = (E[0][1] * E[2][0] - E[0][0] * E[2][1]) / det;
  Ei[2][2] = (E[0][0] * E[1][1] - E[0][1] * E[1][0]) / det;
  double G[4][3];
  for (int k = 0; k < 3; k++)
    for (int c = 0; c < 3; c++) G[k + 1][c] = Ei[c][k];
  for (int c = 0; c < 3; c++) G[0][c] = -(G[1][c] + G[2][c] + G[3][c]);
  double Dm[9];
  for (int e = 0; e < 9; e++) Dm[e] = 0.25 * (Dn[0][e] + Dn[1][e] + Dn[2][e] + Dn[3][e]);
  for (int a = 0; a < 4; a++)
    for (int b = 0; b < 4; b++) {
      Me[4 * a + b] = vol / 20.0 * (a == b ? 2.0 : 1.0);
      double acc = 0.0;
      for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) acc += G[a][r] * Dm[3 * r + c] * G[b][c];
      Ke[4 * a + b] = vol * acc;
    }
  return 0;
}

}  // namespace

bool mf_setup(int elem, int64_t n_nodes, const double* xyz, int64_t n_elems, const int32_t* conn,
              const double* f0, const double* s0, const double* n0, double sigma_l, double sigma_t,
              double sigma_n, double chi, double cm, MfData& out, std::vector<char>& err) {
  if (elem != 27 && elem != 64) {
    set_err(err, "the matrix-free operator takes hexahedra of degree 2 or 3 (27 or 64 nodes)");
    return false;
  }
  if (n_nodes <= 0 || n_elems <= 0) { set_err(err, "empty mesh"); return false; }
  if (!(chi > 0) || !(cm > 0)) { set_err(err, "chi and C_m must be positive"); return false; }
  const int npe = elem, p = elem == 27 ? 2 : 3, n1 = p + 1, Q = n1 * n1 * n1;
  for (int64_t e = 0; e < n_elems * npe; e++)
    if (conn[e] < 0 || conn[e] >= n_nodes) { set_err(err, "connectivity index out of range"); return false; }
  double gp[4], gw[4], z[4];
  gauss_legendre(n1, gp, gw);
  for (int j = 0; j < n1; j++) z[j] = -1.0 + 2.0 * j / p;
  out.p = p;
  out.n_elems = n_elems;
  out.V.assign((size_t)n1 * n1, 0.0);
  out.Dv.assign((size_t)n1 * n1, 0.0);
  for (int q = 0; q < n1; q++)
    for (int j = 0; j < n1; j++) {
      double val = 1.0, der = 0.0;
      for (int m = 0; m < n1; m++) {
        if (m == j) continue;
        const double f = (gp[q] - z[m]) / (z[j] - z[m]);
        der = der * f + val / (z[j] - z[m]);
        val *= f;
      }
      out.V[(size_t)q * n1 + j] = val;
      out.Dv[(size_t)q * n1 + j] = der;
    }
  out.geo.assign((size_t)n_elems * 7 * Q, 0.0);
  const double scale = 1.0 / (chi * cm);
  static const double ex[3] = {1, 0, 0}, ey[3] = {0, 1, 0}, ez[3] = {0, 0, 1};
  std::vector<char> bad(2, 0);
  const std::vector<double>& V = out.V;
  const std::vector<double>& Dv = out.Dv;
  parallel_for(n_elems, [&](int64_t e) {
    double X[64][3], Dn[64][9];
    for (int k = 0; k < npe; k++) {
      const int64_t v = conn[e * npe + k];
      for (int c = 0; c < 3; c++) X[k][c] = xyz[3 * v + c];
      nodal_tensor(f0 ? f0 + 3 * v : ex, s0 ? s0 + 3 * v : ey, n0 ? n0 + 3 * v : ez, sigma_l, sigma_t, sigma_n,
                   scale, Dn[k]);
    }
    double* g = &out.geo[(size_t)e * 7 * Q];
    for (int qz = 0; qz < n1; qz++)
      for (int qy = 0; qy < n1; qy++)
        for (int qx = 0; qx < n1; qx++) {
          const int q = qx + n1 * (qy + n1 * qz);
          double J[3][3] = {{0}}, Dq[9] = {0};
          for (int c = 0; c < n1; c++)
            for (int b = 0; b < n1; b++)
              for (int a = 0; a < n1; a++) {
                const int k = a + n1 * (b + n1 * c);
                const double N = V[qx * n1 + a] * V[qy * n1 + b] * V[qz * n1 + c];
                const double d0 = Dv[qx * n1 + a] * V[qy * n1 + b] * V[qz * n1 + c];
                const double d1 = V[qx * n1 + a] * Dv[qy * n1 + b] * V[qz * n1 + c];
                const double d2 = V[qx * n1 + a] * V[qy * n1 + b] * Dv[qz * n1 + c];
                for (int cc = 0; cc < 3; cc++) {
                  J[0][cc] += d0 * X[k][cc];
                  J[1][cc] += d1 * X[k][cc];
                  J[2][cc] += d2 * X[k][cc];
                }
                for (int t = 0; t < 9; t++) Dq[t] += N * Dn[k][t];
              }
          const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                             J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                             J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
          if (!(det > 0.0)) {
            bad[0] = 1;
            return;
          }
          if (!psd3(Dq)) {
            bad[1] = 1;
            return;
          }
          double Ji[3][3];
          Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
          Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
          Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
          Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
          Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
          Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
          Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
          Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
          Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
          // physical gradient component r of a function = sum_s Ji[r][s] d_s;
          // C[s][u] = w det sum_{r,t} Ji[r][s] Dq[r][t] Ji[t][u]
          const double w = gw[qx] * gw[qy] * gw[qz] * det;
          double DJ[3][3];
          for (int r = 0; r < 3; r++)
            for (int u = 0; u < 3; u++)
              DJ[r][u] = Dq[3 * r] * Ji[0][u] + Dq[3 * r + 1] * Ji[1][u] + Dq[3 * r + 2] * Ji[2][u];
          double C[3][3];
          for (int s2 = 0; s2 < 3; s2++)
            for (int u = 0; u < 3; u++)
              C[s2][u] = w * (Ji[0][s2] * DJ[0][u] + Ji[1][s2] * DJ[1][u] + Ji[2][s2] * DJ[2][u]);
          g[0 * Q + q] = C[0][0];
          g[1 * Q + q] = 0.5 * (C[0][1] + C[1][0]);
          g[2 * Q + q] = 0.5 * (C[0][2] + C[2][0]);
          g[3 * Q + q] = C[1][1];
          g[4 * Q + q] = 0.5 * (C[1][2] + C[2][1]);
          g[5 * Q + q] = C[2][2];
          g[6 * Q + q] = w;
        }
  });
  if (bad[0]) { set_err(err, "degenerate or inverted element"); return false; }
  if (bad[1]) {
    set_err(err, "the diffusion tensor interpolated from the nodal fibers is indefinite at a quadrature point");
    return false;
  }
  // compression: every element's factors equal (product of the point's 1-D
  // Gauss weights) x (an element constant) to rounding.  The Jacobian is
  // interpolated from coordinates of magnitude R on an element of extent d,
  // so its rounding is about eps R / d relative; an affine element passes at
  // 64 eps (1 + R / d), a curved one or a varying tensor (relative changes of
  // the order of the element size) does not
  {
    std::vector<double> wq(Q);
    for (int qz = 0; qz < n1; qz++)
      for (int qy = 0; qy < n1; qy++)
        for (int qx = 0; qx < n1; qx++) wq[qx + n1 * (qy + n1 * qz)] = gw[qx] * gw[qy] * gw[qz];
    std::atomic<bool> uniform{true};
    parallel_for(n_elems, [&](int64_t e) {
      if (!uniform.load(std::memory_order_relaxed)) return;
      const double* g = &out.geo[(size_t)e * 7 * Q];
      double R = 0.0, d = 0.0;
      const int64_t v0 = conn[e * npe];
      for (int k = 0; k < npe; k++) {
        const int64_t v = conn[e * npe + k];
        for (int c = 0; c < 3; c++) {
          R = std::max(R, std::fabs(xyz[3 * v + c]));
          d = std::max(d, std::fabs(xyz[3 * v + c] - xyz[3 * v0 + c]));
        }
      }
      const double tol = 64.0 * DBL_EPSILON * (1.0 + R / d);
      // each part against its own magnitude: the 3x3 factor, and det J
      double scale_c = 0.0;
      for (int c2 = 0; c2 < 6; c2++) scale_c = std::max(scale_c, std::fabs(g[c2 * Q] / wq[0]));
      for (int c = 0; c < 7; c++) {
        const double k = g[c * Q] / wq[0];
        const double scale = c < 6 ? scale_c : std::fabs(k);
        for (int q = 1; q < Q; q++)
          if (std::fabs(g[c * Q + q] - k * wq[q]) > tol * scale * wq[q]) {
            uniform.store(false, std::memory_order_relaxed);
            return;
          }
      }
    });
    if (uniform.load()) {
      std::vector<double> gc((size_t)n_elems * 7);
      for (int64_t e = 0; e < n_elems; e++)
        for (int c = 0; c < 7; c++) gc[(size_t)e * 7 + c] = out.geo[(size_t)e * 7 * Q + (size_t)c * Q] / wq[0];
      out.geo.swap(gc);
      out.cmp = true;
      for (int j = 0; j < n1; j++) out.W[j] = gw[j];
    }
  }
  // node adjacency (element * npe + local index), ascending per node
  out.adj_ptr.assign(n_nodes + 1, 0);
  for (int64_t t = 0; t < n_elems * npe; t++) out.adj_ptr[conn[t] + 1]++;
  for (int64_t i = 0; i < n_nodes; i++) out.adj_ptr[i + 1] += out.adj_ptr[i];
  if (out.adj_ptr[n_nodes] >= (int64_t)INT32_MAX) { set_err(err, "too many element entries for int32"); return false; }
  out.adj.assign(out.adj_ptr[n_nodes], 0);
  std::vector<int64_t> fill(out.adj_ptr.begin(), out.adj_ptr.end() - 1);
  for (int64_t t = 0; t < n_elems * npe; t++) out.adj[fill[conn[t]]++] = (int32_t)t;
  return true;
}

bool assemble_csr(int elem, int64_t n_nodes, const double* xyz, int64_t n_elems,
                  const int32_t* conn, const double* f0, const double* s0, const double* n0,
                  double sigma_l, double sigma_t, double sigma_n, double chi, double cm, Csr& A,
                  std::vector<char>& err, const int32_t* region, const double* region_sigma,
                  const unsigned char* region_on) {
  if (elem != 8 && elem != 4 && elem != 27 && elem != 64 && elem != 125 && elem != 216 && elem != 343 &&
      elem != 10) {
    set_err(err, "element type must be (p + 1)^3 for a hexahedron of degree p = 1..6, 4 (tet) or 10 "
                 "(quadratic tet)");
    return false;
  }
  if (n_nodes <= 0 || n_elems <= 0) { set_err(err, "empty mesh"); return false; }
  if (n_nodes >= (int64_t)INT32_MAX) { set_err(err, "too many nodes for int32 indices"); return false; }
  if (!(chi > 0) || !(cm > 0)) { set_err(err, "chi and C_m must be positive"); return false; }
  const int npe = elem;
  for (int64_t e = 0; e < n_elems * npe; e++)
    if (conn[e] < 0 || conn[e] >= n_nodes) { set_err(err, "connectivity index out of range"); return false; }
  const double scale = 1.0 / (chi * cm);

  // node -> element incidence
  std::vector<int64_t> ne_ptr(n_nodes + 1, 0);
  for (int64_t e = 0; e < n_elems * npe; e++) ne_ptr[conn[e] + 1]++;
  for (int64_t i = 0; i < n_nodes; i++) ne_ptr[i + 1] += ne_ptr[i];
  std::vector<int64_t> ne_idx(ne_ptr[n_nodes]);
  {
    std::vector<int64_t> fill(ne_ptr.begin(), ne_ptr.end() - 1);
    for (int64_t e = 0; e < n_elems; e++)
      for (int k = 0; k < npe; k++) ne_idx[fill[conn[e * npe + k]]++] = e * npe + k;  // element*npe + local
  }

  // sparsity pattern: row i = union of the nodes of its elements
  A.n = n_nodes;
  A.rowptr.assign(n_nodes + 1, 0);
  std::vector<int32_t> rowlen(n_nodes);
  auto gather_row = [&](int64_t i, std::vector<int32_t>& buf) {
    buf.clear();
    for (int64_t t = ne_ptr[i]; t < ne_ptr[i + 1]; t++) {
      const int64_t e = ne_idx[t] / npe;
      for (int k = 0; k < npe; k++) buf.push_back(conn[e * npe + k]);
    }
    std::sort(buf.begin(), buf.end());
    buf.erase(std::unique(buf.begin(), buf.end()), buf.end());
  };
  parallel_for(n_nodes, [&](int64_t i) {
    thread_local std::vector<int32_t> buf;
    gather_row(i, buf);
    rowlen[i] = (int32_t)buf.size();
  });
  for (int64_t i = 0; i < n_nodes; i++) A.rowptr[i + 1] = A.rowptr[i] + rowlen[i];
  const int64_t nnz = A.rowptr[n_nodes];
  A.col.assign(nnz, 0);
  A.valM.assign(nnz, 0.0);
  A.valK.assign(nnz, 0.0);
  parallel_for(n_nodes, [&](int64_t i) {
    thread_local std::vector<int32_t> buf;
    gather_row(i, buf);
    std::copy(buf.begin(), buf.end(), &A.col[A.rowptr[i]]);
  });

  // element matrices, in chunks of elements whose matrices take at most
  // about 256 MiB (a degree-6 element alone holds 343^2 entries of M and K,
  // 1.9 MB), each chunk added row by row into the pattern above
  const int64_t per_elem = (int64_t)npe * npe;
  const int64_t chunk = std::max<int64_t>(1, ((int64_t)1 << 28) / (per_elem * 2 * (int64_t)sizeof(double)));
  std::vector<double> Me((size_t)std::min(chunk, n_elems) * per_elem), Ke(Me.size());
  std::vector<char> bad(2, 0);   // [0]: degenerate or inverted element, [1]: indefinite tensor
  static const double ex[3] = {1, 0, 0}, ey[3] = {0, 1, 0}, ez[3] = {0, 0, 1};
  for (int64_t e0 = 0; e0 < n_elems; e0 += chunk) {
    const int64_t e1 = std::min(n_elems, e0 + chunk);
    parallel_for(e1 - e0, [&](int64_t le) {
      const int64_t e = e0 + le;
      double X[343][3], Dn[343][9];
      const int r = region ? region[e] : 0;
      const double sl = region ? region_sigma[3 * r] : sigma_l;
      const double st = region ? region_sigma[3 * r + 1] : sigma_t;
      const double sn = region ? region_sigma[3 * r + 2] : sigma_n;
      for (int k = 0; k < npe; k++) {
        const int64_t v = conn[e * npe + k];
        for (int c = 0; c < 3; c++) X[k][c] = xyz[3 * v + c];
        const double* f = f0 ? f0 + 3 * v : ex;
        const double* s = s0 ? s0 + 3 * v : ey;
        const double* nn = n0 ? n0 + 3 * v : ez;
        nodal_tensor(f, s, nn, sl, st, sn, scale, Dn[k]);
      }
      double* me = &Me[(size_t)le * per_elem];
      double* ke = &Ke[(size_t)le * per_elem];
      const int rc = (npe >= 125) ? hexp_element(npe == 125 ? 4 : npe == 216 ? 5 : 6, X, Dn, me, ke)
                     : (npe == 64) ? hex64_element(X, Dn, me, ke)
                     : (npe == 27) ? hex27_element(X, Dn, me, ke)
                     : (npe == 10) ? tet10_element(X, Dn, me, ke)
                     : (npe == 8)  ? hex_element(X, Dn, me, ke)
                                   : tet_element(X, Dn, me, ke);
      if (rc == 1) bad[0] = 1;
      if (rc == 2) bad[1] = 1;
      if (region && region_on && !region_on[r])
        for (int64_t k = 0; k < per_elem; k++) me[k] = ke[k] = 0.0;
    });
    if (bad[0]) { set_err(err, "degenerate or inverted element"); return false; }
    if (bad[1]) {
      set_err(err, "the diffusion tensor interpolated from the nodal fibers is indefinite at a quadrature point "
                   "(the fiber field varies too abruptly for this element degree)");
      return false;
    }
    // row i gathers the element rows of its local index, for the elements of
    // this chunk (a node's incidences are listed in increasing element order)
    parallel_for(n_nodes, [&](int64_t i) {
      const int32_t* c = &A.col[A.rowptr[i]];
      const int len = (int)(A.rowptr[i + 1] - A.rowptr[i]);
      double* m = &A.valM[A.rowptr[i]];
      double* kk = &A.valK[A.rowptr[i]];
      const int64_t* lo = std::lower_bound(&ne_idx[ne_ptr[i]], &ne_idx[ne_ptr[i + 1]], e0 * npe);
      for (const int64_t* t = lo; t < &ne_idx[0] + ne_ptr[i + 1] && *t < e1 * npe; t++) {
        const int64_t e = *t / npe;
        const int a = (int)(*t % npe);
        const double* mrow = &Me[((size_t)(e - e0) * npe + a) * npe];
        const double* krow = &Ke[((size_t)(e - e0) * npe + a) * npe];
        for (int b = 0; b < npe; b++) {
          const int32_t j = conn[e * npe + b];
          const int pos = (int)(std::lower_bound(c, c + len, j) - c);
          m[pos] += mrow[b];
          kk[pos] += krow[b];
        }
      }
    });
  }
  return true;
}

std::vector<int64_t> distinct_offsets(const Csr& A) {
  std::vector<int64_t> offs;
  std::vector<char> seen;
  // offsets are bounded by n in magnitude; collect through a sorted merge
  for (int64_t i = 0; i < A.n; i++) {
    for (int64_t t = A.rowptr[i]; t < A.rowptr[i + 1]; t++) {
      const int64_t d = (int64_t)A.col[t] - i;
      offs.push_back(d);
    }
    if (offs.size() > 4096) {
      std::sort(offs.begin(), offs.end());
      offs.erase(std::unique(offs.begin(), offs.end()), offs.end());
      if (offs.size() > 64) return offs;  // far too many for a diagonal format
    }
  }
  std::sort(offs.begin(), offs.end());
  offs.erase(std::unique(offs.begin(), offs.end()), offs.end());
  return offs;
}

}  // namespace ep
