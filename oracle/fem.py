"""Finite-element mass and stiffness matrices (FP64, CPU).  Test infrastructure.

Follows the space discretization of the paper (Section "Cardiac
electrophysiology: numerical discretization"): M_jk is the integral of
phi_k phi_j over the domain, K_jk the integral of D grad(phi_k) . grad(phi_j),
with Gauss quadrature of the fewest points that integrate M exactly:
2x2x2 Gauss-Legendre points for trilinear hexahedra (Q1), 3x3x3 for
triquadratic hexahedra (Q2, the paper's higher-order hexahedral elements),
4x4x4 for tricubic hexahedra (Q3), (p+1)^3 for degree p = 4..6,
the symmetric 4-point degree-2 rule for linear tetrahedra (P1), and a
64-point conical product rule (exact to degree 5) for quadratic tetrahedra
(P2, the paper's higher-order tetrahedral elements, isoparametric like the
hexahedra).

The diffusion tensor is the one of the monodomain model (eq. of the diffusion
tensor): D = sigma_l f f^T + sigma_t s s^T + sigma_n n n^T, rescaled by
1/(chi C_m) (the rescaling stated below the dimensional monodomain equation).
Nodal tensors are interpolated to quadrature points with the FE basis.

Pins: closed-form Q1 / P1 element matrices, K 1 = 0, 1^T M 1 = |Omega|,
the cosine eigenmode of the slab, the 7-point stencil of the Kuhn-split
lattice (tests/test_oracle_fem.py).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def nodal_diffusion(f0, s0, n0, sigma_l, sigma_t, sigma_n, chi, cm):
    """D at every node, [n_nodes, 3, 3], in mm^2/ms (eq. of the diffusion tensor
    divided by chi*C_m)."""
    f0 = np.asarray(f0, np.float64)
    s0 = np.asarray(s0, np.float64)
    n0 = np.asarray(n0, np.float64)
    D = (sigma_l * np.einsum("ni,nj->nij", f0, f0)
         + sigma_t * np.einsum("ni,nj->nij", s0, s0)
         + sigma_n * np.einsum("ni,nj->nij", n0, n0))
    return D / (chi * cm)


# ---------------------------------------------------------------------------
# Q1 hexahedra
# ---------------------------------------------------------------------------

def _q1_reference():
    """Shape values [q, 8] and reference gradients [q, 8, 3] at the 2x2x2
    Gauss points of [-1, 1]^3 (weights all 1).  Local node k = a + 2b + 4c at
    the corner (2a-1, 2b-1, 2c-1)."""
    g = 1.0 / np.sqrt(3.0)
    pts = [(x, y, z) for z in (-g, g) for y in (-g, g) for x in (-g, g)]
    N = np.zeros((8, 8))
    dN = np.zeros((8, 8, 3))
    for q, (x, y, z) in enumerate(pts):
        for c in (0, 1):
            for b in (0, 1):
                for a in (0, 1):
                    k = a + 2 * b + 4 * c
                    sa, sb, sc = 2 * a - 1, 2 * b - 1, 2 * c - 1
                    fx, fy, fz = 1 + sa * x, 1 + sb * y, 1 + sc * z
                    N[q, k] = fx * fy * fz / 8.0
                    dN[q, k] = (sa * fy * fz / 8.0, sb * fx * fz / 8.0, sc * fx * fy / 8.0)
    w = np.ones(8)
    return N, dN, w


def q1_element_matrices(X, Dn):
    """Element mass and stiffness for a batch of trilinear hexahedra.

    X  : [E, 8, 3] corner coordinates (lexicographic local order)
    Dn : [E, 8, 3, 3] nodal diffusion tensors of the element's corners
    returns Me [E, 8, 8], Ke [E, 8, 8]
    """
    N, dN, w = _q1_reference()
    E = X.shape[0]
    Me = np.zeros((E, 8, 8))
    Ke = np.zeros((E, 8, 8))
    for q in range(N.shape[0]):
        # J[e, i, j] = d x_j / d xi_i
        J = np.einsum("ki,ekj->eij", dN[q], X)
        detJ = np.linalg.det(J)
        Jinv = np.linalg.inv(J)
        # physical gradients G[e, k, :] = J^{-1} dN_ref[k]
        G = np.einsum("eij,kj->eki", Jinv, dN[q])
        Dq = np.einsum("k,ekij->eij", N[q], Dn)
        wq = w[q] * detJ
        Me += wq[:, None, None] * np.outer(N[q], N[q])[None]
        Ke += wq[:, None, None] * np.einsum("eai,eij,ebj->eab", G, Dq, G)
    return Me, Ke


# ---------------------------------------------------------------------------
# Q2 hexahedra (27 nodes, triquadratic)
# ---------------------------------------------------------------------------

def _lagrange2(t):
    """Quadratic Lagrange basis on [-1, 1] with nodes -1, 0, 1: values and
    derivatives, each [3]."""
    v = np.array([0.5 * t * (t - 1.0), 1.0 - t * t, 0.5 * t * (t + 1.0)])
    d = np.array([t - 0.5, -2.0 * t, t + 0.5])
    return v, d


def _q2_reference():
    """Shape values [q, 27] and reference gradients [q, 27, 3] at the 3x3x3
    Gauss points of [-1, 1]^3, and the weights.  Local node k = a + 3b + 9c
    sits at the reference point (a - 1, b - 1, c - 1)."""
    g = np.sqrt(0.6)
    x1, w1 = np.array([-g, 0.0, g]), np.array([5.0, 8.0, 5.0]) / 9.0
    pts, wts = [], []
    for iz in range(3):
        for iy in range(3):
            for ix in range(3):
                pts.append((x1[ix], x1[iy], x1[iz]))
                wts.append(w1[ix] * w1[iy] * w1[iz])
    N = np.zeros((27, 27))
    dN = np.zeros((27, 27, 3))
    for q, (x, y, z) in enumerate(pts):
        vx, dx = _lagrange2(x)
        vy, dy = _lagrange2(y)
        vz, dz = _lagrange2(z)
        for c in range(3):
            for b in range(3):
                for a in range(3):
                    k = a + 3 * b + 9 * c
                    N[q, k] = vx[a] * vy[b] * vz[c]
                    dN[q, k] = (dx[a] * vy[b] * vz[c], vx[a] * dy[b] * vz[c], vx[a] * vy[b] * dz[c])
    return N, dN, np.array(wts)


def q2_element_matrices(X, Dn):
    """Element mass and stiffness for a batch of triquadratic hexahedra
    (isoparametric, 27 nodes in the order k = a + 3b + 9c).

    X  : [E, 27, 3]; Dn : [E, 27, 3, 3]; returns Me, Ke [E, 27, 27]
    """
    N, dN, w = _q2_reference()
    E = X.shape[0]
    Me = np.zeros((E, 27, 27))
    Ke = np.zeros((E, 27, 27))
    for q in range(N.shape[0]):
        J = np.einsum("ki,ekj->eij", dN[q], X)
        detJ = np.linalg.det(J)
        Jinv = np.linalg.inv(J)
        G = np.einsum("eij,kj->eki", Jinv, dN[q])
        Dq = np.einsum("k,ekij->eij", N[q], Dn)
        wq = w[q] * detJ
        Me += wq[:, None, None] * np.outer(N[q], N[q])[None]
        Ke += wq[:, None, None] * np.einsum("eai,eij,ebj->eab", G, Dq, G)
    return Me, Ke


def _lagrange3(t):
    """Cubic Lagrange basis on [-1, 1] with the equispaced nodes -1, -1/3,
    1/3, 1: values and derivatives, each [4], from the product formula."""
    nodes = np.array([-1.0, -1.0 / 3.0, 1.0 / 3.0, 1.0])
    v = np.ones(4)
    d = np.zeros(4)
    for j in range(4):
        others = [m for m in range(4) if m != j]
        for m in others:
            v[j] *= (t - nodes[m]) / (nodes[j] - nodes[m])
        for k in others:
            term = 1.0 / (nodes[j] - nodes[k])
            for m in others:
                if m != k:
                    term *= (t - nodes[m]) / (nodes[j] - nodes[m])
            d[j] += term
    return v, d


def _q3_reference():
    """Shape values [q, 64] and reference gradients [q, 64, 3] at the 4x4x4
    Gauss points of [-1, 1]^3, and the weights.  Local node k = a + 4b + 16c
    sits at the reference point (2a/3 - 1, 2b/3 - 1, 2c/3 - 1)."""
    x1, w1 = np.polynomial.legendre.leggauss(4)
    N = np.zeros((64, 64))
    dN = np.zeros((64, 64, 3))
    wts = np.zeros(64)
    q = 0
    for iz in range(4):
        for iy in range(4):
            for ix in range(4):
                vx, dx = _lagrange3(x1[ix])
                vy, dy = _lagrange3(x1[iy])
                vz, dz = _lagrange3(x1[iz])
                wts[q] = w1[ix] * w1[iy] * w1[iz]
                for c in range(4):
                    for b in range(4):
                        for a in range(4):
                            k = a + 4 * b + 16 * c
                            N[q, k] = vx[a] * vy[b] * vz[c]
                            dN[q, k] = (dx[a] * vy[b] * vz[c], vx[a] * dy[b] * vz[c], vx[a] * vy[b] * dz[c])
                q += 1
    return N, dN, wts


def q3_element_matrices(X, Dn):
    """Element mass and stiffness for a batch of tricubic hexahedra
    (isoparametric, 64 nodes in the order k = a + 4b + 16c; the paper's
    hexahedral Q_p spaces with p = 3).

    X  : [E, 64, 3]; Dn : [E, 64, 3, 3]; returns Me, Ke [E, 64, 64]
    """
    N, dN, w = _q3_reference()
    E = X.shape[0]
    Me = np.zeros((E, 64, 64))
    Ke = np.zeros((E, 64, 64))
    for q in range(N.shape[0]):
        J = np.einsum("ki,ekj->eij", dN[q], X)
        detJ = np.linalg.det(J)
        Jinv = np.linalg.inv(J)
        G = np.einsum("eij,kj->eki", Jinv, dN[q])
        Dq = np.einsum("k,ekij->eij", N[q], Dn)
        wq = w[q] * detJ
        Me += wq[:, None, None] * np.outer(N[q], N[q])[None]
        Ke += wq[:, None, None] * np.einsum("eai,eij,ebj->eab", G, Dq, G)
    return Me, Ke


def _lagrange_equispaced(t, p):
    """Lagrange basis of degree p on [-1, 1] with the p + 1 equispaced nodes
    -1 + 2j/p: values and derivatives, each [p + 1], from the product formula."""
    nodes = -1.0 + 2.0 * np.arange(p + 1) / p
    v = np.ones(p + 1)
    d = np.zeros(p + 1)
    for j in range(p + 1):
        others = [m for m in range(p + 1) if m != j]
        for m in others:
            v[j] *= (t - nodes[m]) / (nodes[j] - nodes[m])
        for k in others:
            term = 1.0 / (nodes[j] - nodes[k])
            for m in others:
                if m != k:
                    term *= (t - nodes[m]) / (nodes[j] - nodes[m])
            d[j] += term
    return v, d


def qp_element_matrices(X, Dn, p):
    """Element mass and stiffness for a batch of isoparametric hexahedra of
    degree p (the paper's hexahedral Q_p spaces), (p + 1)^3 nodes in the
    order k = a + (p + 1) b + (p + 1)^2 c at the reference point
    (2a/p - 1, 2b/p - 1, 2c/p - 1), (p + 1)^3 Gauss-Legendre points.

    X  : [E, (p+1)^3, 3]; Dn : [E, (p+1)^3, 3, 3]
    """
    n1 = p + 1
    npe = n1 ** 3
    x1, w1 = np.polynomial.legendre.leggauss(n1)
    E = X.shape[0]
    Me = np.zeros((E, npe, npe))
    Ke = np.zeros((E, npe, npe))
    for iz in range(n1):
        for iy in range(n1):
            for ix in range(n1):
                vx, dx = _lagrange_equispaced(x1[ix], p)
                vy, dy = _lagrange_equispaced(x1[iy], p)
                vz, dz = _lagrange_equispaced(x1[iz], p)
                N = np.einsum("c,b,a->cba", vz, vy, vx).ravel()
                dN = np.stack([np.einsum("c,b,a->cba", vz, vy, dx).ravel(),
                               np.einsum("c,b,a->cba", vz, dy, vx).ravel(),
                               np.einsum("c,b,a->cba", dz, vy, vx).ravel()], axis=1)
                J = np.einsum("ki,ekj->eij", dN, X)
                detJ = np.linalg.det(J)
                G = np.einsum("eij,kj->eki", np.linalg.inv(J), dN)
                Dq = np.einsum("k,ekij->eij", N, Dn)
                wq = w1[ix] * w1[iy] * w1[iz] * detJ
                Me += wq[:, None, None] * np.outer(N, N)[None]
                Ke += wq[:, None, None] * np.einsum("eai,eij,ebj->eab", G, Dq, G)
    return Me, Ke


# ---------------------------------------------------------------------------
# P1 tetrahedra
# ---------------------------------------------------------------------------

_TET_A = 0.5854101966249685
_TET_B = 0.1381966011250105


def _p1_rule():
    """Barycentric points [4, 4] and weights (fractions of the volume) of the
    symmetric 4-point rule, exact for polynomials of degree 2."""
    L = np.full((4, 4), _TET_B)
    np.fill_diagonal(L, _TET_A)
    return L, np.full(4, 0.25)


def p1_element_matrices(X, Dn):
    """Element mass and stiffness for a batch of linear tetrahedra.

    X  : [E, 4, 3]; Dn : [E, 4, 3, 3]
    """
    E = X.shape[0]
    T = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=1)  # rows = edges
    detT = np.linalg.det(T)
    vol = np.abs(detT) / 6.0
    Tinv = np.linalg.inv(T)
    # gradients of barycentric coordinates: grad L_{1..3} = columns of T^{-1}
    G = np.zeros((E, 4, 3))
    G[:, 1:, :] = np.transpose(Tinv, (0, 2, 1))
    G[:, 0, :] = -G[:, 1:, :].sum(axis=1)
    L, w = _p1_rule()
    Me = np.zeros((E, 4, 4))
    Ke = np.zeros((E, 4, 4))
    for q in range(4):
        Dq = np.einsum("k,ekij->eij", L[q], Dn)
        wq = w[q] * vol
        Me += wq[:, None, None] * np.outer(L[q], L[q])[None]
        Ke += wq[:, None, None] * np.einsum("eai,eij,ebj->eab", G, Dq, G)
    return Me, Ke


# ---------------------------------------------------------------------------
# P2 tetrahedra (10 nodes, straight-sided)
# ---------------------------------------------------------------------------

TET10_EDGES = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))


def _collapsed_tet_rule(n=4):
    """Barycentric points [q, 4] and weights (fractions of the volume) of the
    conical product rule: n-point Gauss-Legendre in each direction of the unit
    cube mapped onto the tetrahedron by collapsing (l1 = u, l2 = v (1 - u),
    l3 = w (1 - u)(1 - v), Jacobian 6 (1 - u)^2 (1 - v)).  Exact for
    polynomials of degree 2n - 3 in the barycentric coordinates."""
    x, wx = np.polynomial.legendre.leggauss(n)
    x, wx = 0.5 * (x + 1.0), 0.5 * wx
    L, W = [], []
    for i in range(n):
        for j in range(n):
            for k in range(n):
                u, v, w = x[i], x[j], x[k]
                l1, l2, l3 = u, v * (1 - u), w * (1 - u) * (1 - v)
                L.append((1.0 - l1 - l2 - l3, l1, l2, l3))
                W.append(6.0 * wx[i] * wx[j] * wx[k] * (1 - u) ** 2 * (1 - v))
    return np.array(L), np.array(W)


def _p2_basis(L):
    """Quadratic Lagrange values [10] and derivatives with respect to the
    barycentric coordinates [10, 4] at one point L (vertices first, then the
    midpoints of TET10_EDGES)."""
    N = np.zeros(10)
    dL = np.zeros((10, 4))
    for i in range(4):
        N[i] = L[i] * (2.0 * L[i] - 1.0)
        dL[i, i] = 4.0 * L[i] - 1.0
    for e, (a, b) in enumerate(TET10_EDGES):
        N[4 + e] = 4.0 * L[a] * L[b]
        dL[4 + e, a] = 4.0 * L[b]
        dL[4 + e, b] = 4.0 * L[a]
    return N, dL


def p2_element_matrices(X, Dn):
    """Element mass and stiffness for a batch of isoparametric quadratic
    tetrahedra: the geometry is interpolated with the same 10-node basis, so
    an element whose midside nodes sit off its edge midpoints is integrated on
    its curved shape (for straight-sided elements the map is affine).

    X  : [E, 10, 3]; Dn : [E, 10, 3, 3]; returns Me, Ke [E, 10, 10]
    """
    E = X.shape[0]
    # derivatives of the barycentric coordinates with respect to the three
    # independent reference coordinates (l1, l2, l3), l0 = 1 - l1 - l2 - l3
    dl = np.array([[-1.0, -1.0, -1.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    Lq, wq = _collapsed_tet_rule(4)
    Me = np.zeros((E, 10, 10))
    Ke = np.zeros((E, 10, 10))
    for q in range(Lq.shape[0]):
        N, dL = _p2_basis(Lq[q])
        dN = dL @ dl                                  # reference gradients [10, 3]
        J = np.einsum("kr,ekc->erc", dN, X)           # J[e, r, c] = d x_c / d l_r
        detJ = np.linalg.det(J)
        Jinv = np.linalg.inv(J)
        G = np.einsum("ecr,kr->ekc", Jinv, dN)        # physical gradients [E, 10, 3]
        Dq = np.einsum("k,ekij->eij", N, Dn)
        w = wq[q] / 6.0 * np.abs(detJ)                # the reference tetrahedron has volume 1/6
        Me += w[:, None, None] * np.outer(N, N)[None]
        Ke += w[:, None, None] * np.einsum("eai,eij,ebj->eab", G, Dq, G)
    return Me, Ke


# ---------------------------------------------------------------------------
# Assembly
# ---------------------------------------------------------------------------

def assemble(xyz, conn, Dnodal, chunk: int = 200000):
    """Global M and K (scipy CSR, FP64) by summing element contributions."""
    xyz = np.asarray(xyz, np.float64)
    conn = np.asarray(conn, np.int64)
    n = xyz.shape[0]
    npe = conn.shape[1]
    rows, cols, mv, kv = [], [], [], []
    for e0 in range(0, conn.shape[0], chunk):
        c = conn[e0:e0 + chunk]
        X = xyz[c]
        Dn = Dnodal[c]
        if npe in (125, 216, 343):
            Me, Ke = qp_element_matrices(X, Dn, round(npe ** (1.0 / 3.0)) - 1)
        elif npe == 64:
            Me, Ke = q3_element_matrices(X, Dn)
        elif npe == 27:
            Me, Ke = q2_element_matrices(X, Dn)
        elif npe == 10:
            Me, Ke = p2_element_matrices(X, Dn)
        elif npe == 8:
            Me, Ke = q1_element_matrices(X, Dn)
        elif npe == 4:
            Me, Ke = p1_element_matrices(X, Dn)
        else:
            raise ValueError("element type")
        rows.append(np.repeat(c, npe, axis=1).ravel())
        cols.append(np.tile(c, (1, npe)).ravel())
        mv.append(Me.ravel())
        kv.append(Ke.ravel())
    r = np.concatenate(rows)
    cidx = np.concatenate(cols)
    M = sp.coo_matrix((np.concatenate(mv), (r, cidx)), shape=(n, n)).tocsr()
    K = sp.coo_matrix((np.concatenate(kv), (r, cidx)), shape=(n, n)).tocsr()
    M.sum_duplicates()
    K.sum_duplicates()
    return M, K
