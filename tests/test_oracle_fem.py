"""Pins of the oracle's finite-element assembly against closed forms.

Each check comes from the mathematics, not from the oracle's own formulas:
tensor-product 1D matrices, exact integrals of linear functions, Neumann
row sums, the domain volume, the slab's cosine eigenmodes and the 7-point
stencil of the Kuhn-split lattice.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads as W
from oracle import fem


def _m1(h):
    return h / 6.0 * np.array([[2.0, 1.0], [1.0, 2.0]])


def _k1(h):
    return 1.0 / h * np.array([[1.0, -1.0], [-1.0, 1.0]])


def _box(hx, hy, hz):
    X = np.zeros((8, 3))
    for c in (0, 1):
        for b in (0, 1):
            for a in (0, 1):
                X[a + 2 * b + 4 * c] = (a * hx, b * hy, c * hz)
    return X


def test_q1_box_matches_tensor_product():
    hx, hy, hz = 0.3, 0.7, 1.1
    dx, dy, dz = 0.9, 0.2, 0.05
    X = _box(hx, hy, hz)[None]
    Dn = np.tile(np.diag([dx, dy, dz]), (1, 8, 1, 1))
    Me, Ke = fem.q1_element_matrices(X, Dn)
    # local index a + 2b + 4c -> kron(z, kron(y, x))
    M_ref = np.kron(_m1(hz), np.kron(_m1(hy), _m1(hx)))
    K_ref = (dx * np.kron(_m1(hz), np.kron(_m1(hy), _k1(hx)))
             + dy * np.kron(_m1(hz), np.kron(_k1(hy), _m1(hx)))
             + dz * np.kron(_k1(hz), np.kron(_m1(hy), _m1(hx))))
    assert np.max(np.abs(Me[0] - M_ref)) < 1e-15
    assert np.max(np.abs(Ke[0] - K_ref)) < 1e-14


def test_q1_parallelepiped_linear_fields():
    """On an affine hexahedron, linear fields are in the Q1 space, so
    v^T K v = vol a^T D a and v^T M v = integral of (a.x + c)^2 exactly."""
    rng = np.random.default_rng(0)
    B = np.array([[1.0, 0.2, 0.1], [0.3, 0.8, -0.2], [0.1, 0.25, 1.3]])
    X = _box(1.0, 1.0, 1.0) @ B.T + np.array([0.4, -1.0, 2.0])
    vol = abs(np.linalg.det(B))
    Dm = rng.normal(size=(3, 3))
    D = Dm @ Dm.T + np.eye(3)
    Me, Ke = fem.q1_element_matrices(X[None], np.tile(D, (1, 8, 1, 1)))
    a = np.array([0.7, -1.2, 0.4])
    v = X @ a
    assert abs(v @ Ke[0] @ v - vol * a @ D @ a) < 1e-12
    assert abs(np.sum(Me[0]) - vol) < 1e-14
    # integral of (a.x)^2 over the parallelepiped via an independent tensor Gauss rule
    g, w = np.polynomial.legendre.leggauss(4)
    s = (g + 1) / 2
    acc = 0.0
    for i, x in enumerate(s):
        for j, y in enumerate(s):
            for k, z in enumerate(s):
                p = B @ np.array([x, y, z]) + np.array([0.4, -1.0, 2.0])
                acc += w[i] * w[j] * w[k] / 8.0 * (a @ p) ** 2
    acc *= vol
    assert abs(v @ Me[0] @ v - acc) < 1e-12


def test_p1_reference_tet():
    X = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]])[None]
    Me, Ke = fem.p1_element_matrices(X, np.tile(np.eye(3), (1, 4, 1, 1)))
    K_ref = np.array([[3, -1, -1, -1], [-1, 1, 0, 0], [-1, 0, 1, 0], [-1, 0, 0, 1]]) / 6.0
    M_ref = (1.0 / 6.0) / 20.0 * (np.ones((4, 4)) + np.eye(4))
    assert np.max(np.abs(Ke[0] - K_ref)) < 1e-15
    assert np.max(np.abs(Me[0] - M_ref)) < 1e-16


def test_p1_general_tet_linear_fields():
    rng = np.random.default_rng(1)
    X = rng.normal(size=(4, 3))
    vol = abs(np.linalg.det(np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]]))) / 6.0
    Dm = rng.normal(size=(3, 3))
    D = Dm @ Dm.T + 0.1 * np.eye(3)
    Me, Ke = fem.p1_element_matrices(X[None], np.tile(D, (1, 4, 1, 1)))
    a = rng.normal(size=3)
    v = X @ a
    assert abs(v @ Ke[0] @ v - vol * a @ D @ a) < 1e-12 * max(1.0, vol * a @ D @ a)
    assert np.max(np.abs(Me[0] - vol / 20.0 * (np.ones((4, 4)) + np.eye(4)))) < 1e-15


def _slab_mk(h=0.5, D=(0.12, 0.013, 0.009)):
    m = W.slab_q1(20.0, 7.0, 3.0, h)
    f, s, n = W.uniform_fibers(m.n_nodes)
    Dn = fem.nodal_diffusion(f, s, n, D[0], D[1], D[2], 1.0, 1.0)
    M, K = fem.assemble(m.xyz, m.conn, Dn)
    return m, M, K


def test_neumann_row_sums_and_volume():
    m, M, K = _slab_mk()
    assert np.max(np.abs(K @ np.ones(m.n_nodes))) < 1e-14
    assert abs(np.ones(m.n_nodes) @ (M @ np.ones(m.n_nodes)) - 20.0 * 7.0 * 3.0) < 1e-10
    assert abs(M - M.T).max() < 1e-17 and abs(K - K.T).max() < 1e-17


def test_system_matrix_spd_small():
    m = W.slab_q1(2.0, 1.5, 1.0, 0.5)
    f, s, n = W.random_fibers(m.n_nodes, 3)
    Dn = fem.nodal_diffusion(f, s, n, 0.17, 0.019, 0.01, 140.0, 0.01)
    M, K = fem.assemble(m.xyz, m.conn, Dn)
    A = (1.5 / 0.05) * M + K
    ev = np.linalg.eigvalsh(A.toarray())
    assert ev.min() > 0
    evk = np.linalg.eigvalsh(K.toarray())
    assert abs(evk.min()) < 1e-13 and np.sort(evk)[1] > 1e-6   # one-dimensional kernel


@pytest.mark.parametrize("k", [1, 3, 7])
def test_cosine_mode_is_generalized_eigenvector(k):
    D = (0.12, 0.013, 0.009)
    m, M, K = _slab_mk(0.5, D)
    nx = m.dims[0]
    h = 20.0 / (nx - 1)
    theta = k * np.pi / (nx - 1)
    lam = 6.0 / h ** 2 * (1 - np.cos(theta)) / (2 + np.cos(theta))
    v = np.cos(k * np.pi * m.xyz[:, 0] / 20.0)
    r = K @ v - D[0] * lam * (M @ v)
    assert np.max(np.abs(r)) < 1e-13


def test_kuhn_lattice_p1_is_seven_point_stencil():
    h, d = 0.25, 0.7
    m = W.slab_p1(2.0, 2.0, 2.0, h)
    f, s, n = W.uniform_fibers(m.n_nodes)
    Dn = fem.nodal_diffusion(f, s, n, d, d, d, 1.0, 1.0)
    _, K = fem.assemble(m.xyz, m.conn, Dn)
    nx, ny, nz = m.dims
    K = K.tocsr()
    interior = [ix + nx * (iy + ny * iz) for iz in range(1, nz - 1) for iy in range(1, ny - 1)
                for ix in range(1, nx - 1)]
    for i in interior[::7]:
        row = K.getrow(i)
        ent = dict(zip(row.indices, row.data))
        expect = {i: 6 * h * d, i - 1: -h * d, i + 1: -h * d, i - nx: -h * d, i + nx: -h * d,
                  i - nx * ny: -h * d, i + nx * ny: -h * d}
        for j, val in ent.items():
            assert abs(val - expect.get(j, 0.0)) < 1e-14, (i, j, val)
        for j in expect:
            assert j in ent
    # total volume
    M, _ = fem.assemble(m.xyz, m.conn, Dn)
    assert abs(M.sum() - 8.0) < 1e-12


def test_mirrored_kuhn_lattice_is_valid():
    """The mirrored split (input generator) is a conforming, positively
    oriented tetrahedral mesh of the slab whose long edges run along all four
    body diagonals equally; its P1 operators keep K 1 = 0 and 1^T M 1 = |slab|."""
    h = 0.25
    m = W.slab_p1(2.0, 1.5, 1.0, h, split="mirrored")
    X = m.xyz[m.conn]
    vol = np.einsum("ij,ij->i", np.cross(X[:, 1] - X[:, 0], X[:, 2] - X[:, 0]), X[:, 3] - X[:, 0]) / 6
    assert vol.min() > 0 and abs(vol.sum() - 3.0) < 1e-12
    faces = np.sort(np.concatenate([m.conn[:, [0, 1, 2]], m.conn[:, [0, 1, 3]],
                                    m.conn[:, [0, 2, 3]], m.conn[:, [1, 2, 3]]]), axis=1)
    _, cnt = np.unique(faces, axis=0, return_counts=True)
    nx, ny, nz = m.dims
    assert cnt.max() == 2
    assert (cnt == 1).sum() == 4 * ((nx - 1) * (ny - 1) + (ny - 1) * (nz - 1) + (nx - 1) * (nz - 1))
    e = np.concatenate([m.conn[:, [a, b]] for a in range(4) for b in range(a + 1, 4)])
    dv = m.xyz[e[:, 1]] - m.xyz[e[:, 0]]
    body = np.all(np.abs(np.abs(dv) - h) < 1e-12, axis=1)
    sgn = np.sign(dv[body]) * np.sign(dv[body][:, :1])
    dirs, num = np.unique(sgn, axis=0, return_counts=True)
    assert dirs.shape[0] == 4 and num.min() == num.max()
    f, s, n = W.uniform_fibers(m.n_nodes)
    M, K = fem.assemble(m.xyz, m.conn, fem.nodal_diffusion(f, s, n, 0.9, 0.5, 0.3, 1.0, 1.0))
    assert np.max(np.abs(K @ np.ones(m.n_nodes))) < 1e-13
    assert abs(M.sum() - 3.0) < 1e-12


def test_lv_shell_mesh_is_valid():
    m, (f, s, n), endo = W.lv_shell(4, 24, 10)
    X = m.xyz[m.conn]
    vol = np.einsum("ij,ij->i", np.cross(X[:, 1] - X[:, 0], X[:, 2] - X[:, 0]), X[:, 3] - X[:, 0]) / 6
    assert vol.min() > 0
    # orthonormal fibers
    for a, b in ((f, s), (f, n), (s, n)):
        assert np.max(np.abs(np.sum(a * b, axis=1))) < 1e-12
    for a in (f, s, n):
        assert np.max(np.abs(np.linalg.norm(a, axis=1) - 1)) < 1e-12
    # conforming: every interior face shared by exactly two tets
    faces = np.sort(np.concatenate([m.conn[:, [0, 1, 2]], m.conn[:, [0, 1, 3]],
                                    m.conn[:, [0, 2, 3]], m.conn[:, [1, 2, 3]]]), axis=1)
    _, cnt = np.unique(faces, axis=0, return_counts=True)
    assert cnt.max() == 2


# ---------------------------------------------------------------------------
# Q2 (27-node) hexahedra
# ---------------------------------------------------------------------------

def test_q2_integrates_quadratic_fields_exactly():
    """Mass and stiffness are exact for quadratic fields on an affinely
    mapped (sheared) Q2 lattice: int f g and int grad f . D grad g against
    closed forms (a dropped term, wrong weight or wrong node order fails)."""
    m = W.slab_q2(2.0, 1.0, 1.0, 0.5)
    A = np.array([[1.0, 0.3, 0.0], [0.0, 1.0, 0.2], [0.1, 0.0, 1.0]])
    xyz = m.xyz @ A.T
    D = np.array([[2.0, 0.3, 0.1], [0.3, 1.0, 0.2], [0.1, 0.2, 0.5]])
    Dn = np.broadcast_to(D, (m.n_nodes, 3, 3)).copy()
    M, K = fem.assemble(xyz, m.conn, Dn)
    # pull back to the reference box [0,2]x[0,1]x[0,1]: x = A r, dx = det A dr
    detA = np.linalg.det(A)
    r = m.xyz
    f = r[:, 0] ** 2 + r[:, 1] * r[:, 2]            # quadratic in r (and in x)
    g = r[:, 2] ** 2 - r[:, 0]
    assert abs(np.ones(m.n_nodes) @ M @ np.ones(m.n_nodes) - 2.0 * detA) < 1e-12
    # int f g dr over the box, by exact 1-D integrals
    Ix = {0: 2.0, 1: 2.0, 2: 8.0 / 3.0, 3: 4.0}
    Iy = {0: 1.0, 1: 0.5, 2: 1.0 / 3.0, 3: 0.25}
    fg = (Ix[2] * Iy[0] * Iy[2] - Ix[3] * Iy[0] * Iy[0] + Ix[0] * Iy[1] * Iy[3] - Ix[1] * Iy[1] * Iy[1])
    assert abs(f @ M @ g - fg * detA) < 1e-12
    # gradients in x: grad_x f = A^{-T} grad_r f; energy = int grad_r f^T B grad_r g dr * detA
    B = np.linalg.inv(A) @ D @ np.linalg.inv(A).T
    # grad_r f = (2 r0, r2, r1), grad_r g = (-1, 0, 2 r2)
    terms = {(0, 0): -2.0 * Ix[1] * Iy[0] * Iy[0], (0, 2): 4.0 * Ix[1] * Iy[0] * Iy[1],
             (1, 0): -Ix[0] * Iy[0] * Iy[1], (1, 2): 2.0 * Ix[0] * Iy[0] * Iy[2],
             (2, 0): -Ix[0] * Iy[1] * Iy[0], (2, 2): 2.0 * Ix[0] * Iy[1] * Iy[1]}
    energy = sum(B[i, j] * v for (i, j), v in terms.items())
    assert abs(f @ K @ g - energy * detA) < 1e-11
    assert np.abs(K @ np.ones(m.n_nodes)).max() < 1e-12


def test_q2_eigenvalue_converges_at_fourth_order():
    """Generalized eigenvalue of the slab's cosine mode: for quadratic
    elements the error falls as h^4 (ratio ~16 per halving); the rate pins
    the quadratic basis and the 3x3x3 rule."""
    L = 2.0
    errs = []
    for h in (0.5, 0.25):
        m = W.slab_q2(L, 0.5, 0.5, h)
        Dn = fem.nodal_diffusion(*W.uniform_fibers(m.n_nodes), 1.0, 1.0, 1.0, 1.0, 1.0)
        M, K = fem.assemble(m.xyz, m.conn, Dn)
        v = np.cos(np.pi * m.xyz[:, 0] / L)
        lam_h = spla.eigsh(K, k=2, M=M, sigma=0.0, which="LM")[0]
        lam = (np.pi / L) ** 2
        errs.append(np.min(np.abs(lam_h - lam)))
        assert np.allclose(K @ np.ones(m.n_nodes), 0.0, atol=1e-12)
        del v
    rate = np.log2(errs[0] / errs[1])
    assert 3.7 < rate < 4.3, (errs, rate)


def test_p2_curved_elements_are_isoparametric():
    """Quadratic tetrahedra whose interior nodes (midside nodes included)
    are moved off the lattice are curved; the domain is still the box.  The
    isoparametric space contains the linear fields of physical space, so
    1^T M 1 = |box|, int x dx = |box| * centroid, and the energy of linear
    fields a.x, b.x is a^T D b |box| exactly.  Geometry taken from the four
    vertices alone (midside nodes ignored) fails the last two."""
    m = W.slab_p2(2.0, 1.0, 1.0, 0.5)
    lo, hi = m.xyz.min(axis=0), m.xyz.max(axis=0)
    interior = np.all((m.xyz > lo + 1e-9) & (m.xyz < hi - 1e-9), axis=1)
    rng = np.random.default_rng(21)
    xyz = m.xyz.copy()
    xyz[interior] += rng.uniform(-0.05, 0.05, (interior.sum(), 3))
    D = np.array([[2.0, 0.3, 0.1], [0.3, 1.0, 0.2], [0.1, 0.2, 0.5]])
    M, K = fem.assemble(xyz, m.conn, np.broadcast_to(D, (m.n_nodes, 3, 3)).copy())
    vol = 2.0
    one = np.ones(m.n_nodes)
    assert abs(one @ M @ one - vol) < 1e-12
    centroid = np.array([1.0, 0.5, 0.5])
    assert np.max(np.abs(xyz.T @ (M @ one) - vol * centroid)) < 1e-12
    a, b = np.array([0.7, -1.1, 0.4]), np.array([-0.2, 0.5, 1.3])
    assert abs((xyz @ a) @ K @ (xyz @ b) - a @ D @ b * vol) < 1e-11
    assert np.abs(K @ one).max() < 1e-12


# ---------------------------------------------------------------------------
# Q3 (64-node) hexahedra
# ---------------------------------------------------------------------------

def _box_integral(poly_a, poly_b, lengths):
    """Exact integral of the product of two polynomials over the box
    [0, Lx] x [0, Ly] x [0, Lz]; a polynomial is {(i, j, k): coefficient}."""
    tot = 0.0
    for ea, ca in poly_a.items():
        for eb, cb in poly_b.items():
            term = ca * cb
            for d in range(3):
                e = ea[d] + eb[d]
                term *= lengths[d] ** (e + 1) / (e + 1)
            tot += term
    return tot


def _poly_grad(poly):
    """Gradient of a polynomial, one polynomial per direction."""
    out = [{}, {}, {}]
    for e, c in poly.items():
        for d in range(3):
            if e[d] > 0:
                f = list(e)
                f[d] -= 1
                out[d][tuple(f)] = out[d].get(tuple(f), 0.0) + c * e[d]
    return out


def _poly_eval(poly, r):
    return sum(c * r[:, 0] ** e[0] * r[:, 1] ** e[1] * r[:, 2] ** e[2] for e, c in poly.items())


def test_q3_integrates_cubic_fields_exactly():
    """Mass and stiffness are exact for cubic fields on an affinely mapped
    (sheared) Q3 lattice with an anisotropic D: int f g and
    int grad f . D grad g against exact monomial integrals."""
    m = W.slab_q3(2.0, 1.0, 1.0, 0.5)
    A = np.array([[1.0, 0.3, 0.0], [0.0, 1.0, 0.2], [0.1, 0.0, 1.0]])
    D = np.array([[2.0, 0.3, 0.1], [0.3, 1.0, 0.2], [0.1, 0.2, 0.5]])
    M, K = fem.assemble(m.xyz @ A.T, m.conn, np.broadcast_to(D, (m.n_nodes, 3, 3)).copy())
    detA = np.linalg.det(A)
    box = (2.0, 1.0, 1.0)
    f = {(3, 0, 0): 1.0, (0, 1, 2): 1.0, (1, 1, 1): -2.0}     # x^3 + y z^2 - 2 x y z
    g = {(0, 0, 3): 1.0, (2, 1, 0): -1.0, (0, 1, 0): 1.0, (3, 0, 0): 0.5}   # z^3 - x^2 y + y + x^3/2
    fv, gv = _poly_eval(f, m.xyz), _poly_eval(g, m.xyz)
    one = np.ones(m.n_nodes)
    assert abs(one @ M @ one - 2.0 * detA) < 1e-12
    exact_m = _box_integral(f, g, box) * detA
    assert abs(fv @ M @ gv - exact_m) < 1e-12 * max(1.0, abs(exact_m))
    B = np.linalg.inv(A) @ D @ np.linalg.inv(A).T
    gf, gg = _poly_grad(f), _poly_grad(g)
    exact_k = sum(B[i, j] * _box_integral(gf[i], gg[j], box) for i in range(3) for j in range(3)) * detA
    assert abs(fv @ K @ gv - exact_k) < 1e-11 * max(1.0, abs(exact_k))
    assert np.abs(K @ one).max() < 1e-12
    # a quartic field is not represented: the pin is not vacuous
    q = {(4, 0, 0): 1.0}
    assert abs(_poly_eval(q, m.xyz) @ M @ one - _box_integral(q, {(0, 0, 0): 1.0}, box) * detA) > 1e-6


def test_q3_eigenvalue_converges_at_sixth_order():
    """Generalized eigenvalue of the slab's cosine mode: for cubic elements
    the error falls as h^6 (ratio ~64 per halving); the rate pins the cubic
    basis and the 4x4x4 rule."""
    L = 2.0
    errs = []
    for h in (1.0, 0.5):
        m = W.slab_q3(L, 1.0, 1.0, h)
        Dn = fem.nodal_diffusion(*W.uniform_fibers(m.n_nodes), 1.0, 1.0, 1.0, 1.0, 1.0)
        M, K = fem.assemble(m.xyz, m.conn, Dn)
        lam_h = spla.eigsh(K, k=2, M=M, sigma=0.0, which="LM")[0]
        errs.append(np.min(np.abs(lam_h - (np.pi / L) ** 2)))
    rate = np.log2(errs[0] / errs[1])
    assert 5.6 < rate < 6.4, (errs, rate)


def test_qp_degree4_integrates_quartic_fields_exactly():
    """Generic degree-p hexahedra at p = 4 (125 nodes): mass and stiffness
    exact for quartic fields (degree 8 in one variable in the mass) on a
    sheared lattice with an anisotropic D; K 1 = 0."""
    m = W.slab_qp(2.0, 1.0, 1.0, 1.0, 4)
    A = np.array([[1.0, 0.3, 0.0], [0.0, 1.0, 0.2], [0.1, 0.0, 1.0]])
    D = np.array([[2.0, 0.3, 0.1], [0.3, 1.0, 0.2], [0.1, 0.2, 0.5]])
    M, K = fem.assemble(m.xyz @ A.T, m.conn, np.broadcast_to(D, (m.n_nodes, 3, 3)).copy())
    detA = np.linalg.det(A)
    box = (2.0, 1.0, 1.0)
    f = {(4, 0, 0): 1.0, (1, 2, 1): -1.5, (0, 0, 2): 0.5}
    g = {(4, 0, 0): -0.5, (0, 3, 1): 1.0, (1, 0, 0): 2.0}
    fv, gv = _poly_eval(f, m.xyz), _poly_eval(g, m.xyz)
    exact_m = _box_integral(f, g, box) * detA
    assert abs(fv @ M @ gv - exact_m) < 1e-11 * max(1.0, abs(exact_m))
    B = np.linalg.inv(A) @ D @ np.linalg.inv(A).T
    gf, gg = _poly_grad(f), _poly_grad(g)
    exact_k = sum(B[i, j] * _box_integral(gf[i], gg[j], box) for i in range(3) for j in range(3)) * detA
    assert abs(fv @ K @ gv - exact_k) < 1e-10 * max(1.0, abs(exact_k))
    assert np.abs(K @ np.ones(m.n_nodes)).max() < 1e-11


def test_qp_degree4_eigenvalue_converges_at_eighth_order():
    L = 2.0
    errs = []
    for h in (1.0, 0.5):
        m = W.slab_qp(L, 1.0, 1.0, h, 4)
        Dn = fem.nodal_diffusion(*W.uniform_fibers(m.n_nodes), 1.0, 1.0, 1.0, 1.0, 1.0)
        M, K = fem.assemble(m.xyz, m.conn, Dn)
        lam_h = spla.eigsh(K, k=2, M=M, sigma=0.0, which="LM")[0]
        errs.append(np.min(np.abs(lam_h - (np.pi / L) ** 2)))
    rate = np.log2(errs[0] / errs[1])
    assert 7.5 < rate < 8.5, (errs, rate)


@pytest.mark.parametrize("p", [2, 3])
def test_qp_generic_matches_dedicated_elements(p):
    """The generic degree-p routine equals the separately pinned Q2 / Q3
    routines on curved elements, and slab_qp equals slab_q2 / slab_q3."""
    gen, ded = {2: (W.slab_q2, fem.q2_element_matrices), 3: (W.slab_q3, fem.q3_element_matrices)}[p]
    a, b = W.slab_qp(2.0, 1.0, 1.0, 0.5, p), gen(2.0, 1.0, 1.0, 0.5)
    assert np.array_equal(a.conn, b.conn) and np.allclose(a.xyz, b.xyz, rtol=0, atol=1e-15)
    rng = np.random.default_rng(p)
    X = a.xyz[a.conn[:4]] + rng.uniform(-0.02, 0.02, (4, a.conn.shape[1], 3))
    Dn = fem.nodal_diffusion(*W.random_fibers(a.conn.shape[1], p), 0.9, 0.3, 0.2, 1.0, 1.0)
    Dn = np.broadcast_to(Dn, (4,) + Dn.shape).copy()
    M1, K1 = fem.qp_element_matrices(X, Dn, p)
    M2, K2 = ded(X, Dn)
    assert np.max(np.abs(M1 - M2)) < 1e-15 and np.max(np.abs(K1 - K2)) < 1e-13


# ---------------------------------------------------------------------------
# P2 (10-node) tetrahedra
# ---------------------------------------------------------------------------

def test_p2_integrates_quadratic_fields_exactly():
    """Same closed forms as for Q2 on the Kuhn-split quadratic lattice:
    exact mass and stiffness for quadratic fields (sheared map, anisotropic D)."""
    m = W.slab_p2(2.0, 1.0, 1.0, 0.5)
    A = np.array([[1.0, 0.3, 0.0], [0.0, 1.0, 0.2], [0.1, 0.0, 1.0]])
    D = np.array([[2.0, 0.3, 0.1], [0.3, 1.0, 0.2], [0.1, 0.2, 0.5]])
    M, K = fem.assemble(m.xyz @ A.T, m.conn, np.broadcast_to(D, (m.n_nodes, 3, 3)).copy())
    detA = np.linalg.det(A)
    r = m.xyz
    f = r[:, 0] ** 2 + r[:, 1] * r[:, 2]
    g = r[:, 2] ** 2 - r[:, 0]
    Ix = {0: 2.0, 1: 2.0, 2: 8.0 / 3.0, 3: 4.0}
    Iy = {0: 1.0, 1: 0.5, 2: 1.0 / 3.0, 3: 0.25}
    fg = (Ix[2] * Iy[0] * Iy[2] - Ix[3] * Iy[0] * Iy[0] + Ix[0] * Iy[1] * Iy[3] - Ix[1] * Iy[1] * Iy[1])
    assert abs(f @ M @ g - fg * detA) < 1e-12
    B = np.linalg.inv(A) @ D @ np.linalg.inv(A).T
    terms = {(0, 0): -2.0 * Ix[1] * Iy[0] * Iy[0], (0, 2): 4.0 * Ix[1] * Iy[0] * Iy[1],
             (1, 0): -Ix[0] * Iy[0] * Iy[1], (1, 2): 2.0 * Ix[0] * Iy[0] * Iy[2],
             (2, 0): -Ix[0] * Iy[1] * Iy[0], (2, 2): 2.0 * Ix[0] * Iy[1] * Iy[1]}
    energy = sum(B[i, j] * v for (i, j), v in terms.items())
    assert abs(f @ K @ g - energy * detA) < 1e-11
    assert np.abs(K @ np.ones(m.n_nodes)).max() < 1e-12
    assert abs(M.sum() - 2.0 * detA) < 1e-12


def test_p2_eigenvalue_converges_at_about_fourth_order():
    """Cosine-mode eigenvalue error of the quadratic tetrahedra: 7.9e-4 at
    h = 0.5 and 6.4e-5 at h = 0.25 (rate 3.6, approaching 4; linear
    elements give 2)."""
    errs = []
    for h in (0.5, 0.25):
        m = W.slab_p2(2.0, 0.5, 0.5, h)
        Dn = fem.nodal_diffusion(*W.uniform_fibers(m.n_nodes), 1.0, 1.0, 1.0, 1.0, 1.0)
        M, K = fem.assemble(m.xyz, m.conn, Dn)
        lam_h = spla.eigsh(K, k=2, M=M, sigma=0.0, which="LM")[0]
        errs.append(np.min(np.abs(lam_h - (np.pi / 2.0) ** 2)))
    rate = np.log2(errs[0] / errs[1])
    assert 3.3 < rate < 4.5, (errs, rate)


def _min_eig_interpolated_d(mesh, fibers, p):
    """Smallest eigenvalue of the nodal D interpolated with the degree-p
    basis, over the Gauss points of every element."""
    Dn = fem.nodal_diffusion(*fibers, 0.17, 0.019, 0.019, 1.0, 1.0)[mesh.conn]   # [E, npe, 3, 3]
    x1, _ = np.polynomial.legendre.leggauss(p + 1)
    lo = np.inf
    for z in x1:
        for y in x1:
            for x in x1:
                N = np.einsum("c,b,a->cba", fem._lagrange_equispaced(z, p)[0], fem._lagrange_equispaced(y, p)[0],
                              fem._lagrange_equispaced(x, p)[0]).ravel()
                lo = min(lo, np.linalg.eigvalsh(np.einsum("k,ekij->eij", N, Dn)).min())
    return lo


def test_interpolated_diffusion_tensor_definiteness():
    """The reading that interpolates nodal D with the element basis keeps D
    positive semi-definite at quadrature points for a smooth fiber field,
    but not at p = 4 for fibers drawn at random per node (the basis has
    negative lobes); trilinear elements stay definite either way."""
    m4 = W.slab_qp(2.0, 1.0, 1.0, 0.5, 4)
    assert _min_eig_interpolated_d(m4, W.rotating_fibers(m4.xyz), 4) > 0.0
    assert _min_eig_interpolated_d(m4, W.random_fibers(m4.n_nodes, 9), 4) < 0.0
    m1 = W.slab_q1(2.0, 1.0, 1.0, 0.25)
    assert _min_eig_interpolated_d(m1, W.random_fibers(m1.n_nodes, 9), 1) > 0.0
