"""Seeded synthetic inputs for the monodomain time step.

This module is shared by the FP64 oracle side (tests, CPU baseline) and the
HIP side (tests, bench).  It holds geometry (node coordinates and element
connectivity), fiber fields, stimulus descriptors, random ionic states and the
workload specifications, and nothing of the method's arithmetic: no finite
element integral, no ionic model, no time stepping, no solver.

Units everywhere: mm, ms, mV, mS/mm, 1/mm, uF/mm^2, uA/mm^3.

Workloads follow the paper's test cases (N-version slab, Section "Slab
benchmark"; idealized left ventricle, Section "Idealized left ventricle";
strong-scalability slab, Section "Strong scalability test") with synthetic
meshes in place of the paper's mesh files, which are not available.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

# ---------------------------------------------------------------------------
# Meshes
# ---------------------------------------------------------------------------

HEX8 = 8
TET4 = 4


@dataclasses.dataclass
class Mesh:
    """Unstructured mesh as plain arrays.

    xyz  : float64 [n_nodes, 3] node coordinates in mm
    conn : int32   [n_elems, 8] (hex) or [n_elems, 4] (tet)
    Hex local node k = a + 2 b + 4 c sits at the reference corner (a, b, c)
    (lexicographic order).  dims is the lattice shape (nx, ny, nz) when the
    mesh came from a structured generator, else None.
    """

    xyz: np.ndarray
    conn: np.ndarray
    dims: Optional[Tuple[int, int, int]] = None
    label: str = ""

    @property
    def n_nodes(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_elems(self) -> int:
        return int(self.conn.shape[0])

    @property
    def elem(self) -> int:
        return int(self.conn.shape[1])


def _lattice_xyz(nx: int, ny: int, nz: int, hx: float, hy: float, hz: float,
                 origin=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Lattice nodes, x fastest: node id = ix + nx*(iy + ny*iz)."""
    ix = np.arange(nx, dtype=np.float64)
    iy = np.arange(ny, dtype=np.float64)
    iz = np.arange(nz, dtype=np.float64)
    Z, Y, X = np.meshgrid(iz, iy, ix, indexing="ij")
    xyz = np.stack([origin[0] + X.ravel() * hx,
                    origin[1] + Y.ravel() * hy,
                    origin[2] + Z.ravel() * hz], axis=1)
    return np.ascontiguousarray(xyz)


def _lattice_cells(nx: int, ny: int, nz: int) -> np.ndarray:
    """Base node id of every lattice cell, x fastest."""
    cx = np.arange(nx - 1)
    cy = np.arange(ny - 1)
    cz = np.arange(nz - 1)
    Z, Y, X = np.meshgrid(cz, cy, cx, indexing="ij")
    return (X + nx * (Y + ny * Z)).ravel()


def _cell_corner_offsets(nx: int, ny: int) -> np.ndarray:
    """Node-id offset of reference corner (a, b, c), index a + 2 b + 4 c."""
    off = np.empty(8, dtype=np.int64)
    for c in (0, 1):
        for b in (0, 1):
            for a in (0, 1):
                off[a + 2 * b + 4 * c] = a + nx * b + nx * ny * c
    return off


def slab_q1(Lx: float, Ly: float, Lz: float, h: float, label: str = "") -> Mesh:
    """Structured Q1 hexahedral mesh of [0,Lx]x[0,Ly]x[0,Lz] with spacing ~h.

    The paper's slab benchmark is a 20 x 7 x 3 mm block with the fibers along
    the long (x) axis (Section "Slab benchmark").
    """
    nx = int(round(Lx / h)) + 1
    ny = int(round(Ly / h)) + 1
    nz = int(round(Lz / h)) + 1
    return lattice_q1(nx, ny, nz, Lx / (nx - 1), Ly / (ny - 1), Lz / (nz - 1), label)


def slab_q2(Lx: float, Ly: float, Lz: float, h: float, label: str = "") -> Mesh:
    """Structured triquadratic (27-node) hexahedral mesh of [0,Lx]x[0,Ly]x[0,Lz]
    with element size ~h: nodes on the lattice of spacing h/2, element-local
    node k = a + 3b + 9c at the element's lattice point (a, b, c)."""
    cx = int(round(Lx / h))
    cy = int(round(Ly / h))
    cz = int(round(Lz / h))
    nx, ny, nz = 2 * cx + 1, 2 * cy + 1, 2 * cz + 1
    xyz = _lattice_xyz(nx, ny, nz, Lx / (nx - 1), Ly / (ny - 1), Lz / (nz - 1))
    ex, ey, ez = np.meshgrid(np.arange(cx), np.arange(cy), np.arange(cz), indexing="ij")
    base = (2 * ex + nx * (2 * ey + ny * 2 * ez)).transpose(2, 1, 0).ravel()
    loc = np.array([a + nx * (b + ny * c) for c in range(3) for b in range(3) for a in range(3)])
    conn = (base[:, None] + loc[None, :]).astype(np.int32)
    return Mesh(xyz, conn, (nx, ny, nz), label or f"slab-q2-{Lx}x{Ly}x{Lz}-h{h}")


def slab_q3(Lx: float, Ly: float, Lz: float, h: float, label: str = "") -> Mesh:
    """Structured tricubic (64-node) hexahedral mesh of [0,Lx]x[0,Ly]x[0,Lz]
    with element size ~h: nodes on the lattice of spacing h/3, element-local
    node k = a + 4b + 16c at the element's lattice point (a, b, c)."""
    cx = int(round(Lx / h))
    cy = int(round(Ly / h))
    cz = int(round(Lz / h))
    nx, ny, nz = 3 * cx + 1, 3 * cy + 1, 3 * cz + 1
    xyz = _lattice_xyz(nx, ny, nz, Lx / (nx - 1), Ly / (ny - 1), Lz / (nz - 1))
    ex, ey, ez = np.meshgrid(np.arange(cx), np.arange(cy), np.arange(cz), indexing="ij")
    base = (3 * ex + nx * (3 * ey + ny * 3 * ez)).transpose(2, 1, 0).ravel()
    loc = np.array([a + nx * (b + ny * c) for c in range(4) for b in range(4) for a in range(4)])
    conn = (base[:, None] + loc[None, :]).astype(np.int32)
    return Mesh(xyz, conn, (nx, ny, nz), label or f"slab-q3-{Lx}x{Ly}x{Lz}-h{h}")


def slab_qp(Lx: float, Ly: float, Lz: float, h: float, p: int, label: str = "") -> Mesh:
    """Structured hexahedral mesh of degree p ((p + 1)^3 nodes per element)
    of [0,Lx]x[0,Ly]x[0,Lz] with element size ~h: nodes on the lattice of
    spacing h/p, element-local node k = a + (p + 1) b + (p + 1)^2 c at the
    element's lattice point (a, b, c)."""
    cx = int(round(Lx / h))
    cy = int(round(Ly / h))
    cz = int(round(Lz / h))
    nx, ny, nz = p * cx + 1, p * cy + 1, p * cz + 1
    xyz = _lattice_xyz(nx, ny, nz, Lx / (nx - 1), Ly / (ny - 1), Lz / (nz - 1))
    ex, ey, ez = np.meshgrid(np.arange(cx), np.arange(cy), np.arange(cz), indexing="ij")
    base = (p * ex + nx * (p * ey + ny * p * ez)).transpose(2, 1, 0).ravel()
    r = range(p + 1)
    loc = np.array([a + nx * (b + ny * c) for c in r for b in r for a in r])
    conn = (base[:, None] + loc[None, :]).astype(np.int32)
    return Mesh(xyz, conn, (nx, ny, nz), label or f"slab-q{p}-{Lx}x{Ly}x{Lz}-h{h}")


def lattice_q1(nx: int, ny: int, nz: int, hx: float, hy: float, hz: float,
               label: str = "") -> Mesh:
    xyz = _lattice_xyz(nx, ny, nz, hx, hy, hz)
    base = _lattice_cells(nx, ny, nz)
    conn = (base[:, None] + _cell_corner_offsets(nx, ny)[None, :]).astype(np.int32)
    return Mesh(xyz, np.ascontiguousarray(conn), (nx, ny, nz), label)


# Kuhn (Freudenthal) split of the unit cube into 6 tetrahedra sharing the
# diagonal from corner 0 to corner 7; corner index = a + 2 b + 4 c.  Every
# cell uses the same split, so faces match across cells (conforming mesh).
_KUHN = np.array([[0, 1, 3, 7], [0, 1, 5, 7], [0, 2, 3, 7],
                  [0, 2, 6, 7], [0, 4, 5, 7], [0, 4, 6, 7]], dtype=np.int64)


def _orient_tets(xyz: np.ndarray, tets: np.ndarray) -> np.ndarray:
    """Swap two nodes of negatively oriented tetrahedra (positive volume)."""
    p = xyz[tets]
    v = np.einsum("ij,ij->i", np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]), p[:, 3] - p[:, 0])
    tets = tets.copy()
    neg = v < 0
    tets[neg, 1], tets[neg, 2] = tets[neg, 2].copy(), tets[neg, 1].copy()
    return tets


def slab_p1(Lx: float, Ly: float, Lz: float, h: float, label: str = "", split: str = "kuhn") -> Mesh:
    """Structured P1 tetrahedral slab: the Q1 lattice with each cell Kuhn-split.

    split "kuhn": every cell split the same way, so every long diagonal runs
    along (1, 1, 1).  split "mirrored": the split of a cell is reflected
    across each axis along which the cell's index is odd, so neighbouring
    cells use different body diagonals (no preferred direction on the scale of
    two cells, closer to an unstructured mesh).  Both are conforming: a face
    between two cells is cut along the same diagonal from both sides.
    """
    q = slab_q1(Lx, Ly, Lz, h)
    nx, ny, nz = q.dims
    base = _lattice_cells(nx, ny, nz)
    corner = _cell_corner_offsets(nx, ny)
    if split == "kuhn":
        local = _KUHN[None, :, :]
    elif split == "mirrored":
        # reflecting across axis a maps corner index bit a to its complement
        flip = (base % nx & 1) + 2 * (base // nx % ny & 1) + 4 * (base // (nx * ny) & 1)
        local = _KUHN[None, :, :] ^ flip[:, None, None]
    else:
        raise ValueError(f"unknown split {split!r}")
    tets = (base[:, None, None] + corner[local]).reshape(-1, 4)
    tets = _orient_tets(q.xyz, tets).astype(np.int32)
    return Mesh(q.xyz, np.ascontiguousarray(tets), (nx, ny, nz), label)


# local edges of a 10-node tetrahedron: node 4 + e is the midpoint of edge e
TET10_EDGES = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))


def slab_p2(Lx: float, Ly: float, Lz: float, h: float, label: str = "") -> Mesh:
    """Structured quadratic (10-node) tetrahedral slab: the Kuhn-split cells
    of the lattice of spacing h, nodes on the lattice of spacing h/2.  Local
    nodes 0-3 are the (positively oriented) vertices, node 4 + e the midpoint
    of edge TET10_EDGES[e]."""
    cx = int(round(Lx / h))
    cy = int(round(Ly / h))
    cz = int(round(Lz / h))
    nx, ny, nz = 2 * cx + 1, 2 * cy + 1, 2 * cz + 1
    xyz = _lattice_xyz(nx, ny, nz, Lx / (nx - 1), Ly / (ny - 1), Lz / (nz - 1))
    ex, ey, ez = np.meshgrid(np.arange(cx), np.arange(cy), np.arange(cz), indexing="ij")
    base = np.stack([2 * ex, 2 * ey, 2 * ez], axis=-1).transpose(2, 1, 0, 3).reshape(-1, 3)
    corner = np.array([[2 * (k & 1), 2 * ((k >> 1) & 1), 2 * ((k >> 2) & 1)] for k in range(8)])
    vert = base[:, None, None, :] + corner[_KUHN][None, :, :, :]          # [cells, 6, 4, 3] lattice index
    vert = vert.reshape(-1, 4, 3)
    ids = lambda ijk: ijk[..., 0] + nx * (ijk[..., 1] + ny * ijk[..., 2])
    tv = ids(vert)
    oriented = _orient_tets(xyz, tv)
    swap = oriented[:, 1] != tv[:, 1]
    vert[swap, 1], vert[swap, 2] = vert[swap, 2].copy(), vert[swap, 1].copy()
    mids = np.stack([(vert[:, a] + vert[:, b]) // 2 for a, b in TET10_EDGES], axis=1)
    conn = np.concatenate([ids(vert), ids(mids)], axis=1).astype(np.int32)
    return Mesh(xyz, np.ascontiguousarray(conn), (nx, ny, nz), label or f"slab-p2-{Lx}x{Ly}x{Lz}-h{h}")


# ---------------------------------------------------------------------------
# Fibers
# ---------------------------------------------------------------------------

def uniform_fibers(n_nodes: int, f=(1.0, 0.0, 0.0), s=(0.0, 1.0, 0.0),
                   n=(0.0, 0.0, 1.0)):
    """Per-node (f0, s0, n0) all equal; the slab benchmark has f along x."""
    F = np.tile(np.asarray(f, np.float64), (n_nodes, 1))
    S = np.tile(np.asarray(s, np.float64), (n_nodes, 1))
    N = np.tile(np.asarray(n, np.float64), (n_nodes, 1))
    return F, S, N


def rotating_fibers(xyz: np.ndarray, angle0: float = -60.0, angle1: float = 60.0):
    """Fibers in the x-y plane whose angle to x turns linearly with z from
    angle0 to angle1 degrees across the slab (the transmural rotation of
    myocardial fibers); sheets follow in the plane, normals along z."""
    z = xyz[:, 2]
    t = (z - z.min()) / max(z.max() - z.min(), 1e-300)
    th = np.deg2rad(angle0 + (angle1 - angle0) * t)
    zero = np.zeros_like(th)
    F = np.stack([np.cos(th), np.sin(th), zero], axis=1)
    S = np.stack([-np.sin(th), np.cos(th), zero], axis=1)
    N = np.tile(np.array([0.0, 0.0, 1.0]), (xyz.shape[0], 1))
    return F, S, N


def smooth_fibers(xyz: np.ndarray, seed: int, rate: float = 0.25):
    """Orthonormal triplets that turn smoothly through space in all three
    directions: the fiber's azimuth and elevation and the sheet's roll are
    sums of seeded low-frequency waves of the coordinates, each changing by
    at most about `rate` radians per mm (a varied tensor that stays as smooth
    as a myocardial fiber field)."""
    rng = np.random.default_rng(seed)
    ang = []
    for _ in range(3):
        k = rng.uniform(-1.0, 1.0, (3, 3))
        ph = rng.uniform(0.0, 2.0 * np.pi, 3)
        a = sum(np.sin(xyz @ k[j] + ph[j]) / (3.0 * max(np.abs(k[j]).sum(), 1e-12)) for j in range(3))
        ang.append(rate * 3.0 * a)
    az, el, roll = ang
    f = np.stack([np.cos(az) * np.cos(el), np.sin(az) * np.cos(el), np.sin(el)], axis=1)
    # a unit vector orthogonal to f, then turned about f by the roll angle
    e = np.stack([-np.sin(az), np.cos(az), np.zeros_like(az)], axis=1)
    g = np.cross(f, e)
    s = np.cos(roll)[:, None] * e + np.sin(roll)[:, None] * g
    n = np.cross(f, s)
    return f, s, n


def random_fibers(n_nodes: int, seed: int):
    """Random orthonormal triplets per node (for anisotropy tests)."""
    rng = np.random.default_rng(seed)
    a = rng.normal(size=(n_nodes, 3))
    b = rng.normal(size=(n_nodes, 3))
    f = a / np.linalg.norm(a, axis=1, keepdims=True)
    b = b - np.sum(b * f, axis=1, keepdims=True) * f
    s = b / np.linalg.norm(b, axis=1, keepdims=True)
    n = np.cross(f, s)
    return f, s, n


# ---------------------------------------------------------------------------
# Idealized left ventricle (truncated prolate spheroid shell, P1 tets)
# ---------------------------------------------------------------------------

def lv_shell(n_t: int = 30, n_phi: int = 360, n_theta: int = 140,
             epi=(25.0, 45.0), endo=(15.0, 35.0), apex_hole_deg: float = 4.0,
             helix_endo_deg: float = 60.0, helix_epi_deg: float = -60.0,
             label: str = "lv"):
    """Truncated prolate-spheroid LV shell, tetrahedral, with rule-based fibers.

    Surfaces x^2/r^2 + y^2/r^2 + z^2/l^2 = 1 for the endocardium (r, l) = endo
    and the epicardium (r, l) = epi, blended linearly in the transmural
    coordinate t in [0, 1] (endo -> epi).  The shell is cut at the equatorial
    plane z = 0 (base) and keeps z <= 0 down to a small apical hole of
    apex_hole_deg (the structured (t, phi, theta) grid is singular at the
    apex).  The circumferential direction is periodic.  Each grid cell is
    Kuhn-split into 6 tetrahedra.

    Fibers follow the rule of the paper's ventricular cases: the helix angle
    varies linearly across the wall from +60 deg (endo) to -60 deg (epi);
    f = cos(a) e_circ + sin(a) e_long, n = wall normal, s = n x f.

    Returns (Mesh, (f0, s0, n0), endo_node_ids).
    """
    t = np.linspace(0.0, 1.0, n_t)
    phi = np.arange(n_phi) * (2.0 * np.pi / n_phi)
    theta = np.linspace(0.5 * np.pi, np.pi - np.deg2rad(apex_hole_deg), n_theta)
    r = endo[0] + (epi[0] - endo[0]) * t            # [n_t]
    l = endo[1] + (epi[1] - endo[1]) * t
    # node id = it + n_t*(iphi + n_phi*itheta)   (t fastest)
    TH, PH, IT = np.meshgrid(theta, phi, np.arange(n_t), indexing="ij")
    R = r[IT]
    L = l[IT]
    x = R * np.sin(TH) * np.cos(PH)
    y = R * np.sin(TH) * np.sin(PH)
    z = L * np.cos(TH)
    xyz = np.ascontiguousarray(np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1))

    # tangent frames
    e_circ = np.stack([-np.sin(PH), np.cos(PH), np.zeros_like(PH)], axis=-1)
    d_th = np.stack([R * np.cos(TH) * np.cos(PH), R * np.cos(TH) * np.sin(PH), -L * np.sin(TH)], axis=-1)
    # longitudinal unit vector pointing from apex towards base
    e_long = -d_th / np.linalg.norm(d_th, axis=-1, keepdims=True)
    nrm = np.cross(e_circ, e_long)
    nrm /= np.linalg.norm(nrm, axis=-1, keepdims=True)
    # make the normal point outward (away from the cavity)
    radial = np.stack([x, y, z / (L / R) ** 2], axis=-1)
    sgn = np.sign(np.sum(nrm * radial, axis=-1, keepdims=True))
    sgn[sgn == 0] = 1.0
    nrm *= sgn
    alpha = np.deg2rad(helix_endo_deg + (helix_epi_deg - helix_endo_deg) * (IT / max(n_t - 1, 1)))[..., None]
    f = np.cos(alpha) * e_circ + np.sin(alpha) * e_long
    f /= np.linalg.norm(f, axis=-1, keepdims=True)
    s = np.cross(nrm, f)
    f0 = np.ascontiguousarray(f.reshape(-1, 3))
    s0 = np.ascontiguousarray(s.reshape(-1, 3))
    n0 = np.ascontiguousarray(nrm.reshape(-1, 3))

    def nid(it, ip, ith):
        return it + n_t * ((ip % n_phi) + n_phi * ith)

    it, ip, ith = np.meshgrid(np.arange(n_t - 1), np.arange(n_phi), np.arange(n_theta - 1), indexing="ij")
    it = it.ravel(); ip = ip.ravel(); ith = ith.ravel()
    corners = np.empty((it.size, 8), dtype=np.int64)
    for c in (0, 1):
        for b in (0, 1):
            for a in (0, 1):
                corners[:, a + 2 * b + 4 * c] = nid(it + a, ip + b, ith + c)
    tets = corners[:, _KUHN].reshape(-1, 4)
    tets = _orient_tets(xyz, tets).astype(np.int32)
    endo_ids = np.where(np.tile(np.arange(n_t), n_phi * n_theta) == 0)[0].astype(np.int64)
    return Mesh(xyz, np.ascontiguousarray(tets), None, label), (f0, s0, n0), endo_ids


# ---------------------------------------------------------------------------
# Stimuli
# ---------------------------------------------------------------------------

CUBE, SPHERE, GAUSS = 0, 1, 2


@dataclasses.dataclass
class Stimulus:
    """Applied current descriptor (Section "Slab benchmark", "Applied current").

    shape  : CUBE (size = edge), SPHERE (size = radius) or GAUSS (size = std)
    center : mm
    amp    : uA/mm^3 (volumetric, i.e. chi * I_app per unit membrane area)
    t0, dur, period : ms (period 0 = single pulse)
    """

    shape: int
    center: Tuple[float, float, float]
    size: float
    amp: float
    t0: float = 0.0
    dur: float = 2.0
    period: float = 0.0


def corner_cube_stimulus(amp: float = 50.0, edge: float = 1.5, corner=(0.0, 0.0, 0.0),
                         dims=(20.0, 7.0, 3.0)) -> Stimulus:
    """Cube of the given edge at one slab corner (the N-version slab stimulus)."""
    c = []
    for k in range(3):
        c.append(edge / 2 if corner[k] == 0 else dims[k] - edge / 2)
    return Stimulus(CUBE, tuple(c), edge, amp, 0.0, 2.0, 0.0)


# ---------------------------------------------------------------------------
# Element labels (material ids) for several subdomains
# ---------------------------------------------------------------------------

def element_centroids(mesh: Mesh) -> np.ndarray:
    """Mean of each element's node coordinates, [n_elems, 3]."""
    return mesh.xyz[mesh.conn].mean(axis=1)


def material_layers(mesh: Mesh, axis: int, cuts) -> np.ndarray:
    """Label k for elements whose centroid coordinate along `axis` lies
    between cuts[k-1] and cuts[k] (layers 0 .. len(cuts)), e.g. the
    endocardial / mid-myocardial / epicardial layers of a slab."""
    c = element_centroids(mesh)[:, axis]
    return np.searchsorted(np.asarray(cuts, np.float64), c).astype(np.int32)


def material_box(mesh: Mesh, lo, hi, label: int, base=None) -> np.ndarray:
    """Copy of `base` (zeros when None) with `label` on the elements whose
    centroid lies inside the axis-aligned box [lo, hi] (e.g. a scar)."""
    c = element_centroids(mesh)
    out = np.zeros(mesh.conn.shape[0], np.int32) if base is None else np.array(base, np.int32)
    inside = np.all((c >= np.asarray(lo)) & (c <= np.asarray(hi)), axis=1)
    out[inside] = label
    return out


# ---------------------------------------------------------------------------
# Physical parameter sets of the workloads
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Physics:
    sigma_l: float = 0.17      # mS/mm
    sigma_t: float = 0.019
    sigma_n: float = 0.019
    chi: float = 140.0         # 1/mm
    cm: float = 0.01           # uF/mm^2


# N-version slab benchmark conductivities are given already divided by
# chi*C_m (m^2/s); 1 m^2/s = 1e3 mm^2/ms.  With chi*C_m = 1 they can be fed
# through the same sigma/(chi C_m) map.
NVERSION_D = (0.95298e-4 * 1e3, 0.12576e-4 * 1e3, 0.12576e-4 * 1e3)


@dataclasses.dataclass
class SimSpec:
    """One simulation: mesh, fibers, physics, model, stimuli, time stepping."""

    mesh: Mesh
    fibers: tuple
    phys: Physics
    model: str                 # "passive" | "ap" | "bo" | "ttp06"
    variant: str = ""          # ttp06: endo|mid|epi ; bo: epi
    stimuli: List[Stimulus] = dataclasses.field(default_factory=list)
    dt: float = 0.05
    bdf: int = 1
    n_steps: int = 1
    rtol: float = 1e-10
    label: str = ""


def config_c0() -> SimSpec:
    """Aliev-Panfilov, Q1 slab 20x7x3 mm at h=0.5 mm (4305 nodes), BDF1, 400 steps."""
    m = slab_q1(20.0, 7.0, 3.0, 0.5, "slab-h0.5")
    return SimSpec(m, uniform_fibers(m.n_nodes), Physics(), "ap", "",
                   [corner_cube_stimulus()], 0.05, 1, 400, 1e-10, "C0")


def config_c1(h: float = 0.1, n_steps: int = 2000, variant: str = "endo") -> SimSpec:
    """TTP06 endocardial, Q1 slab at h=0.1 mm (442,401 nodes), BDF2, 100 ms."""
    m = slab_q1(20.0, 7.0, 3.0, h, f"slab-h{h}")
    return SimSpec(m, uniform_fibers(m.n_nodes), Physics(), "ttp06", variant,
                   [corner_cube_stimulus()], 0.05, 2, n_steps, 1e-10, "C1")


def config_c2(scale: float = 1.0, seed: int = 3, n_steps: int = 6000) -> SimSpec:
    """Bueno-Orovio EPI on a P1 LV shell (~1.5M nodes at scale 1), BDF2."""
    n_t = max(3, int(round(30 * scale)))
    n_phi = max(8, int(round(360 * scale)))
    n_th = max(4, int(round(140 * scale)))
    m, fib, endo_ids = lv_shell(n_t, n_phi, n_th)
    rng = np.random.default_rng(seed)
    # area weights of endocardial nodes ~ local circumference radius
    w = np.hypot(m.xyz[endo_ids, 0], m.xyz[endo_ids, 1]) + 1e-12
    pick = rng.choice(endo_ids, size=5, replace=False, p=w / w.sum())
    # paper's Gaussian impulses: std 2.5 mm, 2 ms; amplitude 0.3 /ms in the
    # dimensionless potential = 0.3*85.7 mV/ms = chi*C_m*25.71 uA/mm^3
    amp = 0.3 * 85.7 * 140.0 * 0.01
    stims = [Stimulus(GAUSS, tuple(m.xyz[i]), 2.5, amp, 0.0, 2.0, 0.0) for i in pick]
    return SimSpec(m, fib, Physics(0.17, 0.17 / 4, 0.17 / 4), "bo", "epi", stims,
                   0.05, 2, n_steps, 1e-10, "C2")


def config_c3(seed: int = 4, n_inst: int = 64, n_steps: int = 4000,
              n_min: int = 5000, n_max: int = 200000, h: float = 0.2) -> List[SimSpec]:
    """64 independent slab instances of uneven size (batched form)."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_inst):
        target = rng.uniform(n_min, n_max)
        L = rng.uniform(10.0, 40.0)
        nx = int(round(L / h)) + 1
        cross = max(target / nx, 4.0)
        # 7:3 aspect cross-section
        ny = max(2, int(round(math.sqrt(cross * 7.0 / 3.0))))
        nz = max(2, int(round(cross / ny)))
        m = lattice_q1(nx, ny, nz, h, h, h, f"inst{k}")
        model = "ap" if rng.uniform() < 0.5 else "ttp06"
        scale = rng.uniform(0.7, 1.3)
        corner = tuple(int(b) for b in rng.integers(0, 2, size=3))
        dims = ((nx - 1) * h, (ny - 1) * h, (nz - 1) * h)
        st = corner_cube_stimulus(50.0, min(1.5, min(dims) * 0.5), corner, dims)
        out.append(SimSpec(m, uniform_fibers(m.n_nodes),
                           Physics(0.17 * scale, 0.019 * scale, 0.019 * scale),
                           model, "endo" if model == "ttp06" else "", [st],
                           0.05, 2, n_steps, 1e-10, f"C3-{k}"))
    return out


@dataclasses.dataclass
class Request:
    arrival_s: float
    spec: SimSpec


def serving_trace(seed: int = 5, n_req: int = 128, rate_per_s: float = 4.0,
                  n_min: float = 1e4, n_max: float = 1e6, t_min: float = 50.0,
                  t_max: float = 500.0, dt: float = 0.05, h: float = 0.2,
                  build_meshes: bool = True) -> List[Request]:
    """Poisson arrivals of TTP06 / Bueno-Orovio requests on slabs or LV shells."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(n_req):
        t += rng.exponential(1.0 / rate_per_s)
        model = "ttp06" if rng.uniform() < 0.5 else "bo"
        geom = "slab" if rng.uniform() < 0.5 else "lv"
        n_target = math.exp(rng.uniform(math.log(n_min), math.log(n_max)))
        T = rng.uniform(t_min, t_max)
        scale = rng.uniform(0.7, 1.3)
        site_u = rng.uniform(size=3)
        n_steps = int(round(T / dt))
        if not build_meshes:
            out.append(Request(t, SimSpec(None, None, Physics(), model, "", [], dt, 2, n_steps, 1e-10,
                                          f"req{k}:{geom}:{int(n_target)}")))
            continue
        if geom == "slab":
            # 20 x 7 x 3 proportions scaled to the target node count
            s = (n_target / (101 * 36 * 16)) ** (1.0 / 3.0)
            nx = max(3, int(round(100 * s)) + 1)
            ny = max(3, int(round(35 * s)) + 1)
            nz = max(2, int(round(15 * s)) + 1)
            m = lattice_q1(nx, ny, nz, h, h, h, f"req{k}")
            fib = uniform_fibers(m.n_nodes)
            dims = ((nx - 1) * h, (ny - 1) * h, (nz - 1) * h)
            c = tuple(site_u[i] * dims[i] for i in range(3))
            st = Stimulus(SPHERE, c, max(1.0, 3 * h), 50.0 if model == "ttp06" else 36.0, 0.0, 2.0, 0.0)
            phys = Physics(0.17 * scale, 0.019 * scale, 0.019 * scale)
        else:
            s = (n_target / (30 * 360 * 140)) ** (1.0 / 3.0)
            m, fib, endo_ids = lv_shell(max(3, int(round(30 * s))), max(8, int(round(360 * s))),
                                        max(4, int(round(140 * s))), label=f"req{k}")
            i = endo_ids[int(site_u[0] * (endo_ids.size - 1))]
            st = Stimulus(GAUSS, tuple(m.xyz[i]), 2.5, 0.3 * 85.7 * 1.4 if model == "bo" else 50.0, 0.0, 2.0, 0.0)
            phys = Physics(0.17 * scale, 0.17 / 4 * scale, 0.17 / 4 * scale)
        out.append(Request(t, SimSpec(m, fib, phys, model, "epi" if model == "bo" else "endo", [st],
                                      dt, 2, n_steps, 1e-10, f"req{k}")))
    return out


# ---------------------------------------------------------------------------
# Random ionic states (for single-step tests).  Variable order is the one the
# C-ABI documents for state upload/download.
# ---------------------------------------------------------------------------

STATE_NAMES = {
    "passive": [],
    "ap": ["v"],
    "bo": ["v", "w", "s"],
    "ttp06": ["m", "h", "j", "xr1", "xr2", "xs", "s", "r", "d", "f", "f2", "fcass",
              "cai", "casr", "cass", "nai", "ki", "rr"],
}


def random_state(model: str, n: int, seed: int):
    """(u, w[n_vars, n]) drawn inside physiological ranges of each variable."""
    rng = np.random.default_rng(seed)
    if model == "passive":
        return rng.uniform(-1.0, 1.0, n), np.zeros((0, n))
    if model == "ap":
        u = rng.uniform(-0.05, 1.05, n)
        w = rng.uniform(0.0, 2.5, (1, n))
        return u, w
    if model == "bo":
        u = rng.uniform(-0.05, 1.5, n)
        w = np.stack([rng.uniform(0, 1, n), rng.uniform(0, 1, n), rng.uniform(0, 1, n)])
        return u, w
    if model == "ttp06":
        u = rng.uniform(-90.0, 45.0, n)
        gates = rng.uniform(0.0, 1.0, (12, n))
        cai = 10 ** rng.uniform(-4.3, -3.0, n)
        casr = rng.uniform(1.0, 4.0, n)
        cass = 10 ** rng.uniform(-4.3, -2.5, n)
        nai = rng.uniform(7.0, 11.0, n)
        ki = rng.uniform(130.0, 140.0, n)
        rr = rng.uniform(0.5, 1.0, n)
        return u, np.vstack([gates, cai, casr, cass, nai, ki, rr])
    raise ValueError(model)
