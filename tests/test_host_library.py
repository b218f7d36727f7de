"""Host-side checks of the HIP library (no GPU needed).

- the shared library loads and exports every function include/ep.h declares;
- the library's C++ finite-element assembly matches the oracle's assembly
  (written independently) on hexahedral (trilinear and triquadratic),
  tetrahedral (linear and quadratic) and curved LV meshes;
- invalid input is rejected with a status and a message, including a fiber
  field whose interpolated diffusion tensor is indefinite.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

import workloads as W
from oracle import fem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    txt = open(os.path.join(ROOT, "include", "ep.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ep_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    import paper_2308_01651_amd as ep
    names = _declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(ep.lib, n), n
    # and the binding declares exactly these
    assert set(ep._lib.exported_names()) == set(names)
    assert "gfx950" in ep.version()


def _compare(mesh, fibers, sigma=(0.17, 0.019, 0.021), chi=140.0, cm=0.01):
    import paper_2308_01651_amd as ep
    rowptr, col, vm, vk = ep.assemble_csr(mesh.elem, mesh.xyz, mesh.conn, fibers, sigma, chi, cm)
    n = mesh.n_nodes
    import scipy.sparse as sp
    Mg = sp.csr_matrix((vm, col, rowptr), shape=(n, n))
    Kg = sp.csr_matrix((vk, col, rowptr), shape=(n, n))
    f, s, nn = fibers if fibers is not None else W.uniform_fibers(n)
    Dn = fem.nodal_diffusion(f, s, nn, *sigma, chi, cm)
    Mo, Ko = fem.assemble(mesh.xyz, mesh.conn, Dn)
    dM = abs(Mg - Mo).max()
    dK = abs(Kg - Ko).max()
    assert dM <= 1e-13 * abs(Mo).max(), dM
    assert dK <= 1e-12 * abs(Ko).max(), dK
    # same pattern (no missing couplings)
    assert Mg.nnz == Mo.nnz


def test_assembly_matches_oracle_q1_slab():
    m = W.slab_q1(5.0, 3.0, 2.0, 0.5)
    _compare(m, W.random_fibers(m.n_nodes, 11))


@pytest.mark.parametrize("split", ["kuhn", "mirrored"])
def test_assembly_matches_oracle_p1_slab(split):
    m = W.slab_p1(3.0, 2.0, 1.5, 0.5, split=split)
    _compare(m, W.random_fibers(m.n_nodes, 12))


def test_assembly_matches_oracle_lv_shell():
    m, fib, _ = W.lv_shell(4, 20, 8)
    _compare(m, fib, (0.17, 0.0425, 0.0425))


def test_assembly_matches_oracle_distorted_hex():
    m = W.slab_q1(4.0, 2.0, 2.0, 0.5)
    rng = np.random.default_rng(5)
    m.xyz = m.xyz + rng.uniform(-0.08, 0.08, m.xyz.shape)
    _compare(m, W.random_fibers(m.n_nodes, 13))


def test_assembly_matches_oracle_q2_slab():
    m = W.slab_q2(3.0, 2.0, 1.0, 0.5)
    rng = np.random.default_rng(6)
    m.xyz = m.xyz + rng.uniform(-0.03, 0.03, m.xyz.shape)   # curved (isoparametric) elements
    _compare(m, W.smooth_fibers(m.xyz, 14))


def test_assembly_matches_oracle_q3_slab():
    m = W.slab_q3(2.0, 1.0, 1.0, 0.5)
    rng = np.random.default_rng(16)
    m.xyz = m.xyz + rng.uniform(-0.02, 0.02, m.xyz.shape)   # curved (isoparametric) elements
    _compare(m, W.smooth_fibers(m.xyz, 17))


@pytest.mark.parametrize("p", [4, 5, 6])
def test_assembly_matches_oracle_degree_p_hex(p):
    m = W.slab_qp(2.0, 1.0, 1.0, 1.0, p)
    rng = np.random.default_rng(30 + p)
    # curved (isoparametric) elements; 2 % of the node spacing keeps det J > 0
    m.xyz = m.xyz + rng.uniform(-0.02 / p, 0.02 / p, m.xyz.shape)
    _compare(m, W.smooth_fibers(m.xyz, 19))


@pytest.mark.parametrize("curved", [False, True])
def test_assembly_matches_oracle_p2_slab(curved):
    m = W.slab_p2(3.0, 2.0, 1.0, 0.5)
    if curved:   # edge nodes off the midpoints: isoparametric elements
        rng = np.random.default_rng(18)
        m.xyz = m.xyz + rng.uniform(-0.03, 0.03, m.xyz.shape)
    _compare(m, W.smooth_fibers(m.xyz, 15))


def test_invalid_input_is_rejected():
    import paper_2308_01651_amd as ep
    m = W.slab_q1(1.0, 1.0, 1.0, 0.5)
    bad = m.conn.copy()
    bad[0, 0] = m.n_nodes + 3
    with pytest.raises(ep.EpError) as ei:
        ep.assemble_csr(8, m.xyz, bad)
    assert ei.value.status == ep._lib.EP_EINVAL and "range" in str(ei.value)
    inv = m.conn.copy()
    inv[:, [0, 1]] = inv[:, [1, 0]]   # mirrored hexahedra
    with pytest.raises(ep.EpError):
        ep.assemble_csr(8, m.xyz, inv)


def test_no_device_fails_loudly_without_gpu():
    import paper_2308_01651_amd as ep
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(ep.EpError) as ei:
        ep.Simulation(0)
    assert ei.value.status in (ep._lib.EP_EHIP, ep._lib.EP_EINVAL)


def test_folded_quadratic_tetrahedron_is_rejected():
    """An edge node moved past the far vertex of its edge folds the
    isoparametric map (its Jacobian changes sign inside the element)."""
    import paper_2308_01651_amd as ep
    m = W.slab_p2(1.0, 1.0, 1.0, 1.0)
    xyz = m.xyz.copy()
    el = m.conn[0]
    a, b = W.TET10_EDGES[0]
    xyz[el[4]] = xyz[el[a]] + 1.6 * (xyz[el[b]] - xyz[el[a]])
    with pytest.raises(ep.EpError):
        ep.assemble_csr(m.elem, xyz, m.conn, None, (0.17, 0.019, 0.019), 140.0, 0.01)
    ep.assemble_csr(m.elem, m.xyz, m.conn, None, (0.17, 0.019, 0.019), 140.0, 0.01)


@pytest.mark.parametrize("kind", ["q2", "q4", "p2"])
def test_indefinite_interpolated_tensor_is_rejected(kind):
    """Elements of degree >= 2 interpolate the nodal tensor with a basis that
    has negative lobes: fibers drawn at random per node leave the cone of
    positive semi-definite tensors at some quadrature point, and K would not
    be positive semi-definite.  Assembly refuses such input (EP_EINVAL); the
    same mesh with a smooth field, and linear elements with random fibers,
    are accepted."""
    import paper_2308_01651_amd as ep
    m = {"q2": lambda: W.slab_q2(3.0, 2.0, 1.0, 0.5), "q4": lambda: W.slab_qp(2.0, 1.0, 1.0, 0.5, 4),
         "p2": lambda: W.slab_p2(3.0, 2.0, 1.0, 0.5)}[kind]()
    with pytest.raises(ep.EpError) as ei:
        ep.assemble_csr(m.elem, m.xyz, m.conn, W.random_fibers(m.n_nodes, 9))
    assert ei.value.status == ep._lib.EP_EINVAL and "indefinite" in str(ei.value)
    ep.assemble_csr(m.elem, m.xyz, m.conn, W.smooth_fibers(m.xyz, 9))
    m1 = W.slab_q1(2.0, 1.0, 1.0, 0.25)
    ep.assemble_csr(m1.elem, m1.xyz, m1.conn, W.random_fibers(m1.n_nodes, 9))
    p1 = W.slab_p1(2.0, 1.0, 1.0, 0.25)
    ep.assemble_csr(p1.elem, p1.xyz, p1.conn, W.random_fibers(p1.n_nodes, 9))


def test_degree_six_element_matrices_are_assembled_in_chunks():
    """150 degree-6 hexahedra need 282 MB of element matrices; assembly holds
    at most 256 MiB of them at a time (two chunks here) and the result keeps
    the exact volume and the constants in the kernel of K (the per-degree
    comparison with the oracle above covers a single chunk)."""
    import paper_2308_01651_amd as ep
    m = W.slab_qp(6.0, 5.0, 5.0, 1.0, 6)     # 6 x 5 x 5 elements of 1 mm
    assert m.conn.shape[0] * 343 * 343 * 16 > (1 << 28)
    rowptr, col, vm, vk = ep.assemble_csr(m.elem, m.xyz, m.conn, W.smooth_fibers(m.xyz, 3))
    import scipy.sparse as sp
    M = sp.csr_matrix((vm, col, rowptr), shape=(m.n_nodes, m.n_nodes))
    K = sp.csr_matrix((vk, col, rowptr), shape=(m.n_nodes, m.n_nodes))
    assert abs(M.sum() - 150.0) < 1e-10 * 150.0        # volume of the block
    assert np.max(np.abs(K @ np.ones(m.n_nodes))) < 1e-12 * abs(K).max()


def _c_struct_fields(name):
    """(field, C type) of `typedef struct name { ... } name;` in include/ep.h, in order."""
    txt = open(os.path.join(ROOT, "include", "ep.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (name, name), txt, flags=re.S).group(1)
    out = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        ctype, names = decl.split(None, 1)
        out += [(n.strip(), ctype) for n in names.split(",")]
    return out


def test_stats_struct_matches_the_header():
    """The binding's ep_stats mirror has the header's fields, in order and
    with the same C types (a mismatch would shift every later field)."""
    import ctypes as C
    import paper_2308_01651_amd as ep
    ctypes_of = {"int64_t": C.c_int64, "int32_t": C.c_int32, "double": C.c_double}
    fields = _c_struct_fields("ep_stats")
    assert len(fields) >= 17 and fields[-1][0] == "mf_compressed"
    assert [(n, ctypes_of[t]) for n, t in fields] == list(ep._lib.EpStats._fields_)


def test_binding_constants_match_the_header():
    """Every numeric constant of include/ep.h that the binding names has the
    header's value (status codes in _lib); the binding's kernel-kind list is
    indexed by the header's EP_K_* values."""
    import paper_2308_01651_amd as ep
    txt = open(os.path.join(ROOT, "include", "ep.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    consts = dict(re.findall(r"\b(EP_[A-Z0-9_]+)\s*=\s*(-?\d+)", txt))
    consts.update(re.findall(r"#define\s+(EP_[A-Z0-9_]+)\s+(-?\d+)", txt))
    checked = 0
    for name, v in consts.items():
        if name.startswith("EP_K_") or name == "EP_N_KERNEL_KINDS":
            continue
        mod = ep if hasattr(ep, name) else ep._lib
        assert hasattr(mod, name), name
        assert getattr(mod, name) == int(v), (name, getattr(mod, name), v)
        checked += 1
    assert checked >= 40
    kinds = {n: int(v) for n, v in consts.items() if n.startswith("EP_K_")}
    assert len(ep.KERNEL_KINDS) == int(consts["EP_N_KERNEL_KINDS"]) == len(kinds)
    for n, v in kinds.items():
        assert ep.KERNEL_KINDS[v] == n[len("EP_K_"):].lower(), (n, v, ep.KERNEL_KINDS[v])
