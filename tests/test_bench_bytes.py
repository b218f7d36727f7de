"""bench.py's algorithmic bytes per launch (the numerator of the reported
roofline) against the per-node figures derived by hand for each kernel:
symmetric DIA of the Q1 lattice (14 stored diagonals), FP64 and the FP32
inner solve, and the matrix-free operator with full and compressed
geometry.  CPU only."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

N = 442401          # C1 lattice, 201 x 71 x 31


def _kb(kind, mixed=False, pipe=False):
    return bench.kernel_bytes(kind, N, 0, mixed, 18, "DIA", 14, pipe)


def test_pipelined_cg_iteration_bytes():
    # 14 diagonals x 8 B + m gathered 8 + dinv 8 + z w p s x r read 48 + z s p x r w m' written 56
    assert _kb("cg_pipe") == 232 * N == 102637032
    # FP32 inner form: 14 x 4 + m 4 + dinv 4 + 5 FP32 vectors read 20 + x 8 + 5 written 20 + x 8 + m' 4
    assert _kb("cg_pipe", mixed=True) == 124 * N
    # start kernels: A u_0 with u_0 read, w_0 and m_0 written, dinv read
    assert _kb("cg_spmv", pipe=True) == (14 * 8 + 32) * N
    assert _kb("cg_spmv", mixed=True, pipe=True) == (14 * 4 + 16) * N


def test_chronopoulos_gear_and_step_kernels():
    assert _kb("cg_spmv") == (14 * 8 + 16) * N
    assert _kb("cg_spmv", mixed=True) == (14 * 4 + 8) * N
    assert _kb("cg_update") == 96 * N and _kb("cg_update", mixed=True) == 56 * N
    assert _kb("rhs") == (2 * 14 * 8 + 48) * N
    assert _kb("ir_residual") == (14 * 8 + 28) * N
    assert _kb("ionic") == 320 * N and _kb("ionic", mixed=True) == 192 * N
    assert _kb("activation") == 32 * N
    assert _kb("cg_finalize") == 0


def test_sell_counts_an_index_per_nonzero():
    nnz = 27 * N
    assert bench.kernel_bytes("cg_spmv", N, nnz, False, 18, "SELL") == nnz * 12 + 16 * N
    assert bench.kernel_bytes("cg_spmv", N, nnz, True, 18, "SELL") == nnz * 8 + 8 * N


def test_matrix_free_geometry_bytes():
    n_el, npe = 52500, 27                      # Q2 elements of 0.2 mm on the C1 slab
    ent = n_el * npe
    full = bench.kernel_bytes("cg_spmv", N, 0, False, 18, "MF", 0, False, ent, n_el, False)
    cmp = bench.kernel_bytes("cg_spmv", N, 0, False, 18, "MF", 0, False, ent, n_el, True)
    # per entry: x gathered 8 + node index 4 + element result 8, node sum 8 + 4;
    # geometry 7 x 8 per entry, or per element once compressed
    assert full == 32 * ent + 56 * ent + 24 * N
    assert cmp == 32 * ent + 56 * n_el + 24 * N
    assert full - cmp == 56 * (ent - n_el)
    rhs_full = bench.kernel_bytes("rhs", N, 0, False, 18, "MF", 0, False, ent, n_el, False)
    rhs_cmp = bench.kernel_bytes("rhs", N, 0, False, 18, "MF", 0, False, ent, n_el, True)
    assert rhs_full - rhs_cmp == 64 * (ent - n_el)


def test_counter_keys_name_the_launch_shape():
    assert bench._shape_key("cg_pipe", {"tile_map": 2}) == "@xmap2"
    assert bench._shape_key("rhs", {"tile_map": 0}) == "@xmap0"
    assert bench._shape_key("ionic", {"ionic_npt": 4}) == "@npt4"
    assert bench._shape_key("activation", {}) == ""
