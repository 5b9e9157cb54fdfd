"""Pins of the seeded input generators: closed-form nonzero counts, the
HPCG/HPGMP sizes printed in Table 2, structure (sorted columns, diagonal,
symmetry where expected) and determinism of the SplitMix64 streams."""
import os

import numpy as np
import pytest

import workloads as W
from workloads import rng

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_reference_values():
    # SplitMix64 with seed 0: first outputs of the published generator
    out = rng.raw(0, 3)
    assert [hex(int(v)) for v in out] == ["0xe220a8397b1dcdaf", "0x6e789e6aa1b965f4", "0x6c45d188009454f"]


def test_streams_are_deterministic_and_distinct():
    a = rng.uniform(rng.substream("x"), 1000, -1, 1)
    b = rng.uniform(rng.substream("x"), 1000, -1, 1)
    c = rng.uniform(rng.substream("y"), 1000, -1, 1)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert a.min() >= -1 and a.max() < 1
    z = rng.normal(rng.substream("n"), 200000)
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1) < 0.01


@pytest.mark.parametrize("gen,size,nnz", [
    (W.poisson2d, 64, 5 * 64 ** 2 - 4 * 64),
    (W.poisson3d, 24, 7 * 24 ** 3 - 6 * 24 ** 2),
    (W.convdiff_q1, 12, (3 * 12 - 2) ** 3),
    (W.elasticity_bonds, 9, 9 * (3 * 9 - 2) ** 3),
    (W.varcoef2d, 33, 5 * 33 ** 2 - 4 * 33),
])
def test_closed_form_nnz_and_structure(gen, size, nnz):
    A = gen(size)
    assert A.nnz == nnz
    assert A.row_ptr[0] == 0 and A.row_ptr[-1] == A.nnz
    for i in range(A.n):
        c = A.col_idx[A.row_ptr[i]:A.row_ptr[i + 1]]
        assert np.all(np.diff(c) > 0) and i in c
    S = A.to_scipy()
    assert np.all(S.diagonal() > 0)
    if gen is not W.convdiff_q1:
        assert abs(S - S.T).max() <= 1e-12 * abs(S).max()
    else:
        assert abs(S - S.T).max() > 1e-3 * abs(S).max()  # convection: nonsymmetric


def test_full_size_closed_forms_match_configs():
    # the sizes quoted for the workloads follow from the closed forms
    assert 7 * 128 ** 3 - 6 * 128 ** 2 == 14_581_760
    assert (3 * 100 - 2) ** 3 == 26_463_592
    assert 9 * (3 * 64 - 2) ** 3 == 61_731_000
    assert 5 * 64 ** 2 - 4 * 64 == 20_224


def test_table2_sizes_follow_the_27_point_closed_form():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "table2_stencil_sizes.txt"))
            if l.strip() and not l.startswith("#")]
    for name, n, nnz in rows:
        x, y, z = (int(t) for t in name.split("_")[1:])
        nx, ny, nz = 2 ** x, 2 ** y, 2 ** z
        assert nx * ny * nz == int(n)
        assert (3 * nx - 2) * (3 * ny - 2) * (3 * nz - 2) == int(nnz)
    A = W.hpcg(4, 8, 2)  # small instance of the same generator
    assert A.nnz == (3 * 4 - 2) * (3 * 8 - 2) * (3 * 2 - 2)
    B = W.hpgmp(4, 8, 2)
    assert B.nnz == A.nnz and np.array_equal(B.col_idx, A.col_idx)


def test_hpgmp_changes_only_the_z_couplings():
    # Sec. 5: the HPCG operator with the forward/backward z couplings set to
    # -1 + beta and -1 - beta (beta = 0.5)
    nx, ny, nz = 4, 3, 5
    A, B = W.hpcg(nx, ny, nz).to_scipy().toarray(), W.hpgmp(nx, ny, nz).to_scipy().toarray()
    D = B - A
    plane = nx * ny
    rows, cols = np.nonzero(D)
    assert np.all(np.abs(cols - rows) == plane)
    assert np.allclose(D[rows, cols], np.where(cols > rows, 0.5, -0.5))
    assert len(rows) == 2 * plane * (nz - 1)
    assert not np.allclose(B, B.T)


def test_paper_rhs_is_uniform_on_unit_interval():
    A = W.poisson2d(16)
    b = W.paper_rhs(A, "t")
    assert b.shape == (A.n,) and b.min() >= 0.0 and b.max() < 1.0


def test_elasticity_is_spd_small():
    A = W.elasticity_bonds(5)
    D = A.to_scipy().toarray()
    np.linalg.cholesky(D)
    np.linalg.cholesky(W.varcoef2d(10).to_scipy().toarray())


def test_rhs_is_a_times_xstar():
    A = W.poisson3d(10)
    xs, b = W.rhs(A, "t")
    assert np.allclose(b, A.to_scipy() @ xs, rtol=1e-14, atol=1e-14)
    assert xs.min() >= -1 and xs.max() < 1
