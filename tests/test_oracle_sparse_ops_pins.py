"""Pins of the oracle's sparse addition (section 2.3) and Jacobi-fused product
(section 2.2.2) against facts that do not come from the oracle: dense
arithmetic on tiny inputs, exact special cases and closed forms, and the
paper's statement that C = (I - omega D^-1 A) B has the pattern of A*B when A's
diagonal is present."""
import numpy as np
import pytest

import oracle
from paper_2103_11991_amd import gen

U = 2.0 ** -53


def dense(A):
    D = np.zeros((A.m, A.n))
    rows = np.repeat(np.arange(A.m), A.row_lengths())
    np.add.at(D, (rows, A.col_idx.astype(np.int64)), A.values.astype(np.float64))
    return D


def pattern(A):
    P = np.zeros((A.m, A.n), dtype=bool)
    rows = np.repeat(np.arange(A.m), A.row_lengths())
    P[rows, A.col_idx.astype(np.int64)] = True
    return P


def rows_cols(rp, cols, m):
    return [cols[rp[i]:rp[i + 1]] for i in range(m)]


@pytest.mark.parametrize("seed", range(10))
def test_spadd_is_the_union_pattern_and_the_dense_sum(seed):
    rng = np.random.default_rng(seed)
    m, n = (int(x) for x in rng.integers(0, 20, size=2))
    A = gen.random_csr(m, n, 0, 8, seed=seed, duplicates=seed % 3 == 0, sorted_rows=seed % 2 == 0)
    B = gen.random_csr(m, n, 0, 8, seed=seed + 7, duplicates=seed % 4 == 0, sorted_rows=seed % 5 != 0)
    alpha, beta = float(rng.normal()), float(rng.normal())
    rp, cols, vals, absv = oracle.spadd(A, B, alpha, beta)
    U_ = pattern(A) | pattern(B)
    for i, c in enumerate(rows_cols(rp, cols, m)):
        np.testing.assert_array_equal(c, np.nonzero(U_[i])[0])
    D = alpha * dense(A) + beta * dense(B)
    rows = np.repeat(np.arange(m), np.diff(rp))
    # at most (terms) roundings of size U each on sums of |contributions|
    np.testing.assert_array_less(np.abs(vals - D[rows, cols]), 40 * U * absv + 1e-300)
    Dabs = np.abs(alpha) * dense(A.with_values(np.abs(A.values))) + np.abs(beta) * dense(B.with_values(np.abs(B.values)))
    np.testing.assert_allclose(absv, Dabs[rows, cols], rtol=1e-14)


def test_spadd_keeps_explicit_zeros_of_cancellation_and_is_exact_on_integers():
    A = gen.random_csr(50, 40, 0, 10, seed=3, value_kind="int")
    rp, cols, vals, _ = oracle.spadd(A, A, 1.0, -1.0)
    # A - A: every stored column of A survives as an explicit zero
    for i, c in enumerate(rows_cols(rp, cols, 50)):
        np.testing.assert_array_equal(c, np.unique(A.col_idx[A.row_ptr[i]:A.row_ptr[i + 1]]))
    assert not vals.any()
    B = gen.random_csr(50, 40, 0, 10, seed=4, value_kind="int", duplicates=True)
    rp, cols, vals, _ = oracle.spadd(A, B, 2.0, -3.0)
    rows = np.repeat(np.arange(50), np.diff(rp))
    np.testing.assert_array_equal(vals, (2.0 * dense(A) - 3.0 * dense(B))[rows, cols])


def test_spadd_with_an_empty_matrix_merges_repeats_only():
    A = gen.random_csr(30, 25, 0, 9, seed=5, duplicates=True, sorted_rows=False, value_kind="int")
    Z = gen.Csr(30, 25, np.zeros(31, dtype=np.int32), np.zeros(0, dtype=np.int32), np.zeros(0))
    rp, cols, vals, _ = oracle.spadd(A, Z, 1.0, 5.0)
    rows = np.repeat(np.arange(30), np.diff(rp))
    np.testing.assert_array_equal(vals, dense(A)[rows, cols])
    assert rp[-1] == pattern(A).sum()


def test_spadd_row_ranges_compose():
    A = gen.random_csr(80, 60, 0, 12, seed=6)
    B = gen.random_csr(80, 60, 0, 12, seed=7)
    full = oracle.spadd(A, B, 0.5, 2.0)
    for r0, r1 in ((0, 17), (17, 50), (50, 80)):
        part = oracle.spadd(A, B, 0.5, 2.0, r0, r1)
        s, e = full[0][r0], full[0][r1]
        np.testing.assert_array_equal(part[0], full[0][r0:r1 + 1] - s)
        np.testing.assert_array_equal(part[1], full[1][s:e])
        np.testing.assert_array_equal(part[2], full[2][s:e])


def with_diagonal(m, k, seed, **kw):
    """A square m x m random matrix whose every row stores its diagonal."""
    A = gen.random_csr(m, m, 0, 6, seed=seed, **kw)
    rows = np.concatenate([np.repeat(np.arange(m), A.row_lengths()), np.arange(m)])
    cols = np.concatenate([A.col_idx.astype(np.int64), np.arange(m)])
    vals = np.concatenate([A.values, 4.0 + np.arange(m) % 3])
    order = np.argsort(rows, kind="stable")
    return gen.csr_from_rows_cols(m, m, rows[order], cols[order], vals[order])


@pytest.mark.parametrize("seed", range(8))
def test_jacobi_is_the_dense_smoother_and_has_the_pattern_of_ab(seed):
    rng = np.random.default_rng(seed)
    m, k = int(rng.integers(1, 18)), int(rng.integers(0, 15))
    A = with_diagonal(m, k, seed)
    B = gen.random_csr(m, k, 0, 6, seed=seed + 30)
    d = np.diag(dense(A))
    dinv = 1.0 / d
    omega = 2.0 / 3.0
    rp, cols, vals, absv = oracle.jacobi_spgemm(A, B, omega, dinv)
    # the paper: same pattern as A*B (A's diagonal present)
    rpE, cE, _, _ = oracle.spgemm(A, B)
    np.testing.assert_array_equal(rp, rpE)
    np.testing.assert_array_equal(cols, cE)
    # values: the dense smoother (I - omega D^-1 A) B
    S = (np.eye(m) - omega * dinv[:, None] * dense(A)) @ dense(B)
    rows = np.repeat(np.arange(m), np.diff(rp))
    np.testing.assert_array_less(np.abs(vals - S[rows, cols]), 64 * U * absv + 1e-300)


def test_jacobi_with_zero_omega_is_b_on_the_pattern_of_ab():
    A = with_diagonal(40, 30, 11)
    B = gen.random_csr(40, 30, 0, 7, seed=12)
    rp, cols, vals, _ = oracle.jacobi_spgemm(A, B, 0.0, np.full(40, 3.0))
    rows = np.repeat(np.arange(40), np.diff(rp))
    np.testing.assert_array_equal(vals, dense(B)[rows, cols])
    assert (vals[~pattern(B)[rows, cols]] == 0).all()


def test_jacobi_of_a_diagonal_matrix_scales_b_exactly():
    # A = D: C = (1 - omega) B, exact for omega = 1/2 and integer B
    m = 60
    D = gen.csr_from_rows_cols(m, m, np.arange(m), np.arange(m), 2.0 + np.arange(m) % 5)
    B = gen.random_csr(m, 45, 0, 9, seed=13, value_kind="int")
    rp, cols, vals, _ = oracle.jacobi_spgemm(D, B, 0.5, 1.0 / D.values)
    np.testing.assert_array_equal(rp, B.row_ptr.astype(np.int64))
    np.testing.assert_array_equal(cols, B.col_idx)
    np.testing.assert_array_equal(vals, 0.5 * B.values)


def test_jacobi_smoothing_of_aggregation_on_the_1d_laplacian():
    """Damped Jacobi on the 1D Laplacian (2, -1) with omega = 2/3 applied to
    pairwise aggregation: interior rows of the smoothed prolongator are
    (1/3, 2/3, 1/3)-shaped: C(i, agg(i)) = 1 - omega*(2-1)/2 = 2/3 and the
    neighbouring aggregate gets omega/2 = 1/3."""
    n = 32
    rows = np.concatenate([np.arange(n), np.arange(1, n), np.arange(n - 1)])
    cols = np.concatenate([np.arange(n), np.arange(n - 1), np.arange(1, n)])
    vals = np.concatenate([np.full(n, 2.0), np.full(2 * (n - 1), -1.0)])
    order = np.lexsort((cols, rows))
    A = gen.csr_from_rows_cols(n, n, rows[order], cols[order], vals[order])
    P = gen.csr_from_rows_cols(n, n // 2, np.arange(n), np.arange(n) // 2, np.ones(n))
    rp, c, v, _ = oracle.jacobi_spgemm(A, P, 2.0 / 3.0, np.full(n, 0.5))
    for i in range(2, n - 2):
        row = dict(zip(c[rp[i]:rp[i + 1]].tolist(), v[rp[i]:rp[i + 1]].tolist()))
        other = i // 2 - 1 if i % 2 == 0 else i // 2 + 1
        assert row == pytest.approx({i // 2: 2.0 / 3.0, other: 1.0 / 3.0}, abs=1e-15)
