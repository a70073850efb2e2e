"""Pins of oracle.deflation: the pivoted Cholesky picks a basis of the
column space (rank equal to numpy's matrix_rank on exact low-rank blocks),
dependent columns are reproduced by their coefficients, and the restarted
solve converges on blocks with duplicate and dependent columns, where the
plain block method breaks down, to the dense LU solution.  CPU only."""
import numpy as np
import pytest

import synthetic as S
from oracle import deflation, dirac, solvers


def _rng_block(n, L, rank, seed):
    rng = np.random.default_rng(seed)
    base = rng.standard_normal((n, rank)) + 1j * rng.standard_normal((n, rank))
    mix = rng.standard_normal((rank, L)) + 1j * rng.standard_normal((rank, L))
    return base @ mix


@pytest.mark.parametrize("L,rank", [(6, 6), (6, 3), (8, 1), (12, 7)])
def test_pivoted_cholesky_rank(L, rank):
    R = _rng_block(200, L, rank, L + rank)
    Rn = R / np.linalg.norm(R, axis=0)
    acc = deflation.pivoted_cholesky(Rn.conj().T @ Rn, 1e-6)
    assert len(acc) == np.linalg.matrix_rank(R) == rank
    # the accepted columns span the block
    Q, _ = np.linalg.qr(R[:, acc])
    assert np.abs(R - Q @ (Q.conj().T @ R)).max() < 1e-10 * np.abs(R).max()


def test_plan_coefficients_reproduce_dependent_columns():
    R = _rng_block(150, 7, 4, 3)
    B = R.copy()
    I, C = deflation.plan(R, B, 1e-12, 1e-6)
    assert len(I) == 4
    assert np.abs(R[:, I] @ C - R).max() < 1e-10 * np.abs(R).max()


def test_plan_drops_converged_columns():
    rng = np.random.default_rng(4)
    B = rng.standard_normal((100, 3)) + 0j
    R = B.copy()
    R[:, 1] *= 1e-14
    I, C = deflation.plan(R, B, 1e-12, 1e-6)
    assert 1 not in I and np.all(C[:, 1] == 0)


@pytest.fixture(scope="module")
def small():
    dims = (4, 4, 2, 2)
    U = S.gauge_links(dims, 0.4, 5)
    kappa, csw = 0.125, 1.0
    A = dirac.as_matrix_operator(U, kappa, csw)
    D = dirac.assemble_dense(U, kappa, csw)
    return dims, A, D


def test_duplicate_columns_converge(small):
    """B = [b, b, 2 b + c, c]: the plain block method breaks down on the
    singular Gram matrix; the deflated solve converges to dense LU."""
    dims, A, D = small
    N = 12 * S.volume(dims)
    b = S.gaussian_sources(dims, 1, 6).reshape(N, 1)
    c = S.gaussian_sources(dims, 1, 7).reshape(N, 1)
    B = np.concatenate([b, b, 2 * b + c, c], axis=1)
    _, info0 = solvers.block_bicggr(A, B, 1e-12, 200)
    assert info0["status"] == "breakdown"
    X, info = deflation.solve(A, B, 1e-12)
    assert info["status"] == "converged"
    assert info["widths"][0] == 2
    Xlu = np.linalg.solve(D, B)
    assert np.abs(X - Xlu).max() < 1e-10 * np.abs(Xlu).max()
    assert solvers.true_residual(A, B, X).max() <= 1e-12


def test_independent_columns_are_not_deflated(small):
    dims, A, D = small
    N = 12 * S.volume(dims)
    B = S.gaussian_sources(dims, 5, 8).reshape(N, 5)
    X, info = deflation.solve(A, B, 1e-12)
    assert info["status"] == "converged" and info["widths"][0] == 5
    assert solvers.true_residual(A, B, X).max() <= 1e-12


def test_planted_mistake_wrong_coefficients_fail():
    """Coefficients taken without the Gram matrix (c_d = R_I^H r_d) no
    longer reproduce the dependent columns: the coefficient pin fails."""
    R = _rng_block(150, 7, 4, 3)
    I, C = deflation.plan(R, R.copy(), 1e-12, 1e-6)
    RI = R[:, I]
    bad = C.copy()
    for d in range(R.shape[1]):
        if d not in I:
            bad[:, d] = RI.conj().T @ R[:, d]
    assert np.abs(RI @ bad - R).max() > 1e-3 * np.abs(R).max()


def test_columns_differing_below_the_tolerance_are_dependent():
    """Two residual columns that differ by 1e-4 of their norm, but by far less
    than tol ||b|| (duplicated right-hand sides late in a solve): the floor
    tol ||b|| / 10 keeps the second one out of the block."""
    rng = np.random.default_rng(11)
    b = rng.standard_normal(300) + 1j * rng.standard_normal(300)
    r = 1e-10 * (rng.standard_normal(300) + 1j * rng.standard_normal(300))
    d = 1e-14 * np.linalg.norm(b) * rng.standard_normal(300) / np.sqrt(300)
    R = np.stack([r, r + d], axis=1)
    B = np.stack([b, b], axis=1)
    I, C = deflation.plan(R, B, 1e-12, 1e-6)
    assert len(I) == 1
    # without the floor the relative test alone would keep both
    Rn = R / np.linalg.norm(R, axis=0)
    assert len(deflation.pivoted_cholesky(Rn.conj().T @ Rn, 1e-6)) == 2
