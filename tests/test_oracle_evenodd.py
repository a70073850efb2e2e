"""Pins of oracle.evenodd against dense linear algebra on the assembled
operator of Eq. (1): with the rows of D_W ordered by parity, the even-even
block is site-local, the Schur complement D_ee - D_eo D_oo^{-1} D_oe equals
the oracle's even-site operator, and the reconstructed solution equals the
dense LU solution.  Planted mistakes in the Schur operator fail.  CPU only."""
import numpy as np
import pytest

import synthetic as S
from oracle import dirac, evenodd


def _perm(dims):
    """Row order of the dense matrix that puts the even sites first (each site's 12 rows together)."""
    par = evenodd.parity(dims)
    sites = np.concatenate([np.nonzero(par == 0)[0], np.nonzero(par == 1)[0]])
    return (sites[:, None] * 12 + np.arange(12)[None, :]).reshape(-1)


@pytest.fixture(scope="module", params=[(4, 4, 4, 4), (4, 2, 2, 6)])
def lat(request):
    dims = request.param
    U = S.gauge_links(dims, 0.4, 71)
    kappa, csw = 0.13, 1.6
    D = dirac.assemble_dense(U, kappa, csw)
    p = _perm(dims)
    Dp = D[np.ix_(p, p)]
    ne = 12 * S.volume(dims) // 2
    return dims, U, kappa, csw, D, Dp, ne


def test_compact_order_is_site_over_two(lat):
    dims = lat[0]
    par = evenodd.parity(dims)
    for q in (0, 1):
        sites = np.nonzero(par == q)[0]
        assert np.array_equal(sites // 2, np.arange(len(sites)))


def test_parity_blocks_of_the_dense_operator(lat):
    """Hops join only sites of opposite parity: the even-even and odd-odd
    blocks are site-local (12 x 12 diagonal blocks)."""
    dims, U, kappa, csw, D, Dp, ne = lat
    for blk in (Dp[:ne, :ne], Dp[ne:, ne:]):
        mask = np.kron(np.eye(ne // 12), np.ones((12, 12)))
        assert np.abs(blk * (1 - mask)).max() == 0.0


@pytest.mark.parametrize("dagger", [False, True])
def test_schur_operator_equals_dense_schur_complement(lat, dagger):
    dims, U, kappa, csw, D, Dp, ne = lat
    A = Dp.conj().T if dagger else Dp
    Sd = A[:ne, :ne] - A[:ne, ne:] @ np.linalg.solve(A[ne:, ne:], A[ne:, :ne])
    V = S.volume(dims)
    xe = S.random_spinor(dims, 3, 72).reshape(V, 4, 3, 3)[: V // 2]
    got = evenodd.schur_apply(U, kappa, csw, xe, dagger=dagger).reshape(ne, 3)
    assert np.abs(got - Sd @ xe.reshape(ne, 3)).max() < 1e-13 * np.abs(Sd).max() * np.abs(xe).max() * 12


@pytest.mark.parametrize("dagger", [False, True])
def test_prepare_and_reconstruct_give_the_dense_solution(lat, dagger):
    """Solve S x_e = b^_e densely from the oracle's operator columns, then
    reconstruct: the whole X equals the dense LU solution of D X = B."""
    dims, U, kappa, csw, D, Dp, ne = lat
    V = S.volume(dims)
    B = S.gaussian_sources(dims, 2, 73)
    be = evenodd.prepare(U, kappa, csw, B, dagger=dagger).reshape(ne, 2)
    Scols = evenodd.schur_apply(U, kappa, csw, np.eye(ne).reshape(V // 2, 4, 3, ne), dagger=dagger).reshape(ne, ne)
    xe = np.linalg.solve(Scols, be).reshape(V // 2, 4, 3, 2)
    X = evenodd.reconstruct(U, kappa, csw, B, xe, dagger=dagger)
    A = D.conj().T if dagger else D
    Xlu = np.linalg.solve(A, B.reshape(12 * V, 2))
    assert np.abs(X.reshape(12 * V, 2) - Xlu).max() < 1e-12 * np.abs(Xlu).max()


def test_iterative_solve(lat):
    dims, U, kappa, csw, D, Dp, ne = lat
    V = S.volume(dims)
    B = S.point_sources(dims)
    X, info = evenodd.solve(U, kappa, csw, B, 1e-13, 500)
    assert info["status"] == "converged"
    R = B.reshape(12 * V, 12) - D @ X.reshape(12 * V, 12)
    assert (np.linalg.norm(R, axis=0) / np.linalg.norm(B.reshape(12 * V, 12), axis=0)).max() < 1e-12


def test_odd_extent_rejected():
    dims = (3, 4, 4, 4)
    with pytest.raises(ValueError):
        evenodd.schur_apply(S.gauge_links(dims, 0.4, 1), 0.1, 1.0, np.zeros((S.volume(dims) // 2, 4, 3, 1)))


# ------------------------------------------------------------ planted mistakes

@pytest.mark.parametrize("mistake", ["no_inverse", "plus_kappa2", "same_parity_hop"])
def test_pin_catches_schur_mistakes(lat, monkeypatch, mistake):
    """M_oo in place of its inverse, +kappa^2 in place of -kappa^2, and the
    second hop read back on the odd sites each break the dense pin."""
    dims, U, kappa, csw, D, Dp, ne = lat
    Sd = Dp[:ne, :ne] - Dp[:ne, ne:] @ np.linalg.solve(Dp[ne:, ne:], Dp[ne:, :ne])
    V = S.volume(dims)
    xe = S.random_spinor(dims, 2, 74).reshape(V, 4, 3, 2)[: V // 2]
    if mistake == "no_inverse":
        M = dirac.local_matrix(U, kappa, csw).reshape(V, 12, 12)
        got = evenodd.schur_apply(U, kappa, csw, xe, Minv=M)
    elif mistake == "plus_kappa2":
        # -kappa^2 H M^{-1} H -> +kappa^2 H M^{-1} H, through a negated inverse
        got = evenodd.schur_apply(U, kappa, csw, xe, Minv=-evenodd.local_inverse(U, kappa, csw))
    else:
        orig = evenodd._restrict
        calls = []

        def bad(field, par, dims_):
            calls.append(par)
            return orig(field, 1 if len(calls) == 2 else par, dims_)

        monkeypatch.setattr(evenodd, "_restrict", bad)
        got = evenodd.schur_apply(U, kappa, csw, xe)
    assert np.abs(got.reshape(ne, 2) - Sd @ xe.reshape(ne, 2)).max() > 1e-6
