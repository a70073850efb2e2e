"""Pins of the oracle's gradients (oracle/gradients.py): the leaf factor
lists against the operator's leaves, the link force against central finite
differences of -Re <Lam, D(U) X>, and every gradient of a full solve against
central finite differences of the loss through dense LU solves."""
import numpy as np
import pytest
import scipy.linalg

import synthetic as S
from oracle import dirac, gradients as GR

DIMS = (3, 3, 4, 3)   # extents >= 3: forward and backward neighbours differ


@pytest.fixture(scope="module")
def setup():
    U = S.gauge_links(DIMS, 0.4, 21)
    L = 2
    B = S.gaussian_sources(DIMS, L, 22)
    C = S.gaussian_sources(DIMS, L, 23)
    return U, B, C


def test_leaf_factor_lists_reproduce_the_leaves(setup):
    U = setup[0]
    for mu in range(4):
        for nu in range(4):
            if mu == nu:
                continue
            for p, spec in zip(dirac.leaves(U, mu, nu), GR.leaf_factors(mu, nu)):
                prod = np.broadcast_to(np.eye(3, dtype=complex), U.shape[1:]).copy()
                for f in spec:
                    prod = prod @ GR.factor_value(U, f)
                assert np.abs(prod - p).max() < 1e-14


def test_hopping_and_clover_split_the_operator(setup):
    U, B, _ = setup
    kappa, csw = 0.11, 1.3
    D = dirac.apply(U, kappa, csw, B)
    assert np.abs(D - (B - kappa * csw * GR.clover_apply(U, B) - kappa * GR.hopping(U, B))).max() < 1e-13


def _fd(f, h=1e-6):
    return (f(h) - f(-h)) / (2 * h)


@pytest.mark.parametrize("csw", [0.0, 1.4])
def test_link_force_matches_finite_differences(setup, csw):
    U, X, Lam = setup
    kappa = 0.12
    g = GR.grad_links(U, kappa, csw, X, Lam)
    rng = np.random.default_rng(5)
    for _ in range(10):
        mu = int(rng.integers(4))
        site = tuple(int(rng.integers(n)) for n in U.shape[1:5])
        a, b = int(rng.integers(3)), int(rng.integers(3))
        for unit in (1.0, 1j):
            def f(h):
                Up = U.copy()
                Up[(mu,) + site + (a, b)] += h * unit
                return GR.link_force_check_value(Up, kappa, csw, X, Lam)
            fd = _fd(f)
            want = g[(mu,) + site + (a, b)]
            got = want.real if unit == 1.0 else want.imag
            assert abs(got - fd) <= 1e-7 * (1 + abs(fd)), (mu, site, a, b, unit, got, fd)


def _solve(U, kappa, csw, B):
    N = 12 * S.volume(DIMS)
    L = B.shape[-1]
    D = dirac.assemble_dense(U, kappa, csw)
    return scipy.linalg.solve(D, B.reshape(N, L)).reshape(B.shape), D


def _loss(X, C):
    # l = Re <C, X> + |X|^2 / 2, whose gradient with respect to X is C + X
    return float(np.real(np.vdot(C, X)) + 0.5 * np.vdot(X, X).real)


def test_solve_gradients_match_finite_differences(setup):
    U, B, C = setup
    kappa, csw = 0.12, 1.4
    N = 12 * S.volume(DIMS)
    L = B.shape[-1]
    X, D = _solve(U, kappa, csw, B)
    G = C + X
    Lam = scipy.linalg.solve(D.conj().T, G.reshape(N, L)).reshape(B.shape)
    # adjoint through gamma_5: D^H = gamma_5 D gamma_5
    Lam5 = dirac.gamma5(_solve(U, kappa, csw, dirac.gamma5(G))[0])
    assert np.abs(Lam5 - Lam).max() < 1e-12 * np.abs(Lam).max()

    gk = GR.grad_kappa(U, kappa, csw, X, Lam)
    gc = GR.grad_csw(U, kappa, csw, X, Lam)
    gU = GR.grad_links(U, kappa, csw, X, Lam)

    fk = _fd(lambda h: _loss(_solve(U, kappa + h, csw, B)[0], C))
    fc = _fd(lambda h: _loss(_solve(U, kappa, csw + h, B)[0], C))
    assert abs(gk - fk) <= 1e-6 * abs(fk), (gk, fk)
    assert abs(gc - fc) <= 1e-6 * abs(fc), (gc, fc)

    rng = np.random.default_rng(9)
    for _ in range(4):
        idx = (int(rng.integers(12 * 0 + S.volume(DIMS))), int(rng.integers(4)), int(rng.integers(3)), int(rng.integers(L)))
        site, s, c, l = idx
        coord = np.unravel_index(site, B.shape[:4])
        for unit in (1.0, 1j):
            def fB(h):
                Bp = B.copy()
                Bp[coord + (s, c, l)] += h * unit
                return _loss(_solve(U, kappa, csw, Bp)[0], C)
            fd = _fd(fB)
            want = Lam[coord + (s, c, l)]
            got = want.real if unit == 1.0 else want.imag
            assert abs(got - fd) <= 1e-6 * (1 + abs(fd))
    for _ in range(4):
        mu = int(rng.integers(4))
        site = tuple(int(rng.integers(n)) for n in U.shape[1:5])
        a, b = int(rng.integers(3)), int(rng.integers(3))
        for unit in (1.0, 1j):
            def fU(h):
                Up = U.copy()
                Up[(mu,) + site + (a, b)] += h * unit
                return _loss(_solve(Up, kappa, csw, B)[0], C)
            fd = _fd(fU)
            want = gU[(mu,) + site + (a, b)]
            got = want.real if unit == 1.0 else want.imag
            assert abs(got - fd) <= 1e-6 * (1 + abs(fd)), (mu, site, a, b, unit, got, fd)
