"""Pins of oracle.correlators: the free field by a momentum-space route, gauge
invariance, and the pion as a sum of squares."""
import numpy as np
import pytest

import synthetic as S
from oracle import correlators as C
from oracle import dirac
from oracle.gamma import GAMMA, GAMMA5


def _solve_dense(U, kappa, csw, dims):
    B = S.point_sources(dims)
    V = S.volume(dims)
    X = np.linalg.solve(dirac.assemble_dense(U, kappa, csw), B.reshape(12 * V, 12))
    return X.reshape(B.shape)


@pytest.fixture(scope="module")
def free_333x6():
    dims = (3, 3, 3, 6)
    kappa = 0.12
    return dims, kappa, _solve_dense(S.unit_links(dims), kappa, 1.0, dims)


@pytest.mark.parametrize("G", [GAMMA5, GAMMA[0], GAMMA[1], GAMMA[2], GAMMA[3]])
def test_free_field_matches_momentum_space(free_333x6, G):
    dims, kappa, X = free_333x6
    got = C.meson(X, G)
    ref = C.free_meson_momentum(dims, kappa, G)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_free_field_channels_positive_and_decaying(free_333x6):
    """Free quarks: both channels are positive, fall from the source to the
    middle of the lattice and are symmetric under t -> Lt - t."""
    dims, kappa, X = free_333x6
    lt = dims[3]
    for c in (C.pion(X), C.rho(X)):
        assert (c > 0).all()
        assert all(c[t + 1] < c[t] for t in range(lt // 2))
        assert np.allclose(c[1:], c[1:][::-1], rtol=1e-10)


def _gauge_transform(U, Om):
    out = np.empty_like(U)
    for mu in range(4):
        out[mu] = Om @ U[mu] @ dirac.dag(dirac.shift(Om, mu, +1))
    return out


@pytest.fixture(scope="module")
def pair_3324():
    dims = (3, 3, 2, 4)
    lx, ly, lz, lt = dims
    U = S.gauge_links(dims, 0.4, 31)
    Om = S.random_su3((lt, lz, ly, lx), 32)
    Ug = _gauge_transform(U, Om)
    X = _solve_dense(U, 0.12, 1.3, dims)
    Xg = _solve_dense(Ug, 0.12, 1.3, dims)
    return X, Xg, Om


def test_propagator_transforms_covariantly(pair_3324):
    """The solved propagator obeys S'(x) = Om(x) S(x) Om(0)^dagger, which is
    what makes the contractions below gauge invariant."""
    X, Xg, Om = pair_3324
    Sm, Sg = C.propagator(X), C.propagator(Xg)
    # 1_spin (x) Om(x) in the 3 * spin + colour ordering
    O = np.einsum("st,...ab->...satb", np.eye(4), Om).reshape(Om.shape[:4] + (12, 12))
    O0 = O[0, 0, 0, 0]
    assert np.abs(Sg - O @ Sm @ O0.conj().T).max() < 1e-12


@pytest.mark.parametrize("G", [GAMMA5, GAMMA[0], GAMMA[1], GAMMA[2]])
def test_gauge_invariance(pair_3324, G):
    X, Xg, _ = pair_3324
    a, b = C.meson(X, G), C.meson(Xg, G)
    assert np.abs(a - b).max() <= 1e-11 * np.abs(a).max()


def _meson_with(X, G, mistake):
    """The contraction of ``C.meson`` with one planted mistake."""
    Sm = C.propagator(X)
    g5 = np.kron(GAMMA5, np.eye(3))
    Gs = np.kron(G, np.eye(3))
    Gbar = Gs if mistake == "gbar_is_g" else np.kron(GAMMA[3] @ G.conj().T @ GAMMA[3], np.eye(3))
    Sd = np.swapaxes(Sm, -1, -2)
    if mistake != "no_conjugate":
        Sd = np.conj(Sd)
    if mistake == "no_gamma5":
        M = Gs @ Sm @ Gbar @ Sd
    else:
        M = Gs @ Sm @ (Gbar @ g5) @ Sd @ g5
    tr = np.trace(M, axis1=-2, axis2=-1)
    return -np.real(tr.sum(axis=(1, 2, 3)))


def test_gauge_pin_catches_a_missing_conjugate(pair_3324):
    """S^T in place of S^dagger breaks gauge invariance of the rho channel."""
    X, Xg, _ = pair_3324
    a, b = _meson_with(X, GAMMA[0], "no_conjugate"), _meson_with(Xg, GAMMA[0], "no_conjugate")
    assert np.abs(a - b).max() > 1e-6 * np.abs(a).max()


@pytest.mark.parametrize("mistake", ["gbar_is_g", "no_gamma5"])
def test_free_pin_catches_contraction_mistakes(free_333x6, mistake):
    """Gbar taken as G (gamma_4 conjugation forgotten), or the gamma_5 pair
    of the backward propagator dropped: gauge invariant, but the free-field
    rho channel no longer matches the momentum-space route."""
    dims, kappa, X = free_333x6
    G = GAMMA[0]
    got = _meson_with(X, G, mistake)
    ref = C.free_meson_momentum(dims, kappa, G)
    assert np.abs(got - ref).max() > 1e-6 * np.abs(ref).max()


def test_pion_is_sum_of_squares(pair_3324):
    X, _, _ = pair_3324
    direct = (np.abs(X) ** 2).sum(axis=(1, 2, 3, 4, 5, 6))
    assert np.abs(C.pion(X) - direct).max() <= 1e-12 * direct.max()
    assert (C.pion(X) > 0).all()
