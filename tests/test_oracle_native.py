"""Pins of the plain-C operator of the oracle (oracle/dirac_sites.c through
oracle/native.py), used for whole-lattice residual checks at full size:
equality with the NumPy oracle, the one-link closed form of the clover term
and the free-field plane wave.  CPU only."""
import numpy as np
import pytest

import synthetic as S
from oracle import dirac, native
from oracle.gamma import GAMMA
from tests.test_oracle_clover_pin import DIMS, I_SIGMA_T, M_SITE, _expected_local, _links_with, _rotation_link


@pytest.fixture(scope="module")
def lat_3534():
    dims = (3, 5, 3, 4)
    return dims, S.gauge_links(dims, 0.4, 61)


def test_local_matrix_equals_numpy_oracle(lat_3534):
    dims, U = lat_3534
    M = native.local_matrix(U, 0.13, 1.6)
    ref = dirac.local_matrix(U, 0.13, 1.6).reshape(M.shape)
    assert np.abs(M - ref).max() < 1e-15


@pytest.mark.parametrize("dagger", [False, True])
@pytest.mark.parametrize("L", [1, 5, 64])
def test_apply_equals_numpy_oracle(lat_3534, dagger, L):
    dims, U = lat_3534
    X = S.random_spinor(dims, L, 62 + L)
    M = native.local_matrix(U, 0.13, 1.6)
    Y = native.apply(U, 0.13, M, X, dagger=dagger)
    ref = dirac.apply(U, 0.13, 1.6, X, dagger=dagger)
    assert np.abs(Y - ref).max() < 1e-13 * np.abs(ref).max()


def test_residual_equals_numpy_oracle(lat_3534):
    dims, U = lat_3534
    X = S.random_spinor(dims, 4, 70)
    B = S.gaussian_sources(dims, 4, 71)
    M = native.local_matrix(U, 0.13, 1.6)
    rel, bn = native.residual(U, 0.13, M, X, B)
    N = 12 * S.volume(dims)
    R = B.reshape(N, 4) - dirac.apply(U, 0.13, 1.6, X).reshape(N, 4)
    ref = np.linalg.norm(R, axis=0) / np.linalg.norm(B.reshape(N, 4), axis=0)
    assert np.allclose(rel, ref, rtol=1e-13, atol=0)
    assert np.allclose(bn, np.linalg.norm(B.reshape(N, 4), axis=0), rtol=1e-14)


def test_single_link_clover_closed_form():
    """The closed form of the clover term with one non-unit link (see
    tests/test_oracle_clover_pin.py), for the C version of the local term."""
    D = _rotation_link(0.7)
    U = _links_with(DIMS, 3, M_SITE, D)
    M = native.local_matrix(U, 0.11, 1.7)
    want = _expected_local(DIMS, 3, M_SITE, D, 0.11, 1.7, I_SIGMA_T).reshape(M.shape)
    assert np.abs(M - want).max() < 1e-15


def test_free_field_plane_wave():
    dims = (4, 3, 5, 4)
    U = S.unit_links(dims)
    kappa = 0.1
    lx, ly, lz, lt = dims
    u = np.arange(12).reshape(4, 3) * (0.3 + 0.7j) + 1.0
    M = native.local_matrix(U, kappa, 1.3)
    for k in [(1, 0, 0, 0), (0, 2, 1, 3), (3, 1, 4, 1)]:
        p = [2 * np.pi * k[i] / dims[i] for i in range(4)]
        t, z, y, x = np.meshgrid(range(lt), range(lz), range(ly), range(lx), indexing="ij")
        phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
        X = (phase[..., None, None] * u)[..., None]
        Y = native.apply(U, kappa, M, X)
        Dp = (1 - 2 * kappa * sum(np.cos(q) for q in p)) * np.eye(4) \
            + 2j * kappa * sum(GAMMA[m] * np.sin(p[m]) for m in range(4))
        assert np.abs(Y[..., 0] - phase[..., None, None] * (Dp @ u)).max() < 1e-14 * np.abs(u).max()
