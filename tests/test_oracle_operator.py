"""Pins of the oracle's gamma matrices and operator against facts the paper and
the mathematics fix (closed forms, invariants, printed counts).  CPU only."""
import json
import os

import numpy as np
import pytest

import synthetic as S
from oracle import dirac
from oracle.gamma import GAMMA, GAMMA5, SIGMA

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _paper_constants():
    with open(os.path.join(GOLDEN, "paper_constants.json")) as f:
        return json.load(f)


# ----------------------------------------------------------------- gamma algebra

def test_gamma_hermitian_and_clifford():
    for m in range(4):
        assert np.allclose(GAMMA[m], GAMMA[m].conj().T, atol=0)
        for n in range(4):
            anti = GAMMA[m] @ GAMMA[n] + GAMMA[n] @ GAMMA[m]
            assert np.array_equal(anti, 2.0 * np.eye(4) * (m == n))


def test_gamma5_properties():
    assert np.array_equal(GAMMA5 @ GAMMA5, np.eye(4))
    assert np.array_equal(GAMMA5, GAMMA5.conj().T)
    for m in range(4):
        assert np.array_equal(GAMMA5 @ GAMMA[m] + GAMMA[m] @ GAMMA5, np.zeros((4, 4)))
    # in this convention gamma_5 is minus the product gamma_1 gamma_2 gamma_3 gamma_4
    assert np.array_equal(GAMMA5, -(GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]))


def test_sigma_antisymmetric_traceless():
    for m in range(4):
        assert np.array_equal(SIGMA[m, m], np.zeros((4, 4)))
        for n in range(4):
            assert np.array_equal(SIGMA[m, n], -SIGMA[n, m])
            assert abs(np.trace(SIGMA[m, n])) == 0
            # (i/2) sigma is Hermitian, so the clover term is Hermitian
            h = 0.5j * SIGMA[m, n]
            assert np.allclose(h, h.conj().T)


def test_projectors_rank_two():
    for m in range(4):
        for s in (+1, -1):
            P = np.eye(4) + s * GAMMA[m]
            assert np.linalg.matrix_rank(P) == 2
            # (1 -/+ gamma)/2 are complementary projectors
            assert np.allclose((P / 2) @ (P / 2), P / 2)


# ----------------------------------------------------------------- operator structure

@pytest.fixture(scope="module")
def lat_3435():
    dims = (3, 4, 3, 5)     # non-cubic, all extents >= 3
    U = S.gauge_links(dims, 0.4, 11)
    return dims, U


def test_nnz_per_row_is_51(lat_3435):
    dims, U = lat_3435
    D = dirac.assemble_dense(U, 0.125, 1.0)
    nnz = (np.abs(D) > 1e-14).sum(axis=1)
    assert set(nnz.tolist()) == {_paper_constants()["nonzeros_per_row"]}


def test_gamma5_hermiticity_dense(lat_3435):
    dims, U = lat_3435
    V = S.volume(dims)
    D = dirac.assemble_dense(U, 0.13, 1.6)
    G5 = np.kron(np.eye(V), np.kron(GAMMA5, np.eye(3)))
    assert np.abs(G5 @ D @ G5 - D.conj().T).max() < 1e-15


def test_dagger_is_conjugate_transpose(lat_3435):
    dims, U = lat_3435
    D = dirac.assemble_dense(U, 0.13, 1.6)
    X = S.random_spinor(dims, 3, 5)
    N = 12 * S.volume(dims)
    Yd = dirac.apply(U, 0.13, 1.6, X, dagger=True).reshape(N, 3)
    assert np.abs(Yd - D.conj().T @ X.reshape(N, 3)).max() < 1e-13
    # and equals gamma5 D gamma5
    Y5 = dirac.gamma5(dirac.apply(U, 0.13, 1.6, dirac.gamma5(X))).reshape(N, 3)
    assert np.abs(Yd - Y5).max() < 1e-13


def test_affine_in_csw_and_plain_wilson(lat_3435):
    dims, U = lat_3435
    X = S.random_spinor(dims, 2, 6)
    k = 0.12
    Y0 = dirac.apply(U, k, 0.0, X)
    Y1 = dirac.apply(U, k, 1.0, X)
    Y2 = dirac.apply(U, k, 2.5, X)
    assert np.abs(Y2 - (Y0 + 2.5 * (Y1 - Y0))).max() < 1e-13
    # c_SW = 0: the site-local block is exactly the identity (plain Wilson)
    M0 = dirac.local_matrix(U, k, 0.0)
    assert np.array_equal(M0, np.broadcast_to(np.eye(12), M0.shape))


def test_clover_block_structure(lat_3435):
    dims, U = lat_3435
    F = dirac.field_strength(U)
    for m in range(4):
        assert np.abs(F[m, m]).max() < 1e-15
        for n in range(4):
            assert np.abs(F[m, n] + F[n, m]).max() < 1e-15
            assert np.abs(F[m, n] - dirac.dag(F[m, n])).max() < 1e-15
    M = dirac.local_matrix(U, 0.13, 1.6)
    assert np.abs(M - dirac.dag(M)).max() < 1e-15
    C = (M - np.eye(12)).reshape(M.shape[:4] + (4, 3, 4, 3))
    spin_trace = np.einsum("...sasb->...ab", C)
    assert np.abs(spin_trace).max() < 1e-15
    # block-diagonal after rotating to psi_upper +/- psi_lower
    Q = np.kron(np.block([[np.eye(2), np.eye(2)], [np.eye(2), -np.eye(2)]]), np.eye(3))
    Mt = Q @ M @ np.linalg.inv(Q)
    assert np.abs(Mt[..., :6, 6:]).max() < 1e-14
    assert np.abs(Mt[..., 6:, :6]).max() < 1e-14


# ----------------------------------------------------------------- closed forms

@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (3, 4, 5, 6)])
def test_free_field_plane_wave(dims):
    """U = 1: D acting on e^{i p.n} u equals D(p) u with
    D(p) = 1 - 2 kappa sum cos p_mu + 2 i kappa sum gamma_mu sin p_mu."""
    U = S.unit_links(dims)
    kappa = 0.1
    lx, ly, lz, lt = dims
    rng = np.random.default_rng(3)
    u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    for k in [(0, 0, 0, 0), (1, 0, 0, 0), (0, 1, 2, 3), (2, 3, 1, 5)]:
        p = [2 * np.pi * k[i] / dims[i] for i in range(4)]
        t, z, y, x = np.meshgrid(range(lt), range(lz), range(ly), range(lx), indexing="ij")
        phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
        X = (phase[..., None, None] * u)[..., None]
        Y = dirac.apply(U, kappa, 1.7, X)
        Dp = (1 - 2 * kappa * sum(np.cos(pp) for pp in p)) * np.eye(4) \
            + 2j * kappa * sum(GAMMA[m] * np.sin(p[m]) for m in range(4))
        expect = phase[..., None, None] * (Dp @ u)
        assert np.abs(Y[..., 0] - expect).max() < 1e-14


def _gauge_transform(U, Om):
    """U_mu(n) -> Om(n) U_mu(n) Om(n+mu)^dagger."""
    out = np.empty_like(U)
    for mu in range(4):
        out[mu] = Om @ U[mu] @ dirac.dag(dirac.shift(Om, mu, +1))
    return out


def test_gauge_covariance(lat_3435):
    dims, U = lat_3435
    lx, ly, lz, lt = dims
    Om = S.random_su3((lt, lz, ly, lx), 21)
    Ug = _gauge_transform(U, Om)
    F = dirac.field_strength(U)
    Fg = dirac.field_strength(Ug)
    assert np.abs(Fg - Om @ F @ dirac.dag(Om)).max() < 1e-13
    X = S.random_spinor(dims, 2, 7)
    OmX = np.einsum("...ab,...sbl->...sal", Om, X)
    lhs = dirac.apply(Ug, 0.13, 1.6, OmX)
    rhs = np.einsum("...ab,...sbl->...sal", Om, dirac.apply(U, 0.13, 1.6, X))
    assert np.abs(lhs - rhs).max() < 1e-13


def test_printed_leaves_break_covariance(lat_3435):
    """Documents the reading of the clover leaves: with the first leaf exactly
    as printed (third factor U_nu^dagger(n+nu)) the loop does not close and
    F is not gauge covariant, so the printed form cannot be meant."""
    dims, U = lat_3435
    lx, ly, lz, lt = dims
    Om = S.random_su3((lt, lz, ly, lx), 22)
    Ug = _gauge_transform(U, Om)
    mu, nu = 0, 3

    def printed_p1(U):
        return U[mu] @ dirac.shift(U[nu], mu, +1) @ dirac.dag(dirac.shift(U[nu], nu, +1)) @ dirac.dag(U[nu])

    bad = np.abs(printed_p1(Ug) - Om @ printed_p1(U) @ dirac.dag(Om)).max()
    good_p1 = dirac.leaves(U, mu, nu)[0]
    good = np.abs(dirac.leaves(Ug, mu, nu)[0] - Om @ good_p1 @ dirac.dag(Om)).max()
    assert good < 1e-13 and bad > 1e-2


def test_translation_covariance():
    dims = (4, 3, 5, 4)
    U = S.gauge_links(dims, 0.4, 12)
    X = S.random_spinor(dims, 2, 8)
    Y = dirac.apply(U, 0.13, 1.2, X)
    for mu, step in [(0, 1), (1, 2), (2, -1), (3, 3)]:
        Us = np.stack([dirac.shift(U[m], mu, step) for m in range(4)])
        Ys = dirac.apply(Us, 0.13, 1.2, dirac.shift(X, mu, step))
        assert np.abs(Ys - dirac.shift(Y, mu, step)).max() < 1e-14


def test_kappa_zero_is_identity(lat_3435):
    dims, U = lat_3435
    X = S.random_spinor(dims, 2, 9)
    assert np.array_equal(dirac.apply(U, 0.0, 1.6, X), X)


def test_extent_two_sums_both_neighbours():
    """At extent 2 the forward and backward neighbours coincide; both hopping
    terms are kept (plane-wave check at p = pi)."""
    dims = (2, 2, 2, 2)
    U = S.unit_links(dims)
    u = np.arange(12).reshape(4, 3) + 1j
    t, z, y, x = np.meshgrid(range(2), range(2), range(2), range(2), indexing="ij")
    phase = (-1.0) ** x
    X = (phase[..., None, None] * u)[..., None]
    kappa = 0.1
    Y = dirac.apply(U, kappa, 0.0, X)
    Dp = (1 - 2 * kappa * (-1 + 3)) * np.eye(4)
    assert np.abs(Y[..., 0] - phase[..., None, None] * (Dp @ u)).max() < 1e-14


def test_apply_at_sites_matches_whole_lattice():
    dims = (3, 4, 5, 3)
    U = S.gauge_links(dims, 0.4, 31)
    X = S.random_spinor(dims, 3, 32)
    Y = dirac.apply(U, 0.13, 1.6, X).reshape(S.volume(dims), 4, 3, 3)
    sites = [0, 1, 7, 59, S.volume(dims) - 1]
    Ys = dirac.apply_at_sites(U, 0.13, 1.6, X, sites)
    assert np.abs(Ys - Y[sites]).max() < 1e-14
