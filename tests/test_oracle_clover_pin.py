"""Closed-form pin of the clover term of Eq. (1) (Sec. 2): sign, scale and
orientation of F_{mu nu} and of the (i/2) sigma_{mu nu} factor.

The lattice has unit links except one link U_nu(m) = D.  A clover leaf is a
product of four links around a plaquette, so every leaf that does not
contain this link is the identity, and (P - P^dagger)/(2i) vanishes for it.
The link lies on the six plaquettes with corners m, m + nu, m + nu + s rho,
m + s rho (rho != nu, s = +-1).  Walking each of the four leaves of Sec. 2
around its corner site n in the (rho, nu) plane (read with the standard
loop closures) gives, with f = (D - D^dagger) / (8i):

* F_{rho nu}(n) = +f at n = m - rho and n = m + nu - rho (the leaf crosses
  the link forwards: it is the second factor of leaf 1 at m - rho and the
  third factor of leaf 4 at m + nu - rho);
* F_{rho nu}(n) = -f at n = m + rho and n = m + nu + rho (the link is
  crossed backwards, as the third factor of leaf 2 and the second of leaf 3);
* at m and m + nu the two leaves of each plane through the link cross it in
  opposite directions and cancel; everywhere else F = 0.

With sigma_{rho nu} = gamma_rho gamma_nu for rho != nu and the sum over both
orderings in Eq. (1), the site-local matrix is
    M(n) = 1 - kappa c_SW sum_rho (i sigma_{rho nu}) (x) F_{rho nu}(n).
The matrices i sigma_{rho 4} below were multiplied out by hand from the gamma
matrices printed in Sec. 2 (they are not computed from the oracle's tables).
Extents are at least 3 so that the listed corner sites are distinct.
"""
import numpy as np
import pytest

import synthetic as S
from oracle import dirac
from oracle.gamma import SIGMA

# i * gamma_rho gamma_4 for rho = x, y, z, from the printed matrices of Sec. 2
I_SIGMA_T = {
    0: np.array([[0, 0, 0, -1], [0, 0, -1, 0], [0, -1, 0, 0], [-1, 0, 0, 0]], dtype=np.complex128),
    1: np.array([[0, 0, 0, 1j], [0, 0, -1j, 0], [0, 1j, 0, 0], [-1j, 0, 0, 0]], dtype=np.complex128),
    2: np.array([[0, 0, -1, 0], [0, 0, 0, 1], [-1, 0, 0, 0], [0, 1, 0, 0]], dtype=np.complex128),
}
# i * gamma_1 gamma_2 = diag(-1, 1, -1, 1) for the (x, y) plane
I_SIGMA_XY = np.diag([-1, 1, -1, 1]).astype(np.complex128)

DIMS = (3, 4, 5, 3)   # Lx, Ly, Lz, Lt, non-cubic
M_SITE = (1, 2, 3, 1)  # x, y, z, t of the base m of the non-trivial link


def _diag_link(theta):
    return np.diag([np.exp(1j * theta), np.exp(-1j * theta), 1.0])


def _rotation_link(theta):
    """exp(i theta lambda_2): a real rotation in the first two colours, so
    f = (sin theta / 4) lambda_2 is not symmetric and a transposed colour
    index would show."""
    c, s = np.cos(theta), np.sin(theta)
    return np.array([[c, s, 0], [-s, c, 0], [0, 0, 1]], dtype=np.complex128)


def _links_with(dims, nu, m, D):
    U = S.unit_links(dims).copy()
    x, y, z, t = m
    U[nu, t, z, y, x] = D
    return U


def _shifted(c, mu, s, dims):
    out = list(c)
    out[mu] = (out[mu] + s) % dims[mu]
    return tuple(out)


def _expected_local(dims, nu, m, D, kappa, csw, i_sigma):
    """M(n) for every site from the closed form in the module docstring.
    i_sigma[rho] is i sigma_{rho nu} for the planes through direction nu."""
    lx, ly, lz, lt = dims
    f = (D - D.conj().T) / 8j
    M = np.broadcast_to(np.eye(12, dtype=np.complex128), (lt, lz, ly, lx, 12, 12)).copy()
    mn = _shifted(m, nu, +1, dims)
    for rho, isig in i_sigma.items():
        for corner, sign in ((_shifted(m, rho, -1, dims), +1), (_shifted(mn, rho, -1, dims), +1),
                             (_shifted(m, rho, +1, dims), -1), (_shifted(mn, rho, +1, dims), -1)):
            x, y, z, t = corner
            M[t, z, y, x] -= kappa * csw * sign * np.kron(isig, f)
    return M


def _check(U, dims, nu, D, kappa, csw, i_sigma):
    got = dirac.local_matrix(U, kappa, csw)
    want = _expected_local(dims, nu, M_SITE, D, kappa, csw, i_sigma)
    return np.abs(got - want).max()


@pytest.mark.parametrize("make", [_diag_link, _rotation_link])
def test_single_link_clover_t_planes(make):
    """Link in the t direction: the (x,t), (y,t), (z,t) planes."""
    D = make(0.7)
    nu = 3
    U = _links_with(DIMS, nu, M_SITE, D)
    assert _check(U, DIMS, nu, D, 0.11, 1.7, I_SIGMA_T) < 1e-15


@pytest.mark.parametrize("make", [_diag_link, _rotation_link])
def test_single_link_clover_xy_plane(make):
    """Link in the y direction: the four corners of its (x, y) plaquettes.
    Each of these sites is a corner of only that one plaquette of the link,
    so M there holds the (x, y) term alone."""
    D = make(1.1)
    nu = 1
    kappa, csw = 0.09, 1.3
    U = _links_with(DIMS, nu, M_SITE, D)
    got = dirac.local_matrix(U, kappa, csw)
    f = (D - D.conj().T) / 8j
    # i sigma_{x y} for the ordered plane (rho, nu) = (x, y)
    for corner, sign in ((_shifted(M_SITE, 0, -1, DIMS), +1), (_shifted(_shifted(M_SITE, 1, 1, DIMS), 0, -1, DIMS), +1),
                         (_shifted(M_SITE, 0, +1, DIMS), -1), (_shifted(_shifted(M_SITE, 1, 1, DIMS), 0, +1, DIMS), -1)):
        x, y, z, t = corner
        want = np.eye(12) - kappa * csw * sign * np.kron(I_SIGMA_XY, f)
        assert np.abs(got[t, z, y, x] - want).max() < 1e-15
    # the base and the tip of the link: every plane cancels
    for c in (M_SITE, _shifted(M_SITE, 1, 1, DIMS)):
        x, y, z, t = c
        assert np.abs(got[t, z, y, x] - np.eye(12)).max() < 1e-15


def test_hand_sigma_matches_oracle_tables():
    """The hand-multiplied i sigma matrices agree with the oracle's sigma
    (a consistency check of the two independent write-ups)."""
    for rho, m in I_SIGMA_T.items():
        assert np.array_equal(1j * SIGMA[rho, 3], m)
    assert np.array_equal(1j * SIGMA[0, 1], I_SIGMA_XY)


# ------------------------------------------------------------ planted mistakes

def _with_field_strength(monkeypatch, transform):
    orig = dirac.field_strength
    monkeypatch.setattr(dirac, "field_strength", lambda U: transform(orig(U)))


@pytest.mark.parametrize("mistake", ["negated", "doubled", "halved", "transposed"])
def test_pin_catches_field_strength_mistakes(monkeypatch, mistake):
    """F -> -F (the sign of the whole term), 2F or F/2 (its scale, e.g. a
    sum over mu < nu only), and F^T (a transposed colour index) each break
    the closed form."""
    transform = {
        "negated": lambda F: -F,
        "doubled": lambda F: 2.0 * F,
        "halved": lambda F: 0.5 * F,
        "transposed": lambda F: np.swapaxes(F, -1, -2),
    }[mistake]
    _with_field_strength(monkeypatch, transform)
    D = _rotation_link(0.7)
    U = _links_with(DIMS, 3, M_SITE, D)
    assert _check(U, DIMS, 3, D, 0.11, 1.7, I_SIGMA_T) > 1e-3


def test_pin_catches_minus_i_over_two(monkeypatch):
    """(i/2) sigma replaced by (-i/2) sigma (equivalently sigma_{nu mu} in
    place of sigma_{mu nu})."""
    monkeypatch.setattr(dirac, "SIGMA", -SIGMA)
    D = _diag_link(0.7)
    U = _links_with(DIMS, 3, M_SITE, D)
    assert _check(U, DIMS, 3, D, 0.11, 1.7, I_SIGMA_T) > 1e-3


@pytest.mark.parametrize("which", [0, 1, 2, 3])
def test_pin_catches_a_reversed_leaf(monkeypatch, which):
    """One of the four leaves walked the wrong way round (P_i^dagger in
    place of P_i) changes F at the corners where that leaf holds the link."""
    orig = dirac.leaves

    def bad(U, mu, nu):
        p = list(orig(U, mu, nu))
        p[which] = dirac.dag(p[which])
        return tuple(p)

    monkeypatch.setattr(dirac, "leaves", bad)
    D = _rotation_link(0.7)
    U = _links_with(DIMS, 3, M_SITE, D)
    assert _check(U, DIMS, 3, D, 0.11, 1.7, I_SIGMA_T) > 1e-3
