"""The O(a)-improved Wilson-Dirac operator D_W of Sec. 2, Eq. (1), in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Array conventions (shared with ``synthetic``):

* links ``U``: shape (4, Lt, Lz, Ly, Lx, 3, 3); ``U[mu][t, z, y, x]`` is the
  3x3 matrix U_mu(n) of Sec. 2, mu = 0..3 for x, y, z, t;
* fields ``X``: shape (Lt, Lz, Ly, Lx, 4, 3, L): quark-field index (alpha, a)
  of Sec. 2 for each of the L right-hand sides of Sec. 3.

Boundary conditions are periodic in all four directions for every field
(Sec. 2), so a shift by one site is ``np.roll``.

Readings of the paper used here:

* clover leaves: the printed P_1 and P_4 do not close into loops.  P_1 is read
  with third factor U_mu^dagger(n + nu) and P_4 with second factor U_mu(n - nu)
  (the standard plaquettes; gauge covariance fails otherwise);
* F_{mu nu} is used as printed, without removing its trace;
* the clover sum runs over all ordered pairs (mu, nu) = 1..4 as printed; the
  terms mu = nu vanish because sigma_{mu mu} = 0 and F_{mu mu} = 0.
"""
import numpy as np

from .gamma import GAMMA, GAMMA5, IDENTITY4, SIGMA

# direction mu -> axis of a (Lt, Lz, Ly, Lx, ...) array
AXIS = (3, 2, 1, 0)


def dims_of(field_or_links) -> tuple:
    """(Lx, Ly, Lz, Lt) of a field (Lt,Lz,Ly,Lx,...) or links (4,Lt,Lz,Ly,Lx,...)."""
    s = field_or_links.shape
    if field_or_links.ndim == 7 and s[0] == 4 and s[-2:] == (3, 3):
        s = s[1:]
    return (s[3], s[2], s[1], s[0])


def shift(f: np.ndarray, mu: int, step: int) -> np.ndarray:
    """g(n) = f(n + step * mu_hat) with periodic wrap."""
    return np.roll(f, -step, axis=AXIS[mu])


def dag(m: np.ndarray) -> np.ndarray:
    return np.conj(np.swapaxes(m, -1, -2))


# ---------------------------------------------------------------- clover term

def leaves(U: np.ndarray, mu: int, nu: int):
    """The four clover leaves P_1..P_4 around site n in the (mu, nu) plane
    (Sec. 2, definition of F_{mu nu}), with the two loop closures read as in
    the module docstring.  Each has shape (Lt, Lz, Ly, Lx, 3, 3)."""
    Umu, Unu = U[mu], U[nu]

    def at(link, *steps):
        # link evaluated at n + sum(step * direction)
        out = link
        for d, s in steps:
            out = shift(out, d, s)
        return out

    p1 = Umu @ at(Unu, (mu, +1)) @ dag(at(Umu, (nu, +1))) @ dag(Unu)
    p2 = Unu @ dag(at(Umu, (mu, -1), (nu, +1))) @ dag(at(Unu, (mu, -1))) @ at(Umu, (mu, -1))
    p3 = (dag(at(Umu, (mu, -1))) @ dag(at(Unu, (mu, -1), (nu, -1)))
          @ at(Umu, (mu, -1), (nu, -1)) @ at(Unu, (nu, -1)))
    p4 = dag(at(Unu, (nu, -1))) @ at(Umu, (nu, -1)) @ at(Unu, (mu, +1), (nu, -1)) @ dag(Umu)
    return p1, p2, p3, p4


def field_strength(U: np.ndarray) -> np.ndarray:
    """F_{mu nu}(n) = 1/4 sum_i (P_i - P_i^dagger) / (2i) for all 16 ordered
    (mu, nu); shape (4, 4, Lt, Lz, Ly, Lx, 3, 3)."""
    dims = U.shape[1:5]
    F = np.zeros((4, 4) + dims + (3, 3), dtype=np.complex128)
    for mu in range(4):
        for nu in range(4):
            acc = np.zeros(dims + (3, 3), dtype=np.complex128)
            for p in leaves(U, mu, nu):
                acc += (p - dag(p)) / 2j
            F[mu, nu] = acc / 4.0
    return F


def local_matrix(U: np.ndarray, kappa: float, csw: float) -> np.ndarray:
    """Site-local part of Eq. (1): the identity plus the clover term
    -kappa csw sum_{mu,nu} (i/2) sigma_{mu nu} F_{mu nu}, as a 12x12 matrix per
    site with row index 3*alpha + a.  Shape (Lt, Lz, Ly, Lx, 12, 12)."""
    F = field_strength(U)
    dims = U.shape[1:5]
    C = np.zeros(dims + (12, 12), dtype=np.complex128)
    for mu in range(4):
        for nu in range(4):
            # kron(sigma (4x4 spin), F (3x3 colour)) -> index 3*spin + colour
            term = np.einsum("st,...ab->...satb", SIGMA[mu, nu], F[mu, nu]).reshape(dims + (12, 12))
            C += 0.5j * term
    return np.eye(12, dtype=np.complex128) - kappa * csw * C


# ---------------------------------------------------------------- the operator

def _colour(m: np.ndarray, x: np.ndarray) -> np.ndarray:
    """(m x)(n, alpha, a, l) = sum_b m(n, a, b) x(n, alpha, b, l)."""
    return np.einsum("...ab,...sbl->...sal", m, x)


def _spin(g: np.ndarray, x: np.ndarray) -> np.ndarray:
    """(g x)(n, alpha, a, l) = sum_beta g(alpha, beta) x(n, beta, a, l)."""
    return np.einsum("rs,...sal->...ral", g, x)


def apply_local(M: np.ndarray, X: np.ndarray) -> np.ndarray:
    shp = X.shape
    out = np.einsum("...ij,...jl->...il", M, X.reshape(shp[:4] + (12, shp[-1])))
    return out.reshape(shp)


def apply(U: np.ndarray, kappa: float, csw: float, X: np.ndarray, dagger: bool = False,
          local: np.ndarray = None) -> np.ndarray:
    """Y = D_W X (Eq. (1)) for every column of X; ``dagger`` gives D_W^dagger.

    D_W X(n) = M(n) X(n) - kappa sum_mu [ (1 - gamma_mu) U_mu(n) X(n + mu)
                                         + (1 + gamma_mu) U_mu^dagger(n - mu) X(n - mu) ]
    with M(n) the site-local matrix.  The adjoint (conjugate transpose of the
    N x N matrix) swaps the signs of gamma_mu in the two projectors; M is
    Hermitian.  ``local`` may pass a precomputed ``local_matrix``.
    """
    if local is None:
        local = local_matrix(U, kappa, csw)
    if dagger:
        local = dag(local)
    sgn = -1.0 if dagger else 1.0
    Y = apply_local(local, X)
    for mu in range(4):
        fwd = _colour(U[mu], shift(X, mu, +1))
        bwd = _colour(dag(shift(U[mu], mu, -1)), shift(X, mu, -1))
        Y = Y - kappa * (_spin(IDENTITY4 - sgn * GAMMA[mu], fwd) + _spin(IDENTITY4 + sgn * GAMMA[mu], bwd))
    return Y


def gamma5(X: np.ndarray) -> np.ndarray:
    return _spin(GAMMA5, X)


def assemble_dense(U: np.ndarray, kappa: float, csw: float) -> np.ndarray:
    """The N x N matrix D_W (N = 12 V), column j = D_W e_j, row 12*site + 3*alpha + a."""
    dims = U.shape[1:5]
    V = int(np.prod(dims))
    N = 12 * V
    E = np.eye(N, dtype=np.complex128).reshape(dims + (4, 3, N))
    return apply(U, kappa, csw, E).reshape(N, N)


def as_matrix_operator(U: np.ndarray, kappa: float, csw: float, dagger: bool = False):
    """A callable mapping an (N, L) array to D_W times it (the A of Sec. 3)."""
    dims = U.shape[1:5]
    local = local_matrix(U, kappa, csw)

    def A(X2: np.ndarray) -> np.ndarray:
        L = X2.shape[1]
        return apply(U, kappa, csw, X2.reshape(dims + (4, 3, L)), dagger=dagger, local=local).reshape(X2.shape)

    return A


# ---------------------------------------------------------------- sampled sites

def _site_coords(dims, site):
    lx, ly, lz, lt = dims
    x = site % lx
    y = (site // lx) % ly
    z = (site // (lx * ly)) % lz
    t = site // (lx * ly * lz)
    return [x, y, z, t]


def _site_index(dims, c):
    lx, ly, lz, lt = dims
    return (c[0] % lx) + lx * ((c[1] % ly) + ly * ((c[2] % lz) + lz * (c[3] % lt)))


def apply_at_sites(U: np.ndarray, kappa: float, csw: float, X: np.ndarray, sites) -> np.ndarray:
    """(D_W X)(n) of Eq. (1) at the listed flat site indices only, by explicit
    neighbour indexing (no whole-lattice shifts), for lattices too large for
    ``apply``.  X has shape (V, 4, 3, L) or (Lt, Lz, Ly, Lx, 4, 3, L); U is
    (4, Lt, Lz, Ly, Lx, 3, 3).  Returns shape (len(sites), 4, 3, L)."""
    dims = dims_of(U)
    V = int(np.prod(dims))
    Uf = U.reshape(4, V, 3, 3)
    Xf = X.reshape(V, 4, 3, -1)
    out = []
    for n in sites:
        c = _site_coords(dims, int(n))

        def link(mu, *steps):
            cc = list(c)
            for d, s in steps:
                cc[d] += s
            return Uf[mu, _site_index(dims, cc)]

        def nbr(mu, s):
            cc = list(c)
            cc[mu] += s
            return Xf[_site_index(dims, cc)]

        # F_{mu nu}(n) from the four leaves (same readings as ``leaves``)
        C = np.zeros((12, 12), dtype=np.complex128)
        for mu in range(4):
            for nu in range(4):
                Um, Un = (lambda *st: link(mu, *st)), (lambda *st: link(nu, *st))
                p1 = Um() @ Un((mu, 1)) @ dag(Um((nu, 1))) @ dag(Un())
                p2 = Un() @ dag(Um((mu, -1), (nu, 1))) @ dag(Un((mu, -1))) @ Um((mu, -1))
                p3 = dag(Um((mu, -1))) @ dag(Un((mu, -1), (nu, -1))) @ Um((mu, -1), (nu, -1)) @ Un((nu, -1))
                p4 = dag(Un((nu, -1))) @ Um((nu, -1)) @ Un((mu, 1), (nu, -1)) @ dag(Um())
                F = sum((p - dag(p)) / 2j for p in (p1, p2, p3, p4)) / 4.0
                C += 0.5j * np.kron(SIGMA[mu, nu], F)
        M = np.eye(12) - kappa * csw * C
        y = (M @ Xf[int(n)].reshape(12, -1)).reshape(4, 3, -1)
        for mu in range(4):
            fwd = np.einsum("ab,sbl->sal", link(mu), nbr(mu, +1))
            bwd = np.einsum("ab,sbl->sal", dag(link(mu, (mu, -1))), nbr(mu, -1))
            y = y - kappa * (np.einsum("rs,sal->ral", IDENTITY4 - GAMMA[mu], fwd)
                             + np.einsum("rs,sal->ral", IDENTITY4 + GAMMA[mu], bwd))
        out.append(y)
    return np.array(out)
