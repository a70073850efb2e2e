"""Gradients of a solve X = D_W^{-1} B with respect to B, kappa, c_SW and the
links U, through the adjoint solve (growth of the method of Sec. 3 to
automatic differentiation; derived from Eq. (1) of Sec. 2).  FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Convention (that of complex autograd): for a real loss l of complex data z,
the gradient is g = dl/dRe z + i dl/dIm z, so that dl = Re sum conj(g) dz.

With X = D^{-1} B and G the gradient of l with respect to X:

    dl = Re <G, D^{-1}(dB - dD X)> = Re <Lam, dB> - Re <Lam, dD X>,
    Lam = D^{-H} G  (the adjoint solve; D^H = gamma_5 D gamma_5),

where <a, b> = sum conj(a) b over sites, spins, colours and columns.  Hence

* grad_B = Lam;
* D = M - kappa H with M = 1 - kappa c_SW C, C = sum_{mu,nu} (i/2) sigma_{mu nu}
  F_{mu nu} (all ordered pairs) and H the hopping sum of Eq. (1), so
  dD/dkappa = -(c_SW C + H) and dD/dc_SW = -kappa C:
  grad_kappa = Re <Lam, (c_SW C + H) X>,  grad_csw = kappa Re <Lam, C X>;
* grad_U = the gradient of f(U) = -Re <Lam, D(U) X> at fixed Lam and X.

The link gradient has a hopping part and a clover part.

Hopping part, for link U_mu(n) (P-+ = 1 -+ gamma_mu):
    g += kappa (conj(A) + B^T),
    A_ab = sum_{i, alpha} conj(Lam_{alpha a i}(n)) (P- X(n + mu))_{alpha b i},
    B_ab = sum_{i, alpha} conj(Lam_{alpha a i}(n + mu)) (P+ X(n))_{alpha b i}.

Clover part: F_{mu nu} = (Q - Q^dagger) / (8 i) with Q the sum of the four
leaves at n.  The pairs (mu, nu) and (nu, mu) contribute equally, so
    -Re <Lam, dM X> = Re sum_n sum_{mu<nu} sum_ab dQ^{mu nu}_ab(n) W^{mu nu}_ab(n),
    W = kappa c_SW / (4 i) (K + K^H),
    K_ab = sum_{i, alpha, beta} conj(Lam_{alpha a i}) ((i/2) sigma_{mu nu})_{alpha beta} X_{beta b i}.
For a leaf F1 F2 F3 F4 (site arrays) the derivative through its k-th factor
is sum_xy dF_k,xy M_yx with M = (F_{k+1} .. F4) W^T (F1 .. F_{k-1}); the
link of that factor receives M^H if the factor is a link and M if it is a
daggered link.
"""
import numpy as np

from .dirac import dag, field_strength, shift
from .gamma import GAMMA, IDENTITY4, SIGMA


def _spin(g, x):
    return np.einsum("rs,...sal->...ral", g, x)


def _colour(m, x):
    return np.einsum("...ab,...sbl->...sal", m, x)


def inner(a: np.ndarray, b: np.ndarray) -> complex:
    """<a, b> = sum conj(a) b."""
    return complex(np.vdot(a, b))


def hopping(U: np.ndarray, X: np.ndarray) -> np.ndarray:
    """H X = sum_mu [ (1 - gamma_mu) U_mu(n) X(n + mu) + (1 + gamma_mu) U_mu^dagger(n - mu) X(n - mu) ],
    so that D_W = M - kappa H (Eq. (1))."""
    Y = np.zeros_like(X)
    for mu in range(4):
        fwd = _colour(U[mu], shift(X, mu, +1))
        bwd = _colour(dag(shift(U[mu], mu, -1)), shift(X, mu, -1))
        Y = Y + _spin(IDENTITY4 - GAMMA[mu], fwd) + _spin(IDENTITY4 + GAMMA[mu], bwd)
    return Y


def clover_apply(U: np.ndarray, X: np.ndarray) -> np.ndarray:
    """C X with C = sum_{mu, nu} (i/2) sigma_{mu nu} F_{mu nu} (all ordered pairs)."""
    F = field_strength(U)
    Y = np.zeros_like(X)
    for mu in range(4):
        for nu in range(4):
            Y = Y + 0.5j * _spin(SIGMA[mu, nu], _colour(F[mu, nu], X))
    return Y


def grad_kappa(U, kappa, csw, X, Lam) -> float:
    """Re <Lam, (c_SW C + H) X> = -Re <Lam, (dD/dkappa) X>."""
    return float(np.real(inner(Lam, csw * clover_apply(U, X) + hopping(U, X))))


def grad_csw(U, kappa, csw, X, Lam) -> float:
    """kappa Re <Lam, C X> = -Re <Lam, (dD/dc_SW) X>."""
    return float(kappa * np.real(inner(Lam, clover_apply(U, X))))


def leaf_factors(mu: int, nu: int):
    """The four leaves of ``dirac.leaves`` as lists of factors
    (direction, {direction: step}, daggered): factor = U_dir(n + steps),
    conjugate-transposed if daggered."""
    return [
        [(mu, {}, False), (nu, {mu: 1}, False), (mu, {nu: 1}, True), (nu, {}, True)],
        [(nu, {}, False), (mu, {mu: -1, nu: 1}, True), (nu, {mu: -1}, True), (mu, {mu: -1}, False)],
        [(mu, {mu: -1}, True), (nu, {mu: -1, nu: -1}, True), (mu, {mu: -1, nu: -1}, False), (nu, {nu: -1}, False)],
        [(nu, {nu: -1}, True), (mu, {nu: -1}, False), (nu, {mu: 1, nu: -1}, False), (mu, {}, True)],
    ]


def factor_value(U, spec):
    d, steps, daggered = spec
    v = U[d]
    for e, s in steps.items():
        v = shift(v, e, s)
    return dag(v) if daggered else v


def _shift_back(f, steps):
    """h(m) = f(m - steps): moves a quantity computed at n to the link's site n + steps."""
    for e, s in steps.items():
        f = shift(f, e, -s)
    return f


def grad_links(U, kappa, csw, X, Lam) -> np.ndarray:
    """Gradient of f(U) = -Re <Lam, D_W(U) X> with respect to the links, in the
    convention of the module docstring.  Shape (4, Lt, Lz, Ly, Lx, 3, 3)."""
    g = np.zeros_like(U)
    eye3 = np.broadcast_to(np.eye(3, dtype=np.complex128), U.shape[1:])
    # hopping part
    for mu in range(4):
        Xf = shift(X, mu, +1)
        A = np.einsum("...sal,...sbl->...ab", np.conj(Lam), _spin(IDENTITY4 - GAMMA[mu], Xf))
        B = np.einsum("...sal,...sbl->...ab", np.conj(shift(Lam, mu, +1)), _spin(IDENTITY4 + GAMMA[mu], X))
        g[mu] += kappa * (np.conj(A) + np.swapaxes(B, -1, -2))
    if csw == 0.0:
        return g
    # clover part
    for mu in range(4):
        for nu in range(mu + 1, 4):
            K = np.einsum("...sal,st,...tbl->...ab", np.conj(Lam), 0.5j * SIGMA[mu, nu], X)
            W = kappa * csw / 4j * (K + dag(K))
            Wt = np.swapaxes(W, -1, -2)
            for leaf in leaf_factors(mu, nu):
                vals = [factor_value(U, f) for f in leaf]
                for k, spec in enumerate(leaf):
                    post = eye3
                    for v in vals[k + 1:]:
                        post = post @ v
                    pre = eye3
                    for v in vals[:k]:
                        pre = pre @ v
                    M = post @ Wt @ pre
                    contrib = M if spec[2] else dag(M)
                    g[spec[0]] += _shift_back(contrib, spec[1])
    return g


def link_force_check_value(U, kappa, csw, X, Lam) -> float:
    """f(U) = -Re <Lam, D_W(U) X> (the function ``grad_links`` differentiates)."""
    from .dirac import apply
    return float(-np.real(inner(Lam, apply(U, kappa, csw, X))))


__all__ = ["inner", "hopping", "clover_apply", "grad_kappa", "grad_csw", "leaf_factors", "factor_value",
           "grad_links", "link_force_check_value"]
