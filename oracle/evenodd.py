"""Even-odd (Schur-complement) form of the solve D_W X = B, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

This follows from the structure of Eq. (1) (Sec. 2); the paper does not use
it.  Call a site even when x + y + z + t is even.  With every extent even,
each hop of Eq. (1) joins an even site to an odd one, and the site-local term
M = 1 - kappa c_SW sum (i/2) sigma F acts site by site.  With the rows
ordered by parity, and H the hopping sum (D_W = M - kappa H):

    D_W = [[ M_ee,         -kappa H_eo ],
           [ -kappa H_oe,   M_oo       ]].

Eliminating the odd sites leaves the Schur complement on the even sites,

    S = M_ee - kappa^2 H_eo M_oo^{-1} H_oe,
    S x_e = b_e + kappa H_eo M_oo^{-1} b_o,
    x_o = M_oo^{-1} (b_o + kappa H_oe x_e).

The adjoint system D_W^dagger has the same form with H^dagger in place of H
(M is Hermitian).  Even-site blocks are held compactly, (V/2, 4, 3, L) with
the even sites in increasing site order; with Lx even that position is
site // 2.
"""
import numpy as np

from . import dirac, solvers


def check_dims(dims):
    if any(int(d) % 2 for d in dims):
        raise ValueError("the even-odd split needs every lattice extent even")


def parity(dims) -> np.ndarray:
    """0 for even, 1 for odd sites, flat site order (x fastest)."""
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(range(lt), range(lz), range(ly), range(lx), indexing="ij")
    return ((x + y + z + t) % 2).reshape(-1)


def hopping(U: np.ndarray, X: np.ndarray, dagger: bool = False) -> np.ndarray:
    """H X (or H^dagger X): Eq. (1) with the site-local term taken out and
    kappa = 1, i.e. D_W = M - kappa H."""
    V12 = np.zeros(X.shape[:4] + (12, 12), dtype=np.complex128)
    return -dirac.apply(U, 1.0, 0.0, X, dagger=dagger, local=V12)


def _embed(dims, compact: np.ndarray, par: int) -> np.ndarray:
    """Compact block of the sites of parity `par` -> whole-lattice field (zeros elsewhere)."""
    V = int(np.prod(dims))
    L = compact.shape[-1]
    full = np.zeros((V, 4, 3, L), dtype=np.complex128)
    full[parity(dims) == par] = compact
    lx, ly, lz, lt = dims
    return full.reshape(lt, lz, ly, lx, 4, 3, L)


def _restrict(field: np.ndarray, par: int, dims) -> np.ndarray:
    """Sites of parity `par` of a whole-lattice field, as a compact block."""
    V = int(np.prod(dims))
    return field.reshape(V, 4, 3, -1)[parity(dims) == par]


def local_inverse(U: np.ndarray, kappa: float, csw: float) -> np.ndarray:
    """M(n)^{-1} for every site, (V, 12, 12)."""
    M = dirac.local_matrix(U, kappa, csw)
    V = M.shape[0] * M.shape[1] * M.shape[2] * M.shape[3]
    return np.linalg.inv(M.reshape(V, 12, 12))


def _local(Mflat: np.ndarray, compact: np.ndarray, par: int, dims) -> np.ndarray:
    """Site-local 12 x 12 matrices of the sites of parity `par` times a compact block."""
    Mp = Mflat[parity(dims) == par]
    n, L = compact.shape[0], compact.shape[-1]
    return np.einsum("sij,sjl->sil", Mp, compact.reshape(n, 12, L)).reshape(n, 4, 3, L)


def schur_apply(U, kappa, csw, xe: np.ndarray, dagger: bool = False, Minv=None) -> np.ndarray:
    """S x_e = M_ee x_e - kappa^2 H_eo M_oo^{-1} H_oe x_e on a compact even block."""
    dims = dirac.dims_of(U)
    check_dims(dims)
    V = int(np.prod(dims))
    M = dirac.local_matrix(U, kappa, csw).reshape(V, 12, 12)
    Minv = np.linalg.inv(M) if Minv is None else Minv
    t_o = _restrict(hopping(U, _embed(dims, xe, 0), dagger), 1, dims)  # H_oe x_e
    u_o = _local(Minv, t_o, 1, dims)                                 # M_oo^{-1} H_oe x_e
    w_e = _restrict(hopping(U, _embed(dims, u_o, 1), dagger), 0, dims)  # H_eo M_oo^{-1} H_oe x_e
    return _local(M, xe, 0, dims) - kappa ** 2 * w_e


def prepare(U, kappa, csw, B: np.ndarray, dagger: bool = False) -> np.ndarray:
    """b_e + kappa H_eo M_oo^{-1} b_o (compact even block)."""
    dims = dirac.dims_of(U)
    check_dims(dims)
    Minv = local_inverse(U, kappa, csw)
    u_o = _local(Minv, _restrict(B, 1, dims), 1, dims)
    return _restrict(B, 0, dims) + kappa * _restrict(hopping(U, _embed(dims, u_o, 1), dagger), 0, dims)


def reconstruct(U, kappa, csw, B: np.ndarray, xe: np.ndarray, dagger: bool = False) -> np.ndarray:
    """The whole solution: x_e, and x_o = M_oo^{-1} (b_o + kappa H_oe x_e)."""
    dims = dirac.dims_of(U)
    Minv = local_inverse(U, kappa, csw)
    rhs_o = _restrict(B, 1, dims) + kappa * _restrict(hopping(U, _embed(dims, xe, 0), dagger), 1, dims)
    x_o = _local(Minv, rhs_o, 1, dims)
    return _embed(dims, xe, 0) + _embed(dims, x_o, 1)


def solve(U, kappa, csw, B: np.ndarray, tol: float, max_iter: int, dagger: bool = False):
    """D_W X = B through the Schur complement, solved by the oracle's Block
    BiCGGR on the even sites.  Returns (X, info of the even-site solve)."""
    dims = dirac.dims_of(U)
    V = int(np.prod(dims))
    L = B.shape[-1]
    Minv = local_inverse(U, kappa, csw)
    be = prepare(U, kappa, csw, B, dagger)
    n = 12 * (V // 2)

    def A(X2):
        return schur_apply(U, kappa, csw, X2.reshape(V // 2, 4, 3, -1), dagger, Minv).reshape(n, -1)

    xe, info = solvers.block_bicggr(A, be.reshape(n, L), tol, max_iter)
    return reconstruct(U, kappa, csw, B, xe.reshape(V // 2, 4, 3, L), dagger), info
