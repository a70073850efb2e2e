"""Critical hopping parameter of a lattice (context for every solve).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Eq. (1) reads D_W = 1 - kappa K with K independent of kappa (the hopping term
plus c_SW sum (i/2) sigma F).  D_W first becomes singular at
kappa_c = 1 / max Re lambda(K) for the eigenvalue with the largest real part;
the bare quark mass of Sec. 4.1 is (1/kappa - 1/kappa_c) / 2.
"""
import numpy as np
from scipy.sparse.linalg import LinearOperator, eigs

from . import dirac


def kappa_critical(U: np.ndarray, csw: float, k: int = 4, tol: float = 1e-8) -> float:
    dims = U.shape[1:5]
    N = 12 * int(np.prod(dims))
    probe_kappa = 1.0
    local = dirac.local_matrix(U, probe_kappa, csw)

    def matvec(x):
        X = x.reshape(dims + (4, 3, 1))
        DX = dirac.apply(U, probe_kappa, csw, X, local=local)
        return ((X - DX) / probe_kappa).reshape(-1)

    op = LinearOperator((N, N), matvec=matvec, dtype=np.complex128)
    vals = eigs(op, k=k, which="LR", tol=tol, return_eigenvectors=False)
    return float(1.0 / np.max(vals.real))
