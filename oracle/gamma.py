"""Euclidean gamma matrices of Sec. 2 (defined from Bjorken-Drell ones).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The four gamma_mu and gamma_5 are the matrices printed in Sec. 2 (only their
non-zero entries are printed there).  Indices here are 0-based: row/column
``alpha - 1``.  ``GAMMA[0..3]`` are gamma_1..gamma_4 (x, y, z, t),
``GAMMA5`` is gamma_5.  sigma_{mu nu} is half the commutator, as defined in
Sec. 2.
"""
import numpy as np

_i = 1j

GAMMA = np.zeros((4, 4, 4), dtype=np.complex128)
# gamma_1: entries (1,4) = -i, (2,3) = -i, (3,2) = i, (4,1) = i
GAMMA[0][0, 3] = -_i
GAMMA[0][1, 2] = -_i
GAMMA[0][2, 1] = _i
GAMMA[0][3, 0] = _i
# gamma_2: (1,4) = -1, (2,3) = 1, (3,2) = 1, (4,1) = -1
GAMMA[1][0, 3] = -1
GAMMA[1][1, 2] = 1
GAMMA[1][2, 1] = 1
GAMMA[1][3, 0] = -1
# gamma_3: (1,3) = -i, (2,4) = i, (3,1) = i, (4,2) = -i
GAMMA[2][0, 2] = -_i
GAMMA[2][1, 3] = _i
GAMMA[2][2, 0] = _i
GAMMA[2][3, 1] = -_i
# gamma_4 = diag(1, 1, -1, -1)
GAMMA[3] = np.diag([1, 1, -1, -1]).astype(np.complex128)

# gamma_5: (1,3) = (2,4) = (3,1) = (4,2) = 1
GAMMA5 = np.zeros((4, 4), dtype=np.complex128)
GAMMA5[0, 2] = 1
GAMMA5[1, 3] = 1
GAMMA5[2, 0] = 1
GAMMA5[3, 1] = 1

IDENTITY4 = np.eye(4, dtype=np.complex128)


def sigma(mu: int, nu: int) -> np.ndarray:
    """sigma_{mu nu} = (gamma_mu gamma_nu - gamma_nu gamma_mu) / 2 (Sec. 2)."""
    return 0.5 * (GAMMA[mu] @ GAMMA[nu] - GAMMA[nu] @ GAMMA[mu])


SIGMA = np.array([[sigma(m, n) for n in range(4)] for m in range(4)])
