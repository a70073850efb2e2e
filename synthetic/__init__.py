"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws random numbers and lays them out; it holds none of the
solver's or the operator's arithmetic.  Both the CPU oracle and the HIP path
take their inputs from here, and from nowhere else.

Conventions (they match the paper's notation, Sec. 2):

* lattice dims are given as ``(Lx, Ly, Lz, Lt)``; the flat site index is
  ``site = x + Lx*(y + Ly*(z + Lz*t))`` (x fastest), site 0 is the origin;
* gauge links: complex128 array of shape ``(4, Lt, Lz, Ly, Lx, 3, 3)``,
  direction mu = 0..3 <-> x, y, z, t, i.e. ``U[mu, t, z, y, x, a, b]`` is
  ``U_mu(n, a, b)``;
* spinor blocks: complex array of shape ``(Lt, Lz, Ly, Lx, 4, 3, L)``, i.e.
  ``[site][spin][colour][rhs]`` with the right-hand-side index innermost.
  Row ``12*site + 3*spin + colour`` of the N x L matrix of Sec. 3 is
  ``X.reshape(N, L)``.

The link recipe (not from the paper, whose quenched ensemble is not
available) is U = exp(i*eps*H) with H a traceless Hermitian 3x3 matrix whose
independent real components are standard normal, followed by
re-unitarisation.  Draws are made direction-major, then site-lexicographic,
then in the order (H00, H11, H22, Re H01, Im H01, Re H02, Im H02, Re H12,
Im H12).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "volume", "field_shape", "gauge_links", "unit_links", "random_su3",
    "point_sources", "z2_sources", "gaussian_sources", "random_spinor",
]


def volume(dims) -> int:
    lx, ly, lz, lt = (int(d) for d in dims)
    return lx * ly * lz * lt


def field_shape(dims, L: int):
    lx, ly, lz, lt = (int(d) for d in dims)
    return (lt, lz, ly, lx, 4, 3, int(L))


def _reunitarise(m: np.ndarray) -> np.ndarray:
    """Gram-Schmidt on rows 0 and 1, row 2 = conj(row0 x row1) (det = 1)."""
    r0 = m[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = m[..., 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


def _hermitian_traceless(z: np.ndarray) -> np.ndarray:
    """z[..., 9] standard normals -> traceless Hermitian 3x3 (see module doc)."""
    h = np.zeros(z.shape[:-1] + (3, 3), dtype=np.complex128)
    h[..., 0, 0] = z[..., 0]
    h[..., 1, 1] = z[..., 1]
    h[..., 2, 2] = z[..., 2]
    h[..., 0, 1] = z[..., 3] + 1j * z[..., 4]
    h[..., 0, 2] = z[..., 5] + 1j * z[..., 6]
    h[..., 1, 2] = z[..., 7] + 1j * z[..., 8]
    h[..., 1, 0] = np.conj(h[..., 0, 1])
    h[..., 2, 0] = np.conj(h[..., 0, 2])
    h[..., 2, 1] = np.conj(h[..., 1, 2])
    tr = (h[..., 0, 0] + h[..., 1, 1] + h[..., 2, 2]) / 3.0
    for a in range(3):
        h[..., a, a] -= tr
    return h


def gauge_links(dims, eps: float, seed: int) -> np.ndarray:
    """Quenched-like SU(3) links U = exp(i eps H), seeded (see module doc)."""
    lx, ly, lz, lt = (int(d) for d in dims)
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((4, lt, lz, ly, lx, 9))
    h = _hermitian_traceless(z)
    w, v = np.linalg.eigh(h)
    u = np.einsum("...ak,...k,...bk->...ab", v, np.exp(1j * eps * w), np.conj(v))
    return np.ascontiguousarray(_reunitarise(u))


def unit_links(dims) -> np.ndarray:
    lx, ly, lz, lt = (int(d) for d in dims)
    u = np.zeros((4, lt, lz, ly, lx, 3, 3), dtype=np.complex128)
    for a in range(3):
        u[..., a, a] = 1.0
    return u


def random_su3(shape, seed: int) -> np.ndarray:
    """Random SU(3) matrices (QR of a complex Gaussian, phase-fixed, det 1)."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(tuple(shape) + (3, 3)) + 1j * rng.standard_normal(tuple(shape) + (3, 3))
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    q = q * (d / np.abs(d))[..., None, :]
    # rows 0, 1 of a unitary matrix; row 2 rebuilt so that det = 1
    return _reunitarise(q)


def point_sources(dims, site: int = 0, dtype=np.complex128) -> np.ndarray:
    """The 12 point sources of Sec. 2: column i = colour + 3*spin is the unit
    vector at ``site`` (0 = origin) with that spin and colour."""
    shape = field_shape(dims, 12)
    b = np.zeros(shape, dtype=dtype)
    flat = b.reshape(volume(dims), 4, 3, 12)
    for s in range(4):
        for c in range(3):
            flat[site, s, c, c + 3 * s] = 1.0
    return b


def z2_sources(dims, L: int, seed: int, dtype=np.complex128) -> np.ndarray:
    """Z2 noise: every complex entry is +1 or -1 (imaginary part 0)."""
    rng = np.random.default_rng(seed)
    bits = rng.integers(0, 2, size=field_shape(dims, L))
    return (1.0 - 2.0 * bits).astype(dtype)


def gaussian_sources(dims, L: int, seed: int, dtype=np.complex128) -> np.ndarray:
    """Complex Gaussian noise: real and imaginary parts standard normal."""
    rng = np.random.default_rng(seed)
    shape = field_shape(dims, L)
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(dtype)


def random_spinor(dims, L: int, seed: int, dtype=np.complex128) -> np.ndarray:
    return gaussian_sources(dims, L, seed, dtype)
