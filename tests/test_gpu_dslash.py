"""Parity of the HIP operator (bkwd_apply) with the FP64 oracle, element by
element, on seeded inputs."""
import numpy as np
import pytest

import synthetic as S
from oracle import dirac
from tests.gpu_util import lattice, rel_err, to_dev, to_np

pytestmark = pytest.mark.gpu

CASES = [
    ((4, 4, 4, 4), 12),
    ((2, 2, 2, 2), 3),       # extent 2: forward and backward neighbour coincide
    ((3, 4, 5, 6), 1),       # odd extents, one column
    ((4, 3, 2, 5), 16),
    ((4, 4, 2, 2), 64),      # L at its maximum
    ((8, 6, 4, 6), 7),       # L not dividing the 256-thread workgroup
]


@pytest.mark.parametrize("dims,L", CASES)
@pytest.mark.parametrize("dagger", [False, True])
def test_apply_fp64(dims, L, dagger):
    import torch
    U = S.gauge_links(dims, 0.4, 100 + L)
    X = S.random_spinor(dims, L, 200 + L)
    kappa, csw = 0.13, 1.6
    lat = lattice(U, kappa, csw)
    Y = to_np(lat.apply(to_dev(X), dagger=dagger))
    torch.cuda.synchronize()
    ref = dirac.apply(U, kappa, csw, X, dagger=dagger)
    assert rel_err(Y, ref) < 1e-13


@pytest.mark.parametrize("dims,L", CASES[:4])
@pytest.mark.parametrize("compress", [0, 1])
def test_apply_fp32(dims, L, compress):
    import torch
    U = S.gauge_links(dims, 0.3, 300 + L)
    X = S.random_spinor(dims, L, 400 + L)
    kappa, csw = 0.135, 1.6
    lat = lattice(U, kappa, csw, flags=compress)
    Y = to_np(lat.apply(to_dev(X, torch.complex64)))
    ref = dirac.apply(U, kappa, csw, X)
    assert rel_err(Y.astype(np.complex128), ref) < 2e-6


def test_set_params_rebuilds_clover():
    dims, L = (4, 4, 4, 4), 4
    U = S.gauge_links(dims, 0.4, 7)
    X = S.random_spinor(dims, L, 8)
    lat = lattice(U, 0.1, 1.0)
    lat.set_params(0.125, 1.9)
    Y = to_np(lat.apply(to_dev(X)))
    assert rel_err(Y, dirac.apply(U, 0.125, 1.9, X)) < 1e-13


def test_free_field_plane_wave_gpu():
    """U = 1 closed form on the device: D e^{ip.n} u = D(p) e^{ip.n} u."""
    from oracle.gamma import GAMMA
    dims = (4, 6, 4, 8)
    lx, ly, lz, lt = dims
    U = S.unit_links(dims)
    kappa = 0.11
    k = (1, 2, 3, 5)
    p = [2 * np.pi * k[i] / dims[i] for i in range(4)]
    t, z, y, x = np.meshgrid(range(lt), range(lz), range(ly), range(lx), indexing="ij")
    phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    u = np.arange(12).reshape(4, 3) * (1 + 0.5j) + 1
    X = (phase[..., None, None] * u)[..., None]
    Y = to_np(lattice(U, kappa, 1.3).apply(to_dev(X)))
    Dp = (1 - 2 * kappa * sum(np.cos(q) for q in p)) * np.eye(4) \
        + 2j * kappa * sum(GAMMA[m] * np.sin(p[m]) for m in range(4))
    assert np.abs(Y[..., 0] - phase[..., None, None] * (Dp @ u)).max() < 1e-13


@pytest.mark.parametrize("dims,L,prec", [((24, 24, 24, 48), 12, "fp32"), ((24, 24, 24, 48), 1, "fp64"),
                                         ((16, 16, 16, 32), 12, "fp64")])
def test_apply_full_size_sampled(dims, L, prec):
    """Full workload sizes in the launch shape the solver uses: sampled sites
    against the oracle's site-by-site evaluation of Eq. (1)."""
    import torch
    U = S.gauge_links(dims, 0.3, 3)
    X = S.random_spinor(dims, L, 33, dtype=np.complex64 if prec == "fp32" else np.complex128)
    lat = lattice(U, 0.135, 1.6)
    Y = lat.apply(to_dev(X))
    torch.cuda.synchronize()
    V = S.volume(dims)
    rng = np.random.default_rng(5)
    sites = np.concatenate([[0, V - 1, dims[0] - 1, V - dims[0]], rng.integers(0, V, 60)])
    Yg = to_np(Y).reshape(V, 4, 3, L)[sites]
    ref = dirac.apply_at_sites(U, 0.135, 1.6, X.astype(np.complex128), sites)
    tol = 2e-6 if prec == "fp32" else 1e-13
    err = np.abs(Yg - ref).max() / np.abs(ref).max()
    assert err < tol
