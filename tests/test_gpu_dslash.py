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


def _to_cm(X):
    """site-major (Lt, Lz, Ly, Lx, 4, 3, L) -> component-major (12, V, L)"""
    L = X.shape[-1]
    return np.ascontiguousarray(X.reshape(-1, 12, L).transpose(1, 0, 2))


def _from_cm(Y, shape):
    L = shape[-1]
    return np.ascontiguousarray(Y.reshape(12, -1, L).transpose(1, 0, 2)).reshape(shape)


# FP32 widths of the mixed solve's column blocks, component-major as in the
# Krylov workspace; lattices with a slice of sites that is not a multiple of
# a workgroup's sites (ragged last workgroup per slice)
CM_CASES = [((8, 6, 4, 6), 8), ((5, 3, 4, 6), 8), ((8, 6, 4, 6), 4), ((5, 3, 4, 6), 4), ((4, 4, 4, 4), 12)]


@pytest.mark.parametrize("dims,L", CM_CASES)
@pytest.mark.parametrize("compress", [0, 1])
@pytest.mark.parametrize("dagger", [False, True])
def test_apply_fp32_component_major(dims, L, compress, dagger):
    """bkwd_apply_layout with the solver's component-major blocks in FP32 (the
    launches of the mixed solve's inner iteration) against the oracle."""
    import torch
    U = S.gauge_links(dims, 0.3, 500 + L)
    X = S.random_spinor(dims, L, 600 + L)
    kappa, csw = 0.135, 1.6
    lat = lattice(U, kappa, csw, flags=compress)
    Yc = to_np(lat.apply(to_dev(_to_cm(X), torch.complex64), dagger=dagger, layout="component"))
    Y = _from_cm(Yc, X.shape).astype(np.complex128)
    ref = dirac.apply(U, kappa, csw, X, dagger=dagger)
    assert rel_err(Y, ref) < 2e-6


@pytest.mark.parametrize("L", [1, 12])
def test_apply_fp64_component_major(L):
    dims = (5, 3, 4, 6)
    U = S.gauge_links(dims, 0.3, 700 + L)
    X = S.random_spinor(dims, L, 800 + L)
    lat = lattice(U, 0.13, 1.6)
    Y = _from_cm(to_np(lat.apply(to_dev(_to_cm(X)), layout="component")), X.shape)
    assert rel_err(Y, dirac.apply(U, 0.13, 1.6, X)) < 1e-13


def test_apply_rejects_unknown_layout():
    from paper_0903_4936_amd import bkwd
    import ctypes
    dims = (4, 4, 2, 2)
    lat = lattice(S.gauge_links(dims, 0.4, 5), 0.125, 1.0)
    X = to_dev(S.random_spinor(dims, 2, 6))
    Y = X.clone()
    code = bkwd.lib().bkwd_apply_layout(lat._h, 0, 2, bkwd.FP64, 2, ctypes.c_void_p(X.data_ptr()),
                                        ctypes.c_void_p(Y.data_ptr()), None)
    assert code == bkwd.EINVAL and "layout" in bkwd.last_error()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_single_link_clover_closed_form(prec):
    """The device clover term against the closed form of one non-unit link
    (tests/test_oracle_clover_pin.py), with no oracle in between: applying D
    to the 12 point sources at a site gives the site-local matrix M(n) as the
    block of the result at that site."""
    import torch
    from tests.test_oracle_clover_pin import DIMS, I_SIGMA_T, M_SITE, _expected_local, _links_with, _rotation_link
    D = _rotation_link(0.7)
    kappa, csw = 0.11, 1.7
    U = _links_with(DIMS, 3, M_SITE, D)
    want = _expected_local(DIMS, 3, M_SITE, D, kappa, csw, I_SIGMA_T).reshape(-1, 12, 12)
    lat = lattice(U, kappa, csw)
    V = S.volume(DIMS)
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    tol = 1e-15 if prec == "fp64" else 2e-7
    lx, ly, lz, lt = DIMS
    for site in range(V):
        B = S.point_sources(DIMS, site=site)
        Y = to_np(lat.apply(to_dev(B, dt))).reshape(V, 12, 12)
        assert np.abs(Y[site] - want[site]).max() < tol, site


@pytest.mark.parametrize("dims,L,prec,layout", [((24, 24, 24, 48), 8, "fp32", "component"),
                                                ((24, 24, 24, 48), 4, "fp32", "component"),
                                                ((24, 24, 24, 48), 12, "fp32", "site"),
                                                ((32, 32, 32, 64), 8, "fp32", "component"),
                                                ((24, 24, 24, 48), 1, "fp64", "site"),
                                                ((16, 16, 16, 32), 12, "fp64", "site")])
def test_apply_full_size_whole_lattice(dims, L, prec, layout):
    """Full workload sizes in the launch shapes the solver uses (FP32 blocks
    of 8 and 4 columns in the component-major Krylov layout, the FP64 one-column
    operator of the baseline), every site against the oracle's operator
    (plain-C version of Eq. (1))."""
    import torch
    from oracle import native
    U = S.gauge_links(dims, 0.3, 3)
    X = S.random_spinor(dims, L, 33, dtype=np.complex64 if prec == "fp32" else np.complex128)
    lat = lattice(U, 0.135, 1.6)
    Xd = to_dev(_to_cm(X) if layout == "component" else X)
    Y = to_np(lat.apply(Xd, layout=layout))
    torch.cuda.synchronize()
    del Xd, lat
    if layout == "component":
        Y = _from_cm(Y, X.shape)
    M = native.local_matrix(U, 0.135, 1.6)
    ref = native.apply(U, 0.135, M, X.astype(np.complex128))
    tol = 2e-6 if prec == "fp32" else 1e-13
    assert rel_err(Y.astype(np.complex128), ref) < tol
