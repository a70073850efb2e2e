"""Meson two-point functions on the GPU (bkwd_meson_correlators) against the
oracle's contraction of the same solution block, the free field against its
momentum-space form, and the timed workload at full size."""
import numpy as np
import pytest

import synthetic as S
from oracle import correlators as C
from tests.gpu_util import lattice, to_dev, to_np

pytestmark = pytest.mark.gpu


def _check_same(got, ref, tol):
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max(), (got, ref)


def test_contraction_matches_oracle_small():
    import torch
    dims = (4, 4, 4, 8)
    U = S.gauge_links(dims, 0.3, 61)
    lat = lattice(U, 0.125, 1.4)
    X, info = lat.block_solve(to_dev(S.point_sources(dims)), method="block_bicggr", prec="fp64", tol=1e-12)
    pion, rho = lat.meson_correlators(X)
    torch.cuda.synchronize()
    Xh = to_np(X)
    _check_same(to_np(pion), C.pion(Xh), 1e-12)
    _check_same(to_np(rho), C.rho(Xh), 1e-12)
    assert (to_np(pion) > 0).all()


def test_contraction_of_arbitrary_block():
    """The contraction is linear algebra on any 12-column block: random
    complex data (no solve) against the oracle."""
    import torch
    dims = (3, 4, 5, 6)
    U = S.gauge_links(dims, 0.3, 62)
    lat = lattice(U, 0.12, 1.0)
    Xr = S.random_spinor(dims, 12, 63)
    pion, rho = lat.meson_correlators(to_dev(Xr))
    torch.cuda.synchronize()
    _check_same(to_np(pion), C.pion(Xr), 1e-12)
    _check_same(to_np(rho), C.rho(Xr), 1e-12)


def test_rejects_wrong_blocks():
    import torch
    dims = (2, 2, 2, 4)
    lat = lattice(S.gauge_links(dims, 0.3, 64), 0.12, 1.0)
    with pytest.raises(ValueError):
        lat.meson_correlators(to_dev(S.random_spinor(dims, 12, 65)).to(torch.complex64))
    with pytest.raises(ValueError):
        lat.meson_correlators(to_dev(S.random_spinor(dims, 6, 66)))


def test_free_field_against_momentum_space():
    """U = 1: solve on the GPU, contract on the GPU, compare with the free
    propagator summed in momentum space."""
    import torch
    from oracle.gamma import GAMMA, GAMMA5
    dims = (4, 4, 4, 8)
    kappa = 0.12
    lat = lattice(S.unit_links(dims), kappa, 1.0)
    X, _ = lat.block_solve(to_dev(S.point_sources(dims)), method="block_bicggr", prec="fp64", tol=1e-13)
    pion, rho = lat.meson_correlators(X)
    torch.cuda.synchronize()
    ref_pi = C.free_meson_momentum(dims, kappa, GAMMA5)
    ref_rho = sum(C.free_meson_momentum(dims, kappa, GAMMA[k]) for k in range(3)) / 3
    _check_same(to_np(pion), ref_pi, 1e-9)
    _check_same(to_np(rho), ref_rho, 1e-9)


def test_full_size_timed_workload():
    """24^3 x 48, kappa = 0.135, c_SW = 1.6: the mixed solve of the timed
    workload, its correlators on the GPU against the oracle's contraction of
    the same solution; the pion correlator is positive and falls from the
    source to the middle of the lattice."""
    import torch
    dims = (24, 24, 24, 48)
    U = S.gauge_links(dims, 0.3, 3)
    lat = lattice(U, 0.135, 1.6)
    X, info = lat.block_solve(to_dev(S.point_sources(dims)), method="block_bicggr", prec="mixed", tol=1e-12)
    pion, rho = lat.meson_correlators(X)
    torch.cuda.synchronize()
    Xh = to_np(X)
    del X, lat
    p, r = to_np(pion), to_np(rho)
    _check_same(p, C.pion(Xh), 1e-12)
    _check_same(r, C.rho(Xh), 1e-12)
    assert (p > 0).all()
    assert all(p[t + 1] < p[t] for t in range(dims[3] // 2))
