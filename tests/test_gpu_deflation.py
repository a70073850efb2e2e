"""Deflation of converged and dependent columns between Krylov cycles
(opts.deflate): duplicated and dependent right-hand sides, which break the
block iteration down without it, converge to the dense LU solution of the
oracle's operator; independent columns are unaffected; converged columns are
left out; the full-size 64-column workload reaches 1e-12 by the oracle's
operator over the whole lattice."""
import numpy as np
import pytest

import synthetic as S
from oracle import deflation, dirac, solvers
from tests.gpu_util import lattice, rel_err, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small():
    dims = (4, 4, 2, 2)
    U = S.gauge_links(dims, 0.4, 5)
    kappa, csw = 0.125, 1.0
    D = dirac.assemble_dense(U, kappa, csw)
    return dims, U, kappa, csw, D


def _dependent_block(dims):
    b = S.gaussian_sources(dims, 1, 6)
    c = S.gaussian_sources(dims, 1, 7)
    return np.concatenate([b, b, 2 * b + c, c, 1j * c], axis=-1)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("evenodd", [False, True])
def test_dependent_columns_converge(small, prec, evenodd):
    dims, U, kappa, csw, D = small
    B = _dependent_block(dims)
    N, L = 12 * S.volume(dims), B.shape[-1]
    lat = lattice(U, kappa, csw)
    X, info = lat.block_solve(to_dev(B), method="block_bicggr", prec=prec, tol=1e-12, deflate=True, evenodd=evenodd)
    assert info["converged"] == 1 and info["deflated_columns"] >= 3, info
    Xlu = np.linalg.solve(D, B.reshape(N, L))
    assert rel_err(to_np(X).reshape(N, L), Xlu) < 1e-10
    # the oracle's deflated solve agrees
    Xo, io = deflation.solve(lambda Y: D @ Y, B.reshape(N, L), 1e-12)
    assert io["status"] == "converged" and io["widths"][0] == 2
    assert rel_err(to_np(X).reshape(N, L), Xo) < 1e-9


@pytest.mark.parametrize("method", ["block_bicggr", "block_bicgstab"])
def test_duplicates_without_deflation_break_down(small, method):
    """The failure deflation removes: without it the singular L x L systems of
    the block iteration stop the solve."""
    from paper_0903_4936_amd import NotConverged
    dims, U, kappa, csw, D = small
    b = S.gaussian_sources(dims, 1, 6)
    lat = lattice(U, kappa, csw)
    with pytest.raises(NotConverged) as ei:
        lat.block_solve(to_dev(np.concatenate([b, b], axis=-1)), method=method, prec="fp64", tol=1e-12)
    assert ei.value.code == -5


def test_independent_columns_unaffected(small):
    dims, U, kappa, csw, D = small
    B = S.gaussian_sources(dims, 6, 8)
    N = 12 * S.volume(dims)
    lat = lattice(U, kappa, csw)
    X, info = lat.block_solve(to_dev(B), method="block_bicggr", prec="mixed", tol=1e-12, deflate=True)
    assert info["converged"] == 1
    tr = solvers.true_residual(lambda Y: D @ Y, B.reshape(N, 6), to_np(X).reshape(N, 6))
    assert tr.max() <= 1e-12


def test_converged_column_left_out(small):
    """With X0 exact for column 0 (from a dense solve) only the other columns
    are iterated: one column is deflated in the first cycle."""
    dims, U, kappa, csw, D = small
    B = S.gaussian_sources(dims, 3, 9)
    N = 12 * S.volume(dims)
    X0 = np.zeros_like(B)
    X0[..., 0] = np.linalg.solve(D, B[..., 0].reshape(N)).reshape(X0[..., 0].shape)
    lat = lattice(U, kappa, csw)
    X, info = lat.block_solve(to_dev(B), X=to_dev(X0), method="block_bicggr", prec="fp64", tol=1e-12, deflate=True)
    assert info["converged"] == 1 and info["deflated_columns"] >= 1
    tr = solvers.true_residual(lambda Y: D @ Y, B.reshape(N, 3), to_np(X).reshape(N, 3))
    assert tr.max() <= 1e-12


def test_full_size_deflated_whole_lattice():
    import torch
    from oracle import native
    dims, L = (32, 32, 32, 64), 64
    U = S.gauge_links(dims, 0.3, 4)
    kappa, csw = 0.135, 1.6
    B = S.z2_sources(dims, L, 41)
    lat = lattice(U, kappa, csw)
    X, info = lat.block_solve(to_dev(B), method="block_bicggr", prec="mixed", tol=1e-12, deflate=True)
    torch.cuda.synchronize()
    print(f"deflated 32^3x64 L=64: {info['iterations']} iterations, {info['seconds']:.3f} s, "
          f"{info['deflated_columns']} columns left out", flush=True)
    assert info["converged"] == 1
    Xh = to_np(X)
    del X, lat
    torch.cuda.empty_cache()
    rel, _ = native.residual(U, kappa, native.local_matrix(U, kappa, csw), Xh, B)
    assert rel.max() <= 1e-12, rel.max()
