"""Even-odd preconditioned block solves (opts.evenodd): the Krylov cycles run
on the Schur complement of the even sites.  Parity with dense LU of the
oracle's assembled operator, the adjoint system, and whole-lattice true
residuals by the oracle's operator at full size."""
import numpy as np
import pytest
import scipy.linalg

import synthetic as S
from oracle import dirac, solvers
from tests.gpu_util import lattice, rel_err, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c1():
    dims = (4, 4, 4, 4)
    U = S.gauge_links(dims, 0.4, 1)
    kappa, csw = 0.125, 1.0
    B = S.point_sources(dims)
    N = 12 * S.volume(dims)
    D = dirac.assemble_dense(U, kappa, csw)
    Xlu = scipy.linalg.lu_solve(scipy.linalg.lu_factor(D), B.reshape(N, 12)).reshape(B.shape)
    return dims, U, kappa, csw, B, D, Xlu, np.linalg.cond(D)


@pytest.mark.parametrize("method", ["block_bicggr", "block_bicgstab", "bicgstab"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_evenodd_matches_dense_lu(c1, method, prec):
    dims, U, kappa, csw, B, D, Xlu, cond = c1
    lat = lattice(U, kappa, csw)
    X, info = lat.block_solve(to_dev(B), method=method, prec=prec, tol=1e-12, evenodd=True)
    Xg = to_np(X)
    N = 12 * S.volume(dims)
    tr = solvers.true_residual(lambda Y: D @ Y, B.reshape(N, 12), Xg.reshape(N, 12))
    assert tr.max() <= 1e-12, (tr.max(), info)
    assert abs(info["true_residual_max"] - tr.max()) <= 1e-14 + 1e-3 * tr.max()
    assert rel_err(Xg, Xlu) <= max(1e-10, 2 * cond * 1e-12)
    assert info["converged"] == 1


def test_evenodd_needs_fewer_iterations(c1):
    """The Schur system on the even sites is better conditioned: FP64 block
    BiCGGR needs fewer iterations than on the whole lattice."""
    dims, U, kappa, csw, B, D, Xlu, cond = c1
    lat = lattice(U, 0.135, 1.6)
    _, i_eo = lat.block_solve(to_dev(B), method="block_bicggr", prec="fp64", tol=1e-12, evenodd=True)
    _, i_full = lat.block_solve(to_dev(B), method="block_bicggr", prec="fp64", tol=1e-12)
    assert i_eo["iterations"] < i_full["iterations"], (i_eo["iterations"], i_full["iterations"])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_evenodd_adjoint(c1, prec):
    dims, U, kappa, csw, B, D, Xlu, cond = c1
    G = S.gaussian_sources(dims, 3, 81)
    N = 12 * S.volume(dims)
    lat = lattice(U, kappa, csw)
    X, info = lat.block_solve(to_dev(G), method="block_bicggr", prec=prec, tol=1e-12, evenodd=True, dagger=True)
    ref = np.linalg.solve(D.conj().T, G.reshape(N, 3))
    assert rel_err(to_np(X).reshape(N, 3), ref) <= max(1e-10, 2 * cond * 1e-12)


@pytest.mark.parametrize("dims,L", [((4, 2, 6, 4), 5), ((6, 4, 2, 4), 8), ((4, 4, 4, 2), 12), ((2, 4, 4, 6), 17)])
def test_evenodd_shapes(dims, L):
    """Extent 2, non-cubic lattices, ragged and multi-block column counts."""
    U = S.gauge_links(dims, 0.3, 82)
    kappa, csw = 0.13, 1.6
    B = S.gaussian_sources(dims, L, 83)
    lat = lattice(U, kappa, csw)
    for prec in ("fp64", "mixed"):
        X, info = lat.block_solve(to_dev(B), method="block_bicggr", prec=prec, tol=1e-12, evenodd=True)
        N = 12 * S.volume(dims)
        tr = solvers.true_residual(dirac.as_matrix_operator(U, kappa, csw), B.reshape(N, L), to_np(X).reshape(N, L))
        assert tr.max() <= 1e-12, (prec, tr.max())


@pytest.mark.parametrize("dims", [(4, 4, 4, 6), (6, 2, 4, 6)])
@pytest.mark.parametrize("dagger", [False, True])
def test_evenodd_gram_operator_blocks_match_dense_lu(dims, dagger):
    """Mixed even-odd block BiCGGR on 16 columns runs two blocks of 8, whose
    FP32 cycles form the QR frame's Grams of W' = S T in the second launch of
    the Schur operator S (of D, or of D^dagger).  The solution matches dense
    LU of the assembled operator (its conjugate transpose for D^dagger); on
    (6, 2, 4, 6) the 144 even sites leave a ragged last workgroup."""
    U = S.gauge_links(dims, 0.3, 84)
    kappa, csw = 0.13, 1.6
    L = 16
    B = S.gaussian_sources(dims, L, 85)
    N = 12 * S.volume(dims)
    D = dirac.assemble_dense(U, kappa, csw)
    if dagger:
        D = D.conj().T
    Xlu = scipy.linalg.lu_solve(scipy.linalg.lu_factor(D), B.reshape(N, L))
    lat = lattice(U, kappa, csw)
    X, info = lat.block_solve(to_dev(B), method="block_bicggr", prec="mixed", tol=1e-12, evenodd=True,
                              dagger=dagger)
    assert info["main_width"] == 8 and info["gram_operator"] == 1, info
    assert info["converged"] == 1
    Xg = to_np(X).reshape(N, L)
    tr = np.linalg.norm(D @ Xg - B.reshape(N, L), axis=0) / np.linalg.norm(B.reshape(N, L), axis=0)
    assert tr.max() <= 1e-12, (tr.max(), info)
    assert rel_err(Xg, Xlu) < 1e-9


def test_evenodd_rejects_odd_extents_and_options():
    from paper_0903_4936_amd import BkwdError
    dims = (3, 4, 4, 4)
    lat = lattice(S.gauge_links(dims, 0.4, 5), 0.125, 1.0)
    B = to_dev(S.gaussian_sources(dims, 2, 6))
    with pytest.raises((BkwdError, ValueError)):
        lat.block_solve(B, method="block_bicggr", prec="mixed", tol=1e-12, evenodd=True)
    dims = (4, 4, 4, 4)
    lat = lattice(S.gauge_links(dims, 0.4, 5), 0.125, 1.0)
    B = to_dev(S.gaussian_sources(dims, 2, 6))
    with pytest.raises((BkwdError, ValueError)):
        lat.block_solve(B, method="block_bicggr", prec="mixed", tol=1e-12, evenodd=True, reliable=0.1)


@pytest.mark.parametrize("kappa", [0.130, 0.136])
def test_evenodd_c2_whole_lattice(kappa):
    """16^3 x 32, 12 point sources, c_SW = 1.6: FP64 and mixed even-odd
    block BiCGGR reach a 1e-12 true residual by the oracle's operator over
    the whole lattice, with fewer iterations than without the split."""
    import torch
    from oracle import native
    dims = (16, 16, 16, 32)
    U = S.gauge_links(dims, 0.3, 2)
    B = S.point_sources(dims)
    M = native.local_matrix(U, kappa, 1.6)
    lat = lattice(U, kappa, 1.6)
    for prec in ("fp64", "mixed"):
        X, info = lat.block_solve(to_dev(B), method="block_bicggr", prec=prec, tol=1e-12, evenodd=True)
        _, i_full = lat.block_solve(to_dev(B), method="block_bicggr", prec=prec, tol=1e-12)
        torch.cuda.synchronize()
        rel, _ = native.residual(U, kappa, M, to_np(X), B)
        print(f"kappa {kappa} {prec}: even-odd {info['iterations']} iterations, whole lattice "
              f"{i_full['iterations']}; oracle residual {rel.max():.3e}", flush=True)
        assert rel.max() <= 1e-12, (prec, rel.max())
        assert info["iterations"] < i_full["iterations"]


@pytest.mark.parametrize("dims,seed,L,src", [((24, 24, 24, 48), 3, 12, "point"), ((32, 32, 32, 64), 4, 64, "z2")])
def test_evenodd_full_size_whole_lattice(dims, seed, L, src):
    """The benchmark workloads (kappa 0.135, c_SW 1.6) solved mixed with the
    even-odd split to a 1e-12 true residual, checked column by column over the
    whole lattice with the oracle's operator."""
    import torch
    from oracle import native
    U = S.gauge_links(dims, 0.3, seed)
    kappa, csw = 0.135, 1.6
    B = S.point_sources(dims) if src == "point" else S.z2_sources(dims, L, 41)
    lat = lattice(U, kappa, csw)
    Bd = to_dev(B)
    X, info = lat.block_solve(Bd, method="block_bicggr", prec="mixed", tol=1e-12, evenodd=True)
    torch.cuda.synchronize()
    print(f"{dims} L={L} even-odd: {info['iterations']} iterations, {info['seconds']:.3f} s, library true residual "
          f"{info['true_residual_max']:.3e}", flush=True)
    assert info["converged"] == 1 and info["true_residual_max"] <= 1e-12
    Xh = to_np(X)
    del X, Bd, lat
    torch.cuda.empty_cache()
    M = native.local_matrix(U, kappa, csw)
    rel, _ = native.residual(U, kappa, M, Xh, B)
    print(f"oracle whole-lattice residual: max {rel.max():.3e}", flush=True)
    assert rel.max() <= 1e-12
