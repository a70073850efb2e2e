"""Adjoint solves and gradients on the GPU against the oracle
(oracle/gradients.py, pinned by finite differences on the CPU)."""
import numpy as np
import pytest
import scipy.linalg

import synthetic as S
from oracle import dirac, gradients as GR, solvers
from tests.gpu_util import lattice, rel_err, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("method", ["block_bicggr", "bicgstab"])
def test_dagger_solve(prec, method):
    dims = (4, 4, 4, 6)
    U = S.gauge_links(dims, 0.3, 61)
    kappa, csw = 0.13, 1.6
    L = 5
    B = S.gaussian_sources(dims, L, 62)
    lat = lattice(U, kappa, csw)
    X, info = lat.block_solve(to_dev(B), method=method, prec=prec, tol=1e-12, dagger=True)
    N = 12 * S.volume(dims)
    Ad = dirac.as_matrix_operator(U, kappa, csw, dagger=True)
    tr = solvers.true_residual(Ad, B.reshape(N, L), to_np(X).reshape(N, L))
    assert tr.max() <= 1e-12, (tr.max(), info)
    assert abs(info["true_residual_max"] - tr.max()) <= 1e-14 + 1e-3 * tr.max()


@pytest.mark.parametrize("dims,L,csw", [((4, 4, 4, 6), 3, 1.6), ((4, 4, 4, 6), 2, 0.0), ((8, 8, 8, 16), 12, 1.6),
                                        ((3, 4, 5, 6), 1, 1.2)])
def test_gradient_kernels_match_oracle(dims, L, csw):
    """bkwd_gradients for given X and Lam: grad_kappa, grad_csw and the link
    gradient (hopping + clover leaves) against the oracle's formulas."""
    U = S.gauge_links(dims, 0.3, 63)
    kappa = 0.128
    X = S.gaussian_sources(dims, L, 64)
    Lam = S.gaussian_sources(dims, L, 65)
    lat = lattice(U, kappa, csw)
    g = lat.gradients(to_dev(X), to_dev(Lam))
    gk = GR.grad_kappa(U, kappa, csw, X, Lam)
    gc = GR.grad_csw(U, kappa, csw, X, Lam)
    gU = GR.grad_links(U, kappa, csw, X, Lam)
    assert abs(g["kappa"] - gk) <= 1e-12 * (abs(gk) + 1e-300), (g["kappa"], gk)
    assert abs(g["csw"] - gc) <= 1e-12 * abs(gc) + 1e-13 * abs(gk), (g["csw"], gc)
    got = to_np(g["links"])
    assert got.shape == gU.shape
    assert rel_err(got, gU) <= 1e-12


def test_autograd_solve_matches_oracle():
    """X = D^{-1} B through the differentiable solve, loss Re <C, X> + |X|^2/2:
    U.grad, kappa.grad, csw.grad and B.grad against dense solves and the
    oracle's gradient formulas."""
    import torch
    from paper_0903_4936_amd import block_solve
    dims = (4, 4, 4, 4)
    U = S.gauge_links(dims, 0.4, 66)
    kappa, csw, L = 0.12, 1.4, 3
    B = S.gaussian_sources(dims, L, 67)
    C = S.gaussian_sources(dims, L, 68)
    Ut = torch.from_numpy(U.copy()).requires_grad_(True)
    kt = torch.tensor(kappa, dtype=torch.float64, requires_grad=True)
    ct = torch.tensor(csw, dtype=torch.float64, requires_grad=True)
    Bt = to_dev(B).requires_grad_(True)
    Ct = to_dev(C)
    X = block_solve(Ut, kt, ct, Bt, method="block_bicggr", prec="mixed", tol=1e-13)
    loss = (torch.sum(torch.conj(Ct) * X).real + 0.5 * torch.sum(torch.abs(X) ** 2))
    loss.backward()

    N = 12 * S.volume(dims)
    D = dirac.assemble_dense(U, kappa, csw)
    Xo = scipy.linalg.solve(D, B.reshape(N, L)).reshape(B.shape)
    Lamo = scipy.linalg.solve(D.conj().T, (C + Xo).reshape(N, L)).reshape(B.shape)
    assert rel_err(to_np(X.detach()), Xo) <= 1e-11
    assert rel_err(to_np(Bt.grad), Lamo) <= 1e-10
    gk = GR.grad_kappa(U, kappa, csw, Xo, Lamo)
    gc = GR.grad_csw(U, kappa, csw, Xo, Lamo)
    assert abs(kt.grad.item() - gk) <= 1e-9 * abs(gk)
    assert abs(ct.grad.item() - gc) <= 1e-9 * abs(gc)
    assert rel_err(Ut.grad.numpy(), GR.grad_links(U, kappa, csw, Xo, Lamo)) <= 1e-9


def test_c5_gradients_against_finite_differences():
    """The differentiable-solve workload: 16^3 x 32, kappa = 0.134, c_SW = 1.6,
    12 Gaussian sources, loss = Re sum_i <eta_i, X_i> with Gaussian eta.
    Gradients from the adjoint solve against central finite differences
    (step 1e-6) of the loss through FP64 GPU solves: kappa, c_SW, and
    directional derivatives along random directions in B and in the links."""
    import torch
    from paper_0903_4936_amd import Lattice, block_solve
    dims = (16, 16, 16, 32)
    U = S.gauge_links(dims, 0.3, 5)
    kappa, csw, L = 0.134, 1.6, 12
    B = S.gaussian_sources(dims, L, 51)
    eta = to_dev(S.gaussian_sources(dims, L, 52))
    opts = dict(method="block_bicggr", prec="fp64", tol=1e-13)
    Ut = torch.from_numpy(U.copy()).requires_grad_(True)
    kt = torch.tensor(kappa, dtype=torch.float64, requires_grad=True)
    ct = torch.tensor(csw, dtype=torch.float64, requires_grad=True)
    Bt = to_dev(B).requires_grad_(True)
    X = block_solve(Ut, kt, ct, Bt, **opts)
    torch.sum(torch.conj(eta) * X).real.backward()

    # The difference quotient divides the loss's solver error by 2h: the
    # c_SW derivative is ~300 times smaller than kappa's, and at a 1e-13 solve
    # tolerance that error alone was 1.6e-6 of it, so the finite-difference
    # solves run to 1e-14.
    fd_opts = dict(opts, tol=1e-14)

    def loss(Ul, k, c, Bl):
        lat = Lattice(Ul, k, c)
        Xl, _ = lat.block_solve(to_dev(Bl), **fd_opts)
        return float(torch.sum(torch.conj(eta) * Xl).real)

    h = 1e-6
    rng = np.random.default_rng(7)
    fk = (loss(U, kappa + h, csw, B) - loss(U, kappa - h, csw, B)) / (2 * h)
    fc = (loss(U, kappa, csw + h, B) - loss(U, kappa, csw - h, B)) / (2 * h)
    EB = S.gaussian_sources(dims, L, 53)
    fB = (loss(U, kappa, csw, B + h * EB) - loss(U, kappa, csw, B - h * EB)) / (2 * h)
    EU = (rng.standard_normal(U.shape) + 1j * rng.standard_normal(U.shape)) / np.sqrt(2)
    fU = (loss(U + h * EU, kappa, csw, B) - loss(U - h * EU, kappa, csw, B)) / (2 * h)
    dB = float(np.real(np.vdot(to_np(Bt.grad), EB)))
    dU = float(np.real(np.vdot(Ut.grad.numpy(), EU)))
    errs = {"kappa": abs(kt.grad.item() - fk) / abs(fk), "csw": abs(ct.grad.item() - fc) / abs(fc),
            "B": abs(dB - fB) / abs(fB), "U": abs(dU - fU) / abs(fU)}
    print("relative differences from central finite differences:", errs, flush=True)
    for k, e in errs.items():
        assert e <= 1e-6, (k, e)
