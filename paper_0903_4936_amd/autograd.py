"""Differentiable block solve: X = D_W(U, kappa, c_SW)^{-1} B with gradients
for the links U, kappa, c_SW and B (growth of the method of Sec. 3; the
gradient formulas follow from Eq. (1) of Sec. 2).

Backward runs the adjoint block solve D_W^dagger Lam = G on the same HIP
kernels (D_W^dagger = gamma_5 D_W gamma_5) and then the gradient kernels
(bkwd_gradients): grad_B = Lam, and grad_kappa, grad_csw, grad_U in the
complex-autograd convention (dl = Re sum conj(g) dz).
"""
from __future__ import annotations

import numpy as np

from .bkwd import Lattice


def _torch():
    import torch
    return torch


def _solve_nonzero_columns(lat: Lattice, G, opts: dict):
    """D^dagger Lam = G, columns of G that are zero give zero columns of Lam."""
    torch = _torch()
    L = G.shape[-1]
    norms = G.reshape(-1, L).abs().amax(dim=0)
    nz = torch.nonzero(norms > 0).flatten().tolist()
    Lam = torch.zeros_like(G)
    if not nz:
        return Lam
    if len(nz) == L:
        Lam, _ = lat.block_solve(G.contiguous(), dagger=True, **opts)
        return Lam
    Gs = G[..., nz].contiguous()
    Ls, _ = lat.block_solve(Gs, dagger=True, **opts)
    Lam[..., nz] = Ls
    return Lam


class _LatticeCache:
    """The operator of the last forward call, reused while the links tensor
    (same storage, unmodified since: same version counter), kappa, c_SW and
    the device stay the same, so repeated solves on one gauge field do not
    re-upload the links or rebuild the clover blocks."""

    def __init__(self):
        self.key = None
        self.U = None
        self.lat = None

    def get(self, U, kappa: float, csw: float, device):
        torch = _torch()
        key = (U.data_ptr(), U._version, tuple(U.shape), str(U.device), kappa, csw, str(device))
        if self.lat is None or key != self.key:
            links = U.detach().to("cpu", torch.complex128).numpy()
            self.lat = Lattice(np.ascontiguousarray(links), kappa, csw, device=device)
            self.key = key
            self.U = U  # keeps the storage alive, so its address is not reused
        return self.lat


_CACHE = _LatticeCache()


def _make_function():
    torch = _torch()

    class BlockSolve(torch.autograd.Function):
        @staticmethod
        def forward(ctx, U, kappa, csw, B, opts):
            lat = _CACHE.get(U, float(kappa), float(csw), B.device)
            X, _ = lat.block_solve(B.detach().contiguous(), **opts)
            ctx.k_device = kappa.device
            ctx.c_device = csw.device
            ctx.lat = lat
            ctx.opts = opts
            ctx.u_device = U.device
            ctx.save_for_backward(X)
            return X

        @staticmethod
        def backward(ctx, G):
            (X,) = ctx.saved_tensors
            lat = ctx.lat
            need_U, need_k, need_c, need_B, _ = ctx.needs_input_grad
            Lam = _solve_nonzero_columns(lat, G.to(torch.complex128), ctx.opts)
            g = lat.gradients(X, Lam, links=need_U, scalars=need_k or need_c)
            gU = g["links"].to(ctx.u_device) if need_U else None
            gk = torch.tensor(g["kappa"], dtype=torch.float64, device=ctx.k_device) if need_k else None
            gc = torch.tensor(g["csw"], dtype=torch.float64, device=ctx.c_device) if need_c else None
            return gU, gk, gc, (Lam if need_B else None), None

    return BlockSolve


_FN = None


def block_solve(U, kappa, csw, B, **opts):
    """Differentiable X = D_W^{-1} B.  U: complex128 tensor (4, Lt, Lz, Ly, Lx,
    3, 3); kappa, csw: float64 tensors (or floats); B: complex128 CUDA tensor
    (Lt, Lz, Ly, Lx, 4, 3, L).  ``opts`` are Lattice.make_opts keywords."""
    global _FN
    torch = _torch()
    if _FN is None:
        _FN = _make_function()
    if not isinstance(kappa, torch.Tensor):
        kappa = torch.tensor(float(kappa), dtype=torch.float64)
    if not isinstance(csw, torch.Tensor):
        csw = torch.tensor(float(csw), dtype=torch.float64)
    return _FN.apply(U, kappa, csw, B, opts)
