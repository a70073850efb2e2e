"""Meson two-point functions from the 12 point-source solutions (the downstream
use of the L = 12 solves named in the introduction and Sec. 4: the quark
propagator from one site to all sites).  FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The solution block X of D_W X = B with the 12 point sources of Sec. 2 at the
origin (column i = colour b + 3 * spin beta) is the propagator

    S(x)_{(alpha a), (beta b)} = X[x, alpha, a, 3 beta + b],

a 12 x 12 matrix per site with rows and columns ordered 3 * spin + colour.
For a bilinear O_G = psibar G psi the Wick contraction with the
gamma_5-hermiticity S(0, x) = gamma_5 S(x, 0)^dagger gamma_5 (which D_W has:
gamma_5 D_W gamma_5 = D_W^dagger) gives, summed over the spatial sites of
time slice t (the source sits at t = 0),

    C_G(t) = - sum_x Tr[ G S(x) Gbar gamma_5 S(x)^dagger gamma_5 ],
    Gbar = gamma_4 G^dagger gamma_4,

the trace over spin and colour, the overall sign that of the closed quark
loop.  This is the textbook contraction, not a formula of the paper; the
gamma matrices are those of Sec. 2.

* pion:  G = gamma_5, for which C(t) = sum_x ||S(x)||_F^2 >= 0;
* rho:   G = gamma_k, averaged over k = 1, 2, 3.
"""
import numpy as np

from .gamma import GAMMA, GAMMA5


def propagator(X: np.ndarray) -> np.ndarray:
    """(Lt, Lz, Ly, Lx, 4, 3, 12) solution block -> (Lt, Lz, Ly, Lx, 12, 12)
    propagator matrices, rows (alpha, a) and columns (beta, b) both ordered
    3 * spin + colour."""
    if X.shape[-3:] != (4, 3, 12):
        raise ValueError("X must hold the 12 point-source columns")
    return X.reshape(X.shape[:4] + (12, 12))


def _spin(G: np.ndarray) -> np.ndarray:
    """G acting on spin only: G (x) 1_colour, 12 x 12."""
    return np.kron(G, np.eye(3))


def meson(X: np.ndarray, G: np.ndarray) -> np.ndarray:
    """C_G(t) for t = 0 .. Lt - 1 (real part; the imaginary part vanishes for
    the channels used here)."""
    S = propagator(X)
    g5 = _spin(GAMMA5)
    Gs = _spin(G)
    Gbar = _spin(GAMMA[3] @ G.conj().T @ GAMMA[3])
    Sdag = np.conj(np.swapaxes(S, -1, -2))
    M = Gs @ S @ (Gbar @ g5) @ Sdag @ g5
    tr = np.trace(M, axis1=-2, axis2=-1)
    return -np.real(tr.sum(axis=(1, 2, 3)))


def pion(X: np.ndarray) -> np.ndarray:
    return meson(X, GAMMA5)


def rho(X: np.ndarray) -> np.ndarray:
    return sum(meson(X, GAMMA[k]) for k in range(3)) / 3.0


def free_meson_momentum(dims, kappa: float, G: np.ndarray) -> np.ndarray:
    """C_G(t) at U = 1 by a different route: the free propagator in momentum
    space, S(p) = D(p)^-1 with D(p) = 1 - 2 kappa sum_mu cos p_mu
    + 2 i kappa sum_mu gamma_mu sin p_mu (the Fourier transform of Eq. (1) at
    U = 1, where F_{mu nu} = 0), and the spatial sum over x done as a sum
    over spatial momenta (Parseval):
        sum_x Tr[A S(x,t) B S(x,t)^dagger]
          = (1 / V_s) sum_p Tr[A St(p,t) B St(p,t)^dagger],
        St(p, t) = (1 / Lt) sum_{p4} e^{i p4 t} S(p, p4).
    Colour is the identity, so every colour trace is 3 x the spin trace.
    dims = (Lx, Ly, Lz, Lt); periodic in all directions."""
    lx, ly, lz, lt = dims
    ks = [2 * np.pi * np.arange(n) / n for n in (lx, ly, lz, lt)]
    A = G
    B = GAMMA[3] @ G.conj().T @ GAMMA[3] @ GAMMA5
    out = np.zeros(lt)
    vs = lx * ly * lz
    for p1 in ks[0]:
        for p2 in ks[1]:
            for p3 in ks[2]:
                St = np.zeros((lt, 4, 4), dtype=np.complex128)
                for p4 in ks[3]:
                    p = (p1, p2, p3, p4)
                    D = (1 - 2 * kappa * sum(np.cos(q) for q in p)) * np.eye(4) \
                        + 2j * kappa * sum(GAMMA[m] * np.sin(p[m]) for m in range(4))
                    Sp = np.linalg.inv(D)
                    St += np.exp(1j * p4 * np.arange(lt))[:, None, None] * Sp / lt
                for t in range(lt):
                    out[t] += -3 * np.real(np.trace(A @ St[t] @ B @ St[t].conj().T @ GAMMA5)) / vs
    return out


__all__ = ["propagator", "meson", "pion", "rho", "free_meson_momentum"]
