"""Deflation of converged and linearly dependent columns between Krylov
cycles, FP64 (growth of Sec. 3 for the failure of the block methods on
dependent or nearly dependent right-hand sides that Sec. 4.3 and Sec. 5
report; the paper names no remedy).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Restarted block solve: with X the current iterate and R = B - A X,

1. columns with ||r_i|| <= tol ||b_i|| have converged and are left out;
2. a pivoted Cholesky factorisation of the others' Gram matrix picks,
   largest remaining relative diagonal first, the columns whose part
   orthogonal to those already picked is at least max(drop ||r_i||,
   tol ||b_i|| / 10) in norm: the independent set I.  (The second bound
   keeps columns that differ only at the level the solve does not resolve,
   such as duplicated right-hand sides whose residuals drift apart by
   rounding, out of the block);
3. every other active column d is written in the span of I in the least-
   squares sense, r_d ~ R_I c_d with c_d = (R_I^H R_I)^{-1} R_I^H r_d;
4. one Block BiCGGR cycle solves A E = R_I to a relative `inner_tol`, and
   the correction is x_i += e_i for i in I, x_d += E c_d.

Because A is linear the dependent columns' corrections are exact when r_d
lies in the span of R_I; what is left of r_d is taken up by later cycles.
"""
import numpy as np

from . import solvers


def pivoted_cholesky(G: np.ndarray, drop: float, floor=None):
    """Pivoted Cholesky of a Hermitian positive semi-definite G (n x n):
    returns the pivot order of the accepted columns, in which the squared
    pivot (the squared norm of the column's part orthogonal to the columns
    accepted before it, for G a Gram matrix) is at least drop**2 times its
    diagonal entry and at least floor[i] (default 0).  Stops at the first
    column below that."""
    n = G.shape[0]
    A = G.astype(np.complex128).copy()
    d0 = np.real(np.diag(G)).copy()
    fl = np.zeros(n) if floor is None else np.asarray(floor, dtype=float)
    perm = list(range(n))
    accepted = []
    for k in range(n):
        # largest remaining diagonal relative to the original column norm
        rem = [np.real(A[perm[j], perm[j]]) / d0[perm[j]] if d0[perm[j]] > 0 else 0.0 for j in range(k, n)]
        j = k + int(np.argmax(rem))
        if rem[j - k] < drop ** 2 or np.real(A[perm[j], perm[j]]) < fl[perm[j]]:
            break
        perm[k], perm[j] = perm[j], perm[k]
        p = perm[k]
        piv = np.sqrt(np.real(A[p, p]))
        accepted.append(p)
        # eliminate: A <- A - a a^H / piv^2 on the remaining columns
        col = A[:, p].copy()
        for q in perm[k + 1:]:
            for t in perm[k + 1:]:
                A[q, t] -= col[q] * np.conj(col[t]) / piv ** 2
    return accepted


def plan(R: np.ndarray, B: np.ndarray, tol: float, drop: float):
    """Active and independent columns of a residual block R, and the
    coefficients of the dependent ones: (I, C) with C of shape (len(I), L),
    the correction being E @ C for the cycle's solution E of A E = R[:, I]."""
    L = R.shape[1]
    rn = np.linalg.norm(R, axis=0)
    bn = np.linalg.norm(B, axis=0)
    active = [i for i in range(L) if rn[i] > tol * bn[i]]
    if not active:
        return [], np.zeros((0, L), dtype=np.complex128)
    Ra = R[:, active]
    G = Ra.conj().T @ Ra
    sel = pivoted_cholesky(G, drop, (0.1 * tol * bn[active]) ** 2)
    I = [active[j] for j in sel]
    C = np.zeros((len(I), L), dtype=np.complex128)
    for j, i in enumerate(I):
        C[j, i] = 1.0
    RI = R[:, I]
    GI = RI.conj().T @ RI
    for d in active:
        if d not in I:
            C[:, d] = np.linalg.solve(GI, RI.conj().T @ R[:, d])
    return I, C


def solve(A, B: np.ndarray, tol: float, inner_tol: float = 1e-6, drop: float = 1e-6, max_cycles: int = 50,
          max_iter: int = 1000):
    """Restarted Block BiCGGR with deflation (module docstring).  Returns
    (X, info) with the iterations and the width of every cycle."""
    X = np.zeros_like(B)
    bn = np.linalg.norm(B, axis=0)
    widths, iters = [], 0
    for _ in range(max_cycles):
        R = B - A(X)
        if np.max(np.linalg.norm(R, axis=0) / bn) <= tol:
            return X, {"status": "converged", "widths": widths, "iterations": iters}
        I, C = plan(R, B, tol, drop)
        RI = R[:, I]
        E, info = solvers.block_bicggr(A, RI, inner_tol, max_iter)
        iters += info["iterations"]
        widths.append(len(I))
        X = X + E @ C
    return X, {"status": "maxcycles", "widths": widths, "iterations": iters}
