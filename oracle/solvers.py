"""The three Krylov solvers of Sec. 3 and the true residual of Sec. 4.3, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

A is any callable mapping an (N, L) complex array to A times it.  Blocks are
(N, L) arrays whose column i is x^(i) (Sec. 3).

Readings of points the paper leaves open:

* initial guess X_0 = 0 unless one is passed;
* shadow residual R~_0 = R_0 unless one is passed;
* inner product (x, y) = x^H y (conjugate on the first argument), consistent
  with the block methods' R~_0^H (.);
* the stop test max_i ||r_k^(i)|| / ||b^(i)|| <= eps is made at the top of
  each iteration; ``iterations`` counts completed loop bodies;
* L x L systems are solved by LU with partial pivoting (numpy.linalg.solve);
* BiCGSTAB degenerate step: if A t_k = 0 exactly (t_k = 0, the iterate is
  already exact) zeta_k is taken as 0 instead of 0/0, so the next stop test
  ends the loop.  The same for Tr(Z^H Z) = 0 in block BiCGSTAB;
* a singular L x L system or a non-finite scalar is a breakdown; the solver
  returns the last iterate with status "breakdown".
"""
import numpy as np


def _col_norms(M: np.ndarray) -> np.ndarray:
    return np.sqrt(np.sum(np.abs(M) ** 2, axis=0))


def bicgstab(A, b: np.ndarray, tol: float, max_iter: int, x0=None, r_tilde=None, callback=None):
    """BiCGSTAB for one right-hand side, following the listing in Sec. 3.

    ``b`` is an (N,) or (N, 1) vector.  Returns (x, info).
    """
    shape = b.shape
    b = b.reshape(-1, 1)
    x = np.zeros_like(b) if x0 is None else x0.reshape(-1, 1).copy()
    r = b - A(x)
    p = r.copy()
    rt = r.copy() if r_tilde is None else r_tilde.reshape(-1, 1)
    bnorm = np.linalg.norm(b)
    hist = []
    k = 0
    while True:
        rel = np.linalg.norm(r) / bnorm
        hist.append(rel)
        if rel <= tol:
            return x.reshape(shape), {"iterations": k, "status": "converged", "history": hist}
        if k >= max_iter:
            return x.reshape(shape), {"iterations": k, "status": "maxiter", "history": hist}
        Ap = A(p)
        alpha = np.vdot(rt, r) / np.vdot(rt, Ap)
        t = r - alpha * Ap
        At = A(t)
        den = np.vdot(At, At)
        zeta = 0.0 if den == 0 else np.vdot(At, t) / den
        x = x + alpha * p + zeta * t
        r_new = t - zeta * At
        if zeta == 0:
            beta = 0.0
        else:
            beta = (alpha / zeta) * np.vdot(rt, r_new) / np.vdot(rt, r)
        p = r_new + beta * (p - zeta * Ap)
        r = r_new
        k += 1
        if not np.isfinite(alpha) or not np.isfinite(zeta) or not np.isfinite(beta):
            return x.reshape(shape), {"iterations": k, "status": "breakdown", "history": hist}
        if callback is not None:
            callback(k, {"x": x, "r": r, "p": p})


def block_bicgstab(A, B: np.ndarray, tol: float, max_iter: int, X0=None, R_tilde=None, callback=None):
    """Block BiCGSTAB, following the listing in Sec. 3.  Returns (X, info)."""
    X = np.zeros_like(B) if X0 is None else X0.copy()
    R = B - A(X)
    P = R.copy()
    Rt = R.copy() if R_tilde is None else R_tilde
    bnorm = _col_norms(B)
    hist = []
    k = 0
    while True:
        rel = np.max(_col_norms(R) / bnorm)
        hist.append(rel)
        if rel <= tol:
            return X, {"iterations": k, "status": "converged", "history": hist}
        if k >= max_iter:
            return X, {"iterations": k, "status": "maxiter", "history": hist}
        V = A(P)
        G = Rt.conj().T @ V
        try:
            alpha = np.linalg.solve(G, Rt.conj().T @ R)
        except np.linalg.LinAlgError:
            return X, {"iterations": k, "status": "breakdown", "history": hist}
        T = R - V @ alpha
        Z = A(T)
        den = np.vdot(Z, Z)
        zeta = 0.0 if den == 0 else np.vdot(Z, T) / den
        X = X + P @ alpha + zeta * T
        R = T - zeta * Z
        beta = np.linalg.solve(G, -(Rt.conj().T @ Z))
        P = R + (P - zeta * V) @ beta
        k += 1
        if not (np.all(np.isfinite(alpha)) and np.isfinite(zeta) and np.all(np.isfinite(beta))):
            return X, {"iterations": k, "status": "breakdown", "history": hist}
        if callback is not None:
            callback(k, {"X": X, "R": R, "P": P})


def block_bicggr(A, B: np.ndarray, tol: float, max_iter: int, X0=None, R_tilde=None, callback=None):
    """The new block method of Sec. 3 (Block BiCGGR), following its listing.

    The stabilisation scalar zeta_k is formed from R_k and W_k = A R_k (not from
    an intermediate T_k as in block BiCGSTAB); this is what makes the
    recursively updated R_k track B - A X_k.  Returns (X, info).
    """
    X = np.zeros_like(B) if X0 is None else X0.copy()
    R = B - A(X)
    P = R.copy()
    W = A(R)
    V = W.copy()
    Rt = R.copy() if R_tilde is None else R_tilde
    bnorm = _col_norms(B)
    hist = []
    k = 0
    while True:
        rel = np.max(_col_norms(R) / bnorm)
        hist.append(rel)
        if rel <= tol:
            return X, {"iterations": k, "status": "converged", "history": hist}
        if k >= max_iter:
            return X, {"iterations": k, "status": "maxiter", "history": hist}
        try:
            alpha = np.linalg.solve(Rt.conj().T @ V, Rt.conj().T @ R)
        except np.linalg.LinAlgError:
            return X, {"iterations": k, "status": "breakdown", "history": hist}
        zeta = np.vdot(W, R) / np.vdot(W, W)
        S = P - zeta * V
        U = S @ alpha
        Y = A(U)
        X = X + zeta * R + U
        R_new = R - zeta * W - Y
        W = A(R_new)
        try:
            gamma = np.linalg.solve(Rt.conj().T @ R, (Rt.conj().T @ R_new) / zeta)
        except np.linalg.LinAlgError:
            return X, {"iterations": k + 1, "status": "breakdown", "history": hist}
        P = R_new + U @ gamma
        V = W + Y @ gamma
        R = R_new
        k += 1
        if not (np.all(np.isfinite(alpha)) and np.isfinite(zeta) and np.all(np.isfinite(gamma))):
            return X, {"iterations": k, "status": "breakdown", "history": hist}
        if callback is not None:
            callback(k, {"X": X, "R": R, "P": P, "V": V, "W": W})


def true_residual(A, B: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Per-column ||A x^(i) - b^(i)||_2 / ||b^(i)||_2 (Sec. 4.3); the paper
    reports the max over i."""
    return _col_norms(A(X) - B) / _col_norms(B)


def sequential_bicgstab(A, B: np.ndarray, tol: float, max_iter: int, R_tilde=None):
    """L independent BiCGSTAB solves, one column at a time (the per-RHS
    baseline the block methods are compared against).  Column i of
    ``R_tilde``, if given, is the i-th solve's shadow residual."""
    X = np.zeros_like(B)
    iters = []
    status = "converged"
    for i in range(B.shape[1]):
        rt = None if R_tilde is None else R_tilde[:, i:i + 1]
        x, info = bicgstab(A, B[:, i:i + 1], tol, max_iter, r_tilde=rt)
        X[:, i:i + 1] = x
        iters.append(info["iterations"])
        if info["status"] != "converged":
            status = info["status"]
    return X, {"iterations": iters, "status": status}
