"""The three Krylov solvers of Sec. 3 and the true residual of Sec. 4.3, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

A is any callable mapping an (N, L) complex array to A times it.  Blocks are
(N, L) arrays whose column i is x^(i) (Sec. 3).

All three methods are product-type Lanczos methods: the residual is a
stabilising polynomial in A (built from one scalar per iteration, chosen to
minimise a residual norm) applied to the residual of block BiCG (whose L x L
coefficient matrices make a block orthogonal to the shadow block R~_0).  Each
iteration is written here as two halves with a common driver:

* ``step``: the BiCG coefficients alpha_k, the scalar zeta_k, the new
  iterate X_{k+1} and its recursively updated residual R_{k+1};
* ``directions``: the coefficients of the next search block (beta_k, or
  gamma_k for the new method) and the blocks the next iteration needs.

Readings of points the paper leaves open:

* initial guess X_0 = 0 unless one is passed;
* shadow residual R~_0 = R_0 unless one is passed;
* inner product (x, y) = x^H y (conjugate on the first argument), consistent
  with the block methods' R~_0^H (.);
* the stop test max_i ||r_k^(i)|| / ||b^(i)|| <= eps is made at the top of
  each iteration; ``iterations`` counts completed iterations (a breakdown in
  the second half of an iteration counts that iteration);
* L x L systems are solved by LU with partial pivoting (numpy.linalg.solve);
* BiCGSTAB degenerate step: if A t_k = 0 exactly (t_k = 0, the iterate is
  already exact) zeta_k is taken as 0 instead of 0/0, so the next stop test
  ends the loop.  The same for Tr(Z^H Z) = 0 in block BiCGSTAB;
* a singular L x L system or a non-finite scalar is a breakdown; the solver
  returns the last iterate with status "breakdown".
"""
import numpy as np


class _Breakdown(Exception):
    pass


def _col_norms(M: np.ndarray) -> np.ndarray:
    return np.sqrt(np.sum(np.abs(M) ** 2, axis=0))


def _shadow_solve(Rt: np.ndarray, M: np.ndarray, rhs: np.ndarray) -> np.ndarray:
    """The L x L matrix C with (R~^H M) C = rhs; singular -> breakdown."""
    try:
        return np.linalg.solve(Rt.conj().T @ M, rhs)
    except np.linalg.LinAlgError:
        raise _Breakdown from None


def _min_residual_scalar(Z: np.ndarray, T: np.ndarray):
    """The scalar zeta that minimises ||T - zeta Z||_F, i.e. (Z, T) / (Z, Z)
    with the Frobenius inner product; 0 for Z = 0 (see the module readings)."""
    den = np.vdot(Z, Z)
    return 0.0 if den == 0 else np.vdot(Z, T) / den


def _all_finite(*xs) -> bool:
    return all(np.all(np.isfinite(x)) for x in xs)


def _drive(method, B: np.ndarray, tol: float, max_iter: int, callback):
    """Common iteration loop: stop test on the recursively updated residual,
    the two halves of an iteration, breakdown and non-finite detection."""
    bnorm = _col_norms(B)
    hist = []
    k = 0
    while True:
        rel = np.max(_col_norms(method.R) / bnorm)
        hist.append(rel)
        if rel <= tol:
            status = "converged"
            break
        if k >= max_iter:
            status = "maxiter"
            break
        try:
            method.step()
            k += 1
            method.directions()
        except _Breakdown:
            status = "breakdown"
            break
        if not method.finite():
            status = "breakdown"
            break
        if callback is not None:
            callback(k, method.view())
    return method.X, {"iterations": k, "status": status, "history": hist}


class _BiCGStab:
    """BiCGSTAB for one right-hand side (Sec. 3): BiCG's scalar recurrences
    with residual r_{k+1} = (1 - zeta_k A) (r_k - alpha_k A p_k)."""

    def __init__(self, A, b, x0, r_tilde):
        self.A = A
        self.X = np.zeros_like(b) if x0 is None else x0.reshape(-1, 1).copy()
        self.R = b - A(self.X)
        self.P = self.R.copy()
        self.Rt = self.R.copy() if r_tilde is None else r_tilde.reshape(-1, 1)

    def step(self):
        A, Rt = self.A, self.Rt
        self.AP = A(self.P)
        self.rho = np.vdot(Rt, self.R)                 # (r~, r_k)
        self.alpha = self.rho / np.vdot(Rt, self.AP)   # BiCG: (r~, r_k - alpha A p_k) = 0
        T = self.R - self.alpha * self.AP
        AT = A(T)
        self.zeta = _min_residual_scalar(AT, T)
        self.X = self.X + self.alpha * self.P + self.zeta * T
        self.R = T - self.zeta * AT

    def directions(self):
        z = self.zeta
        self.beta = 0.0 if z == 0 else (self.alpha / z) * np.vdot(self.Rt, self.R) / self.rho
        self.P = self.R + self.beta * (self.P - z * self.AP)

    def finite(self):
        return _all_finite(self.alpha, self.zeta, self.beta)

    def view(self):
        return {"x": self.X, "r": self.R, "p": self.P}


class _BlockBiCGStab:
    """Block BiCGSTAB (Sec. 3): L x L BiCG coefficients against R~_0 and one
    stabilising scalar per iteration, minimising ||T_k - zeta A T_k||_F."""

    def __init__(self, A, B, X0, R_tilde):
        self.A = A
        self.X = np.zeros_like(B) if X0 is None else X0.copy()
        self.R = B - A(self.X)
        self.P = self.R.copy()
        self.Rt = self.R.copy() if R_tilde is None else R_tilde

    def step(self):
        A, Rt = self.A, self.Rt
        self.V = A(self.P)
        self.alpha = _shadow_solve(Rt, self.V, Rt.conj().T @ self.R)   # R~^H (R_k - V alpha) = 0
        T = self.R - self.V @ self.alpha
        self.Z = A(T)
        self.zeta = _min_residual_scalar(self.Z, T)
        self.X = self.X + self.P @ self.alpha + self.zeta * T
        self.R = T - self.zeta * self.Z

    def directions(self):
        Rt = self.Rt
        # same matrix R~^H A P_k as for alpha_k
        self.beta = _shadow_solve(Rt, self.V, -(Rt.conj().T @ self.Z))
        self.P = self.R + (self.P - self.zeta * self.V) @ self.beta

    def finite(self):
        return _all_finite(self.alpha, self.zeta, self.beta)

    def view(self):
        return {"X": self.X, "R": self.R, "P": self.P}


class _BlockBiCGGR:
    """Block BiCGGR, the new method of Sec. 3.  It carries W_k = A R_k and
    V_k = A P_k alongside R_k and P_k; the stabilising scalar minimises
    ||R_k - zeta W_k||_F, and the update of X_k and R_k uses the same block
    U_k = (P_k - zeta_k V_k) alpha_k and its product Y_k = A U_k, which is
    what keeps the recursive R_k close to B - A X_k in finite precision."""

    def __init__(self, A, B, X0, R_tilde):
        self.A = A
        self.X = np.zeros_like(B) if X0 is None else X0.copy()
        self.R = B - A(self.X)
        self.P = self.R.copy()
        self.W = A(self.R)
        self.V = self.W.copy()
        self.Rt = self.R.copy() if R_tilde is None else R_tilde

    def step(self):
        Rt = self.Rt
        self.alpha = _shadow_solve(Rt, self.V, Rt.conj().T @ self.R)
        self.zeta = np.vdot(self.W, self.R) / np.vdot(self.W, self.W)
        self.U = (self.P - self.zeta * self.V) @ self.alpha
        self.Y = self.A(self.U)
        self.X = self.X + self.zeta * self.R + self.U
        self.R_prev = self.R
        self.R = self.R - self.zeta * self.W - self.Y
        self.W = self.A(self.R)

    def directions(self):
        Rt = self.Rt
        self.gamma = _shadow_solve(Rt, self.R_prev, (Rt.conj().T @ self.R) / self.zeta)
        self.P = self.R + self.U @ self.gamma
        self.V = self.W + self.Y @ self.gamma

    def finite(self):
        return _all_finite(self.alpha, self.zeta, self.gamma)

    def view(self):
        return {"X": self.X, "R": self.R, "P": self.P, "V": self.V, "W": self.W}


def bicgstab(A, b: np.ndarray, tol: float, max_iter: int, x0=None, r_tilde=None, callback=None):
    """BiCGSTAB for one right-hand side (Sec. 3).  ``b`` is an (N,) or (N, 1)
    vector.  Returns (x, info) with x of b's shape."""
    shape = b.shape
    x, info = _drive(_BiCGStab(A, b.reshape(-1, 1), x0, r_tilde), b.reshape(-1, 1), tol, max_iter, callback)
    return x.reshape(shape), info


def block_bicgstab(A, B: np.ndarray, tol: float, max_iter: int, X0=None, R_tilde=None, callback=None):
    """Block BiCGSTAB (Sec. 3).  Returns (X, info)."""
    return _drive(_BlockBiCGStab(A, B, X0, R_tilde), B, tol, max_iter, callback)


def block_bicggr(A, B: np.ndarray, tol: float, max_iter: int, X0=None, R_tilde=None, callback=None):
    """Block BiCGGR (Sec. 3).  Returns (X, info)."""
    return _drive(_BlockBiCGGR(A, B, X0, R_tilde), B, tol, max_iter, callback)


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
