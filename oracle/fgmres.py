"""CPU oracle of flexible GMRES, FGMRES(m) (Saad 1993, SIAM J. Sci. Comput. 14, 461), plain NumPy, FP64.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Right-preconditioned GMRES in which the preconditioner may change from one
Arnoldi step to the next: z_j = P_j(v_j), w = A z_j, orthogonalised against
v_0..v_j by modified Gram-Schmidt (the Arnoldi step of the published algorithm),
h_{j+1,j} = ||w||, v_{j+1} = w / h_{j+1,j}.  After k steps the iterate is
x_0 + Z_k y with y minimising ||beta e_1 - Hbar_k y|| (the small least-squares
problem, solved here with the library's lstsq), which by the flexible Arnoldi
relation A Z_k = V_{k+1} Hbar_k equals min ||b - A x|| over x in x_0 + span Z_k.
A cycle ends after m steps (or when the least-squares residual reaches the
tolerance), x is updated and the residual is recomputed from it (restart).

The solver the learned preconditioner is used in (spec configuration 5);
pinned by the exact solution of a small dense system, the minimal-residual
property against a brute-force least-squares fit over the Krylov space, the
flexible Arnoldi relation, and one-step convergence with the exact inverse as
preconditioner (tests/test_oracle_fgmres.py).
"""
from __future__ import annotations

import numpy as np


class FgmresResult:
    def __init__(self, x, iters, cycles, hist, basis):
        self.x = x
        self.iters = iters      # Arnoldi steps over all cycles
        self.cycles = cycles
        self.hist = hist        # ||r|| / norm_ref at the start, then the least-squares residual after each step
        self.basis = basis      # (V, Z, Hbar) of the last cycle


def fgmres(A, b, precond=None, m: int = 32, tol: float = 1e-10, maxiter: int = 1000, x0=None,
           norm_ref: float | None = None) -> FgmresResult:
    """Solve A x = b.  A(v) -> A v; precond(j, v) -> z_j (None: z_j = v_j, plain GMRES).  Stops when the
    residual is <= tol * norm_ref (norm_ref defaults to ||b||) or after maxiter Arnoldi steps."""
    b = np.asarray(b, dtype=np.complex128)
    shape = b.shape
    bf = b.reshape(-1)
    ref = float(np.linalg.norm(bf)) if norm_ref is None else float(norm_ref)
    x = np.zeros_like(bf) if x0 is None else np.asarray(x0, dtype=np.complex128).reshape(-1).copy()

    def op(v):
        return np.asarray(A(v.reshape(shape)), dtype=np.complex128).reshape(-1)

    def pre(j, v):
        if precond is None:
            return v
        return np.asarray(precond(j, v.reshape(shape)), dtype=np.complex128).reshape(-1)

    r = bf - op(x)
    beta = float(np.linalg.norm(r))
    hist = [beta / ref]
    iters = cycles = 0
    basis = None
    while beta > tol * ref and iters < maxiter:
        V = [r / beta]
        Z = []
        H = np.zeros((m + 1, m), dtype=np.complex128)
        y = np.zeros(0, dtype=np.complex128)
        k = 0
        for j in range(m):
            if iters >= maxiter:
                break
            z = pre(j, V[j])
            Z.append(z)
            w = op(z)
            for i in range(j + 1):
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            iters += 1
            k = j + 1
            e1 = np.zeros(j + 2, dtype=np.complex128)
            e1[0] = beta
            y = np.linalg.lstsq(H[: j + 2, : j + 1], e1, rcond=None)[0]
            res = float(np.linalg.norm(e1 - H[: j + 2, : j + 1] @ y))
            hist.append(res / ref)
            if H[j + 1, j] == 0 or res <= tol * ref:
                break
            V.append(w / H[j + 1, j])
        if k == 0:
            break
        x = x + np.stack(Z[:k], axis=1) @ y
        cycles += 1
        basis = (np.stack(V[: k + 1], axis=1) if len(V) > k else np.stack(V, axis=1), np.stack(Z[:k], axis=1),
                 H[: k + 1, :k].copy())
        r = bf - op(x)
        beta = float(np.linalg.norm(r))
    return FgmresResult(x.reshape(shape), iters, cycles, np.asarray(hist), basis)
