"""Pins of the oracle's flexible GMRES (Saad 1993) against what the mathematics fixes."""
import numpy as np
import pytest

from oracle.fgmres import fgmres


def _system(n, seed, spread=0.4):
    rng = np.random.default_rng(seed)
    G = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2 * n)
    A = np.eye(n) + spread * G
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return A, b


def test_full_cycle_solves_a_dense_system_exactly():
    """With m >= n and no preconditioner the Krylov space is the whole space: one cycle gives the exact
    solution (to rounding), in at most n steps."""
    A, b = _system(40, 1)
    res = fgmres(lambda v: A @ v, b, m=40, tol=1e-13, maxiter=40)
    assert res.iters <= 40 and res.cycles == 1
    x = np.linalg.solve(A, b)
    assert np.linalg.norm(res.x - x) / np.linalg.norm(x) < 1e-12


@pytest.mark.parametrize("k", [1, 3, 6])
def test_minimal_residual_over_the_krylov_space(k):
    """After k steps from x0 = 0 the residual (the reported least-squares value) is the minimum of
    ||b - A x|| over x in span{b, A b, ..., A^(k-1) b}, found here by brute force: an orthonormal basis
    of the explicit Krylov matrix and a least-squares fit."""
    A, b = _system(30, 2, spread=0.8)
    res = fgmres(lambda v: A @ v, b, m=k, tol=1e-16, maxiter=k)
    K = np.stack([np.linalg.matrix_power(A, i) @ b for i in range(k)], axis=1)
    Q, _ = np.linalg.qr(K)
    c = np.linalg.lstsq(A @ Q, b, rcond=None)[0]
    best = np.linalg.norm(b - A @ Q @ c)
    assert abs(res.hist[k] * np.linalg.norm(b) - best) <= 1e-10 * best
    assert abs(np.linalg.norm(b - A @ res.x) - best) <= 1e-10 * best


def test_flexible_arnoldi_relation_with_a_changing_preconditioner():
    """A preconditioner that differs at every step (random matrices P_j): the flexible Arnoldi relation
    A Z_k = V_{k+1} Hbar_k holds with orthonormal V, and the iterate minimises ||b - A x|| over span Z_k."""
    n, k = 24, 7
    A, b = _system(n, 3, spread=0.9)
    rng = np.random.default_rng(4)
    P = [np.eye(n) + 0.3 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
         for _ in range(k)]
    res = fgmres(lambda v: A @ v, b, precond=lambda j, v: P[j] @ v, m=k, tol=1e-16, maxiter=k)
    V, Z, H = res.basis
    assert np.abs(V.conj().T @ V - np.eye(V.shape[1])).max() < 1e-12
    assert np.abs(A @ Z - V @ H).max() < 1e-12
    for j in range(k):  # z_j = P_j v_j
        assert np.abs(Z[:, j] - P[j] @ V[:, j]).max() < 1e-13
    c = np.linalg.lstsq(A @ Z, b, rcond=None)[0]
    best = np.linalg.norm(b - A @ Z @ c)
    assert abs(np.linalg.norm(b - A @ res.x) - best) <= 1e-10 * best


def test_exact_inverse_as_preconditioner_converges_in_one_step():
    A, b = _system(20, 5)
    Ainv = np.linalg.inv(A)
    res = fgmres(lambda v: A @ v, b, precond=lambda j, v: Ainv @ v, m=5, tol=1e-12, maxiter=5)
    assert res.iters == 1
    assert np.linalg.norm(b - A @ res.x) / np.linalg.norm(b) < 1e-13


def test_restarts_reach_the_tolerance():
    """GMRES(4) on a system that needs more than one cycle: the residual after each restart is
    recomputed from x and the solve ends below tol."""
    A, b = _system(60, 6, spread=0.6)
    res = fgmres(lambda v: A @ v, b, m=4, tol=1e-11, maxiter=400)
    assert res.cycles > 1
    assert np.linalg.norm(b - A @ res.x) / np.linalg.norm(b) <= 1e-11
    # the least-squares residuals never increase within a cycle
    h = res.hist
    assert np.all(np.diff(h[1:5]) <= 1e-15)
