"""Pins of the oracle's clover fermion force (paper Sec. IV, the force of the clover fermion actions in
HMC) against what the mathematics fixes."""
import numpy as np
import pytest
from scipy.linalg import expm

import lattice_inputs as li
import oracle
from oracle import force as of
from tests import geometry as geo


def _fields(L, seed):
    return li.gaussian_source(L, seed), li.gaussian_source(L, seed + 1)


def _with_link(U, mu, i, m):
    V = int(np.prod(U.shape[1:-2]))
    Uf = U.reshape(4, V, 3, 3).copy()
    Uf[mu, i] = m
    return Uf.reshape(U.shape)


def test_generators_normalised():
    T = of.generators()
    for a in range(8):
        assert np.allclose(T[a], T[a].conj().T) and abs(np.trace(T[a])) < 1e-15
        for b in range(8):
            assert abs(np.trace(T[a] @ T[b]) - 0.5 * (a == b)) < 1e-15


@pytest.mark.parametrize("L,t_bc", [((4, 4, 2, 4), 1), ((2, 4, 4, 2), -1)])
def test_operator_is_affine_in_one_link(L, t_bc):
    """M(U + t V) X is affine in t for a change V of one link, the premise of the secant derivative: the
    second difference vanishes to rounding, while the first is of order one."""
    U = li.random_gauge(L, 0.4, 3)
    X, _ = _fields(L, 4)
    rng = np.random.default_rng(5)
    V = int(np.prod(L))
    for mu, i in ((0, 3), (3, V - 1), (2, V // 2 + 1)):
        D = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
        u = U.reshape(4, V, 3, 3)[mu, i]
        m0 = of.operator_apply(L, U, X, 0.12, 1.3, t_bc)
        m1 = of.operator_apply(L, _with_link(U, mu, i, u + D), X, 0.12, 1.3, t_bc)
        m2 = of.operator_apply(L, _with_link(U, mu, i, u + 2 * D), X, 0.12, 1.3, t_bc)
        first = np.linalg.norm(m1 - m0)
        assert first > 1e-3
        assert np.linalg.norm(m2 - 2 * m1 + m0) < 1e-13 * first


@pytest.mark.parametrize("t_bc", [1, -1])
def test_force_matches_group_finite_difference(t_bc):
    """F^a = 2 Tr(T^a H) equals the central difference of B along exp(+-i eps T^a) U_mu(x) (error O(eps^2))."""
    L = (4, 2, 4, 4)
    U = li.random_gauge(L, 0.4, 6)
    X, Y = _fields(L, 7)
    kappa, csw = 0.12, 1.2
    V = int(np.prod(L))
    links = [(0, 0), (1, 5), (2, V - 3), (3, V // 2 + 7), (3, 2)]
    H = of.force(L, U, X, Y, kappa, csw, t_bc, links).reshape(4, V, 3, 3)
    T = of.generators()
    eps = 1e-5
    for mu, i in links:
        u = U.reshape(4, V, 3, 3)[mu, i]
        for a in (0, 2, 4, 7):
            bp = of.bilinear(L, _with_link(U, mu, i, expm(1j * eps * T[a]) @ u), X, Y, kappa, csw, t_bc)
            bm = of.bilinear(L, _with_link(U, mu, i, expm(-1j * eps * T[a]) @ u), X, Y, kappa, csw, t_bc)
            fd = (bp - bm) / (2 * eps)
            fa = 2 * np.trace(T[a] @ H[mu, i]).real
            assert abs(fd - fa) <= 1e-7 * max(1.0, abs(fa)), (mu, i, a, fd, fa)


def test_two_flavour_hmc_force():
    """S = phi^+ (M^+ M)^-1 phi from dense solves: dS/dw^a along exp(i w T^a) U_mu(x) is -F^a for
    X = (M^+ M)^-1 phi, Y = M X (the force an HMC integrator applies)."""
    L = (4, 2, 2, 4)
    U = li.random_gauge(L, 0.4, 8)
    kappa, csw = 0.12, 1.1
    phi = li.gaussian_source(L, 9)

    def action(Ul):
        M = oracle.dense_matrix(L, Ul, oracle.clover_build(L, Ul), kappa, csw)
        p = phi.reshape(-1)
        return np.vdot(p, np.linalg.solve(M.conj().T @ M, p)).real, M

    S0, M = action(U)
    X = np.linalg.solve(M.conj().T @ M, phi.reshape(-1)).reshape(phi.shape)
    Y = (M @ X.reshape(-1)).reshape(phi.shape)
    V = int(np.prod(L))
    links = [(0, 1), (3, V - 2), (1, V // 2)]
    H = of.force(L, U, X, Y, kappa, csw, 1, links).reshape(4, V, 3, 3)
    T = of.generators()
    eps = 1e-5
    for mu, i in links:
        u = U.reshape(4, V, 3, 3)[mu, i]
        for a in (1, 3, 6):
            sp, _ = action(_with_link(U, mu, i, expm(1j * eps * T[a]) @ u))
            sm, _ = action(_with_link(U, mu, i, expm(-1j * eps * T[a]) @ u))
            fd = (sp - sm) / (2 * eps)
            fa = 2 * np.trace(T[a] @ H[mu, i]).real
            assert abs(fd + fa) <= 1e-6 * max(1.0, abs(fa)), (mu, i, a, fd, fa)


def test_force_gauge_covariant_and_hermitian_traceless():
    """U'_mu(x) = Om(x) U_mu(x) Om(x+mu)^+, X' = Om X, Y' = Om Y give H'_mu(x) = Om(x) H_mu(x) Om(x)^+
    (the variation multiplies the link from the left, at its base site); H is Hermitian and traceless."""
    L = (2, 4, 2, 4)
    U = li.random_gauge(L, 0.4, 10)
    X, Y = _fields(L, 11)
    Om = li.gauge_transform(L, 12)
    Up = geo.transform_gauge(L, U, Om)
    Of = Om.reshape(2, L[3], L[2], L[1], L[0] // 2, 3, 3)
    Xp = np.einsum("...ab,...sb->...sa", Of, X)
    Yp = np.einsum("...ab,...sb->...sa", Of, Y)
    V = int(np.prod(L))
    links = [(0, 0), (1, 9), (2, V - 1), (3, V // 2)]
    H = of.force(L, U, X, Y, 0.125, 1.0, 1, links).reshape(4, V, 3, 3)
    Hp = of.force(L, Up, Xp, Yp, 0.125, 1.0, 1, links).reshape(4, V, 3, 3)
    Ov = Om.reshape(V, 3, 3)
    for mu, i in links:
        h = H[mu, i]
        assert np.abs(h - h.conj().T).max() < 1e-14 * np.abs(h).max() and abs(np.trace(h)) < 1e-13
        assert np.abs(Hp[mu, i] - Ov[i] @ h @ Ov[i].conj().T).max() < 1e-12 * np.abs(h).max()
