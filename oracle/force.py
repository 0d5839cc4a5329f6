"""CPU oracle of the clover fermion force, plain NumPy over the oracle's operator, FP64.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Hybrid Monte Carlo with clover fermions (paper Sec. IV: the clover fermion actions of the N_f = 2 + 1
example, integrated by molecular dynamics) moves the links along the force, the derivative of the
pseudo-fermion action.  For the two-flavour action S = phi^+ (M^+ M)^-1 phi, with X = (M^+ M)^-1 phi
and Y = M X, a variation of the links changes S by -[2 Re(Y^+ dM X)]; a rational approximation
(the multi-shift solves) is a sum of such terms.  So the quantity a force kernel computes is the
derivative of the bilinear B(U) = 2 Re(Y^+ M(U) X) at fixed X, Y along each link and generator:

  F^a_mu(x) = d/dw B(U_w) at w = 0,  U_w: U_mu(x) -> exp(i w T^a) U_mu(x), every other link fixed,

with T^a = lambda^a / 2 (Gell-Mann, Tr T^a T^b = delta^ab / 2), returned as the Hermitian traceless
matrix H_mu(x) = sum_a F^a T^a (so F^a = 2 Tr(T^a H)).

Plain definition used here: M (the hop term and the clover term A = 1 - kappa csw C of Eq. "clover",
C built from the four-leaf F) is real-affine in any single link, because each clover leaf contains a
given link at most once (for every extent >= 2) and the hop term is linear.  The directional
derivative along V = i T^a U_mu(x) is therefore exactly M(U + V) - M(U), and
F^a = 2 Re(Y^+ [M(U + V) - M(U)] X), computed with the oracle's own clover builder and operator.

Pins (tests/test_oracle_force.py): the affinity itself; a central finite difference along the group
direction exp(i eps T^a); the HMC force of the two-flavour action against a finite difference of S
from dense solves; gauge covariance H'_mu(x) = Om(x) H_mu(x) Om(x)^+; Hermitian traceless output.
"""
from __future__ import annotations

import numpy as np

import oracle


def generators() -> np.ndarray:
    """T^a = lambda^a / 2, a = 0..7 (Gell-Mann matrices)."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1], lam[1][1, 0] = -1j, 1j
    lam[2][0, 0], lam[2][1, 1] = 1, -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2], lam[4][2, 0] = -1j, 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2], lam[6][2, 1] = -1j, 1j
    lam[7] = np.diag([1, 1, -2]) / np.sqrt(3)
    return lam / 2


def operator_apply(L, U, X, kappa: float, csw: float, t_bc: int = 1) -> np.ndarray:
    """M(U) X with the clover term built from the given links (which need not be unitary)."""
    return oracle.dirac(L, U, oracle.clover_build(L, U), X, kappa, csw, t_bc)


def bilinear(L, U, X, Y, kappa: float, csw: float, t_bc: int = 1) -> float:
    """B(U) = 2 Re(Y^+ M(U) X)."""
    return 2.0 * np.vdot(Y, operator_apply(L, U, X, kappa, csw, t_bc)).real


def force(L, U, X, Y, kappa: float, csw: float, t_bc: int = 1, links=None) -> np.ndarray:
    """H_mu(x) = sum_a T^a F^a_mu(x) for the links (mu, eo site) in `links` (all links when None), zero for
    the others; shape of the gauge layout."""
    V = int(np.prod(L))
    Uf = np.ascontiguousarray(U, dtype=np.complex128).reshape(4, V, 3, 3)
    T = generators()
    base = operator_apply(L, U, X, kappa, csw, t_bc)
    H = np.zeros((4, V, 3, 3), dtype=np.complex128)
    if links is None:
        links = [(mu, i) for mu in range(4) for i in range(V)]
    for mu, i in links:
        for a in range(8):
            Up = Uf.copy()
            Up[mu, i] = Uf[mu, i] + 1j * T[a] @ Uf[mu, i]
            d = operator_apply(L, Up.reshape(U.shape), X, kappa, csw, t_bc) - base
            H[mu, i] += 2.0 * np.vdot(Y, d).real * T[a]
    return H.reshape(np.shape(U))
