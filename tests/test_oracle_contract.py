"""Pins of the oracle's wall sources and meson two-point contraction (the propagator workflow of
Sec. III.B; conventions in oracle/contract.py) against closed forms and identities."""
import numpy as np
import pytest

import oracle
from oracle import contract
from tests import geometry as geo
import lattice_inputs as li


def _identity_prop(L):
    """S(x) = 1 (12 x 12) at every site."""
    V = int(np.prod(L))
    S = np.zeros((12, V, 4, 3), dtype=np.complex128)
    for k in range(12):
        S[k, :, k // 3, k % 3] = 1.0
    return S


@pytest.mark.parametrize("L", [(4, 4, 4, 8), (2, 6, 4, 4)])
def test_contract_identity_propagator_closed_forms(L):
    """S = 1: C(t) = Tr[G_snk G_src] * 3 * (sites per slice) at zero momentum, and 0 at any momentum
    that is not a multiple of the lattice (a full period of phases)."""
    S = _identity_prop(L)
    slice_sites = L[0] * L[1] * L[2]
    for a, b in ((15, 15), (4, 4), (15, 4), (1, 2), (3, 3)):
        expect = 3 * np.trace(oracle.gamma_bitmask(a) @ oracle.gamma_bitmask(b)) * slice_sites
        got = contract.meson_2pt(L, S, a, b)
        assert np.abs(got - expect).max() < 1e-12 * max(abs(expect), 1.0), (a, b)
    got = contract.meson_2pt(L, S, 15, 15, mom=(1, 0, 1))
    assert np.abs(got).max() < 1e-12 * slice_sites


def test_contract_pion_is_the_propagator_norm():
    """G_snk = G_src = g5 (g5^2 = 1): C(t) = sum_{x in t} e^{-ip.x} ||S(x)||_F^2, here checked with a
    plain loop over sites on a random S."""
    L = (4, 2, 2, 6)
    V = int(np.prod(L))
    rng = np.random.default_rng(5)
    S = rng.standard_normal((12, V, 4, 3)) + 1j * rng.standard_normal((12, V, 4, 3))
    c = geo.coords(L)
    for mom in ((0, 0, 0), (1, 1, 0)):
        p = 2 * np.pi * np.asarray(mom) / np.asarray(L[:3])
        expect = np.zeros(L[3], dtype=complex)
        for x in range(V):
            expect[c[x, 3]] += np.exp(-1j * c[x, :3] @ p) * np.sum(np.abs(S[:, x]) ** 2)
        assert np.abs(contract.meson_2pt(L, S, 15, 15, mom) - expect).max() < 1e-12 * np.abs(expect).max()


def test_contract_gamma_rotation_identity():
    """Tr is cyclic and g5 S^+ g5 enters linearly: replacing S by S U for a constant unitary U (a
    rotation of the source basis commuting with g5 and G_src) leaves C(t) unchanged."""
    L = (2, 2, 2, 4)
    V = int(np.prod(L))
    rng = np.random.default_rng(6)
    S = rng.standard_normal((12, V, 4, 3)) + 1j * rng.standard_normal((12, V, 4, 3))
    # a colour rotation on the source side commutes with every spin matrix
    Uc = np.linalg.qr(rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3)))[0]  # a unitary 3 x 3
    R = np.kron(np.eye(4), Uc)  # acts on k = 3 s0 + c0
    S2 = np.einsum("kxsc,kj->jxsc", S, R)
    for a, b in ((15, 15), (4, 1), (8, 7)):
        assert np.abs(contract.meson_2pt(L, S2, a, b) - contract.meson_2pt(L, S, a, b)).max() < 1e-11 * np.abs(
            contract.meson_2pt(L, S, a, b)).max()


def test_wall_sources_closed_form():
    """eta_k(x) = e^{ip.x} on slice t0, spin-colour k, zero elsewhere; summed over the slice with the
    conjugate phase it gives the slice volume."""
    L = (4, 4, 2, 6)
    t0, mom = 3, (1, 0, 1)
    eta = contract.wall_sources(L, t0, mom)
    c = geo.coords(L)
    p = 2 * np.pi * np.asarray(mom) / np.asarray(L[:3])
    for k in (0, 5, 11):
        f = eta[k]
        assert np.abs(f[c[:, 3] != t0]).max() == 0
        others = [j for j in range(12) if j != k]
        assert np.abs(f.reshape(-1, 12)[:, others]).max() == 0
        v = f.reshape(-1, 12)[:, k]
        assert abs(np.sum(v * np.exp(-1j * c[:, :3] @ p)) - L[0] * L[1] * L[2]) < 1e-12


def test_three_point_sequential_matches_dense_double_sum():
    """The sequential route (eta from S on the sink slice, T = M^{-1} eta, then one trace per y) equals
    the explicit double sum over the sink and insertion slices of Tr[Gamma_f D^{-1}(x,y) G_ins
    D^{-1}(y,0) G_src D^{-1}(0,x)], with D^{-1} the dense inverse of the Dirac matrix (2^2 x 4^2)."""
    L = (2, 2, 4, 4)
    V = int(np.prod(L))
    U = li.random_gauge(L, 0.3, 61)
    C = oracle.clover_build(L, U)
    kappa, csw = 0.11, 1.0
    Dinv = np.linalg.inv(oracle.dense_matrix(L, U, C, kappa, csw))
    # S(y <- 0): the 12 columns of the origin (eo index 0)
    S = Dinv[:, :12].T.reshape(12, V, 4, 3)
    c = geo.coords(L)
    t_f, g_f, g_ins, g_src, pf, q = 3, 15, 8, 15, (0, 1, 1), (1, 0, 0)
    eta = contract.seq_sources(L, S, t_f, g_f, pf)
    T = (Dinv @ eta.reshape(12, V * 12).T).T.reshape(12, V, 4, 3)
    got = contract.contract(L, S, T, g_ins, g_src, q)
    G = [oracle.gamma_bitmask(n) for n in (g_f, g_ins, g_src)]
    blk = lambda a, b: Dinv[12 * a:12 * a + 12, 12 * b:12 * b + 12]  # noqa: E731
    I3 = np.eye(3)
    Gf, Gi, Gs = (np.kron(g, I3) for g in G)
    pp = 2 * np.pi * np.asarray(pf) / np.asarray(L[:3])
    qq = 2 * np.pi * np.asarray(q) / np.asarray(L[:3])
    expect = np.zeros(L[3], dtype=complex)
    for x in np.nonzero(c[:, 3] == t_f)[0]:
        for y in range(V):
            expect[c[y, 3]] += np.exp(-1j * (c[x, :3] @ pp)) * np.exp(-1j * (c[y, :3] @ qq)) * np.trace(
                Gf @ blk(x, y) @ Gi @ blk(y, 0) @ Gs @ blk(0, x))
    assert np.abs(got - expect).max() < 1e-11 * np.abs(expect).max()
