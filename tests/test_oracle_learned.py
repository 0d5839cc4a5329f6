"""Pins of the learned-preconditioner oracle (oracle/learned.py)."""
import numpy as np
import pytest

import lattice_inputs as li
import oracle
from oracle import learned as ln
from tests import geometry as geo


def _rand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_hop_weights_reproduce_the_wilson_hop():
    """A 4-channel layer with W_{+mu} = 1 - g_mu, W_{-mu} = 1 + g_mu (channels = spins) is H."""
    L = (4, 2, 6, 4)
    U = li.random_gauge(L, 0.4, 3)
    V = int(np.prod(L))
    W = np.zeros((9, 4, 4), dtype=complex)
    for mu in range(4):
        g = oracle.gamma(mu)
        W[1 + 2 * mu] = np.eye(4) - g
        W[2 + 2 * mu] = np.eye(4) + g
    psi = li.gaussian_source(L, 4)
    phi = np.transpose(psi.reshape(V, 4, 3), (1, 0, 2))
    out = ln.layer_forward(ln.Transport(L, U), W, phi)
    expect = oracle.hop(L, U, psi)
    assert np.abs(np.transpose(out, (1, 0, 2)).reshape(psi.shape) - expect).max() < 1e-13


def test_adjoint_layer_is_the_adjoint():
    rng = np.random.default_rng(5)
    L = (4, 4, 2, 4)
    T = ln.Transport(L, li.random_gauge(L, 0.5, 6))
    W = _rand(rng, 9, 5, 3)
    phi = _rand(rng, 3, T.V, 3)
    g = _rand(rng, 5, T.V, 3)
    lhs = np.vdot(g, ln.layer_forward(T, W, phi))
    rhs = np.vdot(ln.layer_adjoint(T, W, g), phi)
    assert abs(lhs - rhs) / abs(lhs) < 1e-13


def test_net_gauge_equivariance():
    """P(Om r)[Om U Om^+] = Om P(r)[U] for Haar-random Om."""
    rng = np.random.default_rng(7)
    L = (4, 4, 2, 4)
    V = int(np.prod(L))
    U = li.random_gauge(L, 0.5, 8)
    Om = li.gauge_transform(L, 9).reshape(V, 3, 3)
    Uf = U.reshape(4, V, 3, 3)
    Up = np.empty_like(Uf)
    for mu in range(4):
        fw = geo.shift_table(L, mu, +1)
        Up[mu] = Om @ Uf[mu] @ np.conj(np.swapaxes(Om[fw], -1, -2))
    W1, W2 = _rand(rng, 9, 6, 4), _rand(rng, 9, 4, 6)
    r = _rand(rng, V // 2, 4, 3)
    rp = np.einsum("xab,xsb->xsa", Om[: V // 2], r)
    lhs = ln.net_apply(ln.Transport(L, Up), W1, W2, rp)
    rhs = np.einsum("xab,xsb->xsa", Om[: V // 2], ln.net_apply(ln.Transport(L, U), W1, W2, r))
    assert np.abs(lhs - rhs).max() / np.abs(rhs).max() < 1e-13


def test_gradients_match_central_differences():
    rng = np.random.default_rng(11)
    L = (4, 2, 2, 4)
    V = int(np.prod(L))
    T = ln.Transport(L, li.random_gauge(L, 0.4, 12))
    W1, W2 = 0.3 * _rand(rng, 9, 12, 4), 0.3 * _rand(rng, 9, 4, 12)
    pairs = [(_rand(rng, V // 2, 4, 3), _rand(rng, V // 2, 4, 3)) for _ in range(2)]
    loss, G1, G2 = ln.net_loss_and_grad(T, W1, W2, pairs)
    h = 1e-6
    for W, G, name in ((W1, G1, "W1"), (W2, G2, "W2")):
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in W.shape)
            for part, unit in (("re", 1.0), ("im", 1j)):
                Wp, Wm = W.copy(), W.copy()
                Wp[idx] += h * unit
                Wm[idx] -= h * unit
                args_p = (Wp, W2) if name == "W1" else (W1, Wp)
                args_m = (Wm, W2) if name == "W1" else (W1, Wm)
                fd = (ln.net_loss_and_grad(T, *args_p, pairs)[0] - ln.net_loss_and_grad(T, *args_m, pairs)[0]) / (2 * h)
                an = G[idx].real if part == "re" else G[idx].imag
                assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (name, idx, part, fd, an)


def test_identity_weights_give_identity_map():
    L = (4, 2, 2, 4)
    V = int(np.prod(L))
    T = ln.Transport(L, li.random_gauge(L, 0.4, 13))
    W1 = np.zeros((9, 4, 4), dtype=complex)
    W1[0] = np.eye(4)
    r = li.gaussian_source(L, 14).reshape(V, 4, 3)[: V // 2]
    assert np.abs(ln.net_apply(T, W1, W1, r) - r).max() == 0.0
