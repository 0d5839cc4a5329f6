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


# ---------------------------------------------------------------------------
# Adam (Kingma and Ba 2015): closed forms that follow from the algorithm's definition
# ---------------------------------------------------------------------------
def _adam_run(W0, grads, lr, eps=ln.ADAM_EPS):
    st = ln.AdamState(W0.shape)
    W = W0.copy()
    out = []
    for G in grads:
        W = ln.adam_step(W, G, st, lr, eps=eps)
        out.append(W.copy())
    return out


def test_adam_first_step_is_a_signed_step_of_size_lr():
    """With bias correction m_hat = g and v_hat = g^2 after one step, so each real parameter moves
    by -lr g / (|g| + eps), independently for the real and imaginary parts."""
    rng = np.random.default_rng(20)
    W0 = _rand(rng, 9, 4, 3)
    G = _rand(rng, 9, 4, 3) * np.exp(rng.uniform(-6, 2, (9, 4, 3)))
    lr = 3e-3
    (W1,) = _adam_run(W0, [G], lr)
    expect = W0 - lr * (G.real / (np.abs(G.real) + ln.ADAM_EPS) + 1j * G.imag / (np.abs(G.imag) + ln.ADAM_EPS))
    assert np.abs(W1 - expect).max() < 1e-15


def test_adam_constant_gradient_moves_linearly():
    """For a constant gradient both bias-corrected moments equal g and g^2 at every step, so the
    t-th iterate is W0 - t lr g / (|g| + eps): this fixes the powers of beta1 and beta2."""
    rng = np.random.default_rng(21)
    W0 = _rand(rng, 3, 5)
    G = _rand(rng, 3, 5)
    lr = 1e-3
    Ws = _adam_run(W0, [G] * 7, lr)
    unit = G.real / (np.abs(G.real) + ln.ADAM_EPS) + 1j * G.imag / (np.abs(G.imag) + ln.ADAM_EPS)
    for t, W in enumerate(Ws, 1):
        assert np.abs(W - (W0 - t * lr * unit)).max() < 1e-14, t


def test_adam_reversed_second_gradient():
    """Gradients g then -g: m_2 = -(1 - b1)^2 g, so m_hat = -(1 - b1) g / (1 + b1), and
    v_2 = (1 - b2)(1 + b2) g^2, so v_hat = g^2; the second update is +lr (1 - b1)/(1 + b1) g/|g|
    (eps = 0)."""
    rng = np.random.default_rng(22)
    W0 = _rand(rng, 4, 4)
    G = _rand(rng, 4, 4)
    lr = 2e-3
    W1, W2 = _adam_run(W0, [G, -G], lr, eps=0.0)
    b1 = ln.ADAM_BETA1
    f = (1 - b1) / (1 + b1)
    expect = W1 + lr * f * (np.sign(G.real) + 1j * np.sign(G.imag))
    assert np.abs(W2 - expect).max() < 1e-15


def test_adam_is_invariant_to_gradient_scale():
    """m_hat / sqrt(v_hat) does not change when every gradient is multiplied by c > 0 (eps = 0)."""
    rng = np.random.default_rng(23)
    W0 = _rand(rng, 6, 2)
    grads = [_rand(rng, 6, 2) for _ in range(5)]
    a = _adam_run(W0, grads, 1e-3, eps=0.0)
    b = _adam_run(W0, [1e4 * G for G in grads], 1e-3, eps=0.0)
    for x, y in zip(a, b):
        assert np.abs(x - y).max() < 1e-14


def test_full_batch_training_lowers_the_loss():
    """A few full-batch Adam steps of the two-layer net lower the relative-error loss."""
    rng = np.random.default_rng(24)
    L = (4, 2, 2, 4)
    V = int(np.prod(L))
    T = ln.Transport(L, li.random_gauge(L, 0.3, 25))
    W1 = np.zeros((9, 6, 4), dtype=complex)
    W2 = np.zeros((9, 4, 6), dtype=complex)
    W1[0, :4, :4] = np.eye(4)
    W2[0, :4, :4] = np.eye(4)
    W1 += 0.05 * _rand(rng, *W1.shape)
    W2 += 0.05 * _rand(rng, *W2.shape)
    e = [_rand(rng, V // 2, 4, 3) for _ in range(3)]
    r = [0.5 * x + 0.1 * _rand(rng, V // 2, 4, 3) for x in e]  # e is close to 2 r: learnable
    _, _, losses = ln.train_full_batch(T, W1, W2, list(zip(r, e)), 30, 1e-2)
    assert losses[-1] < 0.5 * losses[0], losses
