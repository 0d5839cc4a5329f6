"""CPU oracle of the learned gauge-covariant preconditioner (plain NumPy, FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper's own accelerator for clover inversions is multigrid (Sec. II.E); the
learned preconditioner follows the published idea of gauge-equivariant
convolutions for lattice Dirac operators (Favoni et al., PRL 2022; Lehner and
Wettig, PRD 2023).  A layer maps channels phi_c (each a colour 3-vector field
on the full lattice) to

    out_{c'}(x) = sum_{a in {0, +-1..+-4}} sum_c W_a[c', c] (T_a phi_c)(x)

with T_0 = 1, (T_{+mu} phi)(x) = U_mu(x) phi(x+mu), (T_{-mu} phi)(x) =
U_mu(x-mu)^+ phi(x-mu).  No bias and no nonlinearity, so the network is a
gauge-covariant linear map.  Hop order of the weight index a: 0, then +mu and
-mu for mu = 0..3, i.e. a = 1 + 2 mu + (0 forward | 1 backward).

The preconditioner of the even-odd Schur system: embed an even-site field in
the full lattice (zero on odd sites), apply the layers, keep the even sites.

Gradients (L real, W complex; dL/dW := dL/dRe W + i dL/dIm W):
    loss L = sum_pairs ||P(r) - e||^2 / ||e||^2
    for a layer out = sum_a W_a T_a phi and upstream g = dL/d conj(out) ... see
    layer_weight_grad: G_a[c', c] = 2 sum_x <T_a phi_c(x), g_{c'}(x)>-style
    contraction; pinned by finite differences in the tests.
Parity unpinned with respect to the paper (it does not define the network);
pinned by: a 4-channel layer whose weights are the Wilson projectors equals the
oracle's hop term, gauge equivariance, and central finite differences.

Training: Adam (Kingma and Ba 2015) on the real and imaginary parts of the
weights, pinned by closed forms of its first steps (the first update is
-lr g / (|g| + eps) per real parameter; a constant gradient gives that update at
every step; a reversed second gradient gives +lr (1 - b1) / (1 + b1) per unit
gradient direction) and by its invariance under a rescaling of the gradient.
"""
from __future__ import annotations

import numpy as np

from . import coords_table

N_HOPS = 9


def _neighbour_tables(L):
    """fwd[mu][i], bwd[mu][i]: eo index of site i +- mu-hat (periodic)."""
    c = coords_table(L)
    Lx, Ly, Lz, Lt = L
    V = Lx * Ly * Lz * Lt

    def index(cc):
        x, y, z, t = cc[:, 0], cc[:, 1], cc[:, 2], cc[:, 3]
        p = (x + y + z + t) % 2
        return p * (V // 2) + ((t * Lz + z) * Ly + y) * (Lx // 2) + x // 2

    fwd, bwd = [], []
    for mu in range(4):
        cp = c.copy()
        cp[:, mu] = (cp[:, mu] + 1) % L[mu]
        fwd.append(index(cp))
        cm = c.copy()
        cm[:, mu] = (cm[:, mu] - 1) % L[mu]
        bwd.append(index(cm))
    return fwd, bwd


class Transport:
    """The nine parallel transports T_a on one gauge field (paper layouts)."""

    def __init__(self, L, U):
        self.L = tuple(L)
        V = int(np.prod(L))
        self.V = V
        self.U = np.asarray(U, dtype=np.complex128).reshape(4, V, 3, 3)
        self.fwd, self.bwd = _neighbour_tables(L)

    def apply(self, a: int, phi: np.ndarray) -> np.ndarray:
        """(T_a phi) for phi of shape (C, V, 3)."""
        if a == 0:
            return phi.copy()
        mu, back = (a - 1) // 2, (a - 1) % 2
        if back == 0:
            # U_mu(x) phi(x + mu)
            return np.einsum("xab,cxb->cxa", self.U[mu], phi[:, self.fwd[mu]])
        # U_mu(x - mu)^+ phi(x - mu)
        j = self.bwd[mu]
        return np.einsum("xba,cxb->cxa", self.U[mu][j].conj(), phi[:, j])

    def adjoint(self, a: int, phi: np.ndarray) -> np.ndarray:
        """(T_a^+ phi): T_0^+ = 1 and T_{+-mu}^+ = T_{-+mu}."""
        if a == 0:
            return phi.copy()
        mu, back = (a - 1) // 2, (a - 1) % 2
        return self.apply(1 + 2 * mu + (1 - back), phi)


def layer_forward(T: Transport, W: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """out[c'] = sum_a sum_c W[a, c', c] T_a phi[c]; W: (9, Cout, Cin), phi: (Cin, V, 3)."""
    out = np.zeros((W.shape[1], T.V, 3), dtype=np.complex128)
    for a in range(N_HOPS):
        out += np.einsum("dc,cxk->dxk", W[a], T.apply(a, phi))
    return out


def layer_adjoint(T: Transport, W: np.ndarray, g: np.ndarray) -> np.ndarray:
    """The adjoint map: sum_a T_a^+ W[a]^+ g, g: (Cout, V, 3) -> (Cin, V, 3)."""
    out = np.zeros((W.shape[2], T.V, 3), dtype=np.complex128)
    for a in range(N_HOPS):
        out += T.adjoint(a, np.einsum("dc,dxk->cxk", W[a].conj(), g))
    return out


def layer_weight_grad(T: Transport, phi: np.ndarray, g: np.ndarray) -> np.ndarray:
    """G[a, c', c] = sum_x sum_colour g[c'](x) conj((T_a phi[c])(x)).

    For a real loss L(out) with g = 2 dL/d conj(out) (so g = 2 (out - target) for
    ||out - target||^2), G equals dL/dRe W + i dL/dIm W.
    """
    G = np.zeros((N_HOPS, g.shape[0], phi.shape[0]), dtype=np.complex128)
    for a in range(N_HOPS):
        G[a] = np.einsum("dxk,cxk->dc", g, T.apply(a, phi).conj())
    return G


def embed_even(L, r_e: np.ndarray) -> np.ndarray:
    """Even-site fermion (Vh, 4, 3) -> channels (4, V, 3) with zeros on odd sites."""
    V = int(np.prod(L))
    phi = np.zeros((4, V, 3), dtype=np.complex128)
    phi[:, : V // 2] = np.transpose(np.asarray(r_e).reshape(V // 2, 4, 3), (1, 0, 2))
    return phi


def restrict_even(L, phi: np.ndarray) -> np.ndarray:
    V = int(np.prod(L))
    return np.transpose(phi[:, : V // 2], (1, 0, 2)).copy()


def net_apply(T: Transport, W1: np.ndarray, W2: np.ndarray, r_e: np.ndarray) -> np.ndarray:
    """Preconditioner P(r_e) on even sites: restrict(layer2(layer1(embed(r_e))))."""
    h = layer_forward(T, W1, embed_even(T.L, r_e))
    return restrict_even(T.L, layer_forward(T, W2, h))


def net_loss_and_grad(T: Transport, W1, W2, pairs):
    """L = sum ||P(r) - e||^2 / ||e||^2 over (r_e, e_e) pairs, and dL/dW1, dL/dW2."""
    L_ = T.L
    G1 = np.zeros_like(W1)
    G2 = np.zeros_like(W2)
    loss = 0.0
    for r_e, e_e in pairs:
        phi0 = embed_even(L_, r_e)
        h = layer_forward(T, W1, phi0)
        z = layer_forward(T, W2, h)
        diff = restrict_even(L_, z) - np.asarray(e_e).reshape(-1, 4, 3)
        en = np.linalg.norm(e_e) ** 2
        loss += np.linalg.norm(diff) ** 2 / en
        gz = 2.0 * embed_even(L_, diff) / en  # 2 dL/d conj(z), zero on odd sites
        G2 += layer_weight_grad(T, h, gz)
        gh = layer_adjoint(T, W2, gz)
        G1 += layer_weight_grad(T, phi0, gh)
    return loss, G1, G2


# ---------------------------------------------------------------------------
# Training step: Adam (Kingma and Ba 2015, Algorithm 1), written out from the
# published algorithm.  The complex weights are treated as pairs of independent
# real parameters (Re W, Im W) with the gradient G = dL/dRe W + i dL/dIm W, so
# every formula below acts on the real and the imaginary parts separately.
# ---------------------------------------------------------------------------
ADAM_BETA1 = 0.9
ADAM_BETA2 = 0.999
ADAM_EPS = 1e-8


class AdamState:
    """First and second moment estimates of one complex weight array, and the step count."""

    def __init__(self, shape):
        self.m_re = np.zeros(shape)
        self.m_im = np.zeros(shape)
        self.v_re = np.zeros(shape)
        self.v_im = np.zeros(shape)
        self.t = 0


def _adam_real(theta, g, m, v, t, lr, b1, b2, eps):
    # biased moment estimates, then their bias-corrected forms, then the step
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    m_hat = m / (1.0 - b1 ** t)
    v_hat = v / (1.0 - b2 ** t)
    return theta - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


def adam_step(W, G, state: AdamState, lr, b1=ADAM_BETA1, b2=ADAM_BETA2, eps=ADAM_EPS):
    """One Adam update of the complex weights W with gradient G; returns the new W (state updated)."""
    state.t += 1
    re, state.m_re, state.v_re = _adam_real(W.real, G.real, state.m_re, state.v_re, state.t, lr, b1, b2, eps)
    im, state.m_im, state.v_im = _adam_real(W.imag, G.imag, state.m_im, state.v_im, state.t, lr, b1, b2, eps)
    return re + 1j * im


def train_full_batch(T: Transport, W1, W2, pairs, steps, lr):
    """`steps` Adam steps, each on the mean gradient of the loss over all `pairs` (the batch is
    the whole set, so the order of the pairs does not matter); returns W1, W2 and the mean loss
    of each step (measured before its update)."""
    s1, s2 = AdamState(W1.shape), AdamState(W2.shape)
    losses = []
    for _ in range(steps):
        loss, G1, G2 = net_loss_and_grad(T, W1, W2, pairs)
        n = len(pairs)
        W1 = adam_step(W1, G1 / n, s1, lr)
        W2 = adam_step(W2, G2 / n, s2, lr)
        losses.append(loss / n)
    return W1, W2, losses
