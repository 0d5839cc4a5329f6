"""Pins of the anisotropic clover operator of the CPU oracle (Sec. III.B, Eq. "clover"):
spatial hops weighted by nu/xi_0, the clover planes (i, t) by c_SW^t and the spatial planes by
c_SW^r/xi_0, 1/kappa = 2 (m_0 + 1 + 3 nu/xi_0).  Each test checks a closed form or an invariant
that does not come from the oracle itself.
"""
import numpy as np
import pytest

import lattice_inputs as li
import oracle
from tests import geometry as geo

# the paper's example action (Sec. III.B): xi_0, nu, m_0, c_SW^t, c_SW^r
XI0, NU, M0, CT, CR = 2.464, 0.95, 0.3, 0.91, 1.07


def _rel(a, b):
    return np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / max(np.linalg.norm(np.asarray(b).ravel()), 1e-300)


def _sigma(mu, nu):
    g = [oracle.gamma(m) for m in range(4)]
    return 0.5 * (g[mu] @ g[nu] - g[nu] @ g[mu])


@pytest.mark.parametrize("L,t_bc", [((4, 4, 4, 4), 1), ((4, 6, 2, 8), -1)])
def test_aniso_free_field_plane_wave(L, t_bc):
    """U = 1, psi = e^{ip.x} u: M psi = [1 - 2 kappa sum_mu w_mu cos p_mu + 2 i kappa sum_mu w_mu g_mu
    sin p_mu] psi with w = (nu/xi_0, nu/xi_0, nu/xi_0, 1); at p = 0 (periodic t) this is 2 kappa m_0,
    the bare mass of the paper's kappa formula."""
    rng = np.random.default_rng(71)
    kappa = oracle.aniso_kappa(M0, XI0, NU)
    w = oracle.aniso_weights(XI0, NU)
    U = li.unit_gauge(L)
    clover = oracle.clover_build(L, U, plane_weights=(CT, CR / XI0))
    assert np.abs(clover).max() == 0.0
    c = geo.coords(L)
    g = [oracle.gamma(mu) for mu in range(4)]
    for trial in range(4):
        n = rng.integers(0, 8, size=4) if trial else np.zeros(4, dtype=int)
        p = 2 * np.pi * n / np.asarray(L)
        if t_bc < 0:
            p[3] = (2 * n[3] + 1) * np.pi / L[3]
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        phase = np.exp(1j * (c @ p))
        psi = (phase[:, None, None] * u[None]).reshape(li.fermion_shape(L))
        Mpsi = oracle.dirac(L, U, clover, psi, kappa, 1.0, t_bc, weights=w)
        K = (1 - 2 * kappa * (w * np.cos(p)).sum()) * np.eye(4) + 2j * kappa * sum(
            w[m] * g[m] * np.sin(p[m]) for m in range(4))
        expect = (phase[:, None, None] * (K @ u)[None]).reshape(li.fermion_shape(L))
        assert _rel(Mpsi, expect) < 1e-14
        if trial == 0 and t_bc > 0:
            assert abs((1 - 2 * kappa * w.sum()) / (2 * kappa) - M0) < 1e-14


@pytest.mark.parametrize("mu", [0, 1, 2, 3])
def test_aniso_single_link_clover_closed_form(mu):
    """All links 1 except U_mu(x0) = diag(e^{i th}, e^{-i th}, 1): the plane (mu, nu) carries
    F_{mu nu} = +-(i sin th / 4) diag(1, -1, 0) at x0 + nu, x0 + mu + nu (+) and x0 - nu, x0 + mu - nu
    (-), weighted by c_SW^t when nu or mu is t and by c_SW^r / xi_0 otherwise."""
    L = (4, 4, 6, 4)
    th = 0.37
    x0 = np.array([1, 2, 3, 1])
    U = li.unit_gauge(L)
    V = int(np.prod(L))
    Uf = U.reshape(4, V, 3, 3)
    Uf[mu, geo.eo_index(L, *x0)] = np.diag([np.exp(1j * th), np.exp(-1j * th), 1.0])
    wt, ws = CT, CR / XI0
    clover, off = oracle.clover_build(L, U, return_offblock=True, plane_weights=(wt, ws))
    assert off == 0.0
    got = oracle.unpack_blocks(clover.reshape(V, 2, 36))
    D = 0.25j * np.sin(th) * np.diag([1.0, -1.0, 0.0])
    expect = np.zeros((V, 12, 12), dtype=complex)
    for nu in range(4):
        if nu == mu:
            continue
        wgt = wt if 3 in (mu, nu) else ws
        e_mu = np.eye(4, dtype=int)[mu]
        e_nu = np.eye(4, dtype=int)[nu]
        for shift, sign in ((e_nu, +1), (e_mu + e_nu, +1), (-e_nu, -1), (e_mu - e_nu, -1)):
            y = (x0 + shift) % np.asarray(L)
            expect[geo.eo_index(L, *y)] += wgt * np.kron(_sigma(mu, nu), sign * D)
    blocks = np.zeros((V, 2, 6, 6), dtype=complex)
    blocks[:, 0] = expect[:, :6, :6]
    blocks[:, 1] = expect[:, 6:, 6:]
    assert np.abs(got - blocks).max() < 1e-15


def test_aniso_reduces_to_isotropic():
    """Unit weights give exactly the isotropic hop and clover."""
    L = (4, 4, 2, 4)
    U = li.random_gauge(L, 0.4, seed=72)
    psi = li.gaussian_source(L, 73)
    assert np.array_equal(oracle.hop(L, U, psi, -1, weights=np.ones(4)), oracle.hop(L, U, psi, -1))
    assert np.array_equal(oracle.clover_build(L, U, plane_weights=(1.0, 1.0)), oracle.clover_build(L, U))


@pytest.mark.parametrize("L,t_bc", [((4, 4, 4, 4), 1), ((6, 4, 2, 4), -1)])
def test_aniso_gamma5_hermiticity_and_gauge_covariance(L, t_bc):
    """(chi, g5 M g5 psi) = (M chi, psi) and M[U'] (Om psi) = Om (M[U] psi) for the anisotropic
    operator (both hold direction by direction, so any weights keep them)."""
    V = int(np.prod(L))
    U = li.random_gauge(L, 0.4, seed=74)
    w = oracle.aniso_weights(XI0, NU)
    kappa = oracle.aniso_kappa(M0, XI0, NU)
    C = oracle.clover_build(L, U, plane_weights=(CT, CR / XI0))
    chi = li.gaussian_source(L, 75)
    psi = li.gaussian_source(L, 76)
    g5 = np.array([1, 1, -1, -1])[:, None]

    def M(v, Ux=U, Cx=C):
        return oracle.dirac(L, Ux, Cx, v, kappa, 1.0, t_bc, weights=w)

    assert abs(np.vdot(chi, g5 * M(g5 * psi)) - np.vdot(M(chi), psi)) / abs(np.vdot(M(chi), psi)) < 1e-13
    Om = li.gauge_transform(L, seed=77).reshape(V, 3, 3)
    Uf = U.reshape(4, V, 3, 3)
    Up = np.empty_like(Uf)
    for mu in range(4):
        fw = geo.shift_table(L, mu, +1)
        Up[mu] = Om @ Uf[mu] @ Om[fw].conj().transpose(0, 2, 1)
    Up = Up.reshape(U.shape)
    Cp = oracle.clover_build(L, Up, plane_weights=(CT, CR / XI0))
    lhs = M(np.einsum("iab,isb->isa", Om, psi.reshape(V, 4, 3)).reshape(psi.shape), Up, Cp)
    rhs = np.einsum("iab,isb->isa", Om, M(psi).reshape(V, 4, 3))
    assert _rel(lhs.reshape(V, 4, 3), rhs) < 1e-13
