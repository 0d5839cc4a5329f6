"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test names the passage (paper section or equation) or the mathematical
fact it checks.  The oracle is test infrastructure; these tests are what make
it trustworthy before any GPU kernel is compared with it.
"""
import json
import os

import numpy as np
import pytest

import lattice_inputs as li
import oracle
from tests import geometry as geo

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rel(a, b):
    return np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / max(np.linalg.norm(np.asarray(b).ravel()), 1e-300)


# ---------------------------------------------------------------------------
# Dirac matrices (Sec. II.A names the DeGrand-Rossi basis)
# ---------------------------------------------------------------------------


def test_gamma_clifford_hermitian_chiral():
    g = [oracle.gamma(mu) for mu in range(4)]
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T, atol=0)
        for nu in range(4):
            anti = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(anti, 2.0 * np.eye(4) * (mu == nu), atol=0)
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    # chiral basis: gamma_5 diagonal, upper spins +1
    assert np.allclose(g5, np.diag([1, 1, -1, -1]), atol=0)
    for mu in range(4):
        for nu in range(4):
            s = 0.5 * (g[mu] @ g[nu] - g[nu] @ g[mu])
            assert np.abs(s[:2, 2:]).max() == 0 and np.abs(s[2:, :2]).max() == 0
            assert np.allclose(s, -s.conj().T)


def test_gamma_bitmask_golden():
    """Sec. III.B: gamma(15) is gamma_5 and gamma(15) @ gamma(4) is gamma_5 gamma_3."""
    with open(os.path.join(GOLDEN, "gamma_bitmask.json")) as f:
        gold = json.load(f)
    g = [oracle.gamma(mu) for mu in range(4)]
    named = {"gamma_1": g[0], "gamma_2": g[1], "gamma_3": g[2], "gamma_4": g[3],
             "gamma_5": g[0] @ g[1] @ g[2] @ g[3]}
    for item in gold["cases"]:
        m = np.eye(4, dtype=complex)
        for name in item["product"]:
            m = m @ named[name]
        got = np.eye(4, dtype=complex)
        for n in item["bitmask_product"]:
            got = got @ oracle.gamma_bitmask(n)
        assert np.allclose(got, m, atol=0), item


# ---------------------------------------------------------------------------
# Geometry (Sec. II.A even-odd layout)
# ---------------------------------------------------------------------------


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (2, 4, 6, 8), (6, 2, 4, 2)])
def test_site_indexing_matches_layout_description(L):
    c = geo.coords(L)
    V = int(np.prod(L))
    assert sorted(geo.eo_index(L, *c.T).tolist()) == list(range(V))
    for i in range(0, V, max(1, V // 37)):
        assert oracle.site_coords(L, i) == tuple(c[i])
        assert oracle.site_index(L, c[i]) == i
    assert np.array_equal(oracle.coords_table(L), c)


# ---------------------------------------------------------------------------
# Free field: closed form of the Wilson operator on a plane wave
# ---------------------------------------------------------------------------


@pytest.mark.parametrize("L,t_bc", [((4, 4, 4, 4), 1), ((4, 6, 2, 8), 1), ((4, 4, 6, 6), -1)])
def test_free_field_plane_wave(L, t_bc):
    """U = 1, psi = e^{ip.x} u: M psi = [1 - 2k sum cos p + 2ik sum g_mu sin p] psi.

    This is 2 kappa [m + sum(1 - cos p) + i sum g sin p] with m = 1/(2 kappa) - 4;
    the clover term vanishes at U = 1.  Antiperiodic time (t_bc = -1, the
    paper's t_boundary option) shifts p_t to odd multiples of pi/Lt.
    """
    rng = np.random.default_rng(7)
    kappa, csw = 0.113, 1.3
    U = li.unit_gauge(L)
    clover = oracle.clover_build(L, U)
    assert np.abs(clover).max() == 0.0
    c = geo.coords(L)
    g = [oracle.gamma(mu) for mu in range(4)]
    for trial in range(3):
        n = rng.integers(0, 8, size=4)
        p = 2 * np.pi * n / np.asarray(L)
        if t_bc < 0:
            p[3] = (2 * n[3] + 1) * np.pi / L[3]
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        phase = np.exp(1j * (c @ p))
        psi = (phase[:, None, None] * u[None]).reshape(li.fermion_shape(L))
        Mpsi = oracle.dirac(L, U, clover, psi, kappa, csw, t_bc)
        K = (1 - 2 * kappa * np.cos(p).sum()) * np.eye(4) + 2j * kappa * sum(g[m] * np.sin(p[m]) for m in range(4))
        expect = (phase[:, None, None] * (K @ u)[None]).reshape(li.fermion_shape(L))
        assert _rel(Mpsi, expect) < 1e-14


# ---------------------------------------------------------------------------
# Invariants of the interacting operator
# ---------------------------------------------------------------------------


@pytest.mark.parametrize("L,t_bc", [((4, 4, 4, 4), 1), ((4, 2, 6, 4), -1)])
def test_gauge_covariance(L, t_bc):
    """M[U'] (Om psi) = Om (M[U] psi) for U'_mu(x) = Om(x) U_mu(x) Om(x+mu)^+."""
    V = int(np.prod(L))
    U = li.random_gauge(L, 0.5, seed=11)
    Om = li.gauge_transform(L, seed=12).reshape(V, 3, 3)
    psi = li.gaussian_source(L, seed=13)
    Up = geo.transform_gauge(L, U, Om)
    kappa, csw = 0.121, 1.7
    C = oracle.clover_build(L, U)
    Cp = oracle.clover_build(L, Up)
    lhs = oracle.dirac(L, Up, Cp, np.einsum("iab,isb->isa", Om, psi.reshape(V, 4, 3)).reshape(psi.shape),
                       kappa, csw, t_bc)
    rhs = np.einsum("iab,isb->isa", Om, oracle.dirac(L, U, C, psi, kappa, csw, t_bc).reshape(V, 4, 3))
    assert _rel(lhs.reshape(V, 4, 3), rhs) < 1e-13


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (6, 4, 2, 4)])
def test_gamma5_hermiticity(L):
    """(chi, g5 M g5 psi) = (M chi, psi): the identity used in Sec. III.A."""
    U = li.random_gauge(L, 0.4, seed=21)
    C = oracle.clover_build(L, U)
    chi = li.gaussian_source(L, 22)
    psi = li.gaussian_source(L, 23)
    kappa, csw = 0.124, 1.1
    g5 = np.array([1, 1, -1, -1])[:, None]

    def M(v):
        return oracle.dirac(L, U, C, v, kappa, csw)

    lhs = np.vdot(chi, g5 * M(g5 * psi))
    rhs = np.vdot(M(chi), psi)
    assert abs(lhs - rhs) / abs(rhs) < 1e-13


# ---------------------------------------------------------------------------
# Clover term (Sec. II.A packing, Eq. "clover")
# ---------------------------------------------------------------------------


def _sigma(mu, nu):
    g = [oracle.gamma(m) for m in range(4)]
    return 0.5 * (g[mu] @ g[nu] - g[nu] @ g[mu])


@pytest.mark.parametrize("mu", [0, 1, 2, 3])
def test_single_link_clover_closed_form(mu):
    """All links 1 except U_mu(x0) = diag(e^{i th}, e^{-i th}, 1).

    For every plane (mu, nu): F_{mu nu} = +(i sin th / 4) diag(1,-1,0) at
    x0+nu and x0+mu+nu, -(i sin th / 4) diag(1,-1,0) at x0-nu and x0+mu-nu,
    zero elsewhere (x0 and x0+mu included: their two affected leaves cancel).
    Planes without mu carry no field.
    """
    L = (4, 4, 6, 4)
    th = 0.37
    x0 = np.array([1, 2, 3, 1])
    U = li.unit_gauge(L)
    V = int(np.prod(L))
    Uf = U.reshape(4, V, 3, 3)
    Uf[mu, geo.eo_index(L, *x0)] = np.diag([np.exp(1j * th), np.exp(-1j * th), 1.0])
    clover, off = oracle.clover_build(L, U, return_offblock=True)
    assert off == 0.0
    got = oracle.unpack_blocks(clover.reshape(V, 2, 36))

    D = 0.25j * np.sin(th) * np.diag([1.0, -1.0, 0.0])
    expect = np.zeros((V, 12, 12), dtype=complex)
    for nu in range(4):
        if nu == mu:
            continue
        e_mu = np.eye(4, dtype=int)[mu]
        e_nu = np.eye(4, dtype=int)[nu]
        for shift, sign in ((e_nu, +1), (e_mu + e_nu, +1), (-e_nu, -1), (e_mu - e_nu, -1)):
            y = (x0 + shift) % np.asarray(L)
            # F_{mu nu} at y; sigma_{mu nu} F_{mu nu} is symmetric in the order of the pair
            expect[geo.eo_index(L, *y)] += np.kron(_sigma(mu, nu), sign * D)
    blocks = np.zeros((V, 2, 6, 6), dtype=complex)
    blocks[:, 0] = expect[:, :6, :6]
    blocks[:, 1] = expect[:, 6:, 6:]
    assert np.abs(expect[:, :6, 6:]).max() == 0
    assert np.abs(got - blocks).max() < 1e-15


def test_clover_packing_trace_hermitian_and_inverse():
    L = (4, 4, 4, 4)
    V = 256
    U = li.random_gauge(L, 0.3, seed=0)
    kappa, csw = 0.12, 1.0
    C, off = oracle.clover_build(L, U, return_offblock=True)
    assert off < 1e-15
    blocks = oracle.unpack_blocks(C.reshape(V, 2, 36))
    # sigma blocks are traceless -> tr C_chi = 0 -> tr A_chi = 6
    assert np.abs(np.trace(blocks, axis1=-2, axis2=-1)).max() < 1e-14
    A = np.eye(6) - kappa * csw * blocks
    assert np.allclose(A, np.conj(np.swapaxes(A, -1, -2)), atol=0)
    # Gauss-Jordan inverse against LAPACK's inverse of the same blocks
    inv, bad = oracle.clover_invert(L, C, kappa, csw)
    assert bad == 0
    inv_blocks = oracle.unpack_blocks(inv.reshape(V, 2, 36))
    assert np.abs(inv_blocks - np.linalg.inv(A)).max() < 1e-14
    # A A^{-1} = 1 through the field-level functions
    psi = li.gaussian_source(L, 5)
    back = oracle.packed_apply(L, inv, oracle.clover_apply(L, C, psi, kappa, csw))
    assert _rel(back, psi) < 1e-14
    # U = 1: A = 1
    C1 = oracle.clover_build(L, li.unit_gauge(L))
    assert _rel(oracle.clover_apply(L, C1, psi, kappa, csw), psi) == 0.0


# ---------------------------------------------------------------------------
# Solver: dense LU, free propagator, even-odd Schur, statuses
# ---------------------------------------------------------------------------


@pytest.fixture(scope="module")
def dense4():
    w = li.WORKLOADS["dense4"]
    L = w["L"]
    U = li.random_gauge(L, w["eps"], w["seed"])
    C = oracle.clover_build(L, U)
    M = oracle.dense_matrix(L, U, C, w["kappa"], w["csw"])
    return L, U, C, M, w


@pytest.mark.slow
def test_dense_lu_4444(dense4):
    """4^4 point source: oracle BiCGStab agrees with LAPACK's dense solve."""
    L, U, C, M, w = dense4
    b = li.point_source(L)
    x_lu = np.linalg.solve(M, b.ravel())
    s = np.linalg.svd(M, compute_uv=False)
    cond = s[0] / s[-1]
    res = oracle.bicgstab(L, U, C, b, w["kappa"], w["csw"], tol=1e-10, maxiter=1000)
    assert res.status == 0
    assert res.true_res <= 1e-10
    assert _rel(res.x.ravel(), x_lu) <= cond * 1e-10
    # gamma5-hermiticity of the assembled matrix: M^+ = G5 M G5
    g5 = np.tile(np.repeat([1, 1, -1, -1], 3), int(np.prod(L)))
    assert np.abs(M.conj().T - g5[:, None] * M * g5[None, :]).max() < 1e-14


def test_even_odd_schur_reproduces_full_solve(dense4):
    """Symmetric even-odd Schur solve + reconstruction equals the dense solve."""
    L, U, C, M, w = dense4
    kappa, csw = w["kappa"], w["csw"]
    Ainv, _ = oracle.clover_invert(L, C, kappa, csw)
    b = li.gaussian_source(L, 3)
    Vh = int(np.prod(L)) // 2
    n = 12 * Vh
    Mhat = np.empty((n, n), dtype=complex)
    e = np.zeros(n, dtype=complex)
    for k in range(n):
        e[:] = 0
        e[k] = 1
        Mhat[:, k] = oracle.schur_matpc(L, U, Ainv, e.reshape(Vh, 4, 3), kappa).ravel()
    bhat = oracle.schur_source(L, U, Ainv, b, kappa)
    xe = np.linalg.solve(Mhat, bhat.ravel())
    x = oracle.schur_reconstruct(L, U, Ainv, b, xe.reshape(Vh, 4, 3), kappa)
    x_lu = np.linalg.solve(M, b.ravel())
    assert _rel(x.ravel(), x_lu) < 1e-12


def _free_propagator_fft(L, kappa, spin, colour):
    """Point-source solution at U = 1 from the momentum-space inverse.

    M(p)^{-1} = [a - i sum b_mu g_mu] / (a^2 + sum b_mu^2), a = 1 - 2k sum cos p,
    b_mu = 2k sin p_mu.
    """
    g = [oracle.gamma(m) for m in range(4)]
    Lx, Ly, Lz, Lt = L
    ps = [2 * np.pi * np.fft.fftfreq(n) for n in (Lx, Ly, Lz, Lt)]
    P = np.meshgrid(*ps, indexing="ij")
    a = 1 - 2 * kappa * sum(np.cos(p) for p in P)
    bs = [2 * kappa * np.sin(p) for p in P]
    den = a ** 2 + sum(b ** 2 for b in bs)
    # spin column `spin` of M(p)^{-1}, for every momentum: (Lx,Ly,Lz,Lt,4)
    col = a[..., None] * np.eye(4)[spin] - 1j * sum(bs[m][..., None] * g[m][:, spin] for m in range(4))
    col = col / den[..., None]
    # x(y) = (1/V) sum_p e^{i p y} M(p)^{-1} u  -> inverse FFT
    xs = np.fft.ifftn(col, axes=(0, 1, 2, 3))
    c = geo.coords(L)
    out = np.zeros((int(np.prod(L)), 4, 3), dtype=complex)
    out[:, :, colour] = xs[c[:, 0], c[:, 1], c[:, 2], c[:, 3]]
    return out.reshape(li.fermion_shape(L))


@pytest.mark.parametrize("L,kappa,spin,colour", [((4, 4, 4, 4), 0.12, 0, 0), ((4, 6, 4, 8), 0.1, 2, 1)])
def test_free_propagator_fft(L, kappa, spin, colour):
    U = li.unit_gauge(L)
    C = oracle.clover_build(L, U)
    b = li.point_source(L, spin, colour)
    res = oracle.bicgstab(L, U, C, b, kappa, 1.0, tol=1e-12, maxiter=2000)
    assert res.status == 0
    expect = _free_propagator_fft(L, kappa, spin, colour)
    assert _rel(res.x, expect) < 1e-10


def test_solver_statuses():
    L = (4, 4, 4, 4)
    U = li.random_gauge(L, 0.3, 0)
    C = oracle.clover_build(L, U)
    b = li.gaussian_source(L, 1)
    r = oracle.bicgstab(L, U, C, b, 0.12, 1.0, tol=1e-10, maxiter=3)
    assert r.status == -4 and r.iters == 3 and r.true_res > 1e-10
    bn = b.copy()
    bn.ravel()[17] = np.nan
    r = oracle.bicgstab(L, U, C, bn, 0.12, 1.0, tol=1e-10, maxiter=30)
    assert r.status == -6
    r = oracle.bicgstab(L, U, C, np.zeros_like(b), 0.12, 1.0)
    assert r.status == 0 and np.abs(r.x).max() == 0
    # residual history starts at 1 (zero guess) and ends at or below tol
    r = oracle.bicgstab(L, U, C, b, 0.12, 1.0, tol=1e-10, maxiter=500)
    assert r.status == 0 and r.res_hist[0] == pytest.approx(1.0) and r.res_hist[-1] <= 1e-10


def test_schur_adjoint_identity():
    """M_hat^+ = g5 A_ee M_hat g5 A_ee^{-1} on even sites (M^+ = g5 M g5 and [A, g5] = 0): the identity the
    GPU normal operator uses, checked on the dense matrices."""
    L = (4, 2, 2, 4)
    U = li.random_gauge(L, 0.4, seed=27)
    kappa, csw = 0.12, 1.2
    C = oracle.clover_build(L, U)
    Ainv, _ = oracle.clover_invert(L, C, kappa, csw)
    M = oracle.schur_dense(L, U, Ainv, kappa)
    Vh = int(np.prod(L)) // 2
    n = 12 * Vh

    def blockwise(packed):  # dense block-diagonal matrix of the even-site packed blocks
        full = oracle.unpack_blocks(np.asarray(packed).reshape(-1, 2, 36))[:Vh]
        D = np.zeros((n, n), dtype=complex)
        for i in range(Vh):
            for chi in range(2):
                # block rows/cols: spins 2 chi, 2 chi + 1 (colour inner) of site i
                idx = 12 * i + 6 * chi + np.arange(6)
                D[np.ix_(idx, idx)] = full[i, chi]
        return D

    Ai = blockwise(Ainv)
    A = np.linalg.inv(Ai)
    g5 = np.kron(np.eye(Vh), np.kron(np.diag([1.0, 1.0, -1.0, -1.0]), np.eye(3)))
    assert np.abs(M.conj().T - g5 @ A @ M @ g5 @ Ai).max() < 1e-12 * np.abs(M).max()
