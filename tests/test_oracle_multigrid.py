"""Pins of the oracle's two-level aggregation multigrid (paper Sec. II.E, Sec. III.B: block sizes per
level, a 2^4 sublattice projected to one coarse site) against what the mathematics fixes."""
import numpy as np
import pytest

import lattice_inputs as li
import oracle
from oracle import multigrid as mg
from oracle.fgmres import fgmres
from tests import geometry as geo


def _vecs(L, N, seed):
    return np.stack([li.gaussian_source(L, seed + k) for k in range(N)])


def _rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b))


def _g5c(nc, N):
    """gamma_5 on coarse vectors: +1 on chirality 0, -1 on chirality 1."""
    return np.tile(np.repeat([1.0, -1.0], N), nc // (2 * N))


def test_block_index_enumerates_blocks():
    """Every coarse site owns exactly |b| fine sites, and those sites lie in one b-block of the lattice
    (checked from coordinates written out independently of the oracle)."""
    L, b = (4, 2, 4, 6), (2, 2, 2, 3)
    blk = mg.block_index(L, b).reshape(-1)
    c = geo.coords(L)
    Lc = mg.coarse_dims(L, b)
    assert np.array_equal(np.bincount(blk), np.full(int(np.prod(Lc)), int(np.prod(b))))
    for i in range(len(blk)):
        q = c[i] // np.array(b)
        assert blk[i] == ((q[3] * Lc[2] + q[2]) * Lc[1] + q[1]) * Lc[0] + q[0]


def test_block_gram_schmidt_matches_qr_and_spans_the_vectors():
    """On each aggregate the block vectors equal the Q of a QR factorisation of the restricted vectors
    (library routine, phases fixed so that R has a positive diagonal); P^+ P = 1; and every input
    vector is reproduced by P P^+."""
    L, b, N = (4, 4, 2, 2), (2, 2, 2, 2), 4
    V = _vecs(L, N, 10)
    W = mg.block_orthonormalize(L, b, V)
    for m in mg._aggregate_masks(L, b):
        A = np.stack([V[k][m] for k in range(N)], axis=1)
        Q, R = np.linalg.qr(A)
        ph = np.diag(R) / np.abs(np.diag(R))
        Q = Q * ph[None, :]
        got = np.stack([W[k][m] for k in range(N)], axis=1)
        assert np.abs(got - Q).max() < 1e-13
    nc = int(np.prod(mg.coarse_dims(L, b))) * 2 * N
    rng = np.random.default_rng(3)
    e = rng.standard_normal(nc) + 1j * rng.standard_normal(nc)
    assert np.abs(mg.restrict(L, b, W, mg.prolong(L, b, W, e)).reshape(-1) - e).max() < 1e-13
    for k in range(N):
        assert _rel(mg.prolong(L, b, W, mg.restrict(L, b, W, V[k])), V[k]) < 1e-13


def test_single_site_aggregates_with_a_full_basis_reproduce_M():
    """b = 1 and N = 6: P is unitary, so D_c = P^+ M P has the eigenvalues of M and P D_c^-1 P^+ = M^-1;
    with that exact coarse solve FGMRES converges in one step."""
    L, b, N = (2, 2, 2, 4), (1, 1, 1, 1), 6
    U = li.random_gauge(L, 0.4, 5)
    C = oracle.clover_build(L, U)
    kappa, csw = 0.12, 1.2
    W = mg.block_orthonormalize(L, b, _vecs(L, N, 20))
    D = mg.coarse_dense(L, b, W, U, C, kappa, csw)
    M = oracle.dense_matrix(L, U, C, kappa, csw)
    ev_d, ev_m = np.linalg.eigvals(D), np.linalg.eigvals(M)
    # the same spectrum: every eigenvalue of one has a partner in the other (greedy matching)
    left = list(ev_m)
    for lam in ev_d:
        j = int(np.argmin(np.abs(np.asarray(left) - lam)))
        assert abs(left[j] - lam) < 1e-10
        left.pop(j)
    rhs = li.gaussian_source(L, 30)
    Dinv = np.linalg.inv(D)
    K = mg.two_level_precond(L, b, W, U, C, kappa, csw, lambda r: (Dinv @ r.reshape(-1)).reshape(r.shape))
    x = np.linalg.solve(M, rhs.reshape(-1)).reshape(rhs.shape)
    assert _rel(K(rhs), x) < 1e-11
    res = fgmres(lambda v: oracle.dirac(L, U, C, v, kappa, csw), rhs, precond=lambda j, v: K(v), m=8, tol=1e-10)
    assert res.iters == 1 and _rel(res.x, x) < 1e-10


@pytest.mark.parametrize("b", [(2, 2, 2, 2), (2, 1, 2, 4)])
def test_free_field_coarse_operator_closed_form(b):
    """U = 1 and near-null vectors constant over the lattice (vector k = 3 s + c: spin s, colour c on
    chirality 0, spin 2 + s on chirality 1).  The block vectors are the normalised constants, and D_c
    is the Wilson operator of the coarse lattice with hop weight 1/b_mu per direction:
      D_c e^{ip.x} u = [1 - 2 kappa sum_mu ((b_mu - 1) + cos p_mu) / b_mu
                          + 2 i kappa sum_mu gamma_mu sin p_mu / b_mu] e^{ip.x} u,
    p_mu = 2 pi n_mu / Lc_mu, with the coarse vector [Vc][2][6] read as spin 2 chi + s, colour c."""
    L = (4, 4, 4, 8)
    Lc = mg.coarse_dims(L, b)
    kappa, csw = 0.11, 1.0
    U = li.unit_gauge(L)
    C = oracle.clover_build(L, U)
    N = 6
    V = np.zeros((N,) + li.fermion_shape(L), dtype=np.complex128)
    for k in range(N):
        s, c = divmod(k, 3)
        V[k][..., s, c] = 1.0
        V[k][..., 2 + s, c] = 1.0
    W = mg.block_orthonormalize(L, b, V)
    Vc = int(np.prod(Lc))
    # coarse coordinates, x fastest
    cc = np.array([(i % Lc[0], (i // Lc[0]) % Lc[1], (i // (Lc[0] * Lc[1])) % Lc[2], i // (Lc[0] * Lc[1] * Lc[2]))
                   for i in range(Vc)])
    g = [oracle.gamma(mu) for mu in range(4)]
    rng = np.random.default_rng(7)
    for n in ([0, 0, 0, 0], [1, 0, 0, 0], [0, 1, 1, 0], [1, 1, 0, 1], [0, 0, 0, Lc[3] // 2]):
        p = 2 * np.pi * np.array(n) / np.array(Lc)
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        phase = np.exp(1j * (cc @ p))
        ec = phase[:, None, None] * u[None]  # [Vc, 4, 3] = [Vc, 2 chi, 2 s, 3 c]
        got = mg.coarse_apply(L, b, W, U, C, ec.reshape(Vc, 2, 6), kappa, csw).reshape(Vc, 4, 3)
        m = np.eye(4, dtype=complex) * (1 - 2 * kappa * sum((b[mu] - 1 + np.cos(p[mu])) / b[mu] for mu in range(4)))
        m = m + 2j * kappa * sum(g[mu] * np.sin(p[mu]) / b[mu] for mu in range(4))
        expect = phase[:, None, None] * (m @ u)[None]
        assert np.abs(got - expect).max() < 1e-13, n


def test_coarse_operator_gamma5_hermitian_and_nearest_neighbour():
    """gamma_5 P = P gamma_5^c (aggregates split by chirality) and gamma_5 M gamma_5 = M^+ give
    gamma_5^c D_c gamma_5^c = D_c^+; the coarse stencil couples only blocks that share a face (here the
    coarse lattice is 4 x 2 x 2 x 2, so blocks two steps apart in x do not couple)."""
    L, b, N = (8, 4, 4, 4), (2, 2, 2, 2), 3
    U = li.random_gauge(L, 0.4, 6)
    C = oracle.clover_build(L, U)
    W = mg.block_orthonormalize(L, b, _vecs(L, N, 40))
    D = mg.coarse_dense(L, b, W, U, C, 0.12, 1.1)
    g5 = _g5c(D.shape[0], N)
    assert np.abs(g5[:, None] * D * g5[None, :] - D.conj().T).max() < 1e-14 * np.abs(D).max() * 10
    Lc = mg.coarse_dims(L, b)
    blk = 2 * N
    for i in range(int(np.prod(Lc))):
        x = i % Lc[0]
        j = (i - x) + (x + 2) % Lc[0]  # two steps along x
        assert np.abs(D[i * blk:(i + 1) * blk, j * blk:(j + 1) * blk]).max() == 0.0


def test_coarse_operator_gauge_invariant():
    """U'_mu(x) = Om(x) U_mu(x) Om(x+mu)^+ and v'_k = Om v_k leave D_c unchanged: the block inner
    products are invariant under the site-wise unitary colour rotation."""
    L, b, N = (4, 4, 2, 2), (2, 2, 1, 2), 3
    U = li.random_gauge(L, 0.4, 8)
    Om = li.gauge_transform(L, 9)
    Up = geo.transform_gauge(L, U, Om)
    V = _vecs(L, N, 50)
    Of = Om.reshape(2, L[3], L[2], L[1], L[0] // 2, 3, 3)
    Vp = np.einsum("...ab,k...sb->k...sa", Of, V)
    kappa, csw = 0.12, 1.0
    D = mg.coarse_dense(L, b, mg.block_orthonormalize(L, b, V), U, oracle.clover_build(L, U), kappa, csw)
    Dp = mg.coarse_dense(L, b, mg.block_orthonormalize(L, b, Vp), Up, oracle.clover_build(L, Up), kappa, csw)
    assert np.abs(D - Dp).max() < 1e-13 * np.abs(D).max()


def test_two_level_fgmres_beats_plain_gmres():
    """Near-null vectors from a few minimal-residual sweeps on M v = 0 from Gaussian starts; the two-level
    preconditioner (exact coarse solve, two smoothing steps) reaches 1e-10 in fewer Arnoldi steps than
    unpreconditioned GMRES, to the dense solution."""
    L, b, N = (4, 4, 4, 4), (2, 2, 2, 2), 6
    U = li.random_gauge(L, 0.3, 0)
    C = oracle.clover_build(L, U)
    kappa, csw = 0.124, 1.0

    def M(v):
        return oracle.dirac(L, U, C, v, kappa, csw)

    V = _vecs(L, N, 60)
    for k in range(N):
        v = V[k]
        for _ in range(20):  # minimal-residual steps on M v = 0: v -= alpha M v
            w = M(v)
            v = v - (np.vdot(M(w), w) / np.vdot(M(w), M(w))) * w
        V[k] = v / np.linalg.norm(v)
    W = mg.block_orthonormalize(L, b, V)
    D = mg.coarse_dense(L, b, W, U, C, kappa, csw)
    Dinv = np.linalg.inv(D)
    K = mg.two_level_precond(L, b, W, U, C, kappa, csw, lambda r: (Dinv @ r.reshape(-1)).reshape(r.shape), nu=2)
    rhs = li.point_source(L, 0, 0)
    plain = fgmres(M, rhs, m=32, tol=1e-10, maxiter=2000)
    pre = fgmres(M, rhs, precond=lambda j, v: K(v), m=32, tol=1e-10, maxiter=2000)
    x = np.linalg.solve(oracle.dense_matrix(L, U, C, kappa, csw), rhs.reshape(-1)).reshape(rhs.shape)
    assert _rel(pre.x, x) < 1e-8
    assert pre.iters < plain.iters / 2, (pre.iters, plain.iters)


def test_dependent_vectors_are_rejected():
    """A vector that is a multiple of an earlier one on an aggregate (here everywhere) has no part outside
    their span beyond rounding and is rejected; an independent set is accepted."""
    L, b = (4, 4, 2, 2), (2, 2, 2, 2)
    V = _vecs(L, 2, 90)
    mg.block_orthonormalize(L, b, V)
    V[1] = (2.0 - 0.5j) * V[0]
    with pytest.raises(ValueError, match="dependent"):
        mg.block_orthonormalize(L, b, V)
