"""GPU parity of the two-level aggregation multigrid (paper Sec. II.E, III.B) against the CPU oracle
(oracle/multigrid.py): block vectors, restriction, prolongation and the Galerkin coarse operator from the
same seeded near-null vectors, to the FP64 bar (1e-13 relative); properties of a set-up that generates
its own vectors; multigrid-preconditioned solves whose true residual the oracle recomputes."""
import numpy as np
import pytest
import torch

import lattice_inputs as li
import oracle
import paper_2411_08461_amd as q
from oracle import multigrid as omg

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.fixture(scope="module")
def ctx():
    c = q.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _vecs(L, N, seed):
    return np.stack([li.gaussian_source(L, seed + k) for k in range(N)])


def _dense_from_stencil(Y, Lc, nc):
    """Dense coarse matrix from the stencil [Vc][9][nc][nc] (entry 0 self, 1 + 2 mu: +mu, 2 + 2 mu: -mu)."""
    Vc = int(np.prod(Lc))
    D = np.zeros((Vc * nc, Vc * nc), dtype=np.complex128)
    for cs in range(Vc):
        c = [cs % Lc[0], (cs // Lc[0]) % Lc[1], (cs // (Lc[0] * Lc[1])) % Lc[2], cs // (Lc[0] * Lc[1] * Lc[2])]
        for d in range(9):
            q_ = list(c)
            if d:
                mu, back = (d - 1) // 2, (d - 1) % 2
                q_[mu] = (q_[mu] + (-1 if back else 1)) % Lc[mu]
            nb = ((q_[3] * Lc[2] + q_[2]) * Lc[1] + q_[1]) * Lc[0] + q_[0]
            D[cs * nc:(cs + 1) * nc, nb * nc:(nb + 1) * nc] += Y[cs, d]
    return D


CASES = [  # (L, block, N): 2^4 blocks (the paper's example) and uneven blocks, ragged hop tiles
    ((4, 4, 4, 8), (2, 2, 2, 2), 4),
    ((6, 4, 2, 6), (2, 2, 2, 3), 3),
    ((8, 8, 8, 16), (4, 4, 4, 4), 6),
]


@pytest.mark.parametrize("L,b,N", CASES)
def test_block_vectors_restrict_prolong_match_oracle(ctx, L, b, N):
    U = li.random_gauge(L, 0.3, 71)
    op = q.Operator(ctx, q.make_lattice(L), dev(U), 0.12, 1.0, "f32")
    V = _vecs(L, N, 700)
    mg = q.Multigrid(op, q.make_mg_params(block=b, nvec=N), vecs=dev(V))
    assert mg.coarse_dims == omg.coarse_dims(L, b)
    W = omg.block_orthonormalize(L, b, V)
    got = torch.empty((N,) + li.fermion_shape(L), dtype=torch.complex128, device="cuda")
    q.qcdw_mg_vectors(mg, got)
    assert rel(host(got), W) < 1e-13
    f = li.gaussian_source(L, 710)
    rc = torch.empty(mg.coarse_len(), dtype=torch.complex128, device="cuda")
    q.qcdw_mg_restrict(mg, dev(f), rc)
    assert rel(host(rc).reshape(-1, 2, N), omg.restrict(L, b, W, f)) < 1e-13
    rng = np.random.default_rng(711)
    ec = rng.standard_normal(mg.coarse_len()) + 1j * rng.standard_normal(mg.coarse_len())
    pf = torch.empty(li.fermion_shape(L), dtype=torch.complex128, device="cuda")
    q.qcdw_mg_prolong(mg, dev(ec), pf)
    assert rel(host(pf), omg.prolong(L, b, W, ec)) < 1e-13
    mg.close()
    op.close()


@pytest.mark.parametrize("L,b,N,t_bc,recon", [((4, 4, 4, 4), (2, 2, 2, 2), 3, 1, 12),
                                               ((4, 4, 2, 8), (2, 2, 2, 4), 2, -1, 18),
                                               ((6, 4, 4, 4), (3, 2, 2, 2), 2, 1, 12)])
def test_coarse_operator_matches_oracle(ctx, L, b, N, t_bc, recon):
    """The coarse stencil assembled densely equals the oracle's P^+ M P column by column, with periodic and
    antiperiodic time, reconstruct-12 and -18 links, and a coarse extent of 2 (both faces of a block
    reach the same neighbour)."""
    U = li.random_gauge(L, 0.3, 72)
    kappa, csw = 0.124, 1.1
    op = q.Operator(ctx, q.make_lattice(L, t_bc), dev(U), kappa, csw, "f32", recon)
    V = _vecs(L, N, 720)
    mg = q.Multigrid(op, q.make_mg_params(block=b, nvec=N), vecs=dev(V))
    Lc = omg.coarse_dims(L, b)
    nc = 2 * N
    Y = torch.empty(int(np.prod(Lc)) * 9 * nc * nc, dtype=torch.complex128, device="cuda")
    q.qcdw_mg_coarse_op(mg, Y)
    D = _dense_from_stencil(host(Y).reshape(-1, 9, nc, nc), Lc, nc)
    W = omg.block_orthonormalize(L, b, V)
    expect = omg.coarse_dense(L, b, W, U, oracle.clover_build(L, U), kappa, csw, t_bc)
    assert rel(D, expect) < 1e-13
    mg.close()
    op.close()


def test_coarse_operator_of_the_anisotropic_action(ctx):
    """The coarse operator carries the anisotropic hop weights and clover coefficients of the operator."""
    xi0, nu, m0, ct, cr = 2.464, 0.95, 0.3, 0.91, 1.07
    L, b, N = (4, 4, 4, 8), (2, 2, 2, 2), 2
    kappa = oracle.aniso_kappa(m0, xi0, nu)
    U = li.random_gauge(L, 0.3, 73)
    op = q.Operator(ctx, q.make_lattice(L, -1), dev(U), kappa, 1.0, "f32", 12, aniso=(xi0, nu, ct, cr))
    V = _vecs(L, N, 730)
    mg = q.Multigrid(op, q.make_mg_params(block=b, nvec=N), vecs=dev(V))
    W = omg.block_orthonormalize(L, b, V)
    C = oracle.clover_build(L, U, plane_weights=(ct, cr / xi0))
    rng = np.random.default_rng(731)
    ec = rng.standard_normal(mg.coarse_len()) + 1j * rng.standard_normal(mg.coarse_len())
    out = torch.empty_like(dev(ec))
    q.qcdw_mg_coarse_apply(mg, dev(ec), out)
    expect = omg.coarse_apply(L, b, W, U, C, ec.reshape(-1, 2, N), kappa, 1.0, -1, oracle.aniso_weights(xi0, nu))
    assert rel(host(out).reshape(-1, 2, N), expect) < 1e-13
    mg.close()
    op.close()


def test_coarse_apply_matches_oracle_at_8x8x8x16(ctx):
    """D_c e for random coarse vectors, 4^4 blocks and 6 vectors (512 coarse sites x 12), against the oracle's
    matrix-free P^+ M P e."""
    L, b, N = (8, 8, 8, 16), (4, 4, 4, 4), 6
    U = li.random_gauge(L, 0.2, 74)
    kappa, csw = 0.125, 1.0
    op = q.Operator(ctx, q.make_lattice(L), dev(U), kappa, csw, "bf16")
    V = _vecs(L, N, 740)
    mg = q.Multigrid(op, q.make_mg_params(block=b, nvec=N), vecs=dev(V))
    W = omg.block_orthonormalize(L, b, V)
    C = oracle.clover_build(L, U)
    rng = np.random.default_rng(741)
    for _ in range(2):
        ec = rng.standard_normal(mg.coarse_len()) + 1j * rng.standard_normal(mg.coarse_len())
        out = torch.empty_like(dev(ec))
        q.qcdw_mg_coarse_apply(mg, dev(ec), out)
        expect = omg.coarse_apply(L, b, W, U, C, ec.reshape(-1, 2, N), kappa, csw)
        assert rel(host(out).reshape(-1, 2, N), expect) < 1e-13
    mg.close()
    op.close()


def _sigma_min(mg):
    nc = 2 * mg.nvec
    Lc = mg.coarse_dims
    Y = torch.empty(int(np.prod(Lc)) * 9 * nc * nc, dtype=torch.complex128, device="cuda")
    q.qcdw_mg_coarse_op(mg, Y)
    D = _dense_from_stencil(host(Y).reshape(-1, 9, nc, nc), Lc, nc)
    return D, np.linalg.svd(D, compute_uv=False).min()


def test_generated_set_up_properties(ctx):
    """A set-up that makes its own near-null vectors: the block vectors are orthonormal per aggregate
    (P^+ P e = e), the coarse operator is gamma_5-hermitian, and the vectors are near-null: the coarse
    operator's smallest singular value is far below that of a set-up from random fields (the coarse space
    captures the low modes of M)."""
    L, b, N = (8, 8, 8, 8), (4, 4, 4, 4), 4
    U = li.random_gauge(L, 0.2, 75)
    kappa, csw = 0.125, 1.0
    op = q.Operator(ctx, q.make_lattice(L), dev(U), kappa, csw, "f32")
    mg = q.Multigrid(op, q.make_mg_params(block=b, nvec=N, setup_iters=60, seed=9))
    rng = np.random.default_rng(751)
    ec = rng.standard_normal(mg.coarse_len()) + 1j * rng.standard_normal(mg.coarse_len())
    f = torch.empty(li.fermion_shape(L), dtype=torch.complex128, device="cuda")
    back = torch.empty_like(dev(ec))
    q.qcdw_mg_prolong(mg, dev(ec), f)
    q.qcdw_mg_restrict(mg, f, back)
    assert rel(host(back), ec) < 1e-13
    D, smin = _sigma_min(mg)
    nc = 2 * N
    g5 = np.tile(np.repeat([1.0, -1.0], N), D.shape[0] // nc)
    assert np.abs(g5[:, None] * D * g5[None, :] - D.conj().T).max() < 1e-13 * np.abs(D).max()
    rnd = q.Multigrid(op, q.make_mg_params(block=b, nvec=N), vecs=dev(_vecs(L, N, 753)))
    _, smin_rnd = _sigma_min(rnd)
    assert smin < 0.3 * smin_rnd, (smin, smin_rnd)
    rnd.close()
    mg.close()
    op.close()


@pytest.mark.parametrize("inner", ["f64", "bf16"])
def test_multigrid_solve_reaches_tol_with_fewer_iterations(ctx, inner):
    """FGMRES with the multigrid preconditioner reaches an FP64 true residual of 1e-10 (recomputed by the
    oracle) in far fewer Arnoldi steps than unpreconditioned FGMRES, near the critical kappa."""
    L = (8, 8, 8, 16)
    U = li.random_gauge(L, 0.15, 76)
    kappa, csw = 0.1268, 1.0
    b_ = li.gaussian_source(L, 760)
    op = q.Operator(ctx, q.make_lattice(L), dev(U), kappa, csw, inner)
    mg = q.Multigrid(op, q.make_mg_params(block=(4, 4, 4, 4), nvec=8, setup_iters=80, coarse_iters=30))
    x = torch.zeros(li.fermion_shape(L), dtype=torch.complex128, device="cuda")
    info = q.qcdw_invert_mg(op, mg, dev(b_), x, q.make_params(tol=1e-10, maxiter=4000, gmres_fallback=0))
    C = oracle.clover_build(L, U)
    tr = np.linalg.norm(b_ - oracle.dirac(L, U, C, host(x), kappa, csw)) / np.linalg.norm(b_)
    assert info.status == q.QCDW_OK and tr <= 1e-10, (info, tr)
    x0 = torch.zeros_like(x)
    plain = q.qcdw_invert_fgmres(op, None, dev(b_), x0, q.make_params(tol=1e-10, maxiter=4000, gmres_fallback=0))
    assert info.iters * 4 < plain.iters, (info.iters, plain.iters)
    mg.close()
    op.close()


def test_multigrid_reused_for_another_mass(ctx):
    """The set-up made at one kappa preconditions the operator of another kappa on the same gauge field (the
    paper's reuse of a light-quark multigrid for heavier masses); the solve still reaches 1e-10."""
    L = (8, 8, 8, 8)
    U = li.random_gauge(L, 0.2, 77)
    b_ = li.gaussian_source(L, 770)
    light = q.Operator(ctx, q.make_lattice(L), dev(U), 0.126, 1.0, "f32")
    heavy = q.Operator(ctx, q.make_lattice(L), dev(U), 0.122, 1.0, "f32")
    mg = q.Multigrid(light, q.make_mg_params(block=(4, 4, 4, 4), nvec=6, setup_iters=60))
    x = torch.zeros(li.fermion_shape(L), dtype=torch.complex128, device="cuda")
    info = q.qcdw_invert_mg(heavy, mg, dev(b_), x, q.make_params(tol=1e-10, maxiter=2000))
    C = oracle.clover_build(L, U)
    tr = np.linalg.norm(b_ - oracle.dirac(L, U, C, host(x), 0.122, 1.0)) / np.linalg.norm(b_)
    assert info.status == q.QCDW_OK and tr <= 1e-10, (info, tr)
    mg.close()
    light.close()
    heavy.close()


def test_multigrid_rejects_bad_set_up(ctx):
    L = (4, 4, 4, 8)
    op = q.Operator(ctx, q.make_lattice(L), dev(li.random_gauge(L, 0.3, 78)), 0.12, 1.0, "f32")
    with pytest.raises(q.QcdwError, match="divide"):
        q.Multigrid(op, q.make_mg_params(block=(3, 2, 2, 2), nvec=2))
    with pytest.raises(q.QcdwError, match="even"):
        q.Multigrid(op, q.make_mg_params(block=(1, 1, 1, 1), nvec=2))
    with pytest.raises(q.QcdwError, match="nvec"):
        q.Multigrid(op, q.make_mg_params(block=(2, 2, 2, 2), nvec=33))
    V = np.zeros((2,) + li.fermion_shape(L), dtype=np.complex128)
    V[0] = li.gaussian_source(L, 780)
    V[1] = 2.0 * V[0]
    with pytest.raises(q.QcdwError, match="dependent"):
        q.Multigrid(op, q.make_mg_params(block=(2, 2, 2, 2), nvec=2), vecs=dev(V))
    op.close()
