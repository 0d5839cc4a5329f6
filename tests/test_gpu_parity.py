"""GPU parity: the HIP kernels, called through the C ABI, against the CPU oracle.

FP64 kernels must agree with the oracle to 1e-13 (relative, max over the
field); solves must reach an FP64 true residual <= 1e-10, recomputed by the
oracle from the returned x.  Lattices include extents whose half volume is not
a multiple of the 64-site tile (ragged tails) and antiperiodic time.
"""
import numpy as np
import pytest
import torch

import lattice_inputs as li
import oracle
import paper_2411_08461_amd as q

pytestmark = pytest.mark.gpu

# (L, ragged?)  Vh = 128, 144 (2.25 tiles), 720 (11.25 tiles), 4096
SMALL = [(4, 4, 4, 4), (6, 4, 2, 6), (10, 6, 4, 6), (8, 8, 8, 16)]


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


def _gauge(L, eps=0.3, seed=0):
    return li.random_gauge(L, eps, seed)


@pytest.mark.parametrize("L", SMALL)
def test_clover_build_matches_oracle(ctx, L):
    U = _gauge(L, 0.4, 1)
    lat = q.make_lattice(L)
    C = torch.empty(oracle.packed_shape(L), dtype=torch.float64, device="cuda")
    q.qcdw_clover_build(ctx, lat, dev(U), C)
    expect = oracle.clover_build(L, U)
    assert rel(host(C), expect) < 1e-13


@pytest.mark.parametrize("L", SMALL[:3])
def test_clover_apply_and_invert_match_oracle(ctx, L):
    U = _gauge(L, 0.4, 2)
    kappa, csw = 0.125, 1.1
    Cn = oracle.clover_build(L, U)
    lat = q.make_lattice(L)
    C = dev(Cn)
    psi = li.gaussian_source(L, 3)
    out = torch.empty(li.fermion_shape(L), dtype=torch.complex128, device="cuda")
    q.qcdw_clover_apply(ctx, lat, C, dev(psi), out, kappa, csw)
    assert rel(host(out), oracle.clover_apply(L, Cn, psi, kappa, csw)) < 1e-13
    inv = torch.empty_like(C)
    q.qcdw_clover_invert(ctx, lat, C, kappa, csw, inv)
    inv_o, bad = oracle.clover_invert(L, Cn, kappa, csw)
    assert bad == 0
    assert rel(host(inv), inv_o) < 1e-13


def test_clover_invert_reports_not_positive_definite(ctx):
    L = (4, 4, 4, 4)
    U = _gauge(L, 1.5, 4)
    Cn = oracle.clover_build(L, U)
    inv = torch.empty(Cn.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(q.QcdwError) as e:
        q.qcdw_clover_invert(ctx, q.make_lattice(L), dev(Cn), 1.0, 50.0, inv)
    assert e.value.status == q.QCDW_ENOTPD


@pytest.mark.parametrize("L", SMALL)
@pytest.mark.parametrize("t_bc", [1, -1])
@pytest.mark.parametrize("parity", [0, 1])
def test_hop_parity_matches_oracle(ctx, L, t_bc, parity):
    U = _gauge(L, 0.3, 5)
    psi = li.gaussian_source(L, 6)
    out = torch.empty(li.fermion_shape(L), dtype=torch.complex128, device="cuda")
    q.qcdw_hop(ctx, q.make_lattice(L, t_bc), dev(U), dev(psi), out, parity)
    # oracle: H_{p,1-p} psi = hop of psi restricted to the other parity, on parity p
    V = int(np.prod(L))
    src = psi.reshape(V, 4, 3).copy()
    src[parity * V // 2:(parity + 1) * V // 2] = 0
    expect = oracle.hop(L, U, src.reshape(psi.shape), t_bc, out_parity=parity)
    assert rel(host(out), expect) < 1e-13


@pytest.mark.parametrize("L", SMALL)
@pytest.mark.parametrize("t_bc", [1, -1])
def test_dslash_full_operator_matches_oracle(ctx, L, t_bc):
    U = _gauge(L, 0.3, 7)
    kappa, csw = 0.124, 1.0
    psi = li.gaussian_source(L, 8)
    lat = q.make_lattice(L, t_bc)
    out = torch.empty(li.fermion_shape(L), dtype=torch.complex128, device="cuda")
    q.qcdw_dslash(ctx, lat, dev(U), None, dev(psi), out, kappa, csw)
    Cn = oracle.clover_build(L, U)
    expect = oracle.dirac(L, U, Cn, psi, kappa, csw, t_bc)
    assert rel(host(out), expect) < 1e-13
    # with a caller-provided clover field
    out2 = torch.empty_like(out)
    q.qcdw_dslash(ctx, lat, dev(U), dev(Cn), dev(psi), out2, kappa, csw)
    assert rel(host(out2), expect) < 1e-13


@pytest.mark.parametrize("L", SMALL)
@pytest.mark.parametrize("recon", [12, 18])
def test_matpc_matches_oracle_schur(ctx, L, recon):
    U = _gauge(L, 0.3, 9)
    kappa, csw = 0.124, 1.0
    lat = q.make_lattice(L)
    op = q.Operator(ctx, lat, dev(U), kappa, csw, "f64", recon)
    Vh = int(np.prod(L)) // 2
    xe = li.gaussian_source(L, 10).reshape(-1, 4, 3)[:Vh].copy()
    out = torch.empty((Vh, 4, 3), dtype=torch.complex128, device="cuda")
    q.qcdw_op_matpc(op, "f64", dev(xe), out)
    Ainv, _ = oracle.clover_invert(L, oracle.clover_build(L, U), kappa, csw)
    expect = oracle.schur_matpc(L, U, Ainv, xe, kappa)
    assert rel(host(out), expect) < 1e-13
    op.close()


@pytest.mark.parametrize("prec,bound", [("f32", 2e-6), ("bf16", 2e-2), ("f16", 4e-3)])
def test_matpc_low_precision_error_bounded(ctx, prec, bound):
    """16-bit / FP32 storage with FP32 arithmetic against the FP64 oracle."""
    L = (8, 8, 8, 16)
    U = _gauge(L, 0.2, 11)
    kappa, csw = 0.124, 1.0
    op = q.Operator(ctx, q.make_lattice(L), dev(U), kappa, csw, prec, 12)
    Vh = int(np.prod(L)) // 2
    xe = li.gaussian_source(L, 12).reshape(-1, 4, 3)[:Vh].copy()
    out = torch.empty((Vh, 4, 3), dtype=torch.complex128, device="cuda")
    q.qcdw_op_matpc(op, prec, dev(xe), out)
    Ainv, _ = oracle.clover_invert(L, oracle.clover_build(L, U), kappa, csw)
    expect = oracle.schur_matpc(L, U, Ainv, xe, kappa)
    err = np.linalg.norm(host(out) - expect) / np.linalg.norm(expect)
    print(f"matpc {prec} relative error {err:.3e}")
    assert err < bound
    op.close()


def _forced_nt_context(tmp_path, monkeypatch, L, nt, cg=0, fma=0):
    """A context whose tuning cache fixes the single-RHS hop's form: nt sites per thread along t,
    groups of cg c-tiles swept along t, and the arithmetic form."""
    cache = tmp_path / f"tune_nt{nt}_cg{cg}_f{fma}_{'x'.join(map(str, L))}.txt"
    cache.write_text("".join(f"hop_nt/p{p}/L{L[0]}x{L[1]}x{L[2]}x{L[3]} {nt + 16 * cg + 4096 * fma}\n"
                             for p in range(4)))
    monkeypatch.setenv("QCDW_TUNE_CACHE", str(cache))
    return q.Context(0)


@pytest.mark.parametrize("L", [(8, 8, 8, 16), (6, 4, 2, 8), (10, 6, 4, 8)])
@pytest.mark.parametrize("nt,cg,fma", [(2, 0, 0), (4, 0, 0), (1, 1, 0), (1, 2, 0), (2, 1, 0), (4, 2, 0),
                                       (1, 0, 1), (2, 0, 1), (4, 0, 1), (1, 1, 1), (2, 1, 1), (1, 1, 2), (1, 2, 3)])
def test_t_stepping_matpc(tmp_path, monkeypatch, L, nt, cg, fma):
    """M_hat through the other single-RHS hop forms (nt sites per thread along t; tiles of one
    t-slice swept along t in groups of cg c-tiles; the multiply-add arithmetic form) equals the
    oracle to 1e-13 in FP64 and the plain one-site-per-thread kernel to rounding in every
    precision (the same operations per site, contracted into FMAs differently); lattices with
    t-slices of several tiles, of a partial tile, and a ragged last tile."""
    nct = (L[0] // 2 * L[1] * L[2] + 63) // 64
    if nct % max(cg, 1) or L[3] % (2 * nt):
        pytest.skip("form does not fit this lattice")
    U = _gauge(L, 0.3, 41)
    kappa, csw = 0.124, 1.0
    Vh = int(np.prod(L)) // 2
    xe = dev(li.gaussian_source(L, 42).reshape(-1, 4, 3)[:Vh].copy())
    outs = {}
    for n, g, f in ((1, 0, 0), (nt, cg, fma)):
        c = _forced_nt_context(tmp_path, monkeypatch, L, n, g, f)
        for prec in ("f64", "bf16", "f16", "f32"):
            op = q.Operator(c, q.make_lattice(L), dev(U), kappa, csw, prec, 12)
            assert q.qcdw_op_hop_form(op, "f64") == (n, g, f) and q.qcdw_op_hop_form(op, prec) == (n, g, f)
            for pr in ("f64", prec):
                out = torch.empty((Vh, 4, 3), dtype=torch.complex128, device="cuda")
                q.qcdw_op_matpc(op, pr, xe, out)
                outs[(n + 16 * g + 4096 * f, prec, pr)] = host(out)
            op.close()
        torch.cuda.synchronize()
        c.close()
    Ainv, _ = oracle.clover_invert(L, oracle.clover_build(L, U), kappa, csw)
    expect = oracle.schur_matpc(L, U, Ainv, host(xe), kappa)
    code = nt + 16 * cg + 4096 * fma
    assert rel(outs[(code, "f64", "f64")], expect) < 1e-13
    bound = {"f64": 1e-14, "f32": 1e-6, "f16": 2e-3, "bf16": 1e-2}
    for key, val in outs.items():
        if key[0] == code:
            assert rel(val, outs[(1,) + key[1:]]) < bound[key[2]], key


@pytest.mark.parametrize("L", [(8, 8, 8, 16), (6, 4, 2, 8), (10, 6, 4, 8)])
def test_lds_staged_hop_bitwise_equals_unstaged(tmp_path, monkeypatch, L):
    """The slice-group hop with its t-neighbour spinors staged in LDS (fma bit 1) runs the same arithmetic
    on the same values as the unstaged form: M_hat is bitwise equal in every precision, for both
    arithmetic forms, on lattices whose t-slices hold several tiles, one partial tile and a ragged last
    tile."""
    U = _gauge(L, 0.3, 43)
    kappa, csw = 0.124, 1.0
    Vh = int(np.prod(L)) // 2
    xe = dev(li.gaussian_source(L, 44).reshape(-1, 4, 3)[:Vh].copy())
    outs = {}
    for f in (0, 1, 2, 3):
        c = _forced_nt_context(tmp_path, monkeypatch, L, 1, 1, f)
        for prec in ("f32", "bf16", "f16"):
            op = q.Operator(c, q.make_lattice(L), dev(U), kappa, csw, prec, 12)
            assert q.qcdw_op_hop_form(op, "f64") == (1, 1, f)
            for pr in ("f64", prec):
                out = torch.empty((Vh, 4, 3), dtype=torch.complex128, device="cuda")
                q.qcdw_op_matpc(op, pr, xe, out)
                outs[(f, prec, pr)] = host(out)
            op.close()
        torch.cuda.synchronize()
        c.close()
    for (f, prec, pr), val in outs.items():
        if f & 2:
            assert np.array_equal(val, outs[(f & 1, prec, pr)]), (f, prec, pr)


# ---------------------------------------------------------------------------
# solver
# ---------------------------------------------------------------------------


def _oracle_true_res(L, U, x, b, kappa, csw, t_bc=1):
    Cn = oracle.clover_build(L, U)
    r = b - oracle.dirac(L, U, Cn, x, kappa, csw, t_bc)
    return np.linalg.norm(r) / np.linalg.norm(b)


def test_invert_dense_lu_4444(ctx):
    """4^4, kappa 0.12, csw 1, eps 0.3, point source: GPU solve vs LAPACK dense LU."""
    w = li.WORKLOADS["dense4"]
    L = w["L"]
    U = li.random_gauge(L, w["eps"], w["seed"])
    b = li.point_source(L)
    Cn = oracle.clover_build(L, U)
    M = oracle.dense_matrix(L, U, Cn, w["kappa"], w["csw"])
    x_lu = np.linalg.solve(M, b.ravel())
    cond = np.linalg.cond(M)
    op = q.Operator(ctx, q.make_lattice(L), dev(U), w["kappa"], w["csw"])
    x = torch.zeros(li.fermion_shape(L), dtype=torch.complex128, device="cuda")
    info = q.qcdw_invert(op, dev(b), x, q.make_params(tol=1e-10))
    print(info)
    assert info.status == q.QCDW_OK
    xh = host(x)
    assert info.true_res <= 1e-10
    assert _oracle_true_res(L, U, xh, b, w["kappa"], w["csw"]) <= 1e-10
    assert np.linalg.norm(xh.ravel() - x_lu) / np.linalg.norm(x_lu) <= cond * 1e-10
    assert info.res_hist[0] == pytest.approx(np.linalg.norm(
        oracle.schur_source(L, U, oracle.clover_invert(L, Cn, w["kappa"], w["csw"])[0], b, w["kappa"]))
        / np.linalg.norm(b), rel=1e-12)
    op.close()


@pytest.mark.parametrize("L,t_bc", [((6, 4, 2, 6), 1), ((10, 6, 4, 6), -1), ((8, 8, 8, 16), 1)])
@pytest.mark.parametrize("inner", ["f64", "f32", "bf16", "f16"])
def test_invert_reaches_tolerance(ctx, L, t_bc, inner):
    U = _gauge(L, 0.25, 13)
    kappa, csw = 0.122, 1.0
    b = li.gaussian_source(L, 14)
    op = q.Operator(ctx, q.make_lattice(L, t_bc), dev(U), kappa, csw, inner)
    x = torch.zeros(li.fermion_shape(L), dtype=torch.complex128, device="cuda")
    info = q.qcdw_invert(op, dev(b), x, q.make_params(tol=1e-10, inner=inner, delta=0.1 if inner == "f32" else 0.2))
    print(inner, info)
    assert info.status == q.QCDW_OK
    tr = _oracle_true_res(L, U, host(x), b, kappa, csw, t_bc)
    print(f"oracle true residual {tr:.3e}")
    assert tr <= 1e-10
    ref = oracle.bicgstab(L, U, oracle.clover_build(L, U), b, kappa, csw, tol=1e-12, maxiter=5000, t_bc=t_bc)
    assert ref.status == 0
    err = np.linalg.norm(host(x) - ref.x) / np.linalg.norm(ref.x)
    print(f"solution error vs oracle {err:.3e}")
    assert err < 1e-8
    op.close()


def test_invert_statuses_and_restarts(ctx):
    L = (8, 8, 8, 16)
    U = _gauge(L, 0.25, 15)
    kappa, csw = 0.122, 1.0
    b = li.gaussian_source(L, 16)
    op = q.Operator(ctx, q.make_lattice(L), dev(U), kappa, csw)
    x = torch.zeros(li.fermion_shape(L), dtype=torch.complex128, device="cuda")
    info = q.qcdw_invert(op, dev(b), x, q.make_params(maxiter=3))
    assert info.status == q.QCDW_ENOCONV and info.iters == 3 and info.true_res > 1e-10
    bn = b.copy()
    bn.ravel()[5] = np.nan
    x.zero_()
    info = q.qcdw_invert(op, dev(bn), x, q.make_params())
    assert info.status == q.QCDW_ENAN
    x.fill_(1.0)
    info = q.qcdw_invert(op, torch.zeros_like(x), x, q.make_params())
    assert info.status == q.QCDW_OK and float(x.abs().max()) == 0.0
    x.zero_()
    info = q.qcdw_invert(op, dev(b), x, q.make_params(fault_inject=5))
    assert info.status == q.QCDW_OK and info.n_restarts == 1
    assert _oracle_true_res(L, U, host(x), b, kappa, csw) <= 1e-10
    # resume from a good guess: converges in (almost) no iterations
    info2 = q.qcdw_invert(op, dev(b), x, q.make_params())
    assert info2.status == q.QCDW_OK and info2.iters <= 2
    op.close()


def test_invert_is_deterministic(ctx):
    L = (10, 6, 4, 6)
    U = _gauge(L, 0.25, 17)
    b = li.gaussian_source(L, 18)
    op = q.Operator(ctx, q.make_lattice(L), dev(U), 0.122, 1.0)
    xs, its = [], []
    for _ in range(3):
        x = torch.zeros(li.fermion_shape(L), dtype=torch.complex128, device="cuda")
        info = q.qcdw_invert(op, dev(b), x, q.make_params())
        xs.append(host(x))
        its.append(info.iters)
    assert its[0] == its[1] == its[2]
    assert np.array_equal(xs[0], xs[1]) and np.array_equal(xs[0], xs[2])
    op.close()


# ---------------------------------------------------------------------------
# invariants checked on the GPU operator itself
# ---------------------------------------------------------------------------


def test_gpu_free_field_plane_wave(ctx):
    L = (8, 4, 6, 8)
    kappa = 0.11
    U = li.unit_gauge(L)
    c = oracle.coords_table(L)
    g = [oracle.gamma(m) for m in range(4)]
    rng = np.random.default_rng(3)
    n = np.array([1, 3, 2, 5])
    p = 2 * np.pi * n / np.asarray(L)
    u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    phase = np.exp(1j * (c @ p))
    psi = (phase[:, None, None] * u[None]).reshape(li.fermion_shape(L))
    out = torch.empty(psi.shape, dtype=torch.complex128, device="cuda")
    q.qcdw_dslash(ctx, q.make_lattice(L), dev(U), None, dev(psi), out, kappa, 1.7)
    K = (1 - 2 * kappa * np.cos(p).sum()) * np.eye(4) + 2j * kappa * sum(g[m] * np.sin(p[m]) for m in range(4))
    expect = (phase[:, None, None] * (K @ u)[None]).reshape(psi.shape)
    assert rel(host(out), expect) < 1e-14


def test_gpu_gamma5_hermiticity(ctx):
    L = (6, 4, 2, 6)
    U = _gauge(L, 0.4, 19)
    kappa, csw = 0.124, 1.2
    chi = li.gaussian_source(L, 20)
    psi = li.gaussian_source(L, 21)
    g5 = np.array([1, 1, -1, -1])[:, None]
    lat = q.make_lattice(L)

    def M(v):
        out = torch.empty(v.shape, dtype=torch.complex128, device="cuda")
        q.qcdw_dslash(ctx, lat, dev(U), None, dev(v), out, kappa, csw)
        return host(out)

    lhs = np.vdot(chi, g5 * M(g5 * psi))
    rhs = np.vdot(M(chi), psi)
    assert abs(lhs - rhs) / abs(rhs) < 1e-13


# ---------------------------------------------------------------------------
# workload sizes of the benchmark
# ---------------------------------------------------------------------------


@pytest.fixture(scope="module")
def wc16():
    w = li.WORKLOADS["wc16x32"]
    L = w["L"]
    U = li.random_gauge(L, w["eps"], w["seed"])
    b = li.z2_source(L, w["source_seed"])
    return L, U, b, w


def test_wc16x32_matpc_full_size(ctx, wc16):
    """16^3x32: the benchmark's FP64 reconstruct-12 M_hat against the oracle on every site."""
    L, U, b, w = wc16
    op = q.Operator(ctx, q.make_lattice(L), dev(U), w["kappa"], w["csw"])
    Vh = int(np.prod(L)) // 2
    xe = b.reshape(-1, 4, 3)[:Vh].copy()
    out = torch.empty((Vh, 4, 3), dtype=torch.complex128, device="cuda")
    q.qcdw_op_matpc(op, "f64", dev(xe), out)
    Ainv, _ = oracle.clover_invert(L, oracle.clover_build(L, U), w["kappa"], w["csw"])
    expect = oracle.schur_matpc(L, U, Ainv, xe, w["kappa"])
    assert rel(host(out), expect) < 1e-13
    op.close()


@pytest.mark.parametrize("inner", ["f64", "f32", "bf16", "f16"])
def test_wc16x32_solve(ctx, wc16, inner):
    """16^3x32, kappa 0.124, Z2 source: every precision reaches the FP64 true residual 1e-10."""
    L, U, b, w = wc16
    op = q.Operator(ctx, q.make_lattice(L), dev(U), w["kappa"], w["csw"], inner)
    x = torch.zeros(li.fermion_shape(L), dtype=torch.complex128, device="cuda")
    info = q.qcdw_invert(op, dev(b), x, q.make_params(tol=1e-10, inner=inner, delta=0.1 if inner != "f16" else 0.2))
    print(inner, info)
    assert info.status == q.QCDW_OK
    tr = _oracle_true_res(L, U, host(x), b, w["kappa"], w["csw"])
    print(f"oracle true residual {tr:.3e}")
    assert tr <= 1e-10
    op.close()


@pytest.mark.parametrize("inner", ["f64", "bf16"])
def test_graph_replay_matches_eager(ctx, inner):
    """Graph-replayed iteration chunks give bitwise the same solve as eager launches.

    Several solves alternate between the two paths (with the program's own eager
    work and synchronisations in between), so every replay of the cached graphs
    is checked against the eager result.
    """
    L = (8, 8, 8, 16)
    U = _gauge(L, 0.25, 23)
    b = li.gaussian_source(L, 24)
    op = q.Operator(ctx, q.make_lattice(L), dev(U), 0.122, 1.0, inner)
    ref = None
    for rep in range(3):
        for graph in (False, True):
            x = torch.zeros(li.fermion_shape(L), dtype=torch.complex128, device="cuda")
            info = q.qcdw_invert(op, dev(b), x, q.make_params(inner=inner, delta=0.2, check_every=5,
                                                             use_graph=graph))
            torch.cuda.synchronize()
            assert info.status == q.QCDW_OK
            xh = host(x)
            if ref is None:
                ref = (xh, info.iters, info.res_hist)
            assert np.array_equal(xh, ref[0]) and info.iters == ref[1], (rep, graph)
            assert info.res_hist == ref[2]
            _ = torch.ones(1000, device="cuda").sum().item()  # unrelated eager work between replays
    op.close()


# ---------------------------------------------------------------------------
# multi-RHS
# ---------------------------------------------------------------------------


@pytest.mark.parametrize("L", [(6, 4, 2, 6), (10, 6, 4, 6)])
@pytest.mark.parametrize("prec,nrhs", [("f64", 3), ("f64", 12), ("bf16", 12), ("f32", 5)])
def test_matpc_multi_matches_oracle(ctx, L, prec, nrhs):
    U = _gauge(L, 0.3, 25)
    kappa, csw = 0.124, 1.0
    op = q.Operator(ctx, q.make_lattice(L), dev(U), kappa, csw, "f64" if prec == "f64" else prec, 12)
    Vh = int(np.prod(L)) // 2
    xs = np.stack([li.gaussian_source(L, 100 + k).reshape(-1, 4, 3)[:Vh] for k in range(nrhs)])
    out = torch.empty(xs.shape, dtype=torch.complex128, device="cuda")
    q.qcdw_op_matpc_multi(op, prec, dev(xs), out)
    Ainv, _ = oracle.clover_invert(L, oracle.clover_build(L, U), kappa, csw)
    got = host(out)
    for k in range(nrhs):
        expect = oracle.schur_matpc(L, U, Ainv, xs[k], kappa)
        if prec == "f64":
            assert rel(got[k], expect) < 1e-13, k
        else:
            err = np.linalg.norm(got[k] - expect) / np.linalg.norm(expect)
            assert err < (2e-6 if prec == "f32" else 2e-2), (k, err)
    # the single-RHS kernel agrees to rounding in the same storage precision
    one = torch.empty((Vh, 4, 3), dtype=torch.complex128, device="cuda")
    q.qcdw_op_matpc(op, prec, dev(xs[nrhs - 1]), one)
    bound = {"f64": 1e-14, "f32": 1e-6, "bf16": 1e-2}[prec]
    assert rel(host(one), got[nrhs - 1]) < bound
    op.close()


@pytest.mark.parametrize("inner", ["f64", "bf16"])
def test_invert_multi_propagator(ctx, inner):
    """12 point sources (all spins and colours): lockstep solve equals 12 single solves."""
    L = (8, 8, 8, 16)
    U = _gauge(L, 0.25, 26)
    kappa, csw = 0.122, 1.1
    op = q.Operator(ctx, q.make_lattice(L), dev(U), kappa, csw, inner)
    bs = np.stack([li.point_source(L, s, c) for s in range(4) for c in range(3)])
    x = torch.zeros(bs.shape, dtype=torch.complex128, device="cuda")
    prm = q.make_params(tol=1e-10, inner=inner, delta=0.2)
    infos = q.qcdw_invert_multi(op, dev(bs), x, prm)
    Cn = oracle.clover_build(L, U)
    xh = host(x)
    for k in range(12):
        assert infos[k].status == q.QCDW_OK, (k, infos[k])
        tr = np.linalg.norm(bs[k] - oracle.dirac(L, U, Cn, xh[k], kappa, csw)) / np.linalg.norm(bs[k])
        assert tr <= 1e-10, (k, tr)
    for k in (0, 7, 11):
        x1 = torch.zeros(li.fermion_shape(L), dtype=torch.complex128, device="cuda")
        info = q.qcdw_invert(op, dev(bs[k]), x1, prm)
        assert info.status == q.QCDW_OK
        assert np.linalg.norm(host(x1) - xh[k]) / np.linalg.norm(xh[k]) < 1e-8
    op.close()


def test_invert_multi_masks_finished_rhs(ctx):
    """A zero RHS and an easy RHS finish early; the others keep iterating alone."""
    L = (6, 4, 2, 6)
    U = _gauge(L, 0.25, 27)
    op = q.Operator(ctx, q.make_lattice(L), dev(U), 0.122, 1.0)
    b = np.stack([li.gaussian_source(L, 30), np.zeros(li.fermion_shape(L)), li.gaussian_source(L, 31)])
    x = torch.zeros(b.shape, dtype=torch.complex128, device="cuda")
    x[2] = dev(oracle.bicgstab(L, U, oracle.clover_build(L, U), b[2], 0.122, 1.0, tol=1e-9).x)
    infos = q.qcdw_invert_multi(op, dev(b), x, q.make_params())
    assert [i.status for i in infos] == [q.QCDW_OK] * 3
    assert float(x[1].abs().max()) == 0.0
    assert infos[2].iters < infos[0].iters
    op.close()


# ---------------------------------------------------------------------------
# batched solves of different lattices and kappas
# ---------------------------------------------------------------------------


@pytest.mark.parametrize("inner", ["f64", "bf16"])
def test_invert_batch_uneven(ctx, inner):
    """Lattices of different sizes and kappas in one lockstep batch; each equals its solo solve."""
    specs = [((4, 4, 4, 4), 0.115), ((6, 4, 2, 6), 0.121), ((8, 8, 8, 16), 0.124), ((10, 6, 4, 6), 0.118),
             ((4, 4, 4, 4), 0.123)]
    ops, Us, bs, xs = [], [], [], []
    for k, (L, kappa) in enumerate(specs):
        U = li.random_gauge(L, 0.25, 100 + k)
        Us.append(U)
        ops.append(q.Operator(ctx, q.make_lattice(L), dev(U), kappa, 1.0, inner))
        bs.append(dev(li.gaussian_source(L, 1100 + k)))
        xs.append(torch.zeros(li.fermion_shape(L), dtype=torch.complex128, device="cuda"))
    batch = q.Batch(ctx, ops)
    prm = q.make_params(tol=1e-10, inner=inner, delta=0.2)
    infos = q.qcdw_invert_batch(batch, bs, xs, prm)
    for k, (L, kappa) in enumerate(specs):
        assert infos[k].status == q.QCDW_OK, (k, infos[k])
        bh = host(bs[k])
        Cn = oracle.clover_build(L, Us[k])
        tr = np.linalg.norm(bh - oracle.dirac(L, Us[k], Cn, host(xs[k]), kappa, 1.0)) / np.linalg.norm(bh)
        assert tr <= 1e-10, (k, tr)
        x1 = torch.zeros_like(xs[k])
        solo = q.qcdw_invert(ops[k], bs[k], x1, prm)
        assert solo.status == q.QCDW_OK
        assert np.linalg.norm(host(x1) - host(xs[k])) / np.linalg.norm(host(x1)) < 1e-8
    # the batch is reusable (cached graphs and tuned grid), with the same result
    xs2 = [torch.zeros_like(x) for x in xs]
    infos2 = q.qcdw_invert_batch(batch, bs, xs2, prm)
    for k in range(len(specs)):
        assert infos2[k].status == q.QCDW_OK and infos2[k].iters == infos[k].iters
        assert np.array_equal(host(xs2[k]), host(xs[k]))
    batch.close()
    for op in ops:
        op.close()


def test_invert_batch_many_small_problems(ctx):
    """More problems than right-hand sides of a propagator (regression: per-problem host staging)."""
    n = 24
    L = (4, 4, 4, 4)
    ops, bs, xs, Us, ks = [], [], [], [], []
    for k in range(n):
        U = li.random_gauge(L, 0.25, 200 + k)
        kappa = 0.115 + 0.0004 * k
        Us.append(U)
        ks.append(kappa)
        ops.append(q.Operator(ctx, q.make_lattice(L), dev(U), kappa, 1.0))
        bs.append(dev(li.gaussian_source(L, 1200 + k)))
        xs.append(torch.zeros(li.fermion_shape(L), dtype=torch.complex128, device="cuda"))
    batch = q.Batch(ctx, ops)
    infos = q.qcdw_invert_batch(batch, bs, xs, q.make_params())
    for k in range(n):
        assert infos[k].status == q.QCDW_OK
        bh = host(bs[k])
        r = bh - oracle.dirac(L, Us[k], oracle.clover_build(L, Us[k]), host(xs[k]), ks[k], 1.0)
        assert np.linalg.norm(r) / np.linalg.norm(bh) <= 1e-10
    batch.close()
    for op in ops:
        op.close()


def test_mixed_solve_escalates_to_f64_after_an_overflow(ctx):
    """An overflow flagged in the low-precision cycle (forced at iteration 5) drops that cycle's
    correction and finishes in FP64; an FP64 solve reports it as ENAN."""
    L = (8, 8, 8, 16)
    U = _gauge(L, 0.25, 15)
    kappa, csw = 0.122, 1.0
    b = li.gaussian_source(L, 16)
    op = q.Operator(ctx, q.make_lattice(L), dev(U), kappa, csw, "bf16")
    x = torch.zeros(li.fermion_shape(L), dtype=torch.complex128, device="cuda")
    info = q.qcdw_invert(op, dev(b), x, q.make_params(inner="bf16", fault_inject=-5))
    assert info.status == q.QCDW_OK and info.fallback == 1 and 0 < info.fallback_iters < info.iters
    assert _oracle_true_res(L, U, host(x), b, kappa, csw) <= 1e-10
    x.zero_()
    plain = q.qcdw_invert(op, dev(b), x, q.make_params(inner="bf16"))
    assert plain.status == q.QCDW_OK and plain.fallback == 0
    x.zero_()
    info64 = q.qcdw_invert(op, dev(b), x, q.make_params(fault_inject=-5))
    assert info64.status == q.QCDW_ENAN
    op.close()


def test_mixed_solve_escalates_near_the_critical_kappa(ctx):
    """Near kappa_c the BF16-rounded operator is too far from the FP64 one for the low-precision
    cycles to converge: the solver detects the stall and finishes in FP64 to the same tolerance."""
    L = (8, 8, 8, 16)
    U = li.random_gauge(L, 0.15, 0)
    kappa, csw = 0.1278, 1.0
    b = li.gaussian_source(L, 1000)
    op = q.Operator(ctx, q.make_lattice(L), dev(U), kappa, csw, "bf16")
    x = torch.zeros(li.fermion_shape(L), dtype=torch.complex128, device="cuda")
    info = q.qcdw_invert(op, dev(b), x, q.make_params(inner="bf16", maxiter=6000))
    print(info, info.fallback, info.fallback_iters)
    assert info.status == q.QCDW_OK and info.fallback == 1
    assert _oracle_true_res(L, U, host(x), b, kappa, csw) <= 1e-10
    op.close()


@pytest.mark.parametrize("nt,cg,fma", [(1, 0, 0), (2, 0, 0), (4, 0, 0), (1, 1, 0), (2, 1, 0), (1, 0, 1), (2, 1, 1),
                                       (1, 1, 3)])
def test_t_stepping_hop_in_solves(tmp_path, monkeypatch, nt, cg, fma):
    """Solves whose single-RHS hops take a forced form (nt sites per thread along t, slice groups,
    arithmetic form; through the tuning cache) reach an oracle-checked true residual <= 1e-10, in
    FP64 and BF16-mixed solves, on a lattice whose t-slices are several tiles and one whose
    t-slice is a partial tile."""
    for L, eps, seed in (((8, 8, 8, 16), 0.25, 31), ((6, 4, 2, 8), 0.3, 32)):
        c = _forced_nt_context(tmp_path, monkeypatch, L, nt, cg, fma)
        U = _gauge(L, eps, seed)
        b = li.gaussian_source(L, seed + 100)
        kappa, csw = 0.121, 1.0
        op = q.Operator(c, q.make_lattice(L), dev(U), kappa, csw, "bf16")
        for inner in ("f64", "bf16"):
            x = torch.zeros(li.fermion_shape(L), dtype=torch.complex128, device="cuda")
            info = q.qcdw_invert(op, dev(b), x, q.make_params(inner=inner))
            assert info.status == q.QCDW_OK, (L, inner, info)
            assert _oracle_true_res(L, U, host(x), b, kappa, csw) <= 1e-10
        op.close()
        torch.cuda.synchronize()
        c.close()


@pytest.mark.parametrize("inner", ["f32", "bf16", "f16"])
def test_mixed_solve_resuming_the_recurrence(ctx, inner):
    """Reliable updates that continue the recurrence (inner_resume) reach the same oracle-checked
    tolerance; on this well-conditioned system they need no more iterations than restarting."""
    L = (8, 8, 8, 16)
    U = li.random_gauge(L, 0.15, 0)
    kappa, csw = 0.124, 1.0
    b = li.gaussian_source(L, 1000)
    op = q.Operator(ctx, q.make_lattice(L), dev(U), kappa, csw, inner)
    its = {}
    for resume in (False, True):
        x = torch.zeros(li.fermion_shape(L), dtype=torch.complex128, device="cuda")
        info = q.qcdw_invert(op, dev(b), x, q.make_params(inner=inner, delta=0.2 if inner == "f16" else 0.1,
                                                            inner_resume=resume))
        assert info.status == q.QCDW_OK, (resume, info)
        assert _oracle_true_res(L, U, host(x), b, kappa, csw) <= 1e-10
        its[resume] = info.iters
    print(inner, its)
    assert its[True] <= its[False]
    op.close()


@pytest.mark.parametrize("variant", [0, 1, 2, 4, 1024, 1028])
def test_multi_rhs_forms(tmp_path, monkeypatch, variant):
    """Lockstep multi-RHS solves with each hop form forced through the tuning cache (register loop,
    L2-reuse per RHS, register loop in slice-group order with groups of 1 or 2 c-tiles, and the
    matrix-core form of the BF16 hop in both tile orders) reach an oracle-checked true residual <= 1e-10
    for every RHS, in FP64 and BF16-mixed, the BF16-mixed ones without falling back to FP64."""
    for L in ((8, 8, 8, 16), (6, 4, 2, 8)):
        nct = (L[0] // 2 * L[1] * L[2] + 63) // 64
        if (variant & 1) == 0 and nct % max((variant & 1023) >> 1, 1):
            continue
        nrhs = 3
        cache = tmp_path / f"tune_mrhs_{variant}_{L[0]}.txt"
        cache.write_text("".join(f"mrhs_hop/p{p}/L{L[0]}x{L[1]}x{L[2]}x{L[3]}/n{nrhs} {variant}\n" for p in range(4)))
        monkeypatch.setenv("QCDW_TUNE_CACHE", str(cache))
        c = q.Context(0)
        U = _gauge(L, 0.25, 51)
        kappa, csw = 0.121, 1.0
        bs = np.stack([li.gaussian_source(L, 52 + k) for k in range(nrhs)])
        op = q.Operator(c, q.make_lattice(L), dev(U), kappa, csw, "bf16")
        for inner in ("f64", "bf16"):
            x = torch.zeros(bs.shape, dtype=torch.complex128, device="cuda")
            infos = q.qcdw_invert_multi(op, dev(bs), x, q.make_params(inner=inner))
            xh = host(x)
            for k in range(nrhs):
                assert infos[k].status == q.QCDW_OK, (L, inner, k, infos[k])
                assert infos[k].fallback == 0, (L, inner, k, infos[k])
                assert _oracle_true_res(L, U, xh[k], bs[k], kappa, csw) <= 1e-10
        op.close()
        torch.cuda.synchronize()
        c.close()
        assert f" {variant}" in cache.read_text()


@pytest.mark.parametrize("L,t_bc,cg", [((6, 4, 2, 6), 1, 0), ((10, 6, 4, 6), -1, 0), ((8, 8, 8, 16), -1, 2)])
@pytest.mark.parametrize("prec", ["bf16", "f16"])
@pytest.mark.parametrize("aniso", [False, True])
def test_matpc_multi_mfma_form(tmp_path, monkeypatch, L, t_bc, cg, prec, aniso):
    """The matrix-core multi-RHS hop (forced through the tuning cache, plain and slice-group tile order)
    gives M_hat within the storage rounding of the oracle for every RHS (the single-RHS bounds), and
    agrees with the vector register loop to the same rounding; lattices with ragged tiles, both time
    boundaries, and the anisotropic weights with antiperiodic time."""
    nrhs = 12
    key = f"mrhs_hop/p{q.PREC[prec]}/L{L[0]}x{L[1]}x{L[2]}x{L[3]}/n{nrhs}"
    cache = tmp_path / "tune_mfma.txt"
    cache.write_text(f"{key} {1024 + 2 * cg}\n")
    monkeypatch.setenv("QCDW_TUNE_CACHE", str(cache))
    c_mfma = q.Context(0)
    monkeypatch.delenv("QCDW_TUNE_CACHE")
    c_vec = q.Context(0)
    U = _gauge(L, 0.3, 61)
    Vh = int(np.prod(L)) // 2
    xs = np.stack([li.gaussian_source(L, 62 + k).reshape(-1, 4, 3)[:Vh] for k in range(nrhs)])
    if aniso:
        xi0, nu, ct, cr = 2.464, 0.95, 0.91, 1.07
        kappa, csw, kw = oracle.aniso_kappa(0.3, xi0, nu), 0.0, dict(aniso=(xi0, nu, ct, cr))
        C = oracle.clover_build(L, U, plane_weights=(ct, cr / xi0))
        Ainv, _ = oracle.clover_invert(L, C, kappa, 1.0)
        weights = oracle.aniso_weights(xi0, nu)
    else:
        kappa, csw, kw = 0.124, 1.0, {}
        Ainv, _ = oracle.clover_invert(L, oracle.clover_build(L, U), kappa, csw)
        weights = None
    outs = []
    for c in (c_mfma, c_vec):
        op = q.Operator(c, q.make_lattice(L, t_bc), dev(U), kappa, csw, prec, 12, **kw)
        out = torch.empty(xs.shape, dtype=torch.complex128, device="cuda")
        q.qcdw_op_matpc_multi(op, prec, dev(xs), out)
        outs.append(host(out))
        op.close()
    bound = {"bf16": 2e-2, "f16": 4e-3}[prec]
    for k in range(nrhs):
        if weights is None:
            expect = oracle.schur_matpc(L, U, Ainv, xs[k], kappa, t_bc)
        else:
            expect = oracle.schur_matpc(L, U, Ainv, xs[k], kappa, t_bc, weights=weights)
        err = np.linalg.norm(outs[0][k] - expect) / np.linalg.norm(expect)
        assert err < bound, (k, err)
        assert np.linalg.norm(outs[0][k] - outs[1][k]) / np.linalg.norm(outs[1][k]) < bound / 2, k
    torch.cuda.synchronize()
    c_mfma.close()
    c_vec.close()


@pytest.mark.parametrize("inner", ["f64", "bf16"])
def test_fused_scalar_steps_match_separate_kernels(ctx, monkeypatch, inner):
    """The BiCGStab scalars formed inside the vector kernels (every block sums the partials) give
    bitwise the same iterations, residual histories and solutions as the single-block finaliser
    kernels: single RHS, lockstep multi-RHS and an uneven batch, in FP64 and BF16-mixed."""
    L = (8, 8, 8, 16)
    U = _gauge(L, 0.25, 61)
    kappa, csw = 0.122, 1.0
    b = li.gaussian_source(L, 62)
    bs = np.stack([li.gaussian_source(L, 63 + k) for k in range(3)])
    specs = [((4, 4, 4, 4), 0.115), ((6, 4, 2, 6), 0.121), ((10, 6, 4, 6), 0.118)]
    op = q.Operator(ctx, q.make_lattice(L), dev(U), kappa, csw, inner)
    bops = [q.Operator(ctx, q.make_lattice(Lb), dev(li.random_gauge(Lb, 0.25, 70 + k)), kb, 1.0, inner)
            for k, (Lb, kb) in enumerate(specs)]
    bbs = [dev(li.gaussian_source(Lb, 80 + k)) for k, (Lb, _) in enumerate(specs)]
    batch = q.Batch(ctx, bops)
    prm = q.make_params(tol=1e-10, inner=inner)
    res = {}
    for fuse in ("0", "1000000"):
        monkeypatch.setenv("QCDW_FUSE_NB", fuse)
        x = torch.zeros(li.fermion_shape(L), dtype=torch.complex128, device="cuda")
        info = q.qcdw_invert(op, dev(b), x, prm)
        xm = torch.zeros(bs.shape, dtype=torch.complex128, device="cuda")
        infos = q.qcdw_invert_multi(op, dev(bs), xm, prm)
        xb = [torch.zeros(li.fermion_shape(Lb), dtype=torch.complex128, device="cuda") for Lb, _ in specs]
        binfos = q.qcdw_invert_batch(batch, bbs, xb, prm)
        for i in [info] + list(infos) + list(binfos):
            assert i.status == q.QCDW_OK, (fuse, i)
        res[fuse] = ([i.iters for i in [info] + list(infos) + list(binfos)],
                     [i.res_hist for i in [info] + list(infos) + list(binfos)],
                     [host(x), host(xm)] + [host(t) for t in xb])
    assert res["0"][0] == res["1000000"][0]
    assert res["0"][1] == res["1000000"][1]
    for a, c in zip(res["0"][2], res["1000000"][2]):
        assert np.array_equal(a, c)
    assert _oracle_true_res(L, U, res["0"][2][0], b, kappa, csw) <= 1e-10
    batch.close()
    for o in [op] + bops:
        o.close()


def test_operators_reuse_cached_device_blocks(ctx):
    """Operators created after others were closed take their device blocks from the cache (the same
    sizes, then other sizes in between): every solve gives bitwise the solution of the first operator
    on the same inputs, and a different lattice created in between still solves to the oracle."""
    L, L2 = (8, 8, 8, 16), (6, 4, 2, 6)
    U = _gauge(L, 0.25, 91)
    U2 = _gauge(L2, 0.25, 92)
    b = dev(li.gaussian_source(L, 93))
    b2 = dev(li.gaussian_source(L2, 94))
    prm = q.make_params(tol=1e-10, inner="bf16")

    def solve(Lx, Ux, bx, kappa):
        op = q.Operator(ctx, q.make_lattice(Lx), dev(Ux), kappa, 1.0, "bf16")
        x = torch.zeros(li.fermion_shape(Lx), dtype=torch.complex128, device="cuda")
        info = q.qcdw_invert(op, bx, x, prm)
        op.close()
        assert info.status == q.QCDW_OK
        return host(x), info.iters

    x0, it0 = solve(L, U, b, 0.122)
    for k in range(3):
        x2, _ = solve(L2, U2, b2, 0.118)
        assert _oracle_true_res(L2, U2, x2, host(b2), 0.118, 1.0) <= 1e-10
        x1, it1 = solve(L, U, b, 0.122)
        assert it1 == it0 and np.array_equal(x1, x0), k
