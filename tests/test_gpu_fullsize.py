"""GPU parity at the benchmark's full sizes, in the launch configurations bench.py times.

- The 24^3x64 FP64 M_hat (kappa 0.125, csw 1.1) element by element against the oracle to 1e-13, with the
  single-RHS hop form forced (slice groups of 27 c-tiles with the multiply-add form, and the plain
  one-site-per-thread form) and with the tuner's own pick; at this size the hop's dot partials exceed the
  fused-scalar threshold, so the separate scalar kernels run.
- The 12-RHS BF16 propagator at 24^3x64 (all spins and colours of a point source, lockstep multi-RHS
  solve): every right-hand side's FP64 true residual recomputed by the oracle.
- The 48-problem uneven batch of the benchmark (16 each of 8^3x16, 12^3x24, 16^3x32), FP64 and
  BF16-mixed: every solution's true residual recomputed by the oracle.
- Gauge covariance of the GPU operator itself: M[U'](Om psi) = Om M[U] psi for a Haar-random transform.
"""
import numpy as np
import pytest
import torch

import lattice_inputs as li
import oracle
import paper_2411_08461_amd as q
from tests import geometry as geo
from tests.fieldgen import random_gauges_in_child

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.fixture(scope="module")
def wc24():
    """The 24^3x64 field of the benchmark, its clover inverse and the oracle's M_hat of a Z2 vector."""
    w = li.WORKLOADS["wc24x64"]
    L, kappa, csw = w["L"], w["kappa"], w["csw"]
    U = li.random_gauge(L, w["eps"], w["seed"])
    Vh = int(np.prod(L)) // 2
    xe = li.z2_source(L, 1000).reshape(-1, 4, 3)[:Vh].copy()
    Ainv, _ = oracle.clover_invert(L, oracle.clover_build(L, U), kappa, csw)
    expect = oracle.schur_matpc(L, U, Ainv, xe, kappa)
    del Ainv
    return L, U, xe, expect, w


def _forced_context(tmp_path, monkeypatch, L, form):
    cache = tmp_path / "tune.txt"
    if form is None:
        monkeypatch.delenv("QCDW_TUNE_CACHE", raising=False)
    else:
        nt, cg, fma = form
        cache.write_text("".join(f"hop_nt/p{p}/L{L[0]}x{L[1]}x{L[2]}x{L[3]} {nt + 16 * cg + 4096 * fma}\n"
                                 for p in range(4)))
        monkeypatch.setenv("QCDW_TUNE_CACHE", str(cache))
    return q.Context(0)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("form", [(1, 27, 1), (1, 0, 0), None], ids=["cg27-fma", "plain", "tuned"])
def test_wc24x64_matpc_matches_oracle(tmp_path, monkeypatch, wc24, form):
    L, U, xe, expect, w = wc24
    c = _forced_context(tmp_path, monkeypatch, L, form)
    op = q.Operator(c, q.make_lattice(L), dev(U), w["kappa"], w["csw"], "bf16", 12)
    got_form = q.qcdw_op_hop_form(op, "f64")
    if form is not None:
        assert got_form == form
    out = torch.empty(xe.shape, dtype=torch.complex128, device="cuda")
    q.qcdw_op_matpc(op, "f64", dev(xe), out)
    err = rel(host(out), expect)
    print(f"24^3x64 M_hat FP64, form {got_form}: max relative error {err:.3e}")
    assert err < 1e-13
    q.qcdw_op_matpc(op, "bf16", dev(xe), out)
    err16 = np.linalg.norm(host(out) - expect) / np.linalg.norm(expect)
    print(f"24^3x64 M_hat BF16 storage: relative error {err16:.3e}")
    assert err16 < 1e-2
    op.close()
    torch.cuda.synchronize()
    c.close()


@pytest.mark.timeout(300)
def test_wc24x64_propagator_bf16_multi_rhs(wc24):
    L, U, _, _, w = wc24
    kappa, csw = w["kappa"], w["csw"]
    ctx = q.Context(0)
    op = q.Operator(ctx, q.make_lattice(L), dev(U), kappa, csw, "bf16", 12)
    bs = torch.zeros((12,) + li.fermion_shape(L), dtype=torch.complex128, device="cuda")
    for s in range(4):
        for c in range(3):
            bs[3 * s + c][0, 0, 0, 0, 0, s, c] = 1.0
    x = torch.zeros_like(bs)
    infos = q.qcdw_invert_multi(op, bs, x, q.make_params(tol=1e-10, maxiter=20000, inner="bf16", delta=0.1))
    op.close()
    torch.cuda.synchronize()
    ctx.close()
    C = oracle.clover_build(L, U)
    for k in range(12):
        assert infos[k].status == q.QCDW_OK, (k, infos[k])
        b = li.point_source(L, k // 3, k % 3)
        tr = np.linalg.norm(b - oracle.dirac(L, U, C, host(x[k]), kappa, csw)) / np.linalg.norm(b)
        print(f"rhs {k}: {infos[k].iters} iterations, oracle true residual {tr:.3e}")
        assert tr <= 1e-10, (k, tr)


@pytest.mark.timeout(400)
def test_batch48_bench_workload(tmp_path):
    specs = li.batch48()
    Us = random_gauges_in_child([(p["L"], p["eps"], p["seed"]) for p in specs], tmp_path)
    ctx = q.Context(0)
    ops = [q.Operator(ctx, q.make_lattice(p["L"]), dev(U), p["kappa"], p["csw"], "bf16", 12)
           for p, U in zip(specs, Us)]
    bs = [li.gaussian_source(p["L"], p["source_seed"]) for p in specs]
    bds = [dev(b) for b in bs]
    bt = q.Batch(ctx, ops)
    sols = {}
    for prec in ("f64", "bf16"):
        xs = [torch.zeros_like(b) for b in bds]
        infos = q.qcdw_invert_batch(bt, bds, xs, q.make_params(tol=1e-10, maxiter=20000, inner=prec, delta=0.1))
        sols[prec] = (infos, [host(x) for x in xs])
    bt.close()
    for op in ops:
        op.close()
    torch.cuda.synchronize()
    ctx.close()
    worst = {}
    for k, (p, U, b) in enumerate(zip(specs, Us, bs)):
        C = oracle.clover_build(p["L"], U)
        for prec, (infos, xs) in sols.items():
            assert infos[k].status == q.QCDW_OK, (prec, k, infos[k])
            tr = np.linalg.norm(b - oracle.dirac(p["L"], U, C, xs[k], p["kappa"], p["csw"])) / np.linalg.norm(b)
            assert tr <= 1e-10, (prec, k, tr)
            worst[prec] = max(worst.get(prec, 0.0), tr)
    print(f"48 problems: worst oracle true residual {worst}")


@pytest.mark.parametrize("L,t_bc", [((6, 4, 2, 6), -1), ((8, 8, 8, 16), 1)])
def test_gpu_operator_gauge_covariance(L, t_bc):
    """The GPU's full operator (clover built on the GPU) is gauge covariant to 1e-13:
    M[U'](Om psi) = Om M[U] psi with U'_mu(x) = Om(x) U_mu(x) Om(x+mu)^+."""
    V = int(np.prod(L))
    U = li.random_gauge(L, 0.4, 61)
    Om = li.gauge_transform(L, 62).reshape(V, 3, 3)
    psi = li.gaussian_source(L, 63)
    Up = geo.transform_gauge(L, U, Om)
    rot = lambda f: np.einsum("iab,isb->isa", Om, f.reshape(V, 4, 3)).reshape(f.shape)  # noqa: E731
    kappa, csw = 0.124, 1.3
    ctx = q.Context(0)
    lat = q.make_lattice(L, t_bc)
    a = torch.empty(li.fermion_shape(L), dtype=torch.complex128, device="cuda")
    b = torch.empty_like(a)
    q.qcdw_dslash(ctx, lat, dev(U), None, dev(psi), a, kappa, csw)
    q.qcdw_dslash(ctx, lat, dev(Up), None, dev(rot(psi)), b, kappa, csw)
    torch.cuda.synchronize()
    ctx.close()
    err = rel(host(b), rot(host(a)))
    print(f"gauge covariance of the GPU operator: {err:.3e}")
    assert err < 1e-13
