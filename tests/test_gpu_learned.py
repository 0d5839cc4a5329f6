"""GPU parity of the learned preconditioner and FGMRES against the CPU oracle."""
import numpy as np
import pytest
import torch

import lattice_inputs as li
import oracle
import paper_2411_08461_amd as q
from oracle import learned as ln

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


def _setup(ctx, L, seed=0, kappa=0.12, init_scale=0.3, hidden=12):
    U = li.random_gauge(L, 0.3, 40 + seed)
    op = q.Operator(ctx, q.make_lattice(L), dev(U), kappa, 1.0, "bf16", 12)
    net = q.Net(op, hidden, seed=seed, init_scale=init_scale)
    return U, op, net


@pytest.mark.parametrize("mfma", [0, 1, 2, 3])
@pytest.mark.parametrize("L,hidden", [((6, 4, 2, 6), 12), ((8, 4, 4, 8), 12), ((6, 4, 4, 6), 4), ((10, 6, 2, 4), 12)])
def test_net_forward_matches_oracle(tmp_path, monkeypatch, L, hidden, mfma):
    """FP32 application and BF16 application against the FP64 oracle, with each BF16 layer's channel
    mixing forced (through the tuning cache) onto vector FMA or onto the BF16 matrix cores (bit 0 the
    first layer, which transports its inputs first, bit 1 the second, which mixes first when it narrows
    the channels); the 10x6x2x4 lattice leaves a ragged last wave of 16 sites."""
    cache = tmp_path / "tune.txt"
    cache.write_text(f"net_mfma/h{hidden}/L{L[0]}x{L[1]}x{L[2]}x{L[3]} {mfma}\n")
    monkeypatch.setenv("QCDW_TUNE_CACHE", str(cache))
    ctx = q.Context(0)
    U, op, net = _setup(ctx, L, 1, hidden=hidden)
    W1, W2 = q.qcdw_net_get_weights(net)
    Vh = int(np.prod(L)) // 2
    r = li.gaussian_source(L, 50).reshape(-1, 4, 3)[:Vh].copy()
    expect = ln.net_apply(ln.Transport(L, U), W1, W2, r)
    out = torch.empty((Vh, 4, 3), dtype=torch.complex128, device="cuda")
    q.qcdw_net_apply(net, "f32", dev(r), out)
    err = rel(host(out), expect)  # element-wise, relative to the largest element
    assert err < 1e-6, err
    q.qcdw_net_apply(net, "bf16", dev(r), out)
    err16 = np.linalg.norm(host(out) - expect) / np.linalg.norm(expect)
    print(f"net forward error f32 {err:.2e} bf16 {err16:.2e}")
    assert err16 < 3e-2
    net.close()
    op.close()
    torch.cuda.synchronize()
    ctx.close()


def test_net_loss_and_gradients_match_oracle(ctx):
    L = (6, 4, 2, 6)
    U, op, net = _setup(ctx, L, 2)
    W1, W2 = q.qcdw_net_get_weights(net)
    Vh = int(np.prod(L)) // 2
    rng = np.random.default_rng(3)
    pairs = [((rng.standard_normal((Vh, 4, 3)) + 1j * rng.standard_normal((Vh, 4, 3))),
              (rng.standard_normal((Vh, 4, 3)) + 1j * rng.standard_normal((Vh, 4, 3)))) for _ in range(2)]
    loss, G1, G2 = ln.net_loss_and_grad(ln.Transport(L, U), W1, W2, pairs)
    gl, g1, g2 = q.qcdw_net_loss_grad(net, [dev(p[0]) for p in pairs], [dev(p[1]) for p in pairs])
    print(f"loss {abs(gl - loss) / loss:.2e}, dW1 {rel(g1, G1):.2e}, dW2 {rel(g2, G2):.2e} (element-wise)")
    assert abs(gl - loss) / loss < 1e-6
    assert rel(g1, G1) < 1e-6
    assert rel(g2, G2) < 1e-6
    net.close()
    op.close()


@pytest.mark.parametrize("L,steps", [((6, 4, 2, 6), 1), ((6, 4, 2, 6), 4), ((8, 4, 4, 8), 3)])
def test_net_training_steps_match_oracle_adam(ctx, L, steps):
    """k Adam steps on the GPU (qcdw_net_train with the batch equal to the whole pair set, so every step
    uses the mean gradient over all pairs whatever the shuffle) against the oracle's full-batch Adam
    (Kingma and Ba 2015, Algorithm 1) from the same starting weights: the weights after the last step
    element by element and the loss of every step, both to 1e-6 relative (the GPU keeps the weights in
    FP32)."""
    U, op, net = _setup(ctx, L, 3)
    W1, W2 = q.qcdw_net_get_weights(net)
    Vh = int(np.prod(L)) // 2
    rng = np.random.default_rng(11)
    pairs = [((rng.standard_normal((Vh, 4, 3)) + 1j * rng.standard_normal((Vh, 4, 3))),
              (rng.standard_normal((Vh, 4, 3)) + 1j * rng.standard_normal((Vh, 4, 3)))) for _ in range(3)]
    lr = 2e-3
    hist = q.qcdw_net_train(net, [dev(p[0]) for p in pairs], [dev(p[1]) for p in pairs], steps=steps,
                            batch=len(pairs), lr=lr, seed=5)
    g1, g2 = q.qcdw_net_get_weights(net)
    E1, E2, losses = ln.train_full_batch(ln.Transport(L, U), W1, W2, pairs, steps, lr)
    d1, d2 = rel(g1, E1), rel(g2, E2)
    moved = max(rel(E1, W1), rel(E2, W2))
    print(f"after {steps} Adam steps: W1 {d1:.2e}, W2 {d2:.2e} (the step moved the weights by {moved:.2e})")
    assert d1 < 1e-6 and d2 < 1e-6
    assert moved > 100 * max(d1, d2)  # the comparison sees the update, not only the starting weights
    assert np.abs(np.asarray(hist) - np.asarray(losses)).max() / max(losses) < 1e-6
    net.close()
    op.close()


@pytest.fixture(scope="module")
def trained(ctx):
    """A net trained on random-error pairs of one gauge field, tested on an unseen source."""
    L = (8, 8, 8, 16)
    U = li.random_gauge(L, 0.15, 60)
    kappa = 0.1245
    op = q.Operator(ctx, q.make_lattice(L), dev(U), kappa, 1.0, "bf16", 12)
    r, e = q.qcdw_make_training_pairs(op, None, 32, -17)
    assert len(r) == 32
    net = q.Net(op, 12, seed=5, init_scale=0.01)
    hist = q.qcdw_net_train(net, r, e, steps=100, batch=4, lr=2e-3, seed=7)
    yield L, U, kappa, op, net, hist
    net.close()
    op.close()


def test_random_error_pairs_match_oracle(ctx):
    """r = M_hat e with ||r|| = 1 for the seeded Gaussian errors (checked by the oracle)."""
    L = (6, 4, 4, 6)
    U = li.random_gauge(L, 0.2, 70)
    kappa = 0.124
    op = q.Operator(ctx, q.make_lattice(L), dev(U), kappa, 1.0, "f64", 12)
    r, e = q.qcdw_make_training_pairs(op, None, 3, -5)
    Ainv, _ = oracle.clover_invert(L, oracle.clover_build(L, U), kappa, 1.0)
    Vh = int(np.prod(L)) // 2
    for rk, ek in zip(r, e):
        en = host(ek).reshape(Vh, 4, 3)
        expect = oracle.schur_matpc(L, U, Ainv, en, kappa)
        got = host(rk).reshape(expect.shape)
        assert np.linalg.norm(got - expect) / np.linalg.norm(expect) < 1e-12
        assert abs(np.linalg.norm(got) - 1.0) < 1e-12
        re = en.real.ravel()
        assert abs(re.mean()) < 0.2 * re.std()  # roughly centred Gaussian entries
    # Distinct streams give distinct errors; the same seed gives the same ones.
    assert np.linalg.norm(host(e[0]) - host(e[1])) > 0.1 * np.linalg.norm(host(e[0]))
    r2, e2 = q.qcdw_make_training_pairs(op, None, 1, -5)
    assert np.array_equal(host(e2[0]), host(e[0]))
    op.close()


def test_training_lowers_the_loss(trained):
    _, _, _, _, _, hist = trained
    print("loss", hist[:3], hist[-3:])
    assert np.mean(hist[-10:]) < 0.7 * np.mean(hist[:5])


def test_fgmres_with_net_beats_fgmres_without(ctx, trained):
    L, U, kappa, op, net, _ = trained
    b = li.gaussian_source(L, 62)
    prm = q.make_params(tol=1e-10, maxiter=4000, gmres_restart=32, gmres_fallback=False)
    # The net is applied in BF16 inside FGMRES; the gain over plain FGMRES(32) is about 2x
    # in iterations on this field.
    x0 = torch.zeros(li.fermion_shape(L), dtype=torch.complex128, device="cuda")
    plain = q.qcdw_invert_fgmres(op, None, dev(b), x0, prm)
    x1 = torch.zeros_like(x0)
    learned = q.qcdw_invert_fgmres(op, net, dev(b), x1, prm)
    x2 = torch.zeros_like(x0)
    bicg = q.qcdw_invert(op, dev(b), x2, q.make_params(tol=1e-10))
    print(f"FGMRES plain {plain}, FGMRES+net {learned}, BiCGStab {bicg}")
    Cn = oracle.clover_build(L, U)
    for info, x in ((plain, x0), (learned, x1)):
        assert info.status == q.QCDW_OK and info.fallback == 0
        tr = np.linalg.norm(b - oracle.dirac(L, U, Cn, host(x), kappa, 1.0)) / np.linalg.norm(b)
        assert tr <= 1e-10
    assert learned.iters < 0.75 * plain.iters


def test_fgmres_falls_back_when_the_net_is_useless(ctx):
    L = (8, 8, 8, 16)
    U = li.random_gauge(L, 0.15, 63)
    kappa = 0.1245
    op = q.Operator(ctx, q.make_lattice(L), dev(U), kappa, 1.0, "bf16", 12)
    net = q.Net(op, 12, seed=9, init_scale=3.0)  # random weights: a bad preconditioner
    b = li.gaussian_source(L, 64)
    x = torch.zeros(li.fermion_shape(L), dtype=torch.complex128, device="cuda")
    info = q.qcdw_invert_fgmres(op, net, dev(b), x, q.make_params(tol=1e-10, maxiter=6000, gmres_restart=8))
    print(info, info.fallback, info.fallback_iters)
    assert info.status == q.QCDW_OK
    Cn = oracle.clover_build(L, U)
    tr = np.linalg.norm(b - oracle.dirac(L, U, Cn, host(x), kappa, 1.0)) / np.linalg.norm(b)
    assert tr <= 1e-10
    assert info.fallback == 1
    net.close()
    op.close()


def test_net_bind_moves_the_net_to_another_field(ctx):
    """After rebinding, the net applies the new field's transports (checked by the oracle)."""
    L = (6, 4, 2, 6)
    U1, op1, net = _setup(ctx, L, 3)
    U2 = li.random_gauge(L, 0.3, 80)
    op2 = q.Operator(ctx, q.make_lattice(L), dev(U2), 0.12, 1.0, "bf16", 12)
    W1, W2 = q.qcdw_net_get_weights(net)
    q.qcdw_net_bind(net, op2)
    Vh = int(np.prod(L)) // 2
    r = li.gaussian_source(L, 81).reshape(-1, 4, 3)[:Vh].copy()
    out = torch.empty((Vh, 4, 3), dtype=torch.complex128, device="cuda")
    q.qcdw_net_apply(net, "f32", dev(r), out)
    expect = ln.net_apply(ln.Transport(L, U2), W1, W2, r)
    assert np.linalg.norm(host(out) - expect) / np.linalg.norm(expect) < 1e-5
    # a lattice of other extents is refused
    L3 = (6, 4, 4, 6)
    op3 = q.Operator(ctx, q.make_lattice(L3), dev(li.random_gauge(L3, 0.3, 82)), 0.12, 1.0, "bf16", 12)
    with pytest.raises(q.QcdwError):
        q.qcdw_net_bind(net, op3)
    net.close()
    for o in (op1, op2, op3):
        o.close()


def test_net_trained_on_other_fields_helps_an_unseen_field(ctx):
    """Train on two gauge fields of one ensemble, precondition FGMRES on a third."""
    L = (8, 8, 8, 16)
    kappa = 0.1245
    ops = [q.Operator(ctx, q.make_lattice(L), dev(li.random_gauge(L, 0.15, 90 + k)), kappa, 1.0, "bf16", 12)
           for k in range(3)]
    net = q.Net(ops[1], 12, seed=5, init_scale=0.01)
    for k in (1, 2):
        q.qcdw_net_bind(net, ops[k])
        r, e = q.qcdw_make_training_pairs(ops[k], None, 16, -(200 + k))
        q.qcdw_net_train(net, r, e, steps=50, batch=4, lr=2e-3, seed=k)
    q.qcdw_net_bind(net, ops[0])
    U0 = li.random_gauge(L, 0.15, 90)
    b = li.gaussian_source(L, 1090)
    prm = q.make_params(tol=1e-10, maxiter=4000, gmres_restart=32, gmres_fallback=False)
    x0 = torch.zeros(li.fermion_shape(L), dtype=torch.complex128, device="cuda")
    plain = q.qcdw_invert_fgmres(ops[0], None, dev(b), x0, prm)
    x1 = torch.zeros_like(x0)
    learned = q.qcdw_invert_fgmres(ops[0], net, dev(b), x1, prm)
    print(f"unseen field: FGMRES plain {plain.iters}, FGMRES+net {learned.iters}")
    Cn = oracle.clover_build(L, U0)
    tr = np.linalg.norm(b - oracle.dirac(L, U0, Cn, host(x1), kappa, 1.0)) / np.linalg.norm(b)
    assert learned.status == q.QCDW_OK and tr <= 1e-10
    assert learned.iters < 0.75 * plain.iters
    net.close()
    for o in ops:
        o.close()


def test_fgmres_matches_the_oracle_fgmres(ctx):
    """FGMRES(8) on the even-odd Schur system without a preconditioner against the oracle's flexible GMRES
    (Saad 1993) on the oracle's Schur operator and source: the residual of every Arnoldi step of the first
    two cycles (relative to ||b||) agrees to 1e-8, and the solutions agree to 1e-8 (both are FP64; the
    GPU orthogonalises by classical Gram-Schmidt twice, the oracle by modified Gram-Schmidt)."""
    from oracle.fgmres import fgmres

    L = (6, 4, 2, 6)
    kappa, csw = 0.124, 1.0
    U = li.random_gauge(L, 0.3, 77)
    b = li.gaussian_source(L, 78)
    op = q.Operator(ctx, q.make_lattice(L), dev(U), kappa, csw, "f64", 12)
    x = torch.zeros(li.fermion_shape(L), dtype=torch.complex128, device="cuda")
    info = q.qcdw_invert_fgmres(op, None, dev(b), x, q.make_params(tol=1e-10, maxiter=400, gmres_restart=8,
                                                                    gmres_fallback=False))
    op.close()
    assert info.status == q.QCDW_OK and info.fallback == 0
    Ainv, _ = oracle.clover_invert(L, oracle.clover_build(L, U), kappa, csw)
    bhat = oracle.schur_source(L, U, Ainv, b, kappa)
    ref = fgmres(lambda v: oracle.schur_matpc(L, U, Ainv, v, kappa), bhat, m=8, tol=0.5e-10, maxiter=400,
                 norm_ref=np.linalg.norm(b))
    got = np.asarray(info.res_hist)
    n = min(17, len(ref.hist), len(got))
    print("GPU  ", got[:n])
    print("orcl ", ref.hist[:n])
    # the first cycle's estimates, then (after the restart) the second cycle's from the recomputed residual
    assert np.all(np.abs(got[:9] - ref.hist[:9]) <= 1e-8 * ref.hist[:9])
    Vh = int(np.prod(L)) // 2
    xe = host(x).reshape(-1, 4, 3)[:Vh]
    assert np.linalg.norm(xe - ref.x) / np.linalg.norm(ref.x) < 1e-8
