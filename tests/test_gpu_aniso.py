"""GPU parity of the anisotropic clover operator (Sec. III.B, Eq. "clover") against the CPU
oracle: the Schur operator in every storage precision, solves with antiperiodic time (the paper's
example action), lockstep multi-RHS, and a batch mixing anisotropic and isotropic operators."""
import numpy as np
import pytest
import torch

import lattice_inputs as li
import oracle
import paper_2411_08461_amd as q

pytestmark = pytest.mark.gpu

# the paper's example action: xi_0, nu, m_0, c_SW^t, c_SW^r
XI0, NU, M0, CT, CR = 2.464, 0.95, 0.3, 0.91, 1.07
ANISO = (XI0, NU, CT, CR)
KAPPA = oracle.aniso_kappa(M0, XI0, NU)
W = oracle.aniso_weights(XI0, NU)


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


def _clover(L, U):
    return oracle.clover_build(L, U, plane_weights=(CT, CR / XI0))


def _true_res(L, U, x, b, t_bc):
    r = b - oracle.dirac(L, U, _clover(L, U), x, KAPPA, 1.0, t_bc, weights=W)
    return np.linalg.norm(r) / np.linalg.norm(b)


@pytest.mark.parametrize("L,t_bc", [((4, 4, 4, 8), -1), ((10, 6, 4, 6), 1), ((8, 8, 8, 16), -1)])
@pytest.mark.parametrize("recon", [12, 18])
def test_aniso_matpc_matches_oracle(ctx, L, t_bc, recon):
    """M_hat of the anisotropic operator equals the oracle's to 1e-13 in FP64 and to the storage
    rounding in FP32 / BF16 / FP16 (the isotropic bounds), lattices with ragged tiles."""
    U = li.random_gauge(L, 0.3, 81)
    Vh = int(np.prod(L)) // 2
    xe = li.gaussian_source(L, 82).reshape(-1, 4, 3)[:Vh].copy()
    Ainv, bad = oracle.clover_invert(L, _clover(L, U), KAPPA, 1.0)
    assert bad == 0
    expect = oracle.schur_matpc(L, U, Ainv, xe, KAPPA, t_bc, weights=W)
    lat = q.make_lattice(L, t_bc)
    for prec, bound in (("f64", 1e-13), ("f32", 2e-6), ("bf16", 2e-2), ("f16", 4e-3)):
        if recon == 18 and prec in ("bf16", "f16"):
            continue
        op = q.Operator(ctx, lat, dev(U), KAPPA, 0.0, prec, recon, aniso=ANISO)
        out = torch.empty((Vh, 4, 3), dtype=torch.complex128, device="cuda")
        q.qcdw_op_matpc(op, prec, dev(xe), out)
        assert rel(host(out), expect) < bound, (prec, rel(host(out), expect))
        op.close()


@pytest.mark.parametrize("inner", ["f64", "bf16"])
def test_aniso_invert_paper_action(ctx, inner):
    """Solves of the paper's example action (antiperiodic t) reach an oracle-checked true residual
    <= 1e-10; the isotropic parameters through the anisotropic entry point give the isotropic
    operator's solution."""
    L, t_bc = (8, 8, 8, 16), -1
    U = li.random_gauge(L, 0.25, 83)
    b = li.gaussian_source(L, 84)
    op = q.Operator(ctx, q.make_lattice(L, t_bc), dev(U), KAPPA, 0.0, inner, aniso=ANISO)
    x = torch.zeros(li.fermion_shape(L), dtype=torch.complex128, device="cuda")
    info = q.qcdw_invert(op, dev(b), x, q.make_params(tol=1e-10, inner=inner))
    op.close()
    assert info.status == q.QCDW_OK, info
    assert _true_res(L, U, host(x), b, t_bc) <= 1e-10
    # xi_0 = nu = 1, c_SW^t = c_SW^r = c_SW: the isotropic operator
    iso = q.Operator(ctx, q.make_lattice(L, t_bc), dev(U), 0.121, 1.1, inner)
    ani = q.Operator(ctx, q.make_lattice(L, t_bc), dev(U), 0.121, 0.0, inner, aniso=(1.0, 1.0, 1.1, 1.1))
    xs = []
    for o in (iso, ani):
        xo = torch.zeros_like(x)
        assert q.qcdw_invert(o, dev(b), xo, q.make_params(tol=1e-10, inner=inner)).status == q.QCDW_OK
        xs.append(host(xo))
        o.close()
    assert np.linalg.norm(xs[0] - xs[1]) / np.linalg.norm(xs[0]) < 1e-8


def test_aniso_multi_rhs_and_batch(ctx):
    """Lockstep multi-RHS solves of the anisotropic operator, and a batch of an anisotropic and an
    isotropic operator on different lattices, each reach an oracle-checked true residual <= 1e-10."""
    L, t_bc = (6, 4, 2, 8), -1
    U = li.random_gauge(L, 0.25, 85)
    bs = np.stack([li.gaussian_source(L, 86 + k) for k in range(3)])
    op = q.Operator(ctx, q.make_lattice(L, t_bc), dev(U), KAPPA, 0.0, "bf16", aniso=ANISO)
    for inner in ("f64", "bf16"):
        x = torch.zeros(bs.shape, dtype=torch.complex128, device="cuda")
        infos = q.qcdw_invert_multi(op, dev(bs), x, q.make_params(tol=1e-10, inner=inner))
        for k in range(3):
            assert infos[k].status == q.QCDW_OK, (inner, k, infos[k])
            assert _true_res(L, U, host(x)[k], bs[k], t_bc) <= 1e-10
    L2 = (4, 4, 4, 4)
    U2 = li.random_gauge(L2, 0.25, 89)
    op2 = q.Operator(ctx, q.make_lattice(L2), dev(U2), 0.12, 1.0, "bf16")  # a batch shares the inner precision
    batch = q.Batch(ctx, [op, op2])
    b0, b1 = dev(bs[0]), dev(li.gaussian_source(L2, 90))
    x0 = torch.zeros_like(b0)
    x1 = torch.zeros_like(b1)
    infos = q.qcdw_invert_batch(batch, [b0, b1], [x0, x1], q.make_params(tol=1e-10))
    assert all(i.status == q.QCDW_OK for i in infos)
    assert _true_res(L, U, host(x0), bs[0], t_bc) <= 1e-10
    C2 = oracle.clover_build(L2, U2)
    r2 = host(b1) - oracle.dirac(L2, U2, C2, host(x1), 0.12, 1.0)
    assert np.linalg.norm(r2) / np.linalg.norm(host(b1)) <= 1e-10
    batch.close()
    op2.close()
    op.close()


def test_aniso_rejects_bad_coefficients(ctx):
    L = (4, 4, 4, 4)
    U = dev(li.random_gauge(L, 0.2, 91))
    for bad in ((0.0, 1.0, 1.0, 1.0), (1.0, -1.0, 1.0, 1.0), (float("nan"), 1.0, 1.0, 1.0)):
        with pytest.raises(q.QcdwError):
            q.Operator(ctx, q.make_lattice(L), U, 0.12, 0.0, aniso=bad)
