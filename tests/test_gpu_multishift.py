"""GPU multi-shift CG on the normal even-odd operator against dense solves of each shifted system
(the oracle's normal_shifted_solve)."""
import numpy as np
import pytest
import torch

import lattice_inputs as li
import oracle
import paper_2411_08461_amd as q

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.fixture(scope="module")
def ctx():
    c = q.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


@pytest.mark.parametrize("L,t_bc", [((4, 4, 2, 4), 1), ((6, 4, 2, 6), -1)])
def test_multishift_matches_dense_solves(ctx, L, t_bc):
    """Every shifted solution has a true normal-equation residual <= 1e-10 (dense N, FP64) and equals
    the dense solve; the reported residuals are those true residuals (recomputed on the GPU)."""
    U = li.random_gauge(L, 0.3, 97)
    kappa, csw = 0.12, 1.0
    Vh = int(np.prod(L)) // 2
    b = li.gaussian_source(L, 98).reshape(-1, 4, 3)[:Vh].copy()
    shifts = [0.0, 0.001, 0.05, 0.7, 3.0]
    op = q.Operator(ctx, q.make_lattice(L, t_bc), dev(U), kappa, csw)
    xs = [torch.empty((Vh, 4, 3), dtype=torch.complex128, device="cuda") for _ in shifts]
    it, res = q.qcdw_invert_multishift(op, dev(b), xs, shifts, tol=1e-10)
    op.close()
    assert it > 0 and max(res) <= 1e-10
    Ainv, _ = oracle.clover_invert(L, oracle.clover_build(L, U), kappa, csw)
    M = oracle.schur_dense(L, U, Ainv, kappa, t_bc)
    N = M.conj().T @ M
    expect = oracle.normal_shifted_solve(L, U, Ainv, b, kappa, shifts, t_bc)
    for x, e, s, rep in zip(xs, expect, shifts, res):
        xh = x.cpu().numpy().reshape(-1)
        r = (N + s * np.eye(N.shape[0])) @ xh - b.reshape(-1)
        tr = np.linalg.norm(r) / np.linalg.norm(b)
        assert tr <= 1e-10, s
        assert abs(rep - tr) <= 1e-2 * tr + 1e-14, (s, rep, tr)
        assert np.linalg.norm(xh - e.reshape(-1)) / np.linalg.norm(e) <= 1e-7, s


def test_multishift_argument_errors(ctx):
    L = (4, 4, 2, 4)
    Vh = int(np.prod(L)) // 2
    op = q.Operator(ctx, q.make_lattice(L), dev(li.random_gauge(L, 0.2, 99)), 0.12, 1.0)
    b = torch.zeros((Vh, 4, 3), dtype=torch.complex128, device="cuda")
    x = torch.empty_like(b)
    with pytest.raises(q.QcdwError):
        q.qcdw_invert_multishift(op, b, [x], [-0.1])
    with pytest.raises(q.QcdwError):
        q.qcdw_invert_multishift(op, b, [b], [0.1])
    it, res = q.qcdw_invert_multishift(op, b, [x], [0.1])  # b = 0: x = 0 at once
    assert it == 0 and float(x.abs().max()) == 0.0
    op.close()


def test_multishift_iteration_cap_and_repeat(ctx):
    """maxiter below the need raises (QCDW_ENOCONV) for every cap, including caps that fall between
    the solver's done-flag reads; a second solve on the same context reproduces the first bit for bit
    (the device state is rebuilt per call); the largest shift alone converges in fewer iterations, and
    in the joint solve its solution is frozen once converged and equals the dense solve."""
    L, t_bc = (6, 4, 2, 6), -1
    U = li.random_gauge(L, 0.3, 101)
    Vh = int(np.prod(L)) // 2
    b = dev(li.gaussian_source(L, 102).reshape(-1, 4, 3)[:Vh].copy())
    op = q.Operator(ctx, q.make_lattice(L, t_bc), dev(U), 0.12, 1.0)
    for cap in (1, 3, 5):
        xs = [torch.empty_like(b) for _ in range(2)]
        with pytest.raises(q.QcdwError):
            q.qcdw_invert_multishift(op, b, xs, [0.0, 0.5], maxiter=cap)
    shifts = [0.0, 0.02, 4.0]
    runs = []
    for _ in range(2):
        xs = [torch.empty_like(b) for _ in shifts]
        it, res = q.qcdw_invert_multishift(op, b, xs, shifts, tol=1e-10)
        runs.append((it, res, [x.cpu().numpy() for x in xs]))
    assert runs[0][0] == runs[1][0] and runs[0][1] == runs[1][1]
    for a, c in zip(runs[0][2], runs[1][2]):
        assert np.array_equal(a, c)
    it_big, _ = q.qcdw_invert_multishift(op, b, [torch.empty_like(b)], [4.0], tol=1e-10)
    assert it_big + 4 < runs[0][0]
    # stopped a few iterations after the shift 4.0 has converged: its solution is already the final one
    # bit for bit, since a converged shift takes no further updates
    xs_cap = [torch.empty_like(b) for _ in shifts]
    with pytest.raises(q.QcdwError):
        q.qcdw_invert_multishift(op, b, xs_cap, shifts, tol=1e-10, maxiter=it_big + 4)
    assert np.array_equal(xs_cap[2].cpu().numpy(), runs[0][2][2])
    assert not np.array_equal(xs_cap[0].cpu().numpy(), runs[0][2][0])
    Ainv, _ = oracle.clover_invert(L, oracle.clover_build(L, U), 0.12, 1.0)
    expect = oracle.normal_shifted_solve(L, U, Ainv, b.cpu().numpy(), 0.12, shifts, t_bc)
    for x, e in zip(runs[0][2], expect):
        assert np.linalg.norm(x.reshape(-1) - e.reshape(-1)) / np.linalg.norm(e) <= 1e-7
    op.close()


def test_multishift_bench_workload_true_residuals(ctx):
    """The benchmark's workload (16^3x32, 8 shifts 1e-4 * 4^k, Gaussian even-site source, tol 1e-10): every
    shifted solution's true residual ||b - (M_hat^+ M_hat + s) x|| / ||b||, with M_hat and the adjoint composed
    on the CPU from the oracle's Schur operator, clover term and clover inverse (M_hat^+ = g5 A_ee M_hat g5
    A_ee^-1, the identity pinned on dense matrices), is within 1e-10 and equals the residual the library reports."""
    w = li.WORKLOADS["wc16x32"]
    L, kappa, csw = w["L"], w["kappa"], w["csw"]
    Vh = int(np.prod(L)) // 2
    U = li.random_gauge(L, w["eps"], w["seed"])
    b = li.gaussian_source(L, 1009).reshape(-1, 4, 3)[:Vh].copy()
    shifts = [1e-4 * 4 ** k for k in range(8)]
    op = q.Operator(ctx, q.make_lattice(L), dev(U), kappa, csw)
    xs = [torch.empty((Vh, 4, 3), dtype=torch.complex128, device="cuda") for _ in shifts]
    it, res = q.qcdw_invert_multishift(op, dev(b), xs, shifts, tol=1e-10)
    op.close()
    assert max(res) <= 1e-10
    C = oracle.clover_build(L, U)
    Ainv, _ = oracle.clover_invert(L, C, kappa, csw)

    def g5(v):
        v = v.copy()
        v[:, 2:, :] *= -1.0
        return v

    def even(full):
        return np.asarray(full).reshape(-1, 4, 3)[:Vh]

    def embed(v):
        full = np.zeros((2 * Vh, 4, 3), dtype=np.complex128)
        full[:Vh] = v
        return full.reshape(li.fermion_shape(L))

    def mhat(v):
        return oracle.schur_matpc(L, U, Ainv, v, kappa)

    def mhat_dag(v):
        t = even(oracle.packed_apply(L, Ainv, embed(v)))
        t = mhat(g5(t))
        return g5(even(oracle.clover_apply(L, C, embed(t), kappa, csw)))

    for x, s, rep in zip(xs, shifts, res):
        xh = x.cpu().numpy()
        r = b - mhat_dag(mhat(xh)) - s * xh
        tr = np.linalg.norm(r) / np.linalg.norm(b)
        assert tr <= 1e-10, s
        assert abs(rep - tr) <= 1e-2 * tr + 1e-14, (s, rep, tr)
