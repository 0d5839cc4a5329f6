"""qcdw_dslash_noalloc (workspace in the library's fixed per-device array) against qcdw_dslash.

Both entry points run the same kernels in the same order, so the results must be bitwise equal;
the oracle's operator checks both to the FP64 bar (1e-13 relative).  Two calls in a row, the
second on a smaller lattice (the array keeps the first call's contents), with and without a
caller-supplied clover field, and a lattice beyond the fixed size rejected before any GPU work.
"""
import numpy as np
import pytest
import torch

import lattice_inputs as li
import oracle
import paper_2411_08461_amd as q

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.fixture(scope="module")
def ctx():
    c = q.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


@pytest.mark.parametrize("with_clover", [False, True])
def test_noalloc_dslash_equals_dslash_on_two_calls(ctx, with_clover):
    # (8^3 x 16: 4096 sites per parity, 64 tiles), then 6x4x2x6 (144 sites per parity, a ragged tile)
    for L, eps, seed, kappa, csw in (((8, 8, 8, 16), 0.3, 11, 0.124, 1.0), ((6, 4, 2, 6), 0.4, 12, 0.12, 1.3)):
        U = li.random_gauge(L, eps, seed)
        psi = li.gaussian_source(L, seed + 1000)
        lat = q.make_lattice(L)
        C = oracle.clover_build(L, U)
        Cd = dev(C) if with_clover else None
        ref = torch.empty(li.fermion_shape(L), dtype=torch.complex128, device="cuda")
        out = torch.full_like(ref, float("nan"))
        q.qcdw_dslash(ctx, lat, dev(U), Cd, dev(psi), ref, kappa, csw)
        q.qcdw_dslash_noalloc(ctx, lat, dev(U), Cd, dev(psi), out, kappa, csw)
        torch.cuda.synchronize()
        a, b = out.cpu().numpy(), ref.cpu().numpy()
        assert np.array_equal(a.view(np.float64), b.view(np.float64)), (L, rel(a, b))
        expect = oracle.dirac(L, U, C, psi, kappa, csw)
        assert rel(a, expect) < 1e-13, L


def test_noalloc_dslash_rejects_lattice_beyond_workspace(ctx):
    L = (16, 16, 16, 32)  # needs ~340 MB of workspace
    lat = q.make_lattice(L)
    V = 16 * 16 * 16 * 32
    U = torch.zeros(36 * V, dtype=torch.complex128, device="cuda")
    psi = torch.zeros(12 * V, dtype=torch.complex128, device="cuda")
    out = torch.zeros_like(psi)
    with pytest.raises(q.QcdwError, match="workspace"):
        q.qcdw_dslash_noalloc(ctx, lat, U, None, psi, out, 0.12, 1.0)
