"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module holds no arithmetic of the method itself: it only draws random
gauge links, gauge transformations and sources, in the paper's field layouts
(Sec. II.A: gauge [Nd, 2, Lt, Lz, Ly, Lx/2, Nc, Nc], fermion
[2, Lt, Lz, Ly, Lx/2, Ns, Nc], even-odd site order).

Recipes (readings of the workload descriptions, stated once here):

* links U = exp(i eps H), H = (A + A^+)/2 with A_ij = N(0,1) + i N(0,1),
  trace removed; U = V diag(exp(i eps lambda)) V^+ from the Hermitian
  eigendecomposition, all in FP64.  Links are drawn in eo-layout order
  [mu][parity][t][z][y][x/2] with NumPy's PCG64 ``default_rng(seed)``;
* Z2 source: each of the 12 V complex entries is (+-1 +- i)/sqrt(2);
* Gaussian source: real and imaginary parts N(0, 1);
* point source: 1 at (0,0,0,0), given spin and colour;
* gauge transformation: Haar-random SU(3) per site from the QR of a complex
  Gaussian matrix, phase-fixed to det = 1.
"""
from __future__ import annotations

import numpy as np


def volume(L) -> int:
    return int(L[0] * L[1] * L[2] * L[3])


def gauge_shape(L):
    Lx, Ly, Lz, Lt = L
    return (4, 2, Lt, Lz, Ly, Lx // 2, 3, 3)


def fermion_shape(L):
    Lx, Ly, Lz, Lt = L
    return (2, Lt, Lz, Ly, Lx // 2, 4, 3)


def check_lattice(L):
    if len(L) != 4 or any(int(l) < 2 or int(l) % 2 for l in L):
        raise ValueError(f"lattice extents must be four even numbers >= 2, got {L}")


def _su3_exp(eps: float, rng: np.random.Generator, n: int, chunk: int = 1 << 20) -> np.ndarray:
    out = np.empty((n, 3, 3), dtype=np.complex128)
    for s in range(0, n, chunk):
        m = min(chunk, n - s)
        a = rng.standard_normal((m, 3, 3)) + 1j * rng.standard_normal((m, 3, 3))
        h = 0.5 * (a + np.conj(np.swapaxes(a, -1, -2)))
        tr = np.trace(h, axis1=-2, axis2=-1).real / 3.0
        h -= tr[:, None, None] * np.eye(3)
        lam, vec = np.linalg.eigh(h)
        ph = np.exp(1j * eps * lam)
        out[s : s + m] = (vec * ph[:, None, :]) @ np.conj(np.swapaxes(vec, -1, -2))
    return out


def random_gauge(L, eps: float, seed: int) -> np.ndarray:
    """Random SU(3) links U = exp(i eps H) in the paper gauge layout."""
    check_lattice(L)
    rng = np.random.default_rng(seed)
    n = 4 * volume(L)
    return _su3_exp(eps, rng, n).reshape(gauge_shape(L))


def _gauge_job(job):
    L, eps, seed = job
    return random_gauge(L, eps, seed)


def random_gauges(jobs, workers: int | None = None):
    """random_gauge(L, eps, seed) for each (L, eps, seed) in jobs, one worker process per field.

    The fields are independent streams, so the result equals the serial calls.  Workers are
    forked: call this before the process has initialised a GPU.
    """
    import multiprocessing as mp
    import os

    jobs = [tuple(j) for j in jobs]
    if workers is None:
        workers = min(len(jobs), os.cpu_count() or 1, 16)
    if workers <= 1 or len(jobs) <= 1:
        return [_gauge_job(j) for j in jobs]
    # close() + join() let the workers finish and exit on their own (the pool's context manager
    # would terminate them with a signal)
    pool = mp.get_context("fork").Pool(workers)
    try:
        out = pool.map(_gauge_job, jobs, chunksize=1)
        pool.close()
    except BaseException:
        pool.terminate()
        raise
    finally:
        pool.join()
    return out


def unit_gauge(L) -> np.ndarray:
    check_lattice(L)
    U = np.zeros(gauge_shape(L), dtype=np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1.0
    return U


def haar_su3(n: int, seed: int) -> np.ndarray:
    """n Haar-random SU(3) matrices (QR of a complex Gaussian, det fixed to 1)."""
    rng = np.random.default_rng(seed)
    z = (rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    q = q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(q)
    q = q / (det ** (1.0 / 3.0))[:, None, None]
    return q


def gauge_transform(L, seed: int) -> np.ndarray:
    """Site field of SU(3) matrices Omega(x), shape [2, Lt, Lz, Ly, Lx/2, 3, 3]."""
    check_lattice(L)
    Lx, Ly, Lz, Lt = L
    return haar_su3(volume(L), seed).reshape(2, Lt, Lz, Ly, Lx // 2, 3, 3)


def z2_source(L, seed: int) -> np.ndarray:
    check_lattice(L)
    rng = np.random.default_rng(seed)
    n = 12 * volume(L)
    re = rng.integers(0, 2, n) * 2 - 1
    im = rng.integers(0, 2, n) * 2 - 1
    return ((re + 1j * im) / np.sqrt(2.0)).reshape(fermion_shape(L))


def gaussian_source(L, seed: int) -> np.ndarray:
    check_lattice(L)
    rng = np.random.default_rng(seed)
    n = 12 * volume(L)
    return (rng.standard_normal(n) + 1j * rng.standard_normal(n)).reshape(fermion_shape(L))


def point_source(L, spin: int = 0, colour: int = 0) -> np.ndarray:
    """1 at the origin (even parity, eo index 0) for one spin and colour."""
    check_lattice(L)
    b = np.zeros(fermion_shape(L), dtype=np.complex128)
    b[0, 0, 0, 0, 0, spin, colour] = 1.0
    return b


# Workloads: lattice extents [Lx, Ly, Lz, Lt] and physics parameters.
WORKLOADS = {
    "dense4": dict(L=(4, 4, 4, 4), kappa=0.12, csw=1.0, eps=0.3, seed=0, source="point"),
    "wc16x32": dict(L=(16, 16, 16, 32), kappa=0.124, csw=1.0, eps=0.2, seed=0, source="z2", source_seed=1000),
    "wc24x64": dict(L=(24, 24, 24, 64), kappa=0.125, csw=1.1, eps=0.2, seed=0, source="point12"),
    # kappa: the smallest value on a 1e-5 grid at which FP64 even-odd BiCGStab from the Gaussian
    # source needs at least 2000 iterations to reach 1e-10 (2729 at 0.12781, 1857 at 0.12780),
    # found by bisection on the GPU solver (bench.py --bisect-kappa)
    "wc32x64": dict(L=(32, 32, 32, 64), kappa=0.12781, csw=1.0, eps=0.15, seed=0, source="gaussian",
                    source_seed=1000),
}


# the 48 uneven problems solved as one batch: 16 each of 8^3x16, 12^3x24, 16^3x32, kappa uniform in
# [0.115, 0.124] (seed 4000), csw 1.0, independent eps = 0.25 fields (seeds 100..147), Gaussian sources
# (seeds 1100..1147)
def batch48():
    kap = np.random.default_rng(4000).uniform(0.115, 0.124, 48)
    Ls = [(8, 8, 8, 16)] * 16 + [(12, 12, 12, 24)] * 16 + [(16, 16, 16, 32)] * 16
    return [dict(L=Ls[k], kappa=float(kap[k]), csw=1.0, eps=0.25, seed=100 + k, source_seed=1100 + k)
            for k in range(48)]


def make_source(kind: str, L, seed: int = 0, spin: int = 0, colour: int = 0) -> np.ndarray:
    if kind == "point":
        return point_source(L, spin, colour)
    if kind == "z2":
        return z2_source(L, seed)
    if kind == "gaussian":
        return gaussian_source(L, seed)
    raise ValueError(kind)
