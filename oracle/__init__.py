"""Plain FP64 CPU oracle for the even-odd Wilson-clover inversion.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the HIP library ``paper_2411_08461_amd`` and never imports it.

The arithmetic lives in ``oracle.c`` (plain C, compiled with gcc); this module
only marshals NumPy arrays and composes the even-odd pieces out of the
full-lattice functions, so each step can be read against the paper:

* field layouts and the DeGrand-Rossi basis: paper Sec. II.A;
* the operator M = A - kappa H, A = 1 - kappa csw sum sigma F:
  paper Sec. III.B, Eq. "clover" in the isotropic limit (xi0 = nu = 1);
* even-odd (red-black) preconditioning of local fields: Sec. II.A/II.D;
* BiCGStab as the clover solver: Sec. II.E.

Functions whose result is only checked through invariants, not against an
independent closed form, are marked "parity unpinned" below.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# tests of the pins themselves load a deliberately broken build of oracle.c through this variable
_LIB_OVERRIDE = os.environ.get("QCDW_ORACLE_LIB")


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            _lib = ctypes.CDLL(_LIB_OVERRIDE)
        else:
            build(force=False)
            _lib = ctypes.CDLL(_LIB)
        d, i, p = ctypes.c_double, ctypes.c_int, ctypes.c_void_p
        _lib.orc_hop.argtypes = [p, i, p, p, p, i]
        _lib.orc_set_threads.argtypes = [i]
        _lib.orc_set_threads.restype = None
        _lib.orc_hop_w.argtypes = [p, i, p, p, p, i, p]
        _lib.orc_clover_build.argtypes = [p, p, p]
        _lib.orc_clover_build.restype = d
        _lib.orc_clover_build_w.argtypes = [p, p, p, d, d]
        _lib.orc_clover_build_w.restype = d
        _lib.orc_dirac_w.argtypes = [p, i, p, p, p, p, d, d, p]
        _lib.orc_packed_apply.argtypes = [p, p, p, p]
        _lib.orc_clover_apply.argtypes = [p, p, p, p, d, d]
        _lib.orc_clover_invert.argtypes = [p, p, d, d, p]
        _lib.orc_clover_invert.restype = ctypes.c_long
        _lib.orc_dirac.argtypes = [p, i, p, p, p, p, d, d]
        _lib.orc_bicgstab.argtypes = [p, i, p, p, d, d, p, p, d, i, p, p]
        _lib.orc_bicgstab.restype = i
        _lib.orc_gamma.argtypes = [i, p]
        _lib.orc_site_index.argtypes = [p, p]
        _lib.orc_site_index.restype = ctypes.c_long
        _lib.orc_site_coords.argtypes = [p, ctypes.c_long, p]
        _lib.orc_num_threads.restype = i
    return _lib


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"], "oracle arrays must be C-contiguous"
    return a.ctypes.data_as(ctypes.c_void_p)


def _dims(L):
    return np.ascontiguousarray(np.asarray(L, dtype=np.int32))


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


# --------------------------------------------------------------------------
# Geometry and Dirac matrices (Sec. II.A)
# --------------------------------------------------------------------------


def gamma(mu: int) -> np.ndarray:
    """gamma_{mu+1} in the DeGrand-Rossi basis as a 4x4 complex matrix."""
    out = np.zeros(32)
    lib().orc_gamma(mu, _ptr(out))
    return out.view(np.complex128).reshape(4, 4).copy()


def gamma_bitmask(n: int) -> np.ndarray:
    """Gamma(n) = g1^{n&1} g2^{(n>>1)&1} g3^{(n>>2)&1} g4^{(n>>3)&1}.

    The bitmask indexing follows the example in Sec. III.B, where the product
    gamma(15) @ gamma(4) stands for gamma_5 gamma_3.
    """
    m = np.eye(4, dtype=np.complex128)
    for mu in range(4):
        if (n >> mu) & 1:
            m = m @ gamma(mu)
    return m


def num_threads() -> int:
    """OpenMP threads the oracle's loops use."""
    return int(lib().orc_num_threads())


def set_threads(n: int) -> None:
    """Set the OpenMP thread count of the oracle's loops (timing on fewer cores)."""
    lib().orc_set_threads(int(n))


def site_index(L, c) -> int:
    return int(lib().orc_site_index(_ptr(_dims(L)), _ptr(np.asarray(c, dtype=np.int32))))


def site_coords(L, i: int):
    c = np.zeros(4, dtype=np.int32)
    lib().orc_site_coords(_ptr(_dims(L)), int(i), _ptr(c))
    return tuple(int(v) for v in c)


def coords_table(L) -> np.ndarray:
    """(V, 4) array of (x, y, z, t) for every eo index (Sec. II.A order)."""
    Lx, Ly, Lz, Lt = L
    V = Lx * Ly * Lz * Lt
    idx = np.arange(V)
    parity = idx // (V // 2)
    r = idx % (V // 2)
    xh = r % (Lx // 2)
    r //= Lx // 2
    y = r % Ly
    r //= Ly
    z = r % Lz
    t = r // Lz
    x = 2 * xh + ((parity + y + z + t) & 1)
    return np.stack([x, y, z, t], axis=1)


def parity_mask(L, parity: int) -> np.ndarray:
    V = int(np.prod(L))
    m = np.zeros(V, dtype=bool)
    m[parity * (V // 2) : (parity + 1) * (V // 2)] = True
    return m


# --------------------------------------------------------------------------
# Operator pieces (Sec. III.B, Eq. "clover")
# --------------------------------------------------------------------------


def hop(L, U, psi, t_bc: int = 1, out_parity: int = -1, weights=None) -> np.ndarray:
    """H psi = sum_mu w_mu [(1-g_mu) U_mu(x) psi(x+mu) + (1+g_mu) U_mu(x-mu)^+ psi(x-mu)].

    Full-lattice fields in the paper layout; with out_parity >= 0 only the
    sites of that parity are computed (the rest are zero), which is the
    parity-to-parity block H_{p, 1-p} when psi vanishes on parity p.
    weights: w_mu for mu = x, y, z, t (default all 1; the anisotropic action of
    Sec. III.B, Eq. "clover", has w = (nu/xi_0, nu/xi_0, nu/xi_0, 1)).
    """
    U, psi = _c128(U), _c128(psi)
    out = np.empty_like(psi)
    if weights is None:
        lib().orc_hop(_ptr(_dims(L)), int(t_bc), _ptr(U), _ptr(psi), _ptr(out), int(out_parity))
    else:
        w = np.ascontiguousarray(weights, dtype=np.float64)
        lib().orc_hop_w(_ptr(_dims(L)), int(t_bc), _ptr(U), _ptr(psi), _ptr(out), int(out_parity), _ptr(w))
    return out


def aniso_weights(xi_0: float, nu: float) -> np.ndarray:
    """Hop weights of the anisotropic clover action (Sec. III.B, Eq. "clover"): nu/xi_0 on the
    three spatial directions, 1 on t."""
    r = nu / xi_0
    return np.array([r, r, r, 1.0])


def aniso_kappa(m_0: float, xi_0: float, nu: float) -> float:
    """kappa from the bare mass of the anisotropic action: 1/kappa = 2 (m_0 + 1 + 3 nu/xi_0) (Sec. III.B)."""
    return 1.0 / (2.0 * (m_0 + 1.0 + 3.0 * nu / xi_0))


def clover_build(L, U, return_offblock: bool = False, plane_weights=None):
    """Packed C = sum_{mu<nu} sigma_{mu nu} F_{mu nu}, [2,Lt,Lz,Ly,Lx/2,2,36] reals.

    F_{mu nu} = (Q - Q^+)/8 traceless, Q the four-leaf sum.  The trace removal
    and the overall sign are readings of Eq. "clover" (pinned by the
    single-link closed form and the invariants in the tests).
    plane_weights = (wt, ws) weights the planes (i, t) by wt and the spatial
    planes by ws: the anisotropic action (Sec. III.B) has C = c_SW^t sum sigma_i4
    F_i4 + (c_SW^r / xi_0) sum sigma_ij F_ij, used with c_SW = 1.
    """
    U = _c128(U)
    V = int(np.prod(L))
    clover = np.empty((V, 2, 36))
    if plane_weights is None:
        off = lib().orc_clover_build(_ptr(_dims(L)), _ptr(U), _ptr(clover))
    else:
        wt, ws = plane_weights
        off = lib().orc_clover_build_w(_ptr(_dims(L)), _ptr(U), _ptr(clover), float(wt), float(ws))
    clover = clover.reshape(packed_shape(L))
    return (clover, off) if return_offblock else clover


def packed_shape(L):
    Lx, Ly, Lz, Lt = L
    return (2, Lt, Lz, Ly, Lx // 2, 2, 36)


def fermion_shape(L):
    Lx, Ly, Lz, Lt = L
    return (2, Lt, Lz, Ly, Lx // 2, 4, 3)


def packed_apply(L, packed, psi) -> np.ndarray:
    """Apply packed Hermitian 6x6 chirality blocks site by site."""
    packed = np.ascontiguousarray(packed, dtype=np.float64)
    psi = _c128(psi)
    out = np.empty_like(psi)
    lib().orc_packed_apply(_ptr(_dims(L)), _ptr(packed), _ptr(psi), _ptr(out))
    return out


def unpack_blocks(packed) -> np.ndarray:
    """Packed [..., 2, 36] reals -> full Hermitian blocks [..., 2, 6, 6]."""
    p = np.asarray(packed, dtype=np.float64)
    out = np.zeros(p.shape[:-1] + (6, 6), dtype=np.complex128)
    for j in range(6):
        out[..., j, j] = p[..., j]
    s = 0
    for j in range(1, 6):
        for k in range(j):
            v = p[..., 6 + 2 * s] + 1j * p[..., 7 + 2 * s]
            out[..., j, k] = v
            out[..., k, j] = np.conj(v)
            s += 1
    return out


def clover_apply(L, clover, psi, kappa: float, csw: float) -> np.ndarray:
    """A psi with A = 1 - kappa csw C."""
    clover = np.ascontiguousarray(clover, dtype=np.float64)
    psi = _c128(psi)
    out = np.empty_like(psi)
    lib().orc_clover_apply(_ptr(_dims(L)), _ptr(clover), _ptr(psi), _ptr(out), float(kappa), float(csw))
    return out


def clover_invert(L, clover, kappa: float, csw: float):
    """Packed A^{-1} per chirality block by Gauss-Jordan; returns (inv, n_singular)."""
    clover = np.ascontiguousarray(clover, dtype=np.float64)
    inv = np.empty_like(clover)
    bad = lib().orc_clover_invert(_ptr(_dims(L)), _ptr(clover), float(kappa), float(csw), _ptr(inv))
    return inv, int(bad)


def dirac(L, U, clover, psi, kappa: float, csw: float, t_bc: int = 1, weights=None) -> np.ndarray:
    """M psi = A psi - kappa H psi on the full lattice (weights: hop weights per direction, as in hop)."""
    U, psi = _c128(U), _c128(psi)
    clover = np.ascontiguousarray(clover, dtype=np.float64)
    out = np.empty_like(psi)
    if weights is None:
        lib().orc_dirac(_ptr(_dims(L)), int(t_bc), _ptr(U), _ptr(clover), _ptr(psi), _ptr(out), float(kappa),
                        float(csw))
    else:
        w = np.ascontiguousarray(weights, dtype=np.float64)
        lib().orc_dirac_w(_ptr(_dims(L)), int(t_bc), _ptr(U), _ptr(clover), _ptr(psi), _ptr(out), float(kappa),
                          float(csw), _ptr(w))
    return out


# --------------------------------------------------------------------------
# Even-odd Schur pieces composed from the full-lattice functions
# (Sec. II.A / II.D: even-odd preconditioning of local fields)
# --------------------------------------------------------------------------


def _embed(L, half, parity):
    """Half-lattice field of one parity -> full field, zero on the other."""
    V = int(np.prod(L))
    full = np.zeros((V, 4, 3), dtype=np.complex128)
    full[parity * (V // 2) : (parity + 1) * (V // 2)] = np.asarray(half).reshape(V // 2, 4, 3)
    return full.reshape(fermion_shape(L))


def _restrict(L, full, parity):
    V = int(np.prod(L))
    return np.asarray(full).reshape(V, 4, 3)[parity * (V // 2) : (parity + 1) * (V // 2)].copy()


def schur_matpc(L, U, clover_inv, psi_e, kappa: float, t_bc: int = 1, weights=None):
    """M_hat psi_e = psi_e - kappa^2 A_ee^{-1} H_eo A_oo^{-1} H_oe psi_e.

    psi_e: (Vh, 4, 3) even-site field.  clover_inv: packed A^{-1}.  weights: hop weights (see hop).
    """
    full = _embed(L, psi_e, 0)
    t = hop(L, U, full, t_bc, out_parity=1, weights=weights)
    t = packed_apply(L, clover_inv, t)
    t = hop(L, U, t, t_bc, out_parity=0, weights=weights)
    t = packed_apply(L, clover_inv, t)
    return np.asarray(psi_e).reshape(-1, 4, 3) - kappa * kappa * _restrict(L, t, 0)


def schur_source(L, U, clover_inv, b, kappa: float, t_bc: int = 1):
    """b_hat_e = A_ee^{-1} (b_e + kappa H_eo A_oo^{-1} b_o)."""
    b = _c128(b)
    bo = _embed(L, _restrict(L, b, 1), 1)
    t = packed_apply(L, clover_inv, bo)
    t = hop(L, U, t, t_bc, out_parity=0)
    t = _c128(b) * parity_mask(L, 0).reshape(fermion_shape(L)[:5] + (1, 1)) + kappa * t
    t = packed_apply(L, clover_inv, t)
    return _restrict(L, t, 0)


def schur_reconstruct(L, U, clover_inv, b, x_e, kappa: float, t_bc: int = 1):
    """x_o = A_oo^{-1} (b_o + kappa H_oe x_e); returns the full solution."""
    xe_full = _embed(L, x_e, 0)
    t = hop(L, U, xe_full, t_bc, out_parity=1)
    t = _c128(b) * parity_mask(L, 1).reshape(fermion_shape(L)[:5] + (1, 1)) + kappa * t
    t = packed_apply(L, clover_inv, t)
    V = int(np.prod(L))
    x = t.reshape(V, 4, 3)
    x[: V // 2] = np.asarray(x_e).reshape(V // 2, 4, 3)
    return x.reshape(fermion_shape(L))


# --------------------------------------------------------------------------
# Solver (Sec. II.E: BiCGStab is the default for Wilson/clover)
# --------------------------------------------------------------------------


class SolveResult:
    def __init__(self, x, status, iters, true_res, restarts, res_hist):
        self.x = x
        self.status = status
        self.iters = iters
        self.true_res = true_res
        self.restarts = restarts
        self.res_hist = res_hist


def bicgstab(L, U, clover, b, kappa: float, csw: float, tol: float = 1e-10, maxiter: int = 10000,
             x0=None, t_bc: int = 1) -> SolveResult:
    """Textbook BiCGStab on the full (unpreconditioned) system M x = b."""
    U, b = _c128(U), _c128(b)
    clover = np.ascontiguousarray(clover, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else _c128(x0).copy()
    hist = np.full(maxiter + 1, np.nan)
    out = np.zeros(3)
    st = lib().orc_bicgstab(_ptr(_dims(L)), int(t_bc), _ptr(U), _ptr(clover), float(kappa), float(csw), _ptr(b),
                            _ptr(x), float(tol), int(maxiter), _ptr(hist), _ptr(out))
    it = int(out[0])
    return SolveResult(x, int(st), it, float(out[1]), int(out[2]), hist[: it + 1].copy())


def dense_matrix(L, U, clover, kappa: float, csw: float, t_bc: int = 1) -> np.ndarray:
    """M as a dense (12V x 12V) matrix, assembled column by column from dirac()."""
    V = int(np.prod(L))
    n = 12 * V
    M = np.empty((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for k in range(n):
        e[:] = 0
        e[k] = 1
        M[:, k] = dirac(L, U, clover, e.reshape(fermion_shape(L)), kappa, csw, t_bc).reshape(n)
    return M


def schur_dense(L, U, clover_inv, kappa: float, t_bc: int = 1) -> np.ndarray:
    """M_hat as a dense (12 Vh x 12 Vh) matrix, assembled column by column from schur_matpc."""
    Vh = int(np.prod(L)) // 2
    n = 12 * Vh
    M = np.empty((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for k in range(n):
        e[:] = 0
        e[k] = 1
        M[:, k] = schur_matpc(L, U, clover_inv, e.reshape(Vh, 4, 3), kappa, t_bc).reshape(n)
    return M


def normal_shifted_solve(L, U, clover_inv, b_e, kappa: float, shifts, t_bc: int = 1):
    """x_i = (M_hat^+ M_hat + shifts[i])^{-1} b_e by dense solves: the definition the multi-shift solver
    reaches (RHMC's rational approximation needs these solves, Sec. IV)."""
    M = schur_dense(L, U, clover_inv, kappa, t_bc)
    N = M.conj().T @ M
    b = np.asarray(b_e, dtype=np.complex128).reshape(-1)
    return [np.linalg.solve(N + s * np.eye(N.shape[0]), b).reshape(-1, 4, 3) for s in shifts]
