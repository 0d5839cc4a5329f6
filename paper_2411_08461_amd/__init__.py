"""qcdw: even-odd preconditioned Wilson-clover inversion for AMD MI355X (gfx950).

Thin ctypes binding of the HIP library ``libqcdw.so`` (C ABI in
``include/qcdw.h``).  Every function has the name of the C entry point it
calls and only marshals arguments: torch tensors on the GPU provide device
memory and the HIP stream, every step of the computation runs in the library's
own kernels.  There is no CPU fallback: importing works without a GPU, but any
call raises if the library or the device is missing.

Field layouts follow arXiv 2411.08461, Sec. II.A (complex128 tensors):
  gauge   [4, 2, Lt, Lz, Ly, Lx/2, 3, 3]
  fermion [2, Lt, Lz, Ly, Lx/2, 4, 3]
  clover  [2, Lt, Lz, Ly, Lx/2, 2, 36] float64
"""
from __future__ import annotations

import atexit
import ctypes
import math
import os
import weakref

import torch  # noqa: F401  (loads the HIP runtime the library binds to)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqcdw.so")

QCDW_OK, QCDW_EINVAL, QCDW_ENOMEM, QCDW_EHIP, QCDW_ENOCONV, QCDW_EBREAKDOWN, QCDW_ENAN, QCDW_ENOTPD = (
    0, -1, -2, -3, -4, -5, -6, -7)
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ENOCONV", -5: "EBREAKDOWN", -6: "ENAN",
                -7: "ENOTPD"}
QCDW_F64, QCDW_F32, QCDW_BF16, QCDW_F16 = 0, 1, 2, 3
PREC = {"f64": QCDW_F64, "f32": QCDW_F32, "bf16": QCDW_BF16, "f16": QCDW_F16}

# every symbol declared in include/qcdw.h
EXPORTED = (
    "qcdw_solver_params_default", "qcdw_ctx_create", "qcdw_ctx_destroy", "qcdw_last_error", "qcdw_ctx_set_stream",
    "qcdw_ctx_tuned",
    "qcdw_clover_build", "qcdw_clover_apply", "qcdw_clover_invert", "qcdw_hop", "qcdw_dslash", "qcdw_dslash_noalloc",
    "qcdw_op_create",
    "qcdw_op_create_aniso", "qcdw_op_destroy", "qcdw_op_hop_form", "qcdw_op_matpc", "qcdw_op_matpc_multi", "qcdw_invert", "qcdw_invert_multi",
    "qcdw_batch_create", "qcdw_batch_destroy", "qcdw_invert_batch",
    "qcdw_net_create", "qcdw_net_destroy", "qcdw_net_bind", "qcdw_net_get_weights", "qcdw_net_set_weights", "qcdw_net_apply",
    "qcdw_net_loss_grad", "qcdw_net_train", "qcdw_make_training_pairs", "qcdw_invert_fgmres",
    "qcdw_wall_sources", "qcdw_meson_2pt", "qcdw_meson_contract", "qcdw_seq_sources", "qcdw_invert_multishift",
    "qcdw_mg_params_default", "qcdw_mg_create", "qcdw_mg_destroy", "qcdw_mg_info", "qcdw_mg_vectors",
    "qcdw_mg_restrict", "qcdw_mg_prolong", "qcdw_mg_coarse_apply", "qcdw_mg_coarse_op", "qcdw_invert_mg",
    "qcdw_clover_force",
)


class QcdwError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class qcdw_lattice(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32 * 4), ("t_bc", ctypes.c_int32)]


class qcdw_solver_params(ctypes.Structure):
    _fields_ = [
        ("tol", ctypes.c_double),
        ("maxiter", ctypes.c_int32),
        ("inner", ctypes.c_int32),
        ("delta", ctypes.c_double),
        ("check_every", ctypes.c_int32),
        ("max_restarts", ctypes.c_int32),
        ("collect_timing", ctypes.c_int32),
        ("fault_inject", ctypes.c_int32),
        ("use_graph", ctypes.c_int32),
        ("gmres_restart", ctypes.c_int32),
        ("gmres_fallback", ctypes.c_int32),
        ("inner_resume", ctypes.c_int32),
    ]


class qcdw_solve_info(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("iters", ctypes.c_int32),
        ("n_reliable", ctypes.c_int32),
        ("n_restarts", ctypes.c_int32),
        ("true_res", ctypes.c_double),
        ("iter_res", ctypes.c_double),
        ("time_ms", ctypes.c_double),
        ("hop_ms", ctypes.c_double * 3),
        ("n_hop", ctypes.c_int32 * 3),
        ("hist_len", ctypes.c_int32),
        ("hist_count", ctypes.c_int32),
        ("fallback", ctypes.c_int32),
        ("fallback_iters", ctypes.c_int32),
        ("res_hist", ctypes.POINTER(ctypes.c_double)),
    ]


class qcdw_mg_params(ctypes.Structure):
    _fields_ = [
        ("block", ctypes.c_int32 * 4),
        ("nvec", ctypes.c_int32),
        ("setup_iters", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("coarse_iters", ctypes.c_int32),
        ("coarse_tol", ctypes.c_double),
        ("smooth_iters", ctypes.c_int32),
    ]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libqcdw.so (built in-tree by ``paper_2411_08461_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2411_08461_amd.build`")
    lib = ctypes.CDLL(path)
    p, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    lat = ctypes.POINTER(qcdw_lattice)
    sig = {
        "qcdw_solver_params_default": (None, [ctypes.POINTER(qcdw_solver_params)]),
        "qcdw_ctx_create": (i, [ctypes.POINTER(p), i, p]),
        "qcdw_ctx_destroy": (None, [p]),
        "qcdw_last_error": (ctypes.c_char_p, [p]),
        "qcdw_ctx_set_stream": (i, [p, p]),
        "qcdw_ctx_tuned": (i, [p, ctypes.c_char_p, ctypes.POINTER(i)]),
        "qcdw_clover_build": (i, [p, lat, p, p]),
        "qcdw_clover_apply": (i, [p, lat, p, p, p, d, d]),
        "qcdw_clover_invert": (i, [p, lat, p, d, d, p]),
        "qcdw_hop": (i, [p, lat, p, p, p, i]),
        "qcdw_dslash": (i, [p, lat, p, p, p, p, d, d]),
        "qcdw_dslash_noalloc": (i, [p, lat, p, p, p, p, d, d]),
        "qcdw_clover_force": (i, [p, lat, p, p, p, d, d, p]),
        "qcdw_mg_params_default": (None, [ctypes.POINTER(qcdw_mg_params)]),
        "qcdw_mg_create": (i, [p, ctypes.POINTER(qcdw_mg_params), p, ctypes.POINTER(p)]),
        "qcdw_mg_destroy": (None, [p]),
        "qcdw_mg_info": (i, [p, ctypes.POINTER(i), ctypes.POINTER(i)]),
        "qcdw_mg_vectors": (i, [p, p]),
        "qcdw_mg_restrict": (i, [p, p, p]),
        "qcdw_mg_prolong": (i, [p, p, p]),
        "qcdw_mg_coarse_apply": (i, [p, p, p]),
        "qcdw_mg_coarse_op": (i, [p, p]),
        "qcdw_invert_mg": (i, [p, p, p, p, ctypes.POINTER(qcdw_solver_params), ctypes.POINTER(qcdw_solve_info)]),
        "qcdw_op_create": (i, [p, lat, p, d, d, i, i, ctypes.POINTER(p)]),
        "qcdw_op_create_aniso": (i, [p, lat, p, d, d, d, d, d, i, i, ctypes.POINTER(p)]),
        "qcdw_wall_sources": (i, [p, lat, i, ctypes.POINTER(i), p]),
        "qcdw_meson_2pt": (i, [p, lat, p, i, i, ctypes.POINTER(i), p]),
        "qcdw_meson_contract": (i, [p, lat, p, p, i, i, ctypes.POINTER(i), p]),
        "qcdw_seq_sources": (i, [p, lat, p, i, i, ctypes.POINTER(i), p]),
        "qcdw_invert_multishift": (i, [p, p, ctypes.POINTER(p), ctypes.POINTER(d), i, d, i, ctypes.POINTER(i),
                                       ctypes.POINTER(d)]),
        "qcdw_op_destroy": (None, [p]),
        "qcdw_op_hop_form": (i, [p, i, ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(i)]),
        "qcdw_op_matpc": (i, [p, i, p, p]),
        "qcdw_op_matpc_multi": (i, [p, i, i, p, p]),
        "qcdw_invert": (i, [p, p, p, ctypes.POINTER(qcdw_solver_params), ctypes.POINTER(qcdw_solve_info)]),
        "qcdw_invert_multi": (i, [p, i, p, p, ctypes.POINTER(qcdw_solver_params), ctypes.POINTER(qcdw_solve_info)]),
        "qcdw_batch_create": (i, [p, i, ctypes.POINTER(p), ctypes.POINTER(p)]),
        "qcdw_batch_destroy": (None, [p]),
        "qcdw_net_create": (i, [p, i, ctypes.c_uint64, d, ctypes.POINTER(p)]),
        "qcdw_net_destroy": (None, [p]),
        "qcdw_net_bind": (i, [p, p]),
        "qcdw_net_get_weights": (i, [p, p, p]),
        "qcdw_net_set_weights": (i, [p, p, p]),
        "qcdw_net_apply": (i, [p, i, p, p]),
        "qcdw_net_loss_grad": (i, [p, i, ctypes.POINTER(p), ctypes.POINTER(p), ctypes.POINTER(d), p, p]),
        "qcdw_net_train": (i, [p, i, ctypes.POINTER(p), ctypes.POINTER(p), i, i, d, ctypes.c_uint64, p]),
        "qcdw_make_training_pairs": (i, [p, p, i, i, ctypes.POINTER(p), ctypes.POINTER(p), ctypes.POINTER(i)]),
        "qcdw_invert_fgmres": (i, [p, p, p, p, ctypes.POINTER(qcdw_solver_params), ctypes.POINTER(qcdw_solve_info)]),
        "qcdw_invert_batch": (i, [p, ctypes.POINTER(p), ctypes.POINTER(p), ctypes.POINTER(qcdw_solver_params),
                                  ctypes.POINTER(qcdw_solve_info)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _ptr(t, dtype=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must live on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")  # Sec. II.B: contiguous arrays only
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


def _volume(lat: qcdw_lattice) -> int:
    return int(lat.L[0]) * int(lat.L[1]) * int(lat.L[2]) * int(lat.L[3])


def _need(t, numel: int, name: str):
    """Reject tensors whose size does not match the layout the kernels index."""
    if t is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, the lattice needs {numel}")


def make_lattice(L, t_bc: int = 1) -> qcdw_lattice:
    lat = qcdw_lattice()
    for k in range(4):
        lat.L[k] = int(L[k])
    lat.t_bc = int(t_bc)
    return lat


def _check(ctx_handle, st: int):
    if st != QCDW_OK:
        lib = load_library()
        msg = lib.qcdw_last_error(ctx_handle)
        raise QcdwError(st, msg.decode() if msg else "")


# Contexts still open when the interpreter exits (a caller that never closed them, or a failure that
# left them referenced) are closed by an exit handler.  It is registered after torch's, so it runs
# before torch releases its streams and device state, while the objects' streams are still valid.
_live_contexts = weakref.WeakSet()


def _close_live_contexts():
    for c in list(_live_contexts):
        try:
            c.close()
        except Exception:
            pass


atexit.register(_close_live_contexts)


class Context:
    """qcdw_ctx bound to one device and one HIP stream (torch's current one by default)."""

    def __init__(self, device: int = 0, stream=None):
        lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the qcdw library has no CPU path")
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.device = device
        self.stream = stream
        self._children = weakref.WeakSet()  # objects that must be destroyed before the context
        h = ctypes.c_void_p()
        st = lib.qcdw_ctx_create(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream))
        if st != QCDW_OK:
            raise QcdwError(st, "qcdw_ctx_create failed")
        self.handle = h
        _live_contexts.add(self)

    def _adopt(self, obj):
        self._children.add(obj)

    def close(self):
        if getattr(self, "handle", None):
            # nets and batches reference operators, operators reference the context
            kids = list(self._children)
            for rank in (0, 1, 2):
                for k in kids:
                    if getattr(k, "_rank", 2) == rank:
                        k.close()
            load_library().qcdw_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def qcdw_solver_params_default() -> qcdw_solver_params:
    prm = qcdw_solver_params()
    load_library().qcdw_solver_params_default(ctypes.byref(prm))
    return prm


def qcdw_clover_build(ctx: Context, lat: qcdw_lattice, U, clover) -> None:
    V = _volume(lat)
    _need(U, 36 * V, "U")
    _need(clover, 72 * V, "clover")
    st = load_library().qcdw_clover_build(ctx.handle, ctypes.byref(lat), _ptr(U, torch.complex128, "U"),
                                          _ptr(clover, torch.float64, "clover"))
    _check(ctx.handle, st)


def qcdw_clover_apply(ctx: Context, lat: qcdw_lattice, clover, psi, out, kappa: float, csw: float) -> None:
    V = _volume(lat)
    _need(clover, 72 * V, "clover")
    _need(psi, 12 * V, "psi")
    _need(out, 12 * V, "out")
    st = load_library().qcdw_clover_apply(ctx.handle, ctypes.byref(lat), _ptr(clover, torch.float64, "clover"),
                                          _ptr(psi, torch.complex128, "psi"), _ptr(out, torch.complex128, "out"),
                                          float(kappa), float(csw))
    _check(ctx.handle, st)


def qcdw_clover_invert(ctx: Context, lat: qcdw_lattice, clover, kappa: float, csw: float, clover_inv) -> None:
    V = _volume(lat)
    _need(clover, 72 * V, "clover")
    _need(clover_inv, 72 * V, "clover_inv")
    st = load_library().qcdw_clover_invert(ctx.handle, ctypes.byref(lat), _ptr(clover, torch.float64, "clover"),
                                           float(kappa), float(csw), _ptr(clover_inv, torch.float64, "clover_inv"))
    _check(ctx.handle, st)


def qcdw_hop(ctx: Context, lat: qcdw_lattice, U, psi, out, out_parity: int) -> None:
    V = _volume(lat)
    _need(U, 36 * V, "U")
    _need(psi, 12 * V, "psi")
    _need(out, 12 * V, "out")
    st = load_library().qcdw_hop(ctx.handle, ctypes.byref(lat), _ptr(U, torch.complex128, "U"),
                                 _ptr(psi, torch.complex128, "psi"), _ptr(out, torch.complex128, "out"),
                                 int(out_parity))
    _check(ctx.handle, st)


def qcdw_dslash(ctx: Context, lat: qcdw_lattice, U, clover, psi, out, kappa: float, csw: float) -> None:
    V = _volume(lat)
    _need(U, 36 * V, "U")
    _need(clover, 72 * V, "clover")
    _need(psi, 12 * V, "psi")
    _need(out, 12 * V, "out")
    st = load_library().qcdw_dslash(ctx.handle, ctypes.byref(lat), _ptr(U, torch.complex128, "U"),
                                    _ptr(clover, torch.float64, "clover"), _ptr(psi, torch.complex128, "psi"),
                                    _ptr(out, torch.complex128, "out"), float(kappa), float(csw))
    _check(ctx.handle, st)


def qcdw_clover_force(ctx: Context, lat: qcdw_lattice, U, X, Y, kappa: float, csw: float, H) -> None:
    """H_mu(x) = sum_a T^a d/dw [2 Re(Y^+ M X)] along exp(i w T^a) U_mu(x) (gauge layout, Hermitian traceless)."""
    V = _volume(lat)
    _need(U, 36 * V, "U")
    _need(X, 12 * V, "X")
    _need(Y, 12 * V, "Y")
    _need(H, 36 * V, "H")
    st = load_library().qcdw_clover_force(ctx.handle, ctypes.byref(lat), _ptr(U, torch.complex128, "U"),
                                          _ptr(X, torch.complex128, "X"), _ptr(Y, torch.complex128, "Y"),
                                          float(kappa), float(csw), _ptr(H, torch.complex128, "H"))
    _check(ctx.handle, st)


NOALLOC_MAX_BYTES = 67108864  # QCDW_NOALLOC_MAX_BYTES of include/qcdw.h


def qcdw_dslash_noalloc(ctx: Context, lat: qcdw_lattice, U, clover, psi, out, kappa: float, csw: float) -> None:
    """qcdw_dslash with its workspace in the library's fixed per-device array (no device allocation)."""
    V = _volume(lat)
    _need(U, 36 * V, "U")
    _need(clover, 72 * V, "clover")
    _need(psi, 12 * V, "psi")
    _need(out, 12 * V, "out")
    st = load_library().qcdw_dslash_noalloc(ctx.handle, ctypes.byref(lat), _ptr(U, torch.complex128, "U"),
                                            _ptr(clover, torch.float64, "clover"), _ptr(psi, torch.complex128, "psi"),
                                            _ptr(out, torch.complex128, "out"), float(kappa), float(csw))
    _check(ctx.handle, st)


class Operator:
    """qcdw_op: packed links, clover inverse and solver workspace for one (U, kappa, csw)."""

    _rank = 2  # destroyed after the nets and batches that use it

    def __init__(self, ctx: Context, lat: qcdw_lattice, U, kappa: float, csw: float, inner="f64", recon: int = 12,
                 aniso=None):
        """aniso = (xi_0, nu, csw_t, csw_r): the anisotropic clover operator (qcdw_op_create_aniso; csw is
        then not used)."""
        self.ctx = ctx
        self.lat = lat
        self.kappa = kappa
        self.csw = csw
        self.aniso = aniso
        self.inner = PREC[inner] if isinstance(inner, str) else int(inner)
        self.volume = _volume(lat)
        _need(U, 36 * self.volume, "U")
        h = ctypes.c_void_p()
        if aniso is None:
            st = load_library().qcdw_op_create(ctx.handle, ctypes.byref(lat), _ptr(U, torch.complex128, "U"),
                                               float(kappa), float(csw), self.inner, int(recon), ctypes.byref(h))
        else:
            xi_0, nu, csw_t, csw_r = (float(v) for v in aniso)
            st = load_library().qcdw_op_create_aniso(ctx.handle, ctypes.byref(lat), _ptr(U, torch.complex128, "U"),
                                                     float(kappa), xi_0, nu, csw_t, csw_r, self.inner, int(recon),
                                                     ctypes.byref(h))
        _check(ctx.handle, st)
        self.handle = h
        self._children = weakref.WeakSet()
        ctx._adopt(self)

    def close(self):
        if getattr(self, "handle", None):
            for k in list(self._children):
                k.close()
            load_library().qcdw_op_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def qcdw_op_create(ctx: Context, lat: qcdw_lattice, U, kappa: float, csw: float, inner="f64", recon: int = 12):
    return Operator(ctx, lat, U, kappa, csw, inner, recon)


def qcdw_op_destroy(op: Operator) -> None:
    op.close()


def qcdw_op_matpc(op: Operator, prec, in_e, out_e) -> None:
    prec = PREC[prec] if isinstance(prec, str) else int(prec)
    _need(in_e, 6 * op.volume, "in_e")
    _need(out_e, 6 * op.volume, "out_e")
    st = load_library().qcdw_op_matpc(op.handle, prec, _ptr(in_e, torch.complex128, "in_e"),
                                      _ptr(out_e, torch.complex128, "out_e"))
    _check(op.ctx.handle, st)


def qcdw_op_matpc_multi(op: Operator, prec, in_e, out_e) -> None:
    """M_hat on nrhs = in_e.shape[0] stacked even-site fields with the multi-RHS kernel."""
    prec = PREC[prec] if isinstance(prec, str) else int(prec)
    nrhs = int(in_e.shape[0])
    _need(in_e, 6 * op.volume * nrhs, "in_e")
    _need(out_e, 6 * op.volume * nrhs, "out_e")
    st = load_library().qcdw_op_matpc_multi(op.handle, prec, nrhs, _ptr(in_e, torch.complex128, "in_e"),
                                            _ptr(out_e, torch.complex128, "out_e"))
    _check(op.ctx.handle, st)


class SolveInfo:
    def __init__(self, info: qcdw_solve_info, hist):
        self.status = info.status
        self.status_name = STATUS_NAMES.get(info.status, str(info.status))
        self.iters = info.iters
        self.n_reliable = info.n_reliable
        self.n_restarts = info.n_restarts
        self.true_res = info.true_res
        self.iter_res = info.iter_res
        self.time_ms = info.time_ms
        self.hop_ms = list(info.hop_ms)
        self.n_hop = list(info.n_hop)
        self.fallback = info.fallback
        self.fallback_iters = info.fallback_iters
        self.res_hist = list(hist[: info.hist_count]) if hist is not None else []

    def __repr__(self):
        return (f"SolveInfo(status={self.status_name}, iters={self.iters}, true_res={self.true_res:.3e}, "
                f"reliable={self.n_reliable}, restarts={self.n_restarts}, time_ms={self.time_ms:.2f})")


def make_params(tol=1e-10, maxiter=10000, inner="f64", delta=0.1, check_every=8, max_restarts=8,
                collect_timing=False, fault_inject=0, use_graph=True, gmres_restart=32,
                gmres_fallback=True, inner_resume=False) -> qcdw_solver_params:
    prm = qcdw_solver_params_default()
    prm.tol = float(tol)
    prm.maxiter = int(maxiter)
    prm.inner = PREC[inner] if isinstance(inner, str) else int(inner)
    prm.delta = float(delta)
    prm.check_every = int(check_every)
    prm.max_restarts = int(max_restarts)
    prm.collect_timing = 1 if collect_timing else 0
    prm.fault_inject = int(fault_inject)
    prm.use_graph = 1 if use_graph else 0
    prm.gmres_restart = int(gmres_restart)
    prm.gmres_fallback = 1 if gmres_fallback else 0
    prm.inner_resume = 1 if inner_resume else 0
    return prm


def qcdw_ctx_tuned(ctx: Context, key: str):
    """The tuned kernel form of a tuning key (see include/qcdw.h), or None if nothing is tuned for it."""
    v = ctypes.c_int()
    st = load_library().qcdw_ctx_tuned(ctx.handle, key.encode(), ctypes.byref(v))
    return v.value if st == QCDW_OK else None


def qcdw_op_hop_form(op: Operator, prec: str = "f64"):
    """(nt, cgroup, fma): the tuned form of the operator's single-RHS hop in precision prec."""
    nt, cg, fma = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(op.ctx.handle, load_library().qcdw_op_hop_form(op.handle, PREC[prec], ctypes.byref(nt), ctypes.byref(cg),
                                                          ctypes.byref(fma)))
    return nt.value, cg.value, fma.value


def qcdw_wall_sources(ctx: Context, lat: qcdw_lattice, t0: int, mom, out):
    """The 12 wall sources on slice t0 with spatial momentum mom into out (12 fermion fields, complex128)."""
    _need(out, 12 * 12 * _volume(lat), "out")
    m = (ctypes.c_int * 3)(*[int(v) for v in mom])
    _check(ctx.handle, load_library().qcdw_wall_sources(ctx.handle, ctypes.byref(lat), int(t0), m,
                                                        _ptr(out, torch.complex128, "out")))


def qcdw_meson_2pt(ctx: Context, lat: qcdw_lattice, S, gamma_snk: int, gamma_src: int, mom, out):
    """C(t) of the 12-field propagator S into out (Lt complex128 on the device)."""
    _need(S, 12 * 12 * _volume(lat), "S")
    _need(out, lat.L[3], "out")
    m = (ctypes.c_int * 3)(*[int(v) for v in mom])
    _check(ctx.handle, load_library().qcdw_meson_2pt(ctx.handle, ctypes.byref(lat), _ptr(S, torch.complex128, "S"),
                                                     int(gamma_snk), int(gamma_src), m,
                                                     _ptr(out, torch.complex128, "out")))


def qcdw_meson_contract(ctx: Context, lat: qcdw_lattice, S, T, gamma_snk: int, gamma_src: int, mom, out):
    """C(t) with the propagator S forward and T in the backward leg into out (Lt complex128 on the device)."""
    _need(S, 12 * 12 * _volume(lat), "S")
    _need(T, 12 * 12 * _volume(lat), "T")
    _need(out, lat.L[3], "out")
    m = (ctypes.c_int * 3)(*[int(v) for v in mom])
    _check(ctx.handle, load_library().qcdw_meson_contract(ctx.handle, ctypes.byref(lat),
                                                          _ptr(S, torch.complex128, "S"), _ptr(T, torch.complex128, "T"),
                                                          int(gamma_snk), int(gamma_src), m,
                                                          _ptr(out, torch.complex128, "out")))


def qcdw_seq_sources(ctx: Context, lat: qcdw_lattice, S, t_f: int, gamma_f: int, mom, out):
    """The 12 sequential sources through the sink slice t_f from the propagator S into out."""
    _need(S, 12 * 12 * _volume(lat), "S")
    _need(out, 12 * 12 * _volume(lat), "out")
    m = (ctypes.c_int * 3)(*[int(v) for v in mom])
    _check(ctx.handle, load_library().qcdw_seq_sources(ctx.handle, ctypes.byref(lat), _ptr(S, torch.complex128, "S"),
                                                       int(t_f), int(gamma_f), m, _ptr(out, torch.complex128, "out")))


def qcdw_invert_multishift(op: Operator, b_e, xs, shifts, tol: float = 1e-10, maxiter: int = 10000):
    """(M_hat^+ M_hat + shifts[i]) xs[i] = b_e on even sites; returns (iterations, residual estimates)."""
    n = len(shifts)
    _need(b_e, 12 * op.volume // 2, "b_e")
    if len(xs) != n:
        raise ValueError("one output field per shift")
    for x in xs:
        _need(x, 12 * op.volume // 2, "x")
    ptrs = (ctypes.c_void_p * n)(*[_ptr(x, torch.complex128, "x") for x in xs])
    sh = (ctypes.c_double * n)(*[float(v) for v in shifts])
    it, res = ctypes.c_int(), (ctypes.c_double * n)()
    _check(op.ctx.handle, load_library().qcdw_invert_multishift(op.handle, _ptr(b_e, torch.complex128, "b_e"), ptrs, sh,
                                                                n, float(tol), int(maxiter), ctypes.byref(it), res))
    return it.value, list(res)


def qcdw_invert(op: Operator, b, x, params: qcdw_solver_params | None = None, raise_on_error: bool = False):
    """Solve M x = b; x holds the initial guess.  Returns a SolveInfo."""
    if params is None:
        params = make_params()
    _need(b, 12 * op.volume, "b")
    _need(x, 12 * op.volume, "x")
    n_hist = max(1, params.maxiter + 2)
    hist = (ctypes.c_double * n_hist)()
    info = qcdw_solve_info()
    info.hist_len = n_hist
    info.res_hist = ctypes.cast(hist, ctypes.POINTER(ctypes.c_double))
    st = load_library().qcdw_invert(op.handle, _ptr(b, torch.complex128, "b"), _ptr(x, torch.complex128, "x"),
                                    ctypes.byref(params), ctypes.byref(info))
    if raise_on_error:
        _check(op.ctx.handle, st)
    elif st in (QCDW_EINVAL, QCDW_ENOMEM, QCDW_EHIP):
        _check(op.ctx.handle, st)
    return SolveInfo(info, hist)


def qcdw_invert_multi(op: Operator, b, x, params: qcdw_solver_params | None = None):
    """Solve for nrhs = b.shape[0] stacked fermion fields; returns a list of SolveInfo."""
    if params is None:
        params = make_params()
    nrhs = int(b.shape[0])
    _need(b, 12 * op.volume * nrhs, "b")
    _need(x, 12 * op.volume * nrhs, "x")
    n_hist = max(1, params.maxiter + 2)
    hists = [(ctypes.c_double * n_hist)() for _ in range(nrhs)]
    infos = (qcdw_solve_info * nrhs)()
    for k in range(nrhs):
        infos[k].hist_len = n_hist
        infos[k].res_hist = ctypes.cast(hists[k], ctypes.POINTER(ctypes.c_double))
    st = load_library().qcdw_invert_multi(op.handle, nrhs, _ptr(b, torch.complex128, "b"),
                                          _ptr(x, torch.complex128, "x"), ctypes.byref(params), infos)
    if st in (QCDW_EINVAL, QCDW_ENOMEM, QCDW_EHIP):
        _check(op.ctx.handle, st)
    return [SolveInfo(infos[k], hists[k]) for k in range(nrhs)]


class Batch:
    """qcdw_batch: operators of different lattices / kappas solved in lockstep."""

    _rank = 1

    def __init__(self, ctx: Context, ops):
        self.ctx = ctx
        self.ops = list(ops)  # keep the operators alive
        arr = (ctypes.c_void_p * len(self.ops))(*[o.handle.value for o in self.ops])
        h = ctypes.c_void_p()
        st = load_library().qcdw_batch_create(ctx.handle, len(self.ops), arr, ctypes.byref(h))
        _check(ctx.handle, st)
        self.handle = h
        ctx._adopt(self)
        for o in self.ops:
            o._children.add(self)

    def close(self):
        if getattr(self, "handle", None):
            load_library().qcdw_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def qcdw_batch_create(ctx: Context, ops) -> Batch:
    return Batch(ctx, ops)


def qcdw_batch_destroy(batch: Batch) -> None:
    batch.close()


def qcdw_invert_batch(batch: Batch, bs, xs, params: qcdw_solver_params | None = None):
    """Solve M_k x_k = b_k for every operator of the batch; returns a list of SolveInfo."""
    if params is None:
        params = make_params()
    n = len(batch.ops)
    if len(bs) != n or len(xs) != n:
        raise ValueError("one source and one solution per operator")
    for k, op in enumerate(batch.ops):
        _need(bs[k], 12 * op.volume, f"b[{k}]")
        _need(xs[k], 12 * op.volume, f"x[{k}]")
    barr = (ctypes.c_void_p * n)(*[_ptr(t, torch.complex128, "b").value for t in bs])
    xarr = (ctypes.c_void_p * n)(*[_ptr(t, torch.complex128, "x").value for t in xs])
    n_hist = max(1, params.maxiter + 2)
    hists = [(ctypes.c_double * n_hist)() for _ in range(n)]
    infos = (qcdw_solve_info * n)()
    for k in range(n):
        infos[k].hist_len = n_hist
        infos[k].res_hist = ctypes.cast(hists[k], ctypes.POINTER(ctypes.c_double))
    st = load_library().qcdw_invert_batch(batch.handle, barr, xarr, ctypes.byref(params), infos)
    if st in (QCDW_EINVAL, QCDW_ENOMEM, QCDW_EHIP):
        _check(batch.ctx.handle, st)
    return [SolveInfo(infos[k], hists[k]) for k in range(n)]


class Net:
    """qcdw_net: the learned gauge-covariant preconditioner of one operator."""

    _rank = 0

    def __init__(self, op: Operator, hidden: int = 12, seed: int = 0, init_scale: float = 0.01):
        self.op = op
        self.hidden = hidden
        h = ctypes.c_void_p()
        st = load_library().qcdw_net_create(op.handle, int(hidden), int(seed), float(init_scale), ctypes.byref(h))
        _check(op.ctx.handle, st)
        self.handle = h
        op.ctx._adopt(self)
        op._children.add(self)

    def close(self):
        if getattr(self, "handle", None):
            load_library().qcdw_net_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def qcdw_net_create(op: Operator, hidden: int = 12, seed: int = 0, init_scale: float = 0.01) -> Net:
    return Net(op, hidden, seed, init_scale)


def qcdw_net_destroy(net: Net) -> None:
    net.close()


def qcdw_net_bind(net: Net, op: Operator) -> None:
    """Move the net to another operator of the same lattice (weights and Adam state kept)."""
    _check(net.op.ctx.handle, load_library().qcdw_net_bind(net.handle, op.handle))
    net.op._children.discard(net)
    net.op = op
    op._children.add(net)


def _wshape(net):
    return (9, net.hidden, 4), (9, 4, net.hidden)


def qcdw_net_get_weights(net: Net):
    """(W1, W2) as complex NumPy arrays [9][hidden][4], [9][4][hidden]."""
    import numpy as np

    s1, s2 = _wshape(net)
    w1 = np.zeros(2 * int(np.prod(s1)))
    w2 = np.zeros(2 * int(np.prod(s2)))
    st = load_library().qcdw_net_get_weights(net.handle, w1.ctypes.data_as(ctypes.c_void_p),
                                             w2.ctypes.data_as(ctypes.c_void_p))
    _check(net.op.ctx.handle, st)
    return w1.view(np.complex128).reshape(s1), w2.view(np.complex128).reshape(s2)


def qcdw_net_set_weights(net: Net, W1, W2) -> None:
    import numpy as np

    s1, s2 = _wshape(net)
    w1 = np.ascontiguousarray(np.asarray(W1, dtype=np.complex128).reshape(s1)).view(np.float64)
    w2 = np.ascontiguousarray(np.asarray(W2, dtype=np.complex128).reshape(s2)).view(np.float64)
    st = load_library().qcdw_net_set_weights(net.handle, w1.ctypes.data_as(ctypes.c_void_p),
                                             w2.ctypes.data_as(ctypes.c_void_p))
    _check(net.op.ctx.handle, st)


def qcdw_net_apply(net: Net, prec, in_e, out_e) -> None:
    prec = PREC[prec] if isinstance(prec, str) else int(prec)
    _need(in_e, 6 * net.op.volume, "in_e")
    _need(out_e, 6 * net.op.volume, "out_e")
    st = load_library().qcdw_net_apply(net.handle, prec, _ptr(in_e, torch.complex128, "in_e"),
                                       _ptr(out_e, torch.complex128, "out_e"))
    _check(net.op.ctx.handle, st)


def _ptr_array(ts, n_each, name):
    for t in ts:
        _need(t, n_each, name)
    return (ctypes.c_void_p * len(ts))(*[_ptr(t, torch.complex128, name).value for t in ts])


def qcdw_net_loss_grad(net: Net, r_e, e_e):
    """(loss, G1, G2) over the pairs; G = dL/dRe W + i dL/dIm W as complex NumPy arrays."""
    import numpy as np

    s1, s2 = _wshape(net)
    g1 = np.zeros(2 * int(np.prod(s1)))
    g2 = np.zeros(2 * int(np.prod(s2)))
    loss = ctypes.c_double()
    n6 = 6 * net.op.volume
    st = load_library().qcdw_net_loss_grad(net.handle, len(r_e), _ptr_array(r_e, n6, "r_e"),
                                           _ptr_array(e_e, n6, "e_e"), ctypes.byref(loss),
                                           g1.ctypes.data_as(ctypes.c_void_p), g2.ctypes.data_as(ctypes.c_void_p))
    _check(net.op.ctx.handle, st)
    return loss.value, g1.view(np.complex128).reshape(s1), g2.view(np.complex128).reshape(s2)


def qcdw_net_train(net: Net, r_e, e_e, steps: int, batch: int = 8, lr: float = 1e-3, seed: int = 0):
    """Adam training on the GPU; returns the per-step batch-mean loss."""
    import numpy as np

    hist = np.zeros(max(1, steps))
    n6 = 6 * net.op.volume
    st = load_library().qcdw_net_train(net.handle, len(r_e), _ptr_array(r_e, n6, "r_e"), _ptr_array(e_e, n6, "e_e"),
                                       int(steps), int(batch), float(lr), int(seed),
                                       hist.ctypes.data_as(ctypes.c_void_p))
    _check(net.op.ctx.handle, st)
    return hist[:steps]


def qcdw_make_training_pairs(op: Operator, b, npairs: int, stride: int):
    """(r_e, e_e) pairs as lists of device tensors [Vh, 4, 3]: errors of a solve of b
    (stride > 0), or seeded Gaussian errors (stride < 0, seed -stride, b unused; may be None)."""
    if stride >= 0 or b is not None:
        _need(b, 12 * op.volume, "b")
    Vh = op.volume // 2
    r = [torch.empty((Vh, 4, 3), dtype=torch.complex128, device="cuda") for _ in range(npairs)]
    e = [torch.empty((Vh, 4, 3), dtype=torch.complex128, device="cuda") for _ in range(npairs)]
    made = ctypes.c_int()
    bp = _ptr(b, torch.complex128, "b") if b is not None else None
    st = load_library().qcdw_make_training_pairs(op.handle, bp, int(npairs), int(stride),
                                                 _ptr_array(r, 6 * op.volume, "r_e"),
                                                 _ptr_array(e, 6 * op.volume, "e_e"), ctypes.byref(made))
    _check(op.ctx.handle, st)
    return r[: made.value], e[: made.value]


def qcdw_invert_fgmres(op: Operator, net, b, x, params: qcdw_solver_params | None = None):
    """FGMRES(m) with the net as right preconditioner (net None: none); returns a SolveInfo."""
    if params is None:
        params = make_params()
    _need(b, 12 * op.volume, "b")
    _need(x, 12 * op.volume, "x")
    n_hist = max(1, params.maxiter + 2)
    hist = (ctypes.c_double * n_hist)()
    info = qcdw_solve_info()
    info.hist_len = n_hist
    info.res_hist = ctypes.cast(hist, ctypes.POINTER(ctypes.c_double))
    st = load_library().qcdw_invert_fgmres(op.handle, net.handle if net is not None else None,
                                           _ptr(b, torch.complex128, "b"), _ptr(x, torch.complex128, "x"),
                                           ctypes.byref(params), ctypes.byref(info))
    if st in (QCDW_EINVAL, QCDW_ENOMEM, QCDW_EHIP):
        _check(op.ctx.handle, st)
    return SolveInfo(info, hist)


# ---------------------------------------------------------------------------
# multigrid
# ---------------------------------------------------------------------------
def make_mg_params(**kw) -> qcdw_mg_params:
    """qcdw_mg_params with the library defaults, then the given fields (block: 4 ints)."""
    prm = qcdw_mg_params()
    load_library().qcdw_mg_params_default(ctypes.byref(prm))
    for k, v in kw.items():
        if k == "block":
            for mu in range(4):
                prm.block[mu] = int(v[mu])
        elif not hasattr(prm, k):
            raise AttributeError(k)
        else:
            setattr(prm, k, v)
    return prm


class Multigrid:
    """qcdw_mg: two-level aggregation multigrid set up on one operator (vecs: None or nvec fermion fields)."""

    _rank = 0

    def __init__(self, op: Operator, params: qcdw_mg_params | None = None, vecs=None):
        self.op = op
        if params is None:
            params = make_mg_params()
        self.params = params
        if vecs is not None:
            _need(vecs, params.nvec * 12 * op.volume, "vecs")
        h = ctypes.c_void_p()
        st = load_library().qcdw_mg_create(op.handle, ctypes.byref(params),
                                           _ptr(vecs, torch.complex128, "vecs") if vecs is not None else None,
                                           ctypes.byref(h))
        _check(op.ctx.handle, st)
        self.handle = h
        dims = (ctypes.c_int * 4)()
        nv = ctypes.c_int()
        _check(op.ctx.handle, load_library().qcdw_mg_info(h, dims, ctypes.byref(nv)))
        self.coarse_dims = tuple(dims)
        self.nvec = nv.value
        self.coarse_sites = int(math.prod(self.coarse_dims))
        op.ctx._adopt(self)
        op._children.add(self)

    def close(self):
        if getattr(self, "handle", None):
            load_library().qcdw_mg_destroy(self.handle)
            self.handle = None

    def coarse_len(self) -> int:
        return self.coarse_sites * 2 * self.nvec


def qcdw_mg_vectors(mg: Multigrid, out) -> None:
    _need(out, mg.nvec * 12 * mg.op.volume, "out")
    _check(mg.op.ctx.handle, load_library().qcdw_mg_vectors(mg.handle, _ptr(out, torch.complex128, "out")))


def qcdw_mg_restrict(mg: Multigrid, fine, coarse) -> None:
    _need(fine, 12 * mg.op.volume, "fine")
    _need(coarse, mg.coarse_len(), "coarse")
    _check(mg.op.ctx.handle, load_library().qcdw_mg_restrict(mg.handle, _ptr(fine, torch.complex128, "fine"),
                                                             _ptr(coarse, torch.complex128, "coarse")))


def qcdw_mg_prolong(mg: Multigrid, coarse, fine) -> None:
    _need(fine, 12 * mg.op.volume, "fine")
    _need(coarse, mg.coarse_len(), "coarse")
    _check(mg.op.ctx.handle, load_library().qcdw_mg_prolong(mg.handle, _ptr(coarse, torch.complex128, "coarse"),
                                                            _ptr(fine, torch.complex128, "fine")))


def qcdw_mg_coarse_apply(mg: Multigrid, cin, cout) -> None:
    _need(cin, mg.coarse_len(), "in")
    _need(cout, mg.coarse_len(), "out")
    _check(mg.op.ctx.handle, load_library().qcdw_mg_coarse_apply(mg.handle, _ptr(cin, torch.complex128, "in"),
                                                                 _ptr(cout, torch.complex128, "out")))


def qcdw_mg_coarse_op(mg: Multigrid, stencil) -> None:
    _need(stencil, mg.coarse_sites * 9 * (2 * mg.nvec) ** 2, "stencil")
    _check(mg.op.ctx.handle, load_library().qcdw_mg_coarse_op(mg.handle, _ptr(stencil, torch.complex128, "stencil")))


def qcdw_invert_mg(op: Operator, mg: Multigrid, b, x, params: qcdw_solver_params | None = None):
    """FGMRES(m) with the multigrid preconditioner; returns a SolveInfo."""
    if params is None:
        params = make_params()
    _need(b, 12 * op.volume, "b")
    _need(x, 12 * op.volume, "x")
    n_hist = max(1, params.maxiter + 2)
    hist = (ctypes.c_double * n_hist)()
    info = qcdw_solve_info()
    info.hist_len = n_hist
    info.res_hist = ctypes.cast(hist, ctypes.POINTER(ctypes.c_double))
    st = load_library().qcdw_invert_mg(op.handle, mg.handle, _ptr(b, torch.complex128, "b"),
                                       _ptr(x, torch.complex128, "x"), ctypes.byref(params), ctypes.byref(info))
    if st in (QCDW_EINVAL, QCDW_ENOMEM, QCDW_EHIP):
        _check(op.ctx.handle, st)
    return SolveInfo(info, hist)
