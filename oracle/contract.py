"""Oracle: wall sources and meson two-point contractions (the steps on either side of the solves in
the paper's propagator workflow, Sec. III.B).  Test infrastructure only, like the rest of `oracle/`.
Plain NumPy written from the definitions; every sum is taken over the full 12 x 12 spin-colour
matrices with explicit gamma matrices, no structure exploited.

Readings (stated once, used by the library too):
  * A propagator is 12 fields S_k, k = 3 s0 + c0 (source spin s0, colour c0), each in the paper's
    fermion layout; S(x)[3 s + c, k] = S_k(x)[s, c].
  * The wall source of component k on time slice t0 with spatial momentum n is
    eta_k(x) = e^{+i p.x} delta(x_t, t0) e_k with p_i = 2 pi n_i / L_i.
  * The meson two-point function for sink and source gammas G_snk = Gamma(a), G_src = Gamma(b) (the
    paper's bitmask Gamma(n)) and momentum n is
        C(t) = sum_{x: x_t = t} e^{-i p.x} Tr[G_snk S(x) G_src g5 S(x)^+ g5],
    the backward propagator written with g5-hermiticity.  For G_snk = G_src = g5 it is
    sum_{x in t} e^{-i p.x} ||S(x)||^2: the pion.  No overall sign or Gamma-bar is applied.
Parity unpinned: the choice of these conventions (signs, the phase sign of the source) is a
reading; the pins below fix the arithmetic given the reading.
"""
import numpy as np

from . import coords_table, gamma_bitmask


def wall_sources(L, t0: int, mom=(0, 0, 0)) -> np.ndarray:
    """The 12 wall sources [12, V, 4, 3] (paper layout per field, eo site order)."""
    V = int(np.prod(L))
    c = coords_table(L)
    p = 2 * np.pi * np.asarray(mom, dtype=np.float64) / np.asarray(L[:3], dtype=np.float64)
    phase = np.exp(1j * (c[:, :3] @ p)) * (c[:, 3] == t0)
    out = np.zeros((12, V, 4, 3), dtype=np.complex128)
    for k in range(12):
        out[k, :, k // 3, k % 3] = phase
    return out


def meson_2pt(L, S, g_snk: int, g_src: int, mom=(0, 0, 0)) -> np.ndarray:
    """C(t) for t = 0 .. Lt-1 from the 12-field propagator S [12, V, 4, 3] (see the module text)."""
    return contract(L, S, S, g_snk, g_src, mom)


def seq_sources(L, S, t_f: int, g_f: int, mom=(0, 0, 0)) -> np.ndarray:
    """Sequential sources through the sink: eta_k(x) = delta(x_t, t_f) e^{+i p.x} G S_k(x) with the spin
    matrix G = g5 Gamma(g_f)^+ g5 acting on the sink spin of S_k(x).  T = M^{-1} eta then gives the
    three-point function contract(S, T, g_ins, g_src, q) = sum_{y_t = tau} e^{-i q.y}
    Tr[G_ins S(y) G_src g5 T(y)^+ g5] = sum_{x_t = t_f, y_t = tau} e^{-i p.x} e^{-i q.y}
    Tr[Gamma(g_f) S(x<-y) G_ins S(y<-0) G_src S(0<-x)] (g5-hermiticity on both backward legs)."""
    V = int(np.prod(L))
    S = np.asarray(S, dtype=np.complex128).reshape(12, V, 4, 3)
    c = coords_table(L)
    p = 2 * np.pi * np.asarray(mom, dtype=np.float64) / np.asarray(L[:3], dtype=np.float64)
    phase = np.exp(1j * (c[:, :3] @ p)) * (c[:, 3] == t_f)
    g5 = gamma_bitmask(15)
    G = g5 @ np.conj(gamma_bitmask(g_f).T) @ g5
    return np.einsum("x,st,kxtc->kxsc", phase, G, S)


def contract(L, S, T, g_snk: int, g_src: int, mom=(0, 0, 0)) -> np.ndarray:
    """C(t) = sum_{x_t = t} e^{-i p.x} Tr[G_snk S(x) G_src g5 T(x)^+ g5] for two 12-field propagators."""
    V = int(np.prod(L))
    S = np.asarray(S, dtype=np.complex128).reshape(12, V, 12)  # [k][x][3 s + c]
    T = np.asarray(T, dtype=np.complex128).reshape(12, V, 12)
    M = np.transpose(S, (1, 2, 0))  # M[x] = S(x), 12 x 12 (row: sink s c, column: source k)
    N = np.transpose(T, (1, 2, 0))
    c = coords_table(L)
    p = 2 * np.pi * np.asarray(mom, dtype=np.float64) / np.asarray(L[:3], dtype=np.float64)
    phase = np.exp(-1j * (c[:, :3] @ p))
    I3 = np.eye(3)
    A = np.kron(gamma_bitmask(g_snk), I3)
    g5 = np.kron(gamma_bitmask(15), I3)
    B = np.kron(gamma_bitmask(g_src), I3)
    back = g5 @ np.conj(np.transpose(N, (0, 2, 1))) @ g5  # g5 T(x)^+ g5, per site
    per_site = np.einsum("ab,xbc,cd,xda->x", A, M, B, back)  # Tr[A S(x) B back(x)]
    out = np.zeros(L[3], dtype=np.complex128)
    np.add.at(out, c[:, 3], phase * per_site)
    return out
