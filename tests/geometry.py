"""Test-side lattice geometry written from the layout description alone.

Even-odd ("cb2") site order [2, Lt, Lz, Ly, Lx/2] with parity (x+y+z+t) mod 2
and x fastest (paper, Sec. II.A).  Used to build shifted fields, gauge
transformations and plane waves independently of the oracle's own indexing.
"""
import numpy as np


def eo_index(L, x, y, z, t):
    Lx, Ly, Lz, Lt = L
    V = Lx * Ly * Lz * Lt
    p = (x + y + z + t) % 2
    return p * (V // 2) + ((t * Lz + z) * Ly + y) * (Lx // 2) + x // 2


def coords(L):
    """(V, 4) coordinates (x, y, z, t) for every eo index, by enumeration."""
    Lx, Ly, Lz, Lt = L
    V = Lx * Ly * Lz * Lt
    out = np.zeros((V, 4), dtype=np.int64)
    for t in range(Lt):
        for z in range(Lz):
            for y in range(Ly):
                for x in range(Lx):
                    out[eo_index(L, x, y, z, t)] = (x, y, z, t)
    return out


def shift_table(L, mu, step):
    """idx[i] = eo index of (site i) + step * mu-hat, periodic."""
    c = coords(L).copy()
    c[:, mu] = (c[:, mu] + step) % L[mu]
    return eo_index(L, c[:, 0], c[:, 1], c[:, 2], c[:, 3])


def transform_gauge(L, U, Om):
    """U'_mu(x) = Om(x) U_mu(x) Om(x+mu)^+ (Om: [V, 3, 3] in eo order)."""
    V = int(np.prod(L))
    Uf = U.reshape(4, V, 3, 3)
    Of = Om.reshape(V, 3, 3)
    out = np.empty_like(Uf)
    for mu in range(4):
        fw = shift_table(L, mu, +1)
        out[mu] = Of @ Uf[mu] @ np.conj(np.swapaxes(Of[fw], -1, -2))
    return out.reshape(U.shape)
