"""CPU oracle of the two-level (aggregation) multigrid preconditioner, plain NumPy, FP64.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper enables QUDA's multigrid solver for Wilson/clover fermions by a block size per level
(Sec. II.E; Sec. III.B: a 2^4 sublattice is projected to one coarse site), set up when the gauge
field is loaded and reused for other masses.  The method (Brannick et al. 2008; Babich et al. 2010,
the algorithm QUDA implements, Clark et al. 2016) written out plainly:

* Aggregates.  The lattice is cut into blocks of b = (bx, by, bz, bt) sites; a coarse site x^ is one
  block, numbered lexicographically on the coarse lattice Lc = L / b with x fastest.  Each block is
  split by chirality chi (spins {0, 1}: chi = 0, spins {2, 3}: chi = 1; gamma_5 = diag(1, 1, -1, -1)
  in the DeGrand-Rossi basis), giving the aggregate (x^, chi) of 6 |b| complex unknowns.
* Prolongator.  Given near-null vectors v_0 .. v_{N-1} (full fermion fields), the restriction of the
  v_k to each aggregate is orthonormalised in the order k = 0, 1, .. by modified Gram-Schmidt; column
  (x^, chi, k) of P is the k-th orthonormal vector of aggregate (x^, chi), zero elsewhere.  So
  P^+ P = 1, P commutes with gamma_5 and each v_k lies in the range of P.  A vector whose part
  outside the span of the earlier ones is below 1e-10 of its norm on some aggregate is rejected
  as linearly dependent.
* Coarse vectors: [Vc][2][N] complex, index (x^ chi k) -> (x^ * 2 + chi) * N + k.
* Coarse operator: D_c = P^+ M P (Galerkin), M the full Wilson-clover matrix of Eq. "clover".
* Two-level preconditioner for M x = b (one application z = K(v)): coarse correction
  z = P D_c^-1 P^+ v, then `nu` steps of minimal-residual smoothing on M: r = v - M z,
  w = M r, alpha = (w, r) / (w, w), z += alpha r.  Used inside FGMRES (oracle/fgmres.py).

Pins (tests/test_oracle_multigrid.py): orthonormality and span; single-site aggregates with N = 6
(P unitary, so D_c is similar to M and P D_c^-1 P^+ = M^-1); the free-field coarse operator of
constant-per-block vectors, a Wilson operator on the coarse lattice with hopping kappa/b and a mass
shift, checked against its plane-wave closed form; gamma_5-hermiticity of D_c; invariance of D_c
under a gauge transformation of links and vectors; the nearest-neighbour coarse stencil.
"""
from __future__ import annotations

import numpy as np

import oracle


# a vector whose part outside the span of the previous ones is below this fraction of its norm on an
# aggregate counts as linearly dependent (rounding leaves ~1e-16 of an exactly dependent vector)
DEPENDENT = 1e-10


def coarse_dims(L, b):
    """Coarse lattice extents L / b (each block extent must divide its lattice extent)."""
    for mu in range(4):
        if b[mu] < 1 or L[mu] % b[mu]:
            raise ValueError(f"block {tuple(b)} does not tile lattice {tuple(L)}")
    return tuple(L[mu] // b[mu] for mu in range(4))


def block_index(L, b) -> np.ndarray:
    """Coarse site of every fine site, in the fermion layout's eo site order: [2, Lt, Lz, Ly, Lx/2]."""
    Lc = coarse_dims(L, b)
    X = oracle.coords_table(L)  # (V, 4) coordinates (x, y, z, t) in eo order
    cx = X // np.asarray(b)[None, :]
    idx = ((cx[:, 3] * Lc[2] + cx[:, 2]) * Lc[1] + cx[:, 1]) * Lc[0] + cx[:, 0]
    return idx.reshape(2, L[3], L[2], L[1], L[0] // 2)


def _aggregate_masks(L, b):
    """Boolean masks over the fermion layout [2, Lt, Lz, Ly, Lx/2, 4, 3], one per (coarse site, chi)."""
    blk = block_index(L, b)
    Vc = int(np.prod(coarse_dims(L, b)))
    fshape = oracle.fermion_shape(L)
    masks = []
    for xc in range(Vc):
        site = (blk == xc)[..., None, None]
        for chi in range(2):
            spin = np.zeros((4, 3), dtype=bool)
            spin[2 * chi: 2 * chi + 2, :] = True
            masks.append(np.broadcast_to(site & spin, fshape))
    return masks


def block_orthonormalize(L, b, vecs):
    """Orthonormal block vectors W[k] (same shape as vecs: [N, fermion layout]): on each aggregate the
    restrictions of v_0 .. v_{N-1} orthonormalised in order by modified Gram-Schmidt."""
    vecs = np.asarray(vecs, dtype=np.complex128)
    N = vecs.shape[0]
    W = np.zeros_like(vecs)
    for m in _aggregate_masks(L, b):
        cols = [vecs[k][m].copy() for k in range(N)]
        for k in range(N):
            w = cols[k]
            n0 = np.linalg.norm(w)
            for j in range(k):
                w = w - np.vdot(cols[j], w) * cols[j]
            nrm = np.linalg.norm(w)
            if not nrm > DEPENDENT * n0:  # (numerically) in the span of the previous vectors, or zero
                raise ValueError("near-null vectors are linearly dependent on an aggregate")
            cols[k] = w / nrm
            W[k][m] = cols[k]
    return W


def prolong(L, b, W, ec):
    """P e_c: ec [Vc, 2, N] complex -> fermion field."""
    blk = block_index(L, b)
    N = W.shape[0]
    ec = np.asarray(ec, dtype=np.complex128).reshape(-1, 2, N)
    out = np.zeros(oracle.fermion_shape(L), dtype=np.complex128)
    chi_of_spin = np.array([0, 0, 1, 1])
    for k in range(N):
        coef = ec[blk][..., chi_of_spin, k]  # [2, Lt, Lz, Ly, Lx/2, 4]
        out += coef[..., None] * W[k]
    return out


def restrict(L, b, W, r):
    """P^+ r: fermion field -> [Vc, 2, N] complex."""
    blk = block_index(L, b).reshape(-1)
    Vc = int(np.prod(coarse_dims(L, b)))
    N = W.shape[0]
    r = np.asarray(r, dtype=np.complex128).reshape(-1, 4, 3)
    out = np.zeros((Vc, 2, N), dtype=np.complex128)
    for k in range(N):
        w = W[k].reshape(-1, 4, 3)
        prod = (np.conj(w) * r).sum(axis=2)  # [V, 4]
        per_chi = np.stack([prod[:, 0] + prod[:, 1], prod[:, 2] + prod[:, 3]], axis=1)  # [V, 2]
        for chi in range(2):
            out[:, chi, k] = np.bincount(blk, weights=per_chi[:, chi].real, minlength=Vc) + \
                1j * np.bincount(blk, weights=per_chi[:, chi].imag, minlength=Vc)
    return out


def coarse_dense(L, b, W, U, clover, kappa: float, csw: float, t_bc: int = 1, weights=None) -> np.ndarray:
    """D_c = P^+ M P as a dense (2 N Vc) x (2 N Vc) matrix, column by column: P e_j, then M, then P^+
    (weights: the hop weights of oracle.dirac, for the anisotropic operator)."""
    N = W.shape[0]
    nc = int(np.prod(coarse_dims(L, b))) * 2 * N
    D = np.zeros((nc, nc), dtype=np.complex128)
    for j in range(nc):
        e = np.zeros(nc, dtype=np.complex128)
        e[j] = 1.0
        D[:, j] = restrict(L, b, W, oracle.dirac(L, U, clover, prolong(L, b, W, e), kappa, csw, t_bc,
                                                 weights)).reshape(-1)
    return D


def coarse_apply(L, b, W, U, clover, ec, kappa: float, csw: float, t_bc: int = 1, weights=None):
    """D_c e_c = P^+ M P e_c without forming D_c (for lattices where the dense matrix is too large)."""
    return restrict(L, b, W, oracle.dirac(L, U, clover, prolong(L, b, W, ec), kappa, csw, t_bc, weights))


def two_level_precond(L, b, W, U, clover, kappa: float, csw: float, Dc_inv, nu: int = 0, t_bc: int = 1):
    """K(v) = P D_c^-1 P^+ v followed by nu minimal-residual smoothing steps on M (Dc_inv: a callable
    solving D_c y = r on coarse vectors [Vc, 2, N])."""
    def M(x):
        return oracle.dirac(L, U, clover, x, kappa, csw, t_bc)

    def K(v):
        z = prolong(L, b, W, Dc_inv(restrict(L, b, W, v)))
        for _ in range(nu):
            r = v - M(z)
            w = M(r)
            z = z + (np.vdot(w, r) / np.vdot(w, w)) * r
        return z

    return K
