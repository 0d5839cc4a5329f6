// Two-level aggregation multigrid preconditioner for the Wilson-clover operator.
//
// The paper runs QUDA's multigrid solver for Wilson/clover fermions by giving a block size per level
// (Sec. II.E; Sec. III.B: a 2^4 sublattice becomes one coarse site), set up when the gauge field is
// loaded and reused for other quark masses.  This is the method (Brannick et al. 2008, Babich et al.
// 2010) written for gfx950:
//   - aggregates: blocks of b sites split by chirality (spins {0,1} and {2,3}); the near-null vectors
//     restricted to each aggregate are orthonormalised by modified Gram-Schmidt, giving the
//     prolongator P (column (coarse site, chirality, k));
//   - the Galerkin coarse operator D_c = P^+ M P is a nearest-neighbour stencil on the coarse lattice
//     (a self term and one (2N x 2N) matrix per direction), built directly from the links, the clover
//     term and the block vectors (one workgroup per coarse site and stencil entry, fixed order);
//   - the preconditioner of the even-odd system M_hat: coarse correction z_e = [P D_c^-1 P^+ (A_ee v_e)]_e
//     (M_hat^-1 = (M^-1)_ee A_ee), the coarse system solved approximately by BiCGStab in FP32 with
//     device-side scalars (no host synchronisation), then minimal-residual smoothing steps on M_hat;
//     FGMRES(m) on M_hat uses it as its right preconditioner.
// Internal layouts: block vectors W [Vc][N][2 parity][|b|/2][4 spin][3 colour] complex (one contiguous
// run per coarse site and vector); coarse vectors [Vc][2 chirality][N] complex; coarse stencil Yt
// [Vc][9][2N column][2N row] complex (entry 0: self, 1 + 2 mu: from x^+mu, 2 + 2 mu: from x^-mu), the
// column-major blocks make the rows of one column contiguous for the threads of a coarse site.
#include <memory>
#include <numeric>

#include "hop_common.h"
#include "host.h"

namespace qcdw {

struct MgDev {
    Geom g;
    int Lc[4], b[4];
    int Vc;  // coarse sites
    int hb;  // fine sites per parity in one block
    int N;   // near-null vectors
    int nc;  // 2 N
    const int* blk_sites;  // [Vc][2][hb] eo site (within its parity)
    const int* fine_loc;   // [2][Vh] coarse site * hb + local index
    const int* cnbr;       // [Vc][8] coarse neighbour in direction 2 mu + (0 forward, 1 backward)
};

__device__ __forceinline__ long w_index(const MgDev& m, int cs, int k, int p, int j)
{
    return ((((long)cs * m.N + k) * 2 + p) * m.hb + j) * 12;
}

// DeGrand-Rossi gamma_mu: one nonzero per row, gamma_mu[s][gperm(mu, s)] = gph(mu, s)
__device__ __forceinline__ int gperm(int mu, int s)
{
    return mu < 2 ? 3 - s : (s + 2) & 3;
}
__device__ __forceinline__ cx<double> gph(int mu, int s)
{
    switch (mu) {
    case 0: return s < 2 ? cx<double>{0.0, 1.0} : cx<double>{0.0, -1.0};
    case 1: return (s == 0 || s == 3) ? cx<double>{-1.0, 0.0} : cx<double>{1.0, 0.0};
    case 2: return (s == 0 || s == 3) ? cx<double>{0.0, 1.0} : cx<double>{0.0, -1.0};
    default: return {1.0, 0.0};
    }
}

// entry (r, c) of the Hermitian 6 x 6 chirality block chi of a clover-type field (reordered packing of
// pack.hip: [d0 d1 d2 | L10 L20 L21 | L30 L31 L32 L40 L41 L42 L50 L51 L52 | d3 d4 d5 | L43 L53 L54])
__device__ __forceinline__ cx<double> herm6(const double* A, int site, int chi, int r, int c)
{
    const long base = clov_index(site, chi, 0);
    if (r == c) return {A[base + (r < 3 ? r : 24 + r)], 0.0};
    const bool lower = r > c;
    const int j = lower ? r : c, k = lower ? c : r;
    int pos;
    if (j < 3) pos = 3 + 2 * (j * (j - 1) / 2 + k);
    else if (k < 3) pos = 9 + 2 * ((j - 3) * 3 + k);
    else pos = 30 + 2 * (j == 4 ? 0 : (k == 3 ? 1 : 2));
    const cx<double> v = {A[base + pos], A[base + pos + 1]};
    return lower ? v : conj(v);
}

// full link U_mu(x) (3 x 3) of the FP64 internal gauge field (row 2 rebuilt for reconstruct-12)
template <int R>
__device__ __forceinline__ void link3(const void* gauge, int mu, int p, int site, int Vh, cx<double> (&u)[9])
{
    constexpr bool soa = link_soa_for(P64::cbytes);
    load_link<P64, R>(gauge, link_base(mu, p, site, Vh, R, soa), link_stride(Vh, soa), u);
}

// ---------------------------------------------------------------------------
// set-up kernels
// ---------------------------------------------------------------------------
// W <- the near-null vectors (N fields in the paper's fermion layout), gathered per block
__global__ void k_mg_gather(MgDev m, const double2* __restrict__ vecs, double2* W)
{
    const long n = (long)m.Vc * m.N * 2 * m.hb * 12;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int sc = (int)(e % 12);
    long r = e / 12;
    const int j = (int)(r % m.hb);
    r /= m.hb;
    const int p = (int)(r % 2);
    r /= 2;
    const int k = (int)(r % m.N);
    const int cs = (int)(r / m.N);
    const int site = m.blk_sites[((long)cs * 2 + p) * m.hb + j];
    W[e] = vecs[(long)k * 12 * 2 * m.g.Vh + ((long)p * m.g.Vh + site) * 12 + sc];
}

// W -> N fields in the paper's fermion layout (the inverse of k_mg_gather)
__global__ void k_mg_scatter(MgDev m, const double2* __restrict__ W, double2* vecs)
{
    const long n = (long)m.Vc * m.N * 2 * m.hb * 12;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int sc = (int)(e % 12);
    long r = e / 12;
    const int j = (int)(r % m.hb);
    r /= m.hb;
    const int p = (int)(r % 2);
    r /= 2;
    const int k = (int)(r % m.N);
    const int cs = (int)(r / m.N);
    const int site = m.blk_sites[((long)cs * 2 + p) * m.hb + j];
    vecs[(long)k * 12 * 2 * m.g.Vh + ((long)p * m.g.Vh + site) * 12 + sc] = W[e];
}

// out = a - b on n complex entries
__global__ void k_mg_sub(const double2* __restrict__ a, const double2* __restrict__ b, double2* out, long n)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const double2 x = a[e], y = b[e];
    out[e] = make_double2(x.x - y.x, x.y - y.y);
}

// sum of a complex value over the 256-thread block in a fixed order, returned to every thread
__device__ __forceinline__ cx<double> block_sum_cx(cx<double> v)
{
    __shared__ double red[2];
    double a[2] = {v.re, v.im};
    block_sum_store<2>(a, red);
    __syncthreads();
    const cx<double> out = {red[0], red[1]};
    __syncthreads();
    return out;
}

constexpr double MG_DEPENDENT = 1e-10;

// Modified Gram-Schmidt of the N vectors on aggregate (coarse site, chirality) = (blockIdx.x / 2,
// blockIdx.x % 2), in the order k = 0, 1, ..; a vanishing vector sets *bad
__global__ __launch_bounds__(256) void k_mg_orth(MgDev m, double2* W, int* bad)
{
    const int cs = blockIdx.x >> 1, chi = blockIdx.x & 1;
    const int len = 2 * m.hb * 6;  // (parity, local site, 2 spins x 3 colours)
    auto at = [&](int k, int e) {
        const int p = e / (m.hb * 6), rem = e - p * m.hb * 6;
        const int j = rem / 6, sc = 6 * chi + rem % 6;
        return w_index(m, cs, k, p, j) + sc;
    };
    for (int k = 0; k < m.N; k++) {
        cx<double> n0 = {0.0, 0.0};
        for (int e = threadIdx.x; e < len; e += blockDim.x) {
            const double2 b = W[at(k, e)];
            n0.re += b.x * b.x + b.y * b.y;
        }
        n0 = block_sum_cx(n0);
        for (int jv = 0; jv < k; jv++) {
            cx<double> d = {0.0, 0.0};
            for (int e = threadIdx.x; e < len; e += blockDim.x) {
                const double2 a = W[at(jv, e)], b = W[at(k, e)];
                d.re += a.x * b.x + a.y * b.y;
                d.im += a.x * b.y - a.y * b.x;
            }
            d = block_sum_cx(d);
            for (int e = threadIdx.x; e < len; e += blockDim.x) {
                const double2 a = W[at(jv, e)];
                double2& b = W[at(k, e)];
                b.x -= d.re * a.x - d.im * a.y;
                b.y -= d.re * a.y + d.im * a.x;
            }
            __syncthreads();
        }
        cx<double> nn = {0.0, 0.0};
        for (int e = threadIdx.x; e < len; e += blockDim.x) {
            const double2 b = W[at(k, e)];
            nn.re += b.x * b.x + b.y * b.y;
        }
        nn = block_sum_cx(nn);
        // numerically in the span of the earlier vectors (or zero): part left below 1e-10 of the norm
        if (!(nn.re > MG_DEPENDENT * MG_DEPENDENT * n0.re) || !isfinite(nn.re)) {
            if (threadIdx.x == 0) atomicAdd(bad, 1);
            return;
        }
        const double inv = 1.0 / sqrt(nn.re);
        for (int e = threadIdx.x; e < len; e += blockDim.x) {
            double2& b = W[at(k, e)];
            b.x *= inv;
            b.y *= inv;
        }
        __syncthreads();
    }
}

// Galerkin coarse operator, one workgroup per (coarse site, stencil entry d): the sum over the fine
// sites x of the block and the hops of M that stay in the block (d = 0, with the clover term A) or leave
// it through the +mu (d = 1 + 2 mu) or -mu (d = 2 + 2 mu) face, of W(x)^+ T W(y) with T = A(x) (y = x),
// T = -kappa w_mu s (1 - g_mu) U_mu(x) (y = x + mu) or -kappa w_mu s (1 + g_mu) U_mu(x - mu)^+ (y = x - mu),
// w_mu the direction's hop weight and s the time-boundary sign.  Entries in registers, G = T W(y) and
// W(x) staged in LDS.
constexpr int MG_MAX_N = 32;
template <int R>
__global__ __launch_bounds__(256) void k_mg_coarse_build(MgDev m, const double2* __restrict__ W, const void* gauge,
                                                          const double* __restrict__ A0, const double* __restrict__ A1,
                                                          double kappa, double2* Yt)
{
    constexpr int MAXE = (2 * MG_MAX_N) * (2 * MG_MAX_N) / 256;
    __shared__ cx<double> Wx[MG_MAX_N][12];
    __shared__ cx<double> G[2 * MG_MAX_N][12];
    const int cs = blockIdx.x / 9, d = blockIdx.x % 9;
    const int N = m.N, nc = m.nc, ne = nc * nc;
    const Geom& g = m.g;
    cx<double> acc[MAXE];
#pragma unroll
    for (int i = 0; i < MAXE; i++) acc[i] = {0.0, 0.0};
    const int dmu = d == 0 ? -1 : (d - 1) >> 1, ddir = d == 0 ? 0 : (d - 1) & 1;
    if (d != 0 && m.Lc[dmu] == 1) {  // no face in this direction: every hop stays in the block
        for (int e = threadIdx.x; e < ne; e += 256) Yt[((long)cs * 9 + d) * ne + e] = make_double2(0.0, 0.0);
        return;
    }
    for (int p = 0; p < 2; p++) {
        for (int j = 0; j < m.hb; j++) {
            const int site = m.blk_sites[((long)cs * 2 + p) * m.hb + j];
            int xc[4];
            site_coords(g, site, p, xc[0], xc[1], xc[2], xc[3]);
            const int L[4] = {g.Lx, g.Ly, g.Lz, g.Lt};
            if (d != 0) {  // only the face sites of this entry's direction contribute (uniform test)
                const int yq = ddir == 0 ? (xc[dmu] + 1 == L[dmu] ? 0 : xc[dmu] + 1)
                                         : (xc[dmu] == 0 ? L[dmu] - 1 : xc[dmu] - 1);
                if (yq / m.b[dmu] == xc[dmu] / m.b[dmu]) continue;
            }
            __syncthreads();  // previous site's Wx no longer read
            for (int e = threadIdx.x; e < N * 12; e += 256) {
                const double2 v = W[w_index(m, cs, e / 12, p, j) + e % 12];
                Wx[e / 12][e % 12] = {v.x, v.y};
            }
            // terms of this site: t = -1 the clover term, else hop 2 mu + dir
            for (int t = -1; t < 8; t++) {
                const int mu = t < 0 ? 0 : t >> 1, dir = t < 0 ? 0 : t & 1;
                int y[4] = {xc[0], xc[1], xc[2], xc[3]};
                bool inside = true;
                if (t >= 0) {
                    y[mu] = dir == 0 ? (xc[mu] + 1 == L[mu] ? 0 : xc[mu] + 1) : (xc[mu] == 0 ? L[mu] - 1 : xc[mu] - 1);
                    inside = (y[mu] / m.b[mu]) == (xc[mu] / m.b[mu]);
                }
                if (d == 0 ? !inside : (t < 0 || mu != dmu || dir != ddir || inside)) continue;
                const int py = (y[0] + y[1] + y[2] + y[3]) & 1;
                const int sy = ((y[3] * g.Lz + y[2]) * g.Ly + y[1]) * g.Lxh + (y[0] >> 1);
                const int loc = m.fine_loc[(long)py * g.Vh + sy];
                const int cy = loc / m.hb, jy = loc - cy * m.hb;
                cx<double> u[9];
                double coef = 0.0;
                if (t >= 0) {
                    if (dir == 0) link3<R>(gauge, mu, p, site, g.Vh, u);
                    else link3<R>(gauge, mu, py, sy, g.Vh, u);
                    const double wt = mu < 3 ? g.xs : 1.0;
                    const bool cross = mu == 3 && ((dir == 0 && xc[3] == g.Lt - 1) || (dir == 1 && xc[3] == 0));
                    coef = -kappa * wt * ((g.t_bc < 0 && cross) ? -1.0 : 1.0);
                }
                __syncthreads();  // Wx staged; previous G no longer read
                // G[col][s][c] = (T P_chi' W_k'(y))[s][c], col = chi' N + k'
                for (int e = threadIdx.x; e < nc * 12; e += 256) {
                    const int col = e / 12, sc = e % 12, s = sc / 3, c = sc % 3;
                    const int chi2 = col / N, k2 = col - chi2 * N;
                    const long wb = w_index(m, cy, k2, py, jy);
                    cx<double> out = {0.0, 0.0};
                    if (t < 0) {
                        if ((s >> 1) == chi2) {
                            const double* A = p == 0 ? A0 : A1;
                            for (int s2 = 2 * chi2; s2 < 2 * chi2 + 2; s2++)
                                for (int c2 = 0; c2 < 3; c2++) {
                                    const double2 wv = W[wb + 3 * s2 + c2];
                                    out = out + herm6(A, site, chi2, 3 * (s & 1) + c, 3 * (s2 & 1) + c2) *
                                                    cx<double>{wv.x, wv.y};
                                }
                        }
                    } else {
                        // (1 -/+ g_mu) applied to U w (forward) or U^+ w (backward), w = P_chi' W_k'(y)
                        const int s_other = gperm(mu, s);
                        const cx<double> ph = gph(mu, s);
                        cx<double> us = {0.0, 0.0}, uo = {0.0, 0.0};
                        for (int c2 = 0; c2 < 3; c2++) {
                            const cx<double> uc = dir == 0 ? u[3 * c + c2] : conj(u[3 * c2 + c]);
                            if ((s >> 1) == chi2) {
                                const double2 wv = W[wb + 3 * s + c2];
                                us = us + uc * cx<double>{wv.x, wv.y};
                            }
                            if ((s_other >> 1) == chi2) {
                                const double2 wv = W[wb + 3 * s_other + c2];
                                uo = uo + uc * cx<double>{wv.x, wv.y};
                            }
                        }
                        const cx<double> gu = ph * uo;
                        out = dir == 0 ? us - gu : us + gu;
                        out = coef * out;
                    }
                    G[col][sc] = out;
                }
                __syncthreads();
                // entries: row = chi N + k, column col: sum over the spins of chi of conj(W_k(x)) G[col]
#pragma unroll
                for (int i = 0; i < MAXE; i++) {
                    const int e = threadIdx.x + 256 * i;
                    if (e >= ne) break;
                    const int col = e / nc, row = e - col * nc;
                    const int chi = row / N, k = row - chi * N;
                    cx<double> a = acc[i];
                    for (int sc = 6 * chi; sc < 6 * chi + 6; sc++) a = a + cmul_conj(Wx[k][sc], G[col][sc]);
                    acc[i] = a;
                }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < MAXE; i++) {
        const int e = threadIdx.x + 256 * i;
        if (e < ne) Yt[((long)cs * 9 + d) * ne + e] = make_double2(acc[i].re, acc[i].im);
    }
}

// ---------------------------------------------------------------------------
// restriction, prolongation, coarse operator
// ---------------------------------------------------------------------------
// out[cs][chi][k] = sum over the block's sites of parity p < np and the spins of chi of conj(W_k) f, for
// f = (f0, f1) internal fields of the two parities (f1 unused when np = 1).  Block (cs, kb): wave w handles
// vector k = 4 kb + w, its lanes stride over the contiguous run of W_k in chunks of 16 sites x 12 components
// (lane l takes components l, l + 64, l + 128 of each chunk: fixed (site offset, spin-colour) pairs, so the
// loop has no divisions).
template <class PW, class PF>
__global__ __launch_bounds__(256) void k_mg_restrict(MgDev m, const void* W, const void* f0, const void* f1, int np,
                                                      double2* out)
{
    const int kb = blockIdx.x % ((m.N + 3) / 4), cs = blockIdx.x / ((m.N + 3) / 4);
    const int lane = threadIdx.x & 63;
    const int k = 4 * kb + (threadIdx.x >> 6);
    if (k >= m.N) return;  // whole waves
    int dj[3], sc[3];
#pragma unroll
    for (int i = 0; i < 3; i++) {
        dj[i] = (lane + 64 * i) / 12;
        sc[i] = (lane + 64 * i) % 12;
    }
    double a[4] = {0.0, 0.0, 0.0, 0.0};  // (re, im) for chirality 0, then 1
    for (int p = 0; p < np; p++) {
        const void* f = p == 0 ? f0 : f1;
        const long wb = w_index(m, cs, k, p, 0);
        const int* sites = m.blk_sites + ((long)cs * 2 + p) * m.hb;
        for (int j0 = 0; j0 < m.hb; j0 += 16) {
#pragma unroll
            for (int i = 0; i < 3; i++) {
                const int j = j0 + dj[i];
                if (j < m.hb) {
                    const int site = sites[j];
                    const auto wk = PW::ld(W, wb + (long)j * 12 + sc[i]);
                    const auto fv = PF::ld(f, sp_idx(sc[i] / 3, site, sc[i] % 3, m.g.Vh));
                    const double wr = wk.re, wi = wk.im, fr = fv.re, fi = fv.im;
                    const int h = sc[i] < 6 ? 0 : 2;
                    a[h] += wr * fr + wi * fi;
                    a[h + 1] += wr * fi - wi * fr;
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 4; q++) a[q] = wave_sum(a[q]);
    if (lane == 0) {
        out[((long)cs * 2 + 0) * m.N + k] = make_double2(a[0], a[1]);
        out[((long)cs * 2 + 1) * m.N + k] = make_double2(a[2], a[3]);
    }
}

// f_p = scale * sum_k W_k e[chi][k] on the sites of parity p < np (scale = sqrt(*norm2) when norm2 is
// given, else 1); one block per coarse site, the block's coarse vector staged in LDS
template <class PW, class PE, class PF>
__global__ __launch_bounds__(256) void k_mg_prolong(MgDev m, const void* W, const void* e, const double* norm2,
                                                     void* f0, void* f1, int np)
{
    __shared__ cx<double> ec[2 * MG_MAX_N];
    const int cs = blockIdx.x;
    const double scale = norm2 ? sqrt(*norm2) : 1.0;
    for (int i = threadIdx.x; i < m.nc; i += 256) {
        const auto v = PE::ld(e, (long)cs * m.nc + i);
        ec[i] = {scale * (double)v.re, scale * (double)v.im};
    }
    __syncthreads();
    const int len = np * m.hb * 12;
    using T = typename PF::real;
    for (int el = threadIdx.x; el < len; el += 256) {
        const int p = el / (m.hb * 12), rem = el - p * m.hb * 12;
        const int j = rem / 12, sc = rem % 12;
        const int chi = sc < 6 ? 0 : 1;
        cx<double> acc = {0.0, 0.0};
        for (int k = 0; k < m.N; k++) {
            const auto wk = PW::ld(W, w_index(m, cs, k, p, j) + sc);
            acc = acc + cx<double>{(double)wk.re, (double)wk.im} * ec[chi * m.N + k];
        }
        const int site = m.blk_sites[((long)cs * 2 + p) * m.hb + j];
        PF::st(p == 0 ? f0 : f1, sp_idx(sc / 3, site, sc % 3, m.g.Vh), cx<T>{(T)acc.re, (T)acc.im});
    }
}

// out = D_c in, one block per coarse site: thread items (stencil entry d, row) form the partial sums over the
// columns of entry d (consecutive threads read consecutive rows of a column), which are then summed over d in
// a fixed order; red = RED_WDOT: partials of (w, out); RED_TS: partials of (out, y) and ||out||^2 (one
// partial per coarse site); nothing when *stop != 0 (the solve has finished)
// (PY: storage of the stencil, P: of the vectors)
template <class PY, class P, int RED>
__global__ __launch_bounds__(256) void k_mg_coarse_apply(MgDev m, const void* Yt, const void* in, void* out,
                                                          const void* y, double* partials, const int* stop)
{
    if (stop && *stop) return;
    using T = typename P::real;
    __shared__ cx<T> part[9][2 * MG_MAX_N];
    const int nc = m.nc, cs = blockIdx.x;
    const long ne = (long)nc * nc;
    for (int it = threadIdx.x; it < 9 * nc; it += 256) {
        const int d = it / nc, row = it - d * nc;
        const int nb = d == 0 ? cs : m.cnbr[(long)cs * 8 + (d - 1)];
        const long yb = ((long)cs * 9 + d) * ne + row;
        const long ib = (long)nb * nc;
        cx<T> acc = {T(0), T(0)};
        for (int col = 0; col < nc; col++) {
            const auto yv = PY::ld(Yt, yb + (long)col * nc);
            cmac(acc, cx<T>{(T)yv.re, (T)yv.im}, P::ld(in, ib + col));
        }
        part[d][row] = acc;
    }
    __syncthreads();
    const int row = threadIdx.x;
    const bool valid = row < nc;
    const long tid = (long)cs * nc + row;
    cx<T> acc = {T(0), T(0)};
    if (valid) {
        acc = part[0][row];
#pragma unroll
        for (int d = 1; d < 9; d++) acc = acc + part[d][row];
        P::st(out, tid, acc);
    }
    if constexpr (RED != RED_NONE) {
        double v[3] = {0.0, 0.0, 0.0};
        if (valid) {
            const cx<T> o = P::rt(acc);
            if constexpr (RED == RED_WDOT) {
                const cx<T> w = P::ld(y, tid);
                v[0] = (double)w.re * o.re + (double)w.im * o.im;
                v[1] = (double)w.re * o.im - (double)w.im * o.re;
            } else {
                const cx<T> yv = P::ld(y, tid);
                v[0] = (double)o.re * yv.re + (double)o.im * yv.im;
                v[1] = (double)o.re * yv.im - (double)o.im * yv.re;
                v[2] = (double)o.re * o.re + (double)o.im * o.im;
            }
        }
        block_sum_store<3>(v, partials + 3L * blockIdx.x);
    }
}

// [Vc][9][row][col] (natural) <-> Yt [Vc][9][col][row]; also an FP32 copy of Yt
__global__ void k_mg_transpose(const double2* __restrict__ in, double2* out, long nblk, int nc)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long ne = (long)nc * nc;
    if (e >= nblk * ne) return;
    const long blk = e / ne;
    const int r = (int)(e % ne) / nc, c = (int)(e % ne) % nc;
    out[blk * ne + (long)c * nc + r] = in[e];
}

// coarse solve set-up: scale = 1 / ||r_c|| (0 for a zero right-hand side), BiCGStab stops below tol^2
__global__ void k_mg_coarse_init(Scal* S, const double* norm2, double tol2, double* scale)
{
    const double n2 = *norm2;
    const bool zero = !(n2 > 0.0);
    *scale = zero ? 0.0 : 1.0 / sqrt(n2);
    S->stop_rr = zero ? 1.0 : tol2;
    S->iter = 0;
    S->flags = 0;
    S->fault_iter = 0;
    S->hist_len = 0;
    S->hist_norm = 1.0;
}

// minimal-residual step: partials of (w, r) and ||w||^2 (vectors in storage precision P)
template <class P>
__global__ __launch_bounds__(256) void k_mg_mr_dots(const void* w, const void* r, long n, double* partials)
{
    double v[3] = {0.0, 0.0, 0.0};
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long)gridDim.x * 256) {
        const auto a = P::ld(w, e), b = P::ld(r, e);
        v[0] += (double)a.re * b.re + (double)a.im * b.im;
        v[1] += (double)a.re * b.im - (double)a.im * b.re;
        v[2] += (double)a.re * a.re + (double)a.im * a.im;
    }
    block_sum_store<3>(v, partials + 3L * blockIdx.x);
}

// alpha = (w, r) / (w, w) from nb partials (every block sums them in the same order), z += alpha r (z in
// PZ), r -= alpha w (r, w in P)
template <class P, class PZ>
__global__ __launch_bounds__(256) void k_mg_mr_update(void* z, void* r, const void* w, long n, const double* partials,
                                                      int nb)
{
    __shared__ double tot[3];
    double v[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += 256)
        for (int k = 0; k < 3; k++) v[k] += partials[3L * b + k];
    block_sum_store<3>(v, tot);
    __syncthreads();
    const double ww = tot[2];
    const double ar = ww > 0.0 ? tot[0] / ww : 0.0, ai = ww > 0.0 ? tot[1] / ww : 0.0;
    using T = typename P::real;
    using TZ = typename PZ::real;
    const cx<T> al = {(T)ar, (T)ai};
    const cx<TZ> alz = {(TZ)ar, (TZ)ai};
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long)gridDim.x * 256) {
        const auto rv = P::ld(r, e), wv = P::ld(w, e);
        const auto zv = PZ::ld(z, e);
        PZ::st(z, e, zv + alz * cx<TZ>{(TZ)rv.re, (TZ)rv.im});
        P::st(r, e, rv - al * wv);
    }
}

}  // namespace qcdw

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
// Storage of the coarse stencil in the preconditioner's coarse solve (QCDW_MG_YPREC: 0 FP32, 1 BF16,
// 2 FP16) and the smoother's precision (QCDW_MG_SMOOTH_F64 = 1: FP64, else the operator's inner one).
#ifndef QCDW_MG_YPREC
#define QCDW_MG_YPREC 1
#endif
#ifndef QCDW_MG_SMOOTH_F64
#define QCDW_MG_SMOOTH_F64 0
#endif
namespace qcdw {
using MG_YP = std::conditional_t<QCDW_MG_YPREC == 0, P32, std::conditional_t<QCDW_MG_YPREC == 1, PBF16, PF16>>;
constexpr int MG_YPREC = QCDW_MG_YPREC == 0 ? F32 : QCDW_MG_YPREC == 1 ? BF16 : F16;
}  // namespace qcdw

struct qcdw_mg {
    qcdw_op* op = nullptr;  // operator the set-up and the coarse operator were made with
    qcdw_ctx* ctx = nullptr;
    qcdw_mg_params prm{};
    MgDev md{};
    PoolBuf blk_sites, fine_loc, cnbr;
    PoolBuf W64, W32;        // block vectors
    PoolBuf Yt64, Ylo;       // coarse stencil, column-major blocks: FP64 (API), MG_YP (the preconditioner's solve)
    PoolBuf rc, ec, ec64;    // coarse right-hand side (FP64), solution (FP32), FP64 scratch
    PoolBuf ck[6];           // coarse BiCGStab vectors r, r0, p, v, s, t (FP32)
    PoolBuf scal, dpart, dpart2, dnorm, dscale;
    PoolBuf t64, r64, w64, tmpo;  // fine even-site FP64 scratch of the preconditioner
    PoolBuf rlo, wlo, zlo, tmplo;  // smoother vectors in the operator's inner precision (z accumulated in FP32)
    long n_c = 0;                  // complex entries of a coarse vector
    int nb_apply = 0, nb_blas = 0, nb_fine = 0;
};

namespace {

using qcdw::MgDev;

qcdw_status mg_tables(qcdw_mg* mg)
{
    qcdw_ctx* ctx = mg->ctx;
    MgDev& m = mg->md;
    const Geom& g = m.g;
    std::vector<int> blk((size_t)m.Vc * 2 * m.hb, -1), loc(2L * g.Vh), nbr((size_t)m.Vc * 8);
    std::vector<int> fill((size_t)m.Vc * 2, 0);
    for (int p = 0; p < 2; p++)
        for (int i = 0; i < g.Vh; i++) {
            const int xh = i % g.Lxh;
            int r = i / g.Lxh;
            const int y = r % g.Ly;
            r /= g.Ly;
            const int z = r % g.Lz, t = r / g.Lz;
            const int x = 2 * xh + ((p + y + z + t) & 1);
            const int cx = x / m.b[0], cy = y / m.b[1], cz = z / m.b[2], ct = t / m.b[3];
            const int cs = ((ct * m.Lc[2] + cz) * m.Lc[1] + cy) * m.Lc[0] + cx;
            int& f = fill[(size_t)cs * 2 + p];
            if (f >= m.hb) return fail(ctx, QCDW_EINVAL, "block %d has more than %d sites of parity %d", cs, m.hb, p);
            blk[((size_t)cs * 2 + p) * m.hb + f] = i;
            loc[(size_t)p * g.Vh + i] = cs * m.hb + f;
            f++;
        }
    for (int cs = 0; cs < m.Vc; cs++) {
        int c[4] = {cs % m.Lc[0], (cs / m.Lc[0]) % m.Lc[1], (cs / (m.Lc[0] * m.Lc[1])) % m.Lc[2],
                    cs / (m.Lc[0] * m.Lc[1] * m.Lc[2])};
        for (int mu = 0; mu < 4; mu++)
            for (int dir = 0; dir < 2; dir++) {
                int q[4] = {c[0], c[1], c[2], c[3]};
                q[mu] = (q[mu] + (dir == 0 ? 1 : m.Lc[mu] - 1)) % m.Lc[mu];
                nbr[(size_t)cs * 8 + 2 * mu + dir] = ((q[3] * m.Lc[2] + q[2]) * m.Lc[1] + q[1]) * m.Lc[0] + q[0];
            }
    }
    HIPCHK(ctx, mg->blk_sites.alloc(blk.size() * sizeof(int)));
    HIPCHK(ctx, mg->fine_loc.alloc(loc.size() * sizeof(int)));
    HIPCHK(ctx, mg->cnbr.alloc(nbr.size() * sizeof(int)));
    hipStream_t s = ctx->stream;
    HIPCHK(ctx, hipMemcpyAsync(mg->blk_sites.p, blk.data(), blk.size() * sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(ctx, hipMemcpyAsync(mg->fine_loc.p, loc.data(), loc.size() * sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(ctx, hipMemcpyAsync(mg->cnbr.p, nbr.data(), nbr.size() * sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(ctx, hipStreamSynchronize(s));  // host vectors go out of scope
    m.blk_sites = (const int*)mg->blk_sites.p;
    m.fine_loc = (const int*)mg->fine_loc.p;
    m.cnbr = (const int*)mg->cnbr.p;
    return QCDW_OK;
}

inline dim3 g256(long n) { return dim3((unsigned)((n + 255) / 256)); }

// coarse stencil of the operator op from the FP64 block vectors (and its FP32 copy)
qcdw_status mg_build_coarse(qcdw_mg* mg, qcdw_op* op)
{
    qcdw_ctx* ctx = mg->ctx;
    hipStream_t s = ctx->stream;
    const MgDev& m = mg->md;
    const long nst = (long)m.Vc * 9 * m.nc * m.nc;
    HIPCHK(ctx, mg->Yt64.alloc(nst * 16));
    HIPCHK(ctx, mg->Ylo.alloc(nst * MG_YP::cbytes));
    const PrecView v = view(op, F64);
    if (v.recon == 12)
        hipLaunchKernelGGL(k_mg_coarse_build<6>, dim3(m.Vc * 9), dim3(256), 0, s, m, (const double2*)mg->W64.p,
                           v.gauge, (const double*)op->A64[0].p, (const double*)op->A64[1].p, op->kappa,
                           (double2*)mg->Yt64.p);
    else
        hipLaunchKernelGGL(k_mg_coarse_build<9>, dim3(m.Vc * 9), dim3(256), 0, s, m, (const double2*)mg->W64.p,
                           v.gauge, (const double*)op->A64[0].p, (const double*)op->A64[1].p, op->kappa,
                           (double2*)mg->Yt64.p);
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, launch_convert(s, F64, MG_YPREC, mg->Yt64.p, mg->Ylo.p, nst, 1.0));
    return QCDW_OK;
}

template <class PY, class P, int RED>
hipError_t coarse_apply(hipStream_t s, const qcdw_mg* mg, const void* Yt, const void* in, void* out, const void* y,
                        double* partials, const int* stop)
{
    hipLaunchKernelGGL((k_mg_coarse_apply<PY, P, RED>), dim3(mg->nb_apply), dim3(256), 0, s, mg->md, Yt, in, out, y,
                       partials, stop);
    return hipGetLastError();
}

// Preconditioner of M_hat on FP64 even-site internal fields: z = K(v)
qcdw_status mg_precondition(qcdw_mg* mg, qcdw_op* op, const void* v, void* z)
{
    qcdw_ctx* ctx = mg->ctx;
    hipStream_t s = ctx->stream;
    const MgDev& m = mg->md;
    const long n = 12L * m.g.Vh;
    // coarse right-hand side P^+ (A_ee v) on the even sites
    HIPCHK(ctx, launch_clov_apply_internal(s, F64, m.g, op->A64[0].p, v, mg->t64.p));
    hipLaunchKernelGGL((k_mg_restrict<P32, P64>), dim3(m.Vc * ((m.N + 3) / 4)), dim3(256), 0, s, m, mg->W32.p,
                       mg->t64.p, nullptr, 1,
                       (double2*)mg->rc.p);
    HIPCHK(ctx, hipGetLastError());
    // coarse BiCGStab on the normalised right-hand side, FP32 vectors, scalars on the device
    Scal* S = (Scal*)mg->scal.p;
    double* dn2 = (double*)mg->dnorm.p;
    HIPCHK(ctx, launch_norm2(s, F64, mg->rc.p, mg->n_c, (double*)mg->dpart2.p, dn2));
    hipLaunchKernelGGL(k_mg_coarse_init, dim3(1), dim3(1), 0, s, S, dn2, mg->prm.coarse_tol * mg->prm.coarse_tol,
                       (double*)mg->dscale.p);
    void *r = mg->ck[0].p, *r0 = mg->ck[1].p, *p = mg->ck[2].p, *vv = mg->ck[3].p, *sv = mg->ck[4].p,
         *t = mg->ck[5].p;
    double* dpart = (double*)mg->dpart.p;
    double* dpart2 = (double*)mg->dpart2.p;
    HIPCHK(ctx, launch_cycle_start(s, F32, mg->rc.p, r, r0, p, mg->ec.p, mg->n_c, (const double*)mg->dscale.p, S,
                                   dpart2, 1, nullptr, 0, false));
    for (int it = 0; it < mg->prm.coarse_iters; it++) {
        HIPCHK(ctx, (coarse_apply<MG_YP, P32, RED_WDOT>(s, mg, mg->Ylo.p, p, vv, r0, dpart, &S->flags)));
        HIPCHK(ctx, launch_fin_alpha(s, S, dpart, mg->nb_apply, 1, nullptr));
        HIPCHK(ctx, launch_bicg_s(s, F32, sv, r, vv, mg->n_c, S, 1, nullptr, 0, nullptr, 0, nullptr));
        HIPCHK(ctx, (coarse_apply<MG_YP, P32, RED_TS>(s, mg, mg->Ylo.p, sv, t, sv, dpart, &S->flags)));
        HIPCHK(ctx, launch_fin_omega(s, S, dpart, mg->nb_apply, 1, nullptr));
        HIPCHK(ctx, launch_bicg_xr(s, F32, F32, mg->ec.p, p, sv, r, t, r0, mg->n_c, S, dpart2, 1, nullptr, 0, nullptr,
                                   0, nullptr));
        HIPCHK(ctx, launch_fin_beta(s, S, dpart2, mg->nb_blas, nullptr, 1));
        HIPCHK(ctx, launch_bicg_p(s, F32, p, r, vv, mg->n_c, S, 1, nullptr, 0, nullptr, 0, nullptr));
    }
    // z = P e (even sites), undoing the normalisation
    hipLaunchKernelGGL((k_mg_prolong<P32, P32, P64>), dim3(m.Vc), dim3(256), 0, s, m, mg->W32.p, mg->ec.p, dn2, z,
                       nullptr, 1);
    HIPCHK(ctx, hipGetLastError());
    // minimal-residual smoothing on M_hat in the operator's inner precision: r = v - M_hat z, then
    // z_s += alpha r, r -= alpha w with w = M_hat r (alpha = (w, r) / (w, w)), and finally z += z_s
    if (mg->prm.smooth_iters > 0) {
        const int lp = QCDW_MG_SMOOTH_F64 ? (int)F64 : op->inner;
        const PrecView vl = view(op, lp);
        HIPCHK(ctx, launch_convert(s, F64, lp, z, mg->zlo.p, n, 1.0));          // z in the inner precision
        HIPCHK(ctx, matpc(s, op, vl, mg->zlo.p, mg->wlo.p, mg->tmplo.p, RED_NONE, nullptr, nullptr, nullptr));
        HIPCHK(ctx, launch_convert(s, F64, lp, v, mg->rlo.p, n, 1.0));
        HIPCHK(ctx, launch_convert(s, lp, F64, mg->wlo.p, mg->w64.p, n, 1.0));
        HIPCHK(ctx, launch_xmy_norm2(s, F64, F64, v, mg->w64.p, mg->r64.p, n, dpart2, dn2));
        HIPCHK(ctx, launch_convert(s, F64, lp, mg->r64.p, mg->rlo.p, n, 1.0));  // r = v - M_hat z
        HIPCHK(ctx, launch_convert(s, F64, F32, mg->r64.p, mg->zlo.p, n, 0.0));  // z_s = 0 (FP32)
        for (int it = 0; it < mg->prm.smooth_iters; it++) {
            HIPCHK(ctx, matpc(s, op, vl, mg->rlo.p, mg->wlo.p, mg->tmplo.p, RED_NONE, nullptr, nullptr, nullptr));
            switch (lp) {
#define QCDW_MR_CASE(PREC, P)                                                                                      \
    case PREC:                                                                                                     \
        hipLaunchKernelGGL(k_mg_mr_dots<P>, dim3(mg->nb_fine), dim3(256), 0, s, mg->wlo.p, mg->rlo.p, n, dpart2);   \
        hipLaunchKernelGGL((k_mg_mr_update<P, P32>), dim3(mg->nb_fine), dim3(256), 0, s, mg->zlo.p, mg->rlo.p,       \
                           mg->wlo.p, n, (const double*)dpart2, mg->nb_fine);                                      \
        break;
                QCDW_MR_CASE(F64, P64)
                QCDW_MR_CASE(F32, P32)
                QCDW_MR_CASE(BF16, PBF16)
                QCDW_MR_CASE(F16, PF16)
#undef QCDW_MR_CASE
            }
            HIPCHK(ctx, hipGetLastError());
        }
        HIPCHK(ctx, launch_axpy_hi(s, F32, 1.0, nullptr, mg->zlo.p, z, n));  // z += z_s
    }
    return QCDW_OK;
}

}  // namespace

extern "C" void qcdw_mg_params_default(qcdw_mg_params* p)
{
    if (!p) return;
    p->block[0] = p->block[1] = p->block[2] = p->block[3] = 4;
    p->nvec = 12;
    p->setup_iters = 100;
    p->seed = 1234;
    p->coarse_iters = 24;
    p->coarse_tol = 0.1;
    p->smooth_iters = 2;
}

extern "C" qcdw_status qcdw_mg_create(qcdw_op* op, const qcdw_mg_params* params, const void* vecs, qcdw_mg** out)
{
    if (!op || !out) return QCDW_EINVAL;
    *out = nullptr;
    qcdw_ctx* ctx = op->ctx;
    DeviceGuard dg(ctx->device);
    qcdw_mg_params prm;
    if (params) prm = *params;
    else qcdw_mg_params_default(&prm);
    const Geom& g = op->g;
    const int L[4] = {g.Lx, g.Ly, g.Lz, g.Lt};
    long bvol = 1;
    for (int mu = 0; mu < 4; mu++) {
        if (prm.block[mu] < 1 || L[mu] % prm.block[mu])
            return fail(ctx, QCDW_EINVAL, "block extent %d does not divide the lattice extent %d (direction %d)",
                        prm.block[mu], L[mu], mu);
        bvol *= prm.block[mu];
    }
    if (bvol % 2) return fail(ctx, QCDW_EINVAL, "the block volume must be even (some block extent even)");
    if (prm.nvec < 1 || prm.nvec > MG_MAX_N || prm.nvec > 6 * bvol)
        return fail(ctx, QCDW_EINVAL, "nvec = %d must lie in [1, %d] and be at most 6 |block|", prm.nvec, MG_MAX_N);
    if (prm.coarse_iters < 0 || prm.smooth_iters < 0 || !(prm.coarse_tol > 0.0) || prm.setup_iters < 1)
        return fail(ctx, QCDW_EINVAL, "coarse_iters, smooth_iters >= 0, setup_iters >= 1 and coarse_tol > 0 required");
    if (vecs) CHK(check_dev(ctx, vecs, "vecs"));
    auto mg = std::make_unique<qcdw_mg>();
    mg->op = op;
    mg->ctx = ctx;
    mg->prm = prm;
    MgDev& m = mg->md;
    m.g = g;
    for (int mu = 0; mu < 4; mu++) {
        m.b[mu] = prm.block[mu];
        m.Lc[mu] = L[mu] / prm.block[mu];
    }
    m.Vc = m.Lc[0] * m.Lc[1] * m.Lc[2] * m.Lc[3];
    m.hb = (int)(bvol / 2);
    m.N = prm.nvec;
    m.nc = 2 * prm.nvec;
    CHK(mg_tables(mg.get()));
    hipStream_t s = ctx->stream;
    const long nw = (long)m.Vc * m.N * 2 * m.hb * 12;  // = N * 12 V
    HIPCHK(ctx, mg->W64.alloc(nw * 16));
    HIPCHK(ctx, mg->W32.alloc(nw * 8));
    // near-null vectors: given, or x_k ~ M^-1 eta_k (setup_iters BiCGStab iterations from zero on a Gaussian
    // eta_k, so the slowly converging low modes dominate x_k)
    if (vecs) {
        hipLaunchKernelGGL(k_mg_gather, g256(nw), dim3(256), 0, s, m, (const double2*)vecs, (double2*)mg->W64.p);
        HIPCHK(ctx, hipGetLastError());
    } else {
        // relaxation of M x = 0 from a Gaussian x_0 = eta: BiCGStab on M y = M eta from y = 0 for setup_iters
        // iterations leaves the error x = eta - y = p(M) eta, p the method's residual polynomial (p(0) = 1),
        // in which the modes of small |lambda| survive and the rest are damped
        const long nf = 24L * g.Vh;  // complex entries of one full field
        const size_t vb = 12UL * g.Vh * 16;
        PoolBuf eta, rhs, xs, tmp;
        HIPCHK(ctx, eta.alloc(nf * 16));
        HIPCHK(ctx, rhs.alloc(nf * 16));
        HIPCHK(ctx, tmp.alloc(3 * vb));
        HIPCHK(ctx, xs.alloc((size_t)m.N * nf * 16));
        qcdw_solver_params sp;
        qcdw_solver_params_default(&sp);
        sp.tol = 1e-14;
        sp.maxiter = prm.setup_iters;
        sp.inner = (qcdw_prec)op->inner;
        sp.delta = 1e-2;
        const PrecView v64 = view(op, F64);
        void* in[2] = {tmp.p, (char*)tmp.p + vb};
        void* res = (char*)tmp.p + 2 * vb;
        for (int k = 0; k < m.N; k++) {
            HIPCHK(ctx, launch_gaussian(s, eta.p, nf, prm.seed, (uint64_t)k));
            for (int p = 0; p < 2; p++) HIPCHK(ctx, launch_pack_spinor(s, F64, g, eta.p, p, in[p], 1.0));
            for (int p = 0; p < 2; p++) {  // rhs_p = A_p eta_p - kappa H eta_{1-p}
                HopArgs a = hop_args(g, p);
                a.psi = in[1 - p];
                a.out = res;
                a.gauge = v64.gauge;
                a.clov = op->A64[p].p;
                a.y = in[p];
                a.a = op->kappa;
                HIPCHK(ctx, launch_hop(s, F64, v64.recon, EPI_XPAY_CLOVY, RED_NONE, a));
                HIPCHK(ctx, launch_unpack_spinor(s, F64, g, res, p, rhs.p, 1.0));
            }
            void* xk = (char*)xs.p + (size_t)k * nf * 16;
            HIPCHK(ctx, hipMemsetAsync(xk, 0, nf * 16, s));
            qcdw_solve_info si{};
            const qcdw_status st = qcdw_invert(op, rhs.p, xk, &sp, &si);
            if (st != QCDW_OK && st != QCDW_ENOCONV) return st;
            hipLaunchKernelGGL(k_mg_sub, g256(nf), dim3(256), 0, s, (const double2*)eta.p, (const double2*)xk,
                               (double2*)xk, nf);
            HIPCHK(ctx, hipGetLastError());
        }
        hipLaunchKernelGGL(k_mg_gather, g256(nw), dim3(256), 0, s, m, (const double2*)xs.p, (double2*)mg->W64.p);
        HIPCHK(ctx, hipGetLastError());
        HIPCHK(ctx, hipStreamSynchronize(s));  // eta and xs go back to the block cache
    }
    HIPCHK(ctx, hipMemsetAsync(ctx->dev_int, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_mg_orth, dim3(2 * m.Vc), dim3(256), 0, s, m, (double2*)mg->W64.p, ctx->dev_int);
    HIPCHK(ctx, hipGetLastError());
    int bad = 0;
    HIPCHK(ctx, hipMemcpyAsync(ctx->host_d, ctx->dev_int, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    memcpy(&bad, ctx->host_d, sizeof(int));
    if (bad) return fail(ctx, QCDW_EINVAL, "near-null vectors are linearly dependent on %d aggregates", bad);
    HIPCHK(ctx, launch_convert(s, F64, F32, mg->W64.p, mg->W32.p, nw, 1.0));
    CHK(mg_build_coarse(mg.get(), op));
    // solve workspace
    mg->n_c = (long)m.Vc * m.nc;
    mg->nb_apply = m.Vc;  // one block (and one reduction partial) per coarse site
    mg->nb_blas = blas_blocks(mg->n_c);
    const long nfe = 12L * g.Vh;
    mg->nb_fine = blas_blocks(nfe);
    HIPCHK(ctx, mg->rc.alloc(mg->n_c * 16));
    HIPCHK(ctx, mg->ec64.alloc(mg->n_c * 16));
    HIPCHK(ctx, mg->ec.alloc(mg->n_c * 8));
    for (auto& b : mg->ck) HIPCHK(ctx, b.alloc(mg->n_c * 8));
    HIPCHK(ctx, mg->scal.alloc(sizeof(Scal)));
    HIPCHK(ctx, mg->dpart.alloc(3L * std::max(mg->nb_apply, 1) * sizeof(double)));
    HIPCHK(ctx, mg->dpart2.alloc(3L * std::max<long>(std::max(mg->nb_blas, mg->nb_fine), 4096) * sizeof(double)));
    HIPCHK(ctx, mg->dnorm.alloc(64));
    HIPCHK(ctx, mg->dscale.alloc(64));
    HIPCHK(ctx, mg->t64.alloc(nfe * 16));
    HIPCHK(ctx, mg->r64.alloc(nfe * 16));
    HIPCHK(ctx, mg->w64.alloc(nfe * 16));
    HIPCHK(ctx, mg->tmpo.alloc(nfe * 16));
    HIPCHK(ctx, mg->rlo.alloc(nfe * 16));
    HIPCHK(ctx, mg->wlo.alloc(nfe * 16));
    HIPCHK(ctx, mg->zlo.alloc(nfe * 16));
    HIPCHK(ctx, mg->tmplo.alloc(nfe * 16));
    HIPCHK(ctx, hipStreamSynchronize(s));
    *out = mg.release();
    return QCDW_OK;
}

extern "C" void qcdw_mg_destroy(qcdw_mg* mg)
{
    if (!mg) return;
    DeviceGuard dg(mg->ctx->device);
    (void)hipStreamSynchronize(mg->ctx->stream);
    delete mg;
}

extern "C" qcdw_status qcdw_mg_vectors(qcdw_mg* mg, void* vecs)
{
    if (!mg) return QCDW_EINVAL;
    qcdw_ctx* ctx = mg->ctx;
    DeviceGuard dg(ctx->device);
    CHK(check_dev(ctx, vecs, "vecs"));
    const MgDev& m = mg->md;
    const long nw = (long)m.Vc * m.N * 2 * m.hb * 12;
    hipLaunchKernelGGL(k_mg_scatter, g256(nw), dim3(256), 0, ctx->stream, m, (const double2*)mg->W64.p, (double2*)vecs);
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return QCDW_OK;
}

extern "C" qcdw_status qcdw_mg_restrict(qcdw_mg* mg, const void* fine, void* coarse)
{
    if (!mg) return QCDW_EINVAL;
    qcdw_ctx* ctx = mg->ctx;
    DeviceGuard dg(ctx->device);
    CHK(check_dev(ctx, fine, "fine"));
    CHK(check_dev(ctx, coarse, "coarse"));
    const MgDev& m = mg->md;
    hipStream_t s = ctx->stream;
    const long vb = 12L * m.g.Vh * 16;
    PoolBuf f;
    HIPCHK(ctx, f.alloc(2 * vb));
    HIPCHK(ctx, launch_pack_spinor(s, F64, m.g, fine, 0, f.p, 1.0));
    HIPCHK(ctx, launch_pack_spinor(s, F64, m.g, fine, 1, (char*)f.p + vb, 1.0));
    hipLaunchKernelGGL((k_mg_restrict<P64, P64>), dim3(m.Vc * ((m.N + 3) / 4)), dim3(256), 0, s, m, mg->W64.p, f.p,
                       (const char*)f.p + vb, 2, (double2*)coarse);
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, hipStreamSynchronize(s));
    return QCDW_OK;
}

extern "C" qcdw_status qcdw_mg_prolong(qcdw_mg* mg, const void* coarse, void* fine)
{
    if (!mg) return QCDW_EINVAL;
    qcdw_ctx* ctx = mg->ctx;
    DeviceGuard dg(ctx->device);
    CHK(check_dev(ctx, fine, "fine"));
    CHK(check_dev(ctx, coarse, "coarse"));
    const MgDev& m = mg->md;
    hipStream_t s = ctx->stream;
    const long vb = 12L * m.g.Vh * 16;
    PoolBuf f;
    HIPCHK(ctx, f.alloc(2 * vb));
    hipLaunchKernelGGL((k_mg_prolong<P64, P64, P64>), dim3(m.Vc), dim3(256), 0, s, m, mg->W64.p, coarse, nullptr,
                       f.p, (char*)f.p + vb, 2);
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, launch_unpack_spinor(s, F64, m.g, f.p, 0, fine, 1.0));
    HIPCHK(ctx, launch_unpack_spinor(s, F64, m.g, (const char*)f.p + vb, 1, fine, 1.0));
    HIPCHK(ctx, hipStreamSynchronize(s));
    return QCDW_OK;
}

extern "C" qcdw_status qcdw_mg_coarse_apply(qcdw_mg* mg, const void* in, void* out)
{
    if (!mg) return QCDW_EINVAL;
    qcdw_ctx* ctx = mg->ctx;
    DeviceGuard dg(ctx->device);
    CHK(check_dev(ctx, in, "in"));
    CHK(check_dev(ctx, out, "out"));
    if (in == out) return fail(ctx, QCDW_EINVAL, "out must not alias in");
    HIPCHK(ctx, (coarse_apply<P64, P64, RED_NONE>(ctx->stream, mg, mg->Yt64.p, in, out, nullptr, nullptr, nullptr)));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return QCDW_OK;
}

extern "C" qcdw_status qcdw_mg_coarse_op(qcdw_mg* mg, void* stencil)
{
    if (!mg) return QCDW_EINVAL;
    qcdw_ctx* ctx = mg->ctx;
    DeviceGuard dg(ctx->device);
    CHK(check_dev(ctx, stencil, "stencil"));
    const MgDev& m = mg->md;
    const long nblk = (long)m.Vc * 9;
    // Yt is column-major per block; the transpose of a column-major block is its row-major form
    hipLaunchKernelGGL(k_mg_transpose, g256(nblk * m.nc * m.nc), dim3(256), 0, ctx->stream, (const double2*)mg->Yt64.p,
                       (double2*)stencil, nblk, m.nc);
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return QCDW_OK;
}

extern "C" qcdw_status qcdw_mg_info(const qcdw_mg* mg, int* coarse_dims, int* nvec)
{
    if (!mg || !coarse_dims || !nvec) return QCDW_EINVAL;
    for (int mu = 0; mu < 4; mu++) coarse_dims[mu] = mg->md.Lc[mu];
    *nvec = mg->md.N;
    return QCDW_OK;
}

extern "C" qcdw_status qcdw_invert_mg(qcdw_op* op, qcdw_mg* mg, const void* b, void* x,
                                     const qcdw_solver_params* params, qcdw_solve_info* info)
{
    if (!op || !mg) return QCDW_EINVAL;
    const Geom& g = op->g, &h = mg->md.g;
    if (mg->ctx != op->ctx || g.Lx != h.Lx || g.Ly != h.Ly || g.Lz != h.Lz || g.Lt != h.Lt)
        return fail(op->ctx, QCDW_EINVAL, "the multigrid set-up belongs to another context or lattice");
    const Precond pmg = [mg, op](const void* v, void* z) { return mg_precondition(mg, op, v, z); };
    return fgmres_run(op, &pmg, b, x, params, info);
}
