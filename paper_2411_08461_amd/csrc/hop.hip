// Parity hop kernel of the Wilson-clover operator with fused epilogues.
//
// Computes on the sites of one parity (paper, Sec. III.B, Eq. "clover", the
// Wilson hopping term written out):
//   (H psi)(x) = sum_mu (1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^+ psi(x-mu)
// with periodic wrap computed in the kernel and the time boundary sign t_bc.
//
// Work split: four lanes per site.  Lane q = 2 gq + k handles directions
// mu = 2 gq and 2 gq + 1 (forward and backward), and only row k of the
// half-spinor that (1 -/+ g_mu) projects onto.  In the DeGrand-Rossi basis the
// projection is  h_k = psi_k + c psi_l  with a unit coefficient c and
// l = 3 - k (mu = x, y) or 2 + k (mu = z, t); the projected product W h_k
// adds to spin k and conj(c) W h_k to spin l.  So every lane reads just two
// spins (6 complex) of each neighbour plus the link, and owns partial sums of
// two output spins; one in-quad shuffle gives lane q the finished spin q.
// That keeps register use low and gives 4 Vh threads per launch.
#include <hip/hip_ext.h>

#include "internal.h"

#ifndef QCDW_HOP_PREFETCH
#define QCDW_HOP_PREFETCH 0
#endif
// 1: links and clover entries (read once per launch) are loaded non-temporally, so the
// neighbour spinors, which are re-read by the tiles of adjacent t-slices, stay in L2
#ifndef QCDW_HOP_NT
#define QCDW_HOP_NT 0
#endif
#ifndef QCDW_HOP_WAVES_PER_EU
#define QCDW_HOP_WAVES_PER_EU 0
#endif
#if QCDW_HOP_WAVES_PER_EU > 0
#define QCDW_HOP_ATTR __attribute__((amdgpu_waves_per_eu(QCDW_HOP_WAVES_PER_EU, QCDW_HOP_WAVES_PER_EU)))
#else
#define QCDW_HOP_ATTR
#endif

namespace qcdw {

template <class P, int R>
__device__ __forceinline__ void load_link(const void* gauge, long off, cx<typename P::real> (&u)[9])
{
    if constexpr (R == 9) {
#pragma unroll
        for (int e = 0; e < 9; e++) u[e] = QCDW_HOP_NT ? P::ldn(gauge, off + e) : P::ld(gauge, off + e);
    } else {
#pragma unroll
        for (int e = 0; e < 6; e++) u[e] = QCDW_HOP_NT ? P::ldn(gauge, off + e) : P::ld(gauge, off + e);
        // third row of an SU(3) matrix: complex conjugate of row0 x row1
        u[6] = conj(u[1] * u[5] - u[2] * u[4]);
        u[7] = conj(u[2] * u[3] - u[0] * u[5]);
        u[8] = conj(u[0] * u[4] - u[1] * u[3]);
    }
}

// Rows 3h..3h+2 of a Hermitian 6x6 block times the 6-vector (own | other),
// own = the 3 entries of this lane's spin.  `win` holds the lane's 27-real
// window of the reordered packing:
//   [d0 d1 d2 | L10 L20 L21 | L30 L31 L32 L40 L41 L42 L50 L51 L52 | d3 d4 d5 | L43 L53 L54]
//   half 0 reads entries 0..26, half 1 reads entries 9..35.
template <typename T>
__device__ __forceinline__ void herm_rows(const T (&win)[27], int h, const cx<T> (&vo)[3], const cx<T> (&vx)[3],
                                          cx<T> (&out)[3])
{
    T d[3], lo[6], Xr[9], Xi[9];
#pragma unroll
    for (int i = 0; i < 3; i++) d[i] = h ? win[18 + i] : win[i];
#pragma unroll
    for (int i = 0; i < 6; i++) lo[i] = h ? win[21 + i] : win[3 + i];
#pragma unroll
    for (int m = 0; m < 9; m++) {
        Xr[m] = h ? win[2 * m] : win[9 + 2 * m];
        Xi[m] = h ? win[2 * m + 1] : win[10 + 2 * m];
    }
    const cx<T> l10 = {lo[0], lo[1]}, l20 = {lo[2], lo[3]}, l21 = {lo[4], lo[5]};
    cx<T> own[3][3];
    own[0][0] = {d[0], T(0)};
    own[1][1] = {d[1], T(0)};
    own[2][2] = {d[2], T(0)};
    own[1][0] = l10;
    own[2][0] = l20;
    own[2][1] = l21;
    own[0][1] = conj(l10);
    own[0][2] = conj(l20);
    own[1][2] = conj(l21);
#pragma unroll
    for (int a = 0; a < 3; a++) {
        cx<T> s = {T(0), T(0)};
#pragma unroll
        for (int b = 0; b < 3; b++) s = s + own[a][b] * vo[b];
#pragma unroll
        for (int b = 0; b < 3; b++) {
            // cross block: rows of this half, columns of the other half
            cx<T> cb = h ? cx<T>{Xr[3 * a + b], Xi[3 * a + b]} : cx<T>{Xr[3 * b + a], -Xi[3 * b + a]};
            s = s + cb * vx[b];
        }
        out[a] = s;
    }
}

template <class P>
__device__ __forceinline__ void load_window(const void* clov, int site, int q, typename P::real (&win)[27])
{
    const long base = ((long)site * 2 + (q >> 1)) * 36 + 9 * (q & 1);
#pragma unroll
    for (int e = 0; e < 27; e++) win[e] = QCDW_HOP_NT ? P::ldrn(clov, base + e) : P::ldr(clov, base + e);
}

template <typename T>
__device__ __forceinline__ cx<T> shfl_cx(cx<T> v, int src)
{
    return {__shfl(v.re, src, 64), __shfl(v.im, src, 64)};
}
template <typename T>
__device__ __forceinline__ cx<T> shfl_xor_cx(cx<T> v, int m)
{
    return {__shfl_xor(v.re, m, 64), __shfl_xor(v.im, m, 64)};
}

// One 64-site tile of the hop with its epilogue; `part` receives the tile's
// reduction partials (RED != RED_NONE).  All 256 threads of the block call it.
template <class P, int R, int EPI, int RED>
__device__ __forceinline__ void hop_tile(const HopArgs& a, int tile, double* part)
{
    using T = typename P::real;
    const Geom g = a.g;
    const int q = threadIdx.x & 3;
    const int site = tile * HOP_SITES_PER_BLOCK + (threadIdx.x >> 2);
    const bool valid = site < g.Vh;
    const int gq = q >> 1, k = q & 1;
    const int p = a.parity;
    const long Vh = g.Vh;

    cx<T> acc_u[3], acc_l[3];
#pragma unroll
    for (int c = 0; c < 3; c++) acc_u[c] = acc_l[c] = {T(0), T(0)};

    if (valid) {
        int x, y, z, t;
        site_coords(g, site, p, x, y, z, t);
        const int xh = site % g.Lxh;
        const int su = k, sl = gq == 0 ? 3 - k : 2 + k;
        const int Sy = g.Lxh, Sz = g.Lxh * g.Ly, St = g.Lxh * g.Ly * g.Lz;
        // the four hops of this lane: h = 2 j + dir, mu = 2 gq + j, dir 0 forward / 1 backward
        int nbh[4];
        long loff[4];
        T cre[4], cim[4], fsg[4];
#pragma unroll
        for (int j = 0; j < 2; j++) {
            const int mu = 2 * gq + j;
            int fwd, bwd;
            bool fcross = false, bcross = false;
            T c_re, c_im;  // projection coefficient of the forward hop
            if (j == 0) {
                if (gq == 0) {  // x: the neighbour lies in the same row of the other parity
                    const int row = site - xh;
                    const int xp = (x + 1 == g.Lx) ? 0 : x + 1;
                    const int xm = (x == 0) ? g.Lx - 1 : x - 1;
                    fwd = row + (xp >> 1);
                    bwd = row + (xm >> 1);
                    c_re = T(0);
                    c_im = T(-1);
                } else {  // z
                    fwd = (z + 1 == g.Lz) ? site - (g.Lz - 1) * Sz : site + Sz;
                    bwd = (z == 0) ? site + (g.Lz - 1) * Sz : site - Sz;
                    c_re = T(0);
                    c_im = k == 0 ? T(-1) : T(1);
                }
            } else {
                if (gq == 0) {  // y
                    fwd = (y + 1 == g.Ly) ? site - (g.Ly - 1) * Sy : site + Sy;
                    bwd = (y == 0) ? site + (g.Ly - 1) * Sy : site - Sy;
                    c_re = k == 0 ? T(1) : T(-1);
                    c_im = T(0);
                } else {  // t
                    fwd = (t + 1 == g.Lt) ? site - (g.Lt - 1) * St : site + St;
                    bwd = (t == 0) ? site + (g.Lt - 1) * St : site - St;
                    fcross = (t + 1 == g.Lt);
                    bcross = (t == 0);
                    c_re = T(-1);
                    c_im = T(0);
                }
            }
            // forward: U_mu(x) psi(x+mu) with (1 - g_mu); backward: U_mu(x-mu)^+ psi(x-mu)
            // with (1 + g_mu), which flips the projection coefficient
            nbh[2 * j] = fwd;
            nbh[2 * j + 1] = bwd;
            loff[2 * j] = ((long)(mu * 2 + p) * Vh + site) * R;
            loff[2 * j + 1] = ((long)(mu * 2 + (1 - p)) * Vh + bwd) * R;
            cre[2 * j] = c_re;
            cim[2 * j] = c_im;
            cre[2 * j + 1] = -c_re;
            cim[2 * j + 1] = -c_im;
            fsg[2 * j] = (g.t_bc < 0 && fcross) ? T(-1) : T(1);
            fsg[2 * j + 1] = (g.t_bc < 0 && bcross) ? T(-1) : T(1);
        }
#if QCDW_HOP_PREFETCH
        // issue every load of the four hops before any arithmetic
        cx<T> ur[4][R], pu[4][3], pl[4][3];
#pragma unroll
        for (int h = 0; h < 4; h++) {
#pragma unroll
            for (int e = 0; e < R; e++) ur[h][e] = P::ld(a.gauge, loff[h] + e);
#pragma unroll
            for (int c = 0; c < 3; c++) {
                pu[h][c] = P::ld(a.psi, ((long)su * Vh + nbh[h]) * 3 + c);
                pl[h][c] = P::ld(a.psi, ((long)sl * Vh + nbh[h]) * 3 + c);
            }
        }
#endif
#pragma unroll
        for (int h = 0; h < 4; h++) {
            const int dir = h & 1;
            const cx<T> cc = {cre[h], cim[h]};
            cx<T> u[9];
#if QCDW_HOP_PREFETCH
#pragma unroll
            for (int e = 0; e < R; e++) u[e] = ur[h][e];
            if constexpr (R == 6) {
                u[6] = conj(u[1] * u[5] - u[2] * u[4]);
                u[7] = conj(u[2] * u[3] - u[0] * u[5]);
                u[8] = conj(u[0] * u[4] - u[1] * u[3]);
            }
#else
            load_link<P, R>(a.gauge, loff[h], u);
#endif
            cx<T> hv[3];
#pragma unroll
            for (int c = 0; c < 3; c++) {
#if QCDW_HOP_PREFETCH
                hv[c] = pu[h][c] + cc * pl[h][c];
#else
                const cx<T> pu_ = P::ld(a.psi, ((long)su * Vh + nbh[h]) * 3 + c);
                const cx<T> pl_ = P::ld(a.psi, ((long)sl * Vh + nbh[h]) * 3 + c);
                hv[c] = pu_ + cc * pl_;
#endif
            }
            cx<T> w[3];
#pragma unroll
            for (int r = 0; r < 3; r++) {
                cx<T> sacc = {T(0), T(0)};
#pragma unroll
                for (int c = 0; c < 3; c++)
                    sacc = dir == 0 ? sacc + u[3 * r + c] * hv[c] : sacc + cmul_conj(u[3 * c + r], hv[c]);
                w[r] = sacc;
            }
            const cx<T> cd = conj(cc);
#pragma unroll
            for (int r = 0; r < 3; r++) {
                const cx<T> wr = fsg[h] * w[r];
                acc_u[r] = acc_u[r] + wr;
                acc_l[r] = acc_l[r] + cd * wr;
            }
        }
    }

    // gather: lane q finishes spin q
    const int lane = threadIdx.x & 63;
    const int src = (lane & ~3) + (q < 2 ? q + 2 : 3 - q);
    cx<T> res[3];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const cx<T> mine = gq == 0 ? acc_u[c] : acc_l[c];
        const cx<T> theirs = gq == 0 ? acc_l[c] : acc_u[c];
        res[c] = mine + shfl_cx(theirs, src);
    }

    cx<T> outv[3];
    cx<T> yv[3];
    if constexpr (EPI == EPI_CLOV_XPAY || EPI == EPI_XPAY_CLOVY || RED == RED_TS) {
#pragma unroll
        for (int c = 0; c < 3; c++) yv[c] = valid ? P::ld(a.y, ((long)q * Vh + site) * 3 + c) : cx<T>{T(0), T(0)};
    }
    if constexpr (EPI == EPI_NONE) {
#pragma unroll
        for (int c = 0; c < 3; c++) outv[c] = res[c];
    } else {
        T win[27];
        if (valid) {
            load_window<P>(a.clov, site, q, win);
        } else {
#pragma unroll
            for (int e = 0; e < 27; e++) win[e] = T(0);
        }
        const T aa = (T)a.a;
        if constexpr (EPI == EPI_XPAY_CLOVY) {
            cx<T> ox[3], by[3];
#pragma unroll
            for (int c = 0; c < 3; c++) ox[c] = shfl_xor_cx(yv[c], 1);
            herm_rows(win, q & 1, yv, ox, by);
#pragma unroll
            for (int c = 0; c < 3; c++) outv[c] = by[c] - aa * res[c];
        } else {
            cx<T> ox[3], br[3];
#pragma unroll
            for (int c = 0; c < 3; c++) ox[c] = shfl_xor_cx(res[c], 1);
            herm_rows(win, q & 1, res, ox, br);
            if constexpr (EPI == EPI_CLOV) {
#pragma unroll
                for (int c = 0; c < 3; c++) outv[c] = br[c];
            } else {
#pragma unroll
                for (int c = 0; c < 3; c++) outv[c] = yv[c] - aa * br[c];
            }
        }
    }

    // reductions use the values as stored, so the solver's scalars match the
    // vectors it reads back
#pragma unroll
    for (int c = 0; c < 3; c++) outv[c] = P::rt(outv[c]);
    if (valid) {
#pragma unroll
        for (int c = 0; c < 3; c++) P::st(a.out, ((long)q * Vh + site) * 3 + c, outv[c]);
    }

    if constexpr (RED != RED_NONE) {
        double v[3] = {0.0, 0.0, 0.0};
        if (valid) {
#pragma unroll
            for (int c = 0; c < 3; c++) {
                const cx<T> o = outv[c];
                if constexpr (RED == RED_WDOT) {
                    const cx<T> wv = P::ld(a.w, ((long)q * Vh + site) * 3 + c);
                    v[0] += (double)wv.re * o.re + (double)wv.im * o.im;
                    v[1] += (double)wv.re * o.im - (double)wv.im * o.re;
                } else {
                    v[0] += (double)o.re * yv[c].re + (double)o.im * yv[c].im;
                    v[1] += (double)o.re * yv[c].im - (double)o.im * yv[c].re;
                    v[2] += (double)o.re * o.re + (double)o.im * o.im;
                }
            }
        }
        block_sum_store<3>(v, part);
    }
}

template <class P, int R, int EPI, int RED>
__global__ __launch_bounds__(256) QCDW_HOP_ATTR void hop_kernel(HopArgs a)
{
    if (a.stop && *a.stop) return;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    hop_tile<P, R, EPI, RED>(a, tile, a.partials + 3 * (long)tile);
}

// Multi-RHS hop, L2-reuse form: block -> (tile, rhs) with rhs fastest, so the
// blocks applying one tile's links and clover entries to all right-hand sides
// run back to back on one XCD and re-read them from its L2; each block is the
// single-RHS tile code.  Finished RHS (flags set) are skipped.
template <class P, int EPI, int RED>
__global__ __launch_bounds__(256) void hop_rhs_kernel(HopArgs a, const Scal* S)
{
    const int nrhs = a.nrhs;
    const int logical = xcd_tile(blockIdx.x, gridDim.x);
    const int tile = logical / nrhs, r = logical - tile * nrhs;
    if (S && S[r].flags) return;
    const long off = (long)r * 12 * a.g.Vh * P::cbytes;
    HopArgs b = a;
    b.psi = (const char*)a.psi + off;
    b.out = (char*)a.out + off;
    if (a.y) b.y = (const char*)a.y + off;
    if (a.w) b.w = (const char*)a.w + off;
    hop_tile<P, 6, EPI, RED>(b, tile, a.partials + 3 * ((long)r * hop_blocks(a.g.Vh) + tile));
}

// Batched hop: a persistent grid walks the tiles of every problem in a device
// table (problems of different lattice sizes and kappas).  Tile t belongs to
// the problem whose [tile0, tile0 + ntiles) contains it; finished problems
// (flags set) are skipped; partials go to [problem][tile][3].
template <class P, int EPI, int RED>
__global__ __launch_bounds__(256) void hop_batch_kernel(BatchHopArgs b)
{
    for (int t = blockIdx.x; t < b.total_tiles; t += gridDim.x) {
        int lo = 0, hi = b.nprob - 1;
        while (lo < hi) {  // last problem with tile0 <= t
            const int mid = (lo + hi + 1) >> 1;
            if (b.tab[mid].tile0 <= t) lo = mid;
            else hi = mid - 1;
        }
        const BatchEntry& e = b.tab[lo];
        if (b.S && b.S[lo].flags) continue;  // uniform over the block
        HopArgs a{};
        a.g = e.g;
        a.parity = b.parity;
        a.gauge = e.gauge;
        a.clov = e.clov[b.parity];
        a.psi = (const char*)b.psi + e.off * P::cbytes;
        a.out = (char*)b.out + e.off * P::cbytes;
        a.y = b.y ? (const char*)b.y + e.off * P::cbytes : nullptr;
        a.w = b.w ? (const char*)b.w + e.off * P::cbytes : nullptr;
        a.a = b.use_kappa2 ? e.kappa2 : b.a;
        a.nrhs = 1;
        const int tile = t - e.tile0;
        hop_tile<P, 6, EPI, RED>(a, tile, b.partials + 3 * ((long)lo * b.nbmax + tile));
        __syncthreads();  // shared reduction buffer reused by the next tile
    }
}

template <class P, int R>
static hipError_t launch_hop_pr(hipStream_t s, int epi, int red, const HopArgs& a, hipEvent_t e0, hipEvent_t e1)
{
    dim3 grid(hop_blocks(a.g.Vh)), block(256);
    // with events, they are recorded by the dispatch itself (exact kernel time)
#define QCDW_HOP_CASE(E, D)                                                                          \
    if (epi == E && red == D) {                                                                     \
        if (e0)                                                                                     \
            hipExtLaunchKernelGGL((hop_kernel<P, R, E, D>), grid, block, 0, s, e0, e1, 0, a);        \
        else                                                                                        \
            hipLaunchKernelGGL((hop_kernel<P, R, E, D>), grid, block, 0, s, a);                      \
        return hipGetLastError();                                                                   \
    }
    QCDW_HOP_CASE(EPI_NONE, RED_NONE)
    QCDW_HOP_CASE(EPI_CLOV, RED_NONE)
    QCDW_HOP_CASE(EPI_CLOV_XPAY, RED_NONE)
    QCDW_HOP_CASE(EPI_CLOV_XPAY, RED_WDOT)
    QCDW_HOP_CASE(EPI_CLOV_XPAY, RED_TS)
    QCDW_HOP_CASE(EPI_XPAY_CLOVY, RED_NONE)
#undef QCDW_HOP_CASE
    return hipErrorInvalidValue;
}

template <class P>
static hipError_t launch_rhs_p(hipStream_t s, int epi, int red, const HopArgs& a, const Scal* S, hipEvent_t e0,
                               hipEvent_t e1)
{
    const dim3 grid(hop_blocks(a.g.Vh) * a.nrhs), block(256);
#define QCDW_RHS_CASE(E, D)                                                                     \
    if (epi == E && red == D) {                                                                \
        if (e0)                                                                                \
            hipExtLaunchKernelGGL((hop_rhs_kernel<P, E, D>), grid, block, 0, s, e0, e1, 0, a, S); \
        else                                                                                   \
            hipLaunchKernelGGL((hop_rhs_kernel<P, E, D>), grid, block, 0, s, a, S);             \
        return hipGetLastError();                                                              \
    }
    QCDW_RHS_CASE(EPI_CLOV, RED_NONE)
    QCDW_RHS_CASE(EPI_CLOV_XPAY, RED_NONE)
    QCDW_RHS_CASE(EPI_CLOV_XPAY, RED_WDOT)
    QCDW_RHS_CASE(EPI_CLOV_XPAY, RED_TS)
#undef QCDW_RHS_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_hop_rhs(hipStream_t s, int prec, int epi, int red, const HopArgs& a, const Scal* S, hipEvent_t e0,
                          hipEvent_t e1)
{
    if (a.g.Vh <= 0 || a.nrhs <= 0) return hipSuccess;
    switch (prec) {
    case F64: return launch_rhs_p<P64>(s, epi, red, a, S, e0, e1);
    case F32: return launch_rhs_p<P32>(s, epi, red, a, S, e0, e1);
    case BF16: return launch_rhs_p<PBF16>(s, epi, red, a, S, e0, e1);
    case F16: return launch_rhs_p<PF16>(s, epi, red, a, S, e0, e1);
    }
    return hipErrorInvalidValue;
}

template <class P>
static hipError_t launch_batch_p(hipStream_t s, int epi, int red, const BatchHopArgs& b, int grid, hipEvent_t e0,
                                 hipEvent_t e1)
{
#define QCDW_BATCH_CASE(E, D)                                                                             \
    if (epi == E && red == D) {                                                                          \
        if (e0)                                                                                          \
            hipExtLaunchKernelGGL((hop_batch_kernel<P, E, D>), dim3(grid), dim3(256), 0, s, e0, e1, 0, b); \
        else                                                                                             \
            hipLaunchKernelGGL((hop_batch_kernel<P, E, D>), dim3(grid), dim3(256), 0, s, b);             \
        return hipGetLastError();                                                                        \
    }
    QCDW_BATCH_CASE(EPI_CLOV, RED_NONE)
    QCDW_BATCH_CASE(EPI_CLOV_XPAY, RED_WDOT)
    QCDW_BATCH_CASE(EPI_CLOV_XPAY, RED_TS)
#undef QCDW_BATCH_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_hop_batch(hipStream_t s, int prec, int epi, int red, const BatchHopArgs& b, int grid,
                            hipEvent_t e0, hipEvent_t e1)
{
    if (b.total_tiles <= 0) return hipSuccess;
    if (grid <= 0 || grid > b.total_tiles) grid = b.total_tiles;
    switch (prec) {
    case F64: return launch_batch_p<P64>(s, epi, red, b, grid, e0, e1);
    case F32: return launch_batch_p<P32>(s, epi, red, b, grid, e0, e1);
    case BF16: return launch_batch_p<PBF16>(s, epi, red, b, grid, e0, e1);
    case F16: return launch_batch_p<PF16>(s, epi, red, b, grid, e0, e1);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_hop(hipStream_t s, int prec, int recon, int epi, int red, const HopArgs& a, hipEvent_t e0,
                      hipEvent_t e1)
{
    if (a.g.Vh <= 0) return hipSuccess;
    if (recon == 18) {
        if (prec == F64) return launch_hop_pr<P64, 9>(s, epi, red, a, e0, e1);
        if (prec == F32) return launch_hop_pr<P32, 9>(s, epi, red, a, e0, e1);
        return hipErrorInvalidValue;
    }
    switch (prec) {
    case F64: return launch_hop_pr<P64, 6>(s, epi, red, a, e0, e1);
    case F32: return launch_hop_pr<P32, 6>(s, epi, red, a, e0, e1);
    case BF16: return launch_hop_pr<PBF16, 6>(s, epi, red, a, e0, e1);
    case F16: return launch_hop_pr<PF16, 6>(s, epi, red, a, e0, e1);
    }
    return hipErrorInvalidValue;
}

}  // namespace qcdw
