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

#include "hop_common.h"

// arithmetic form of the clover epilogue (see herm_rows): the multiply-add form measured faster
#ifndef QCDW_CLOV_FMA
#define QCDW_CLOV_FMA 1
#endif
#ifndef QCDW_HOP_WAVES_PER_EU
#define QCDW_HOP_WAVES_PER_EU 0
#endif
#if QCDW_HOP_WAVES_PER_EU > 0
#define QCDW_HOP_ATTR __attribute__((amdgpu_waves_per_eu(QCDW_HOP_WAVES_PER_EU, QCDW_HOP_WAVES_PER_EU)))
#else
#define QCDW_HOP_ATTR
#endif
// t-stepping hop: minimum waves per SIMD the compiler must allow (0: its own choice) and
// whether the steps are unrolled
#ifndef QCDW_TKERNEL_WAVES
#define QCDW_TKERNEL_WAVES 0
#endif
#if QCDW_TKERNEL_WAVES > 0
#define QCDW_TKERNEL_ATTR __attribute__((amdgpu_waves_per_eu(QCDW_TKERNEL_WAVES)))
#else
#define QCDW_TKERNEL_ATTR
#endif
#ifndef QCDW_TKERNEL_UNROLL
#define QCDW_TKERNEL_UNROLL 1
#endif

namespace qcdw {

// Gather of the lane partial sums (lane q finishes spin q), epilogue, store, and
// this site's contribution to the fused reduction (added to v).
template <class P, int EPI, int RED>
__device__ __forceinline__ void hop_finish(const HopArgs& a, int site, bool valid, int q,
                                           const cx<typename P::real> (&acc_u)[3],
                                           const cx<typename P::real> (&acc_l)[3], double (&v)[3])
{
    using T = typename P::real;
    const long Vh = a.g.Vh;
    const int gq = q >> 1;
    cx<T> res[3];
#pragma unroll
    for (int c = 0; c < 3; c++) {  // partner lane: q < 2 ? q + 2 : 3 - q
        const cx<T> mine = gq == 0 ? acc_u[c] : acc_l[c];
        const cx<T> theirs = gq == 0 ? acc_l[c] : acc_u[c];
        res[c] = mine + quad_dpp_cx<QUAD_PARTNER>(theirs);
    }

    cx<T> outv[3];
    cx<T> yv[3];
    if constexpr (EPI == EPI_CLOV_XPAY || EPI == EPI_XPAY_CLOVY || RED == RED_TS) {
#pragma unroll
        for (int c = 0; c < 3; c++) yv[c] = valid ? P::ld(a.y, sp_idx(q, site, c, Vh)) : cx<T>{T(0), T(0)};
    }
    if constexpr (EPI == EPI_NONE) {
#pragma unroll
        for (int c = 0; c < 3; c++) outv[c] = res[c];
    } else {
        T win[27];
        if constexpr (QCDW_WIN_SHARE != 0) {
            load_window_shared<P>(a.clov, Vh, site, q, valid, win);
        } else if (valid) {
            load_window<P>(a.clov, Vh, site, q, win);
        } else {
#pragma unroll
            for (int e = 0; e < 27; e++) win[e] = T(0);
        }
        const T aa = (T)a.a;
        if constexpr (EPI == EPI_XPAY_CLOVY) {
            cx<T> ox[3], by[3];
#pragma unroll
            for (int c = 0; c < 3; c++) ox[c] = quad_dpp_cx<QUAD_XOR1>(yv[c]);
            herm_rows<QCDW_CLOV_FMA != 0>(win, q & 1, yv, ox, by);
#pragma unroll
            for (int c = 0; c < 3; c++) outv[c] = by[c] - aa * res[c];
        } else {
            cx<T> ox[3], br[3];
#pragma unroll
            for (int c = 0; c < 3; c++) ox[c] = quad_dpp_cx<QUAD_XOR1>(res[c]);
            herm_rows<QCDW_CLOV_FMA != 0>(win, q & 1, res, ox, br);
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
        for (int c = 0; c < 3; c++) P::st(a.out, sp_idx(q, site, c, Vh), outv[c]);
    }

    if constexpr (RED != RED_NONE) {
        if (valid) {
#pragma unroll
            for (int c = 0; c < 3; c++) {
                const cx<T> o = outv[c];
                if constexpr (RED == RED_WDOT) {
                    const cx<T> wv = P::ld(a.w, sp_idx(q, site, c, Vh));
                    v[0] += (double)wv.re * o.re + (double)wv.im * o.im;
                    v[1] += (double)wv.re * o.im - (double)wv.im * o.re;
                } else {
                    v[0] += (double)o.re * yv[c].re + (double)o.im * yv[c].im;
                    v[1] += (double)o.re * yv[c].im - (double)o.im * yv[c].re;
                    v[2] += (double)o.re * o.re + (double)o.im * o.im;
                }
            }
        }
    }
}

// The hop with its epilogue at one site per 4 lanes (site valid or not: every
// thread of the block calls it); `part` receives the block's reduction partials
// (RED != RED_NONE).  F: the multiply-add form of the hop arithmetic (hop_rows);
// which form is faster depends on the lattice, so the operator's tuner picks it.
// STG: the t-neighbours of the block's 64 sites were staged in LDS by the caller (stg: [t+1 | t-1][spin]
// [site in tile][colour]); the t-lanes read them from there.
template <class P, int R, int EPI, int RED, bool F = false, bool STG = false>
__device__ __forceinline__ void hop_site(const HopArgs& a, int site, bool valid, double* part,
                                         const cx<typename P::real>* stg = nullptr)
{
    using T = typename P::real;
    const Geom g = a.g;
    const int q = threadIdx.x & 3;
    const int gq = q >> 1, k = q & 1;
    const int su = k, sl = gq == 0 ? 3 - k : 2 + k;

    cx<T> acc_u[3], acc_l[3];
#pragma unroll
    for (int c = 0; c < 3; c++) acc_u[c] = acc_l[c] = {T(0), T(0)};
    if (valid) {
        LaneHops<T, R> L;
        lane_hops<T, R, link_soa_for(P::cbytes)>(g, site, a.parity, q, L);
#pragma unroll
        for (int h = 0; h < 4; h++) {
            cx<T> pu[3], pl[3], hv[3];
            if (STG && gq == 1 && h >= 2) {
                const int j = threadIdx.x >> 2;
                const cx<T>* b = stg + (h - 2) * (4 * HOP_SITES_PER_BLOCK * 3);
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    pu[c] = b[(su * HOP_SITES_PER_BLOCK + j) * 3 + c];
                    pl[c] = b[(sl * HOP_SITES_PER_BLOCK + j) * 3 + c];
                }
            } else {
                load_pair<P>(a.psi, g.Vh, su, sl, L.nbh[h], pu, pl);
            }
            project<F>(pu, pl, L.cs[h], h < 2, hv);
            hop_apply<F, P, R>(a.gauge, L, h, hv, acc_u, acc_l);
        }
    }
    double v[3] = {0.0, 0.0, 0.0};
    hop_finish<P, EPI, RED>(a, site, valid, q, acc_u, acc_l, v);
    if constexpr (RED != RED_NONE) block_sum_store<3>(v, part);
}

// One 64-site tile (consecutive eo indices) of the hop with its epilogue.
template <class P, int R, int EPI, int RED, bool F = false>
__device__ __forceinline__ void hop_tile(const HopArgs& a, int tile, double* part)
{
    const int site = tile * HOP_SITES_PER_BLOCK + (threadIdx.x >> 2);
    hop_site<P, R, EPI, RED, F>(a, site, site < a.g.Vh, part);
}

// Single-RHS hop, one site per 4 lanes.  With cgroup = G > 0 the tiles are 64
// consecutive c (eo index within a t-slice) of one slice, and the launch sweeps
// t inside each group of G c-tiles: (c-tile in group, then t, then group).  The
// input slice t is read by the output slices t - 1, t, t + 1, which then run
// G tiles apart instead of a whole slice apart, so its spinors stay in L2.
//
// STG (slice groups only): the tile's 64 sites share t, so their t-neighbours are the same 64 c of
// slices t + 1 and t - 1.  The block first copies those two runs (all spins) into LDS, each thread
// loading consecutive elements of the contiguous runs, and the t-lanes then read their neighbour
// spins from LDS instead of with per-lane strided loads.
template <class P, int R, int EPI, int RED, bool F, bool STG>
__global__ __launch_bounds__(256) QCDW_HOP_ATTR void hop_kernel(HopArgs a)
{
    if (a.stop && *a.stop) return;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    double* part = a.partials + 3 * (long)tile;
    if (a.cgroup > 0) {
        const Geom& g = a.g;
        const int G = a.cgroup, St = g.Lxh * g.Ly * g.Lz;
        const int grp = tile / (G * g.Lt), r = tile - grp * G * g.Lt;
        const int t = r / G, ct = grp * G + (r - t * G);
        const int c = ct * HOP_SITES_PER_BLOCK + (threadIdx.x >> 2);
        if constexpr (STG) {
            using T = typename P::real;
            constexpr int RUN = 4 * HOP_SITES_PER_BLOCK * 3;  // complex per staged slice run
            __shared__ cx<T> stg[2 * RUN];
            const int c0 = ct * HOP_SITES_PER_BLOCK;
            const int tp = t + 1 == g.Lt ? 0 : t + 1, tm = t == 0 ? g.Lt - 1 : t - 1;
            for (int e = threadIdx.x; e < 2 * RUN; e += 256) {
                const int d = e / RUN, rem = e - d * RUN;  // rem = (spin * 64 + j) * 3 + colour
                const int col = rem % 3, sj = rem / 3, sp = sj / HOP_SITES_PER_BLOCK, j = sj % HOP_SITES_PER_BLOCK;
                cx<T> v = {T(0), T(0)};
                if (c0 + j < St) v = P::ld(a.psi, sp_idx(sp, (d == 0 ? tp : tm) * St + c0 + j, col, g.Vh));
                stg[e] = v;
            }
            __syncthreads();
            hop_site<P, R, EPI, RED, F, true>(a, t * St + c, c < St, part, stg);
        } else {
            hop_site<P, R, EPI, RED, F>(a, t * St + c, c < St, part);
        }
    } else {
        hop_tile<P, R, EPI, RED, F>(a, tile, part);
    }
}

// Hop with NT output sites per thread along t.  Output sites of one parity are
// (c, t) with eo index t St + c, c in [0, St); for fixed c and t stepping by 2 the
// physical (x, y, z) is fixed, and the input site (c, t + 1) is both the forward
// t-neighbour of (c, t) and the backward t-neighbour of (c, t + 2).  A thread
// walks t = e + 2 (tg NT + j), j < NT, and carries that half-spinor from one
// step to the next, so the t-neighbour spinors are read once per chain instead
// of being re-fetched by the tiles of the adjacent t-slices.  Blocks: 64
// consecutive c; the order is e, then c-tile (within its group of cgroup
// c-tiles), then chain group tg, then c-tile group.  Requires Lt % (2 NT) == 0.
template <class P, int R, int EPI, int RED, int NT, bool F>
__global__ __launch_bounds__(256) QCDW_TKERNEL_ATTR void hop_tkernel(HopArgs a)
{
    if (a.stop && *a.stop) return;
    using T = typename P::real;
    const Geom g = a.g;
    const int nct = hop_ctiles(g);
    const int blk = xcd_tile(blockIdx.x, gridDim.x);
    // e fastest: the two chains over one t-range read the same input slices (one for its x, y, z
    // hops, the other for its t hops), so they run back to back; then the c-tile within its group
    // of G, then the t-range, then the group (G = all c-tiles of a slice without grouping)
    const int G = a.cgroup > 0 ? a.cgroup : nct, ntg = g.Lt / (2 * NT);
    const int e = blk & 1, rest = blk >> 1;
    const int grp = rest / (G * ntg), r = rest - grp * G * ntg;
    const int tg = r / G, ct = grp * G + (r - tg * G);
    const int St = g.Lxh * g.Ly * g.Lz;
    const int q = threadIdx.x & 3;
    const int c = ct * 64 + (threadIdx.x >> 2);
    const bool valid = c < St;
    const int gq = q >> 1, k = q & 1;
    const int su = k, sl = gq == 0 ? 3 - k : 2 + k;
    double v[3] = {0.0, 0.0, 0.0};
    cx<T> carry[3];  // t-lanes: projected backward half-spinor for the next step
#pragma unroll
    for (int cc = 0; cc < 3; cc++) carry[cc] = {T(0), T(0)};
#if QCDW_TKERNEL_UNROLL
#pragma unroll
#else
#pragma unroll 1
#endif
    for (int j = 0; j < NT; j++) {
        const int t = e + 2 * (tg * NT + j);
        const int site = t * St + c;
        cx<T> acc_u[3], acc_l[3];
#pragma unroll
        for (int cc = 0; cc < 3; cc++) acc_u[cc] = acc_l[cc] = {T(0), T(0)};
        if (valid) {
            LaneHops<T, R> L;
            lane_hops<T, R, link_soa_for(P::cbytes)>(g, site, a.parity, q, L);
            cx<T> next[3];  // this step's forward t-neighbour, projected for the next step
#pragma unroll
            for (int h = 0; h < 4; h++) {
                cx<T> hv[3];
                if (gq == 1 && h == 3 && j > 0) {
                    // backward t-hop: the input site is the previous step's forward t-neighbour
#pragma unroll
                    for (int cc = 0; cc < 3; cc++) hv[cc] = carry[cc];
                } else {
                    cx<T> pu[3], pl[3];
                    load_pair<P>(a.psi, g.Vh, su, sl, L.nbh[h], pu, pl);
                    project<F>(pu, pl, L.cs[h], h < 2, hv);
                    if (gq == 1 && h == 2) project<F>(pu, pl, -L.cs[h], false, next);
                }
                hop_apply<F, P, R>(a.gauge, L, h, hv, acc_u, acc_l);
            }
            if (gq == 1) {
#pragma unroll
                for (int cc = 0; cc < 3; cc++) carry[cc] = next[cc];
            }
        }
        hop_finish<P, EPI, RED>(a, site, valid, q, acc_u, acc_l, v);
    }
    if constexpr (RED != RED_NONE) block_sum_store<3>(v, a.partials + 3 * (long)blk);
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

template <class P, int R, int NT, bool F, bool STG = false>
static hipError_t launch_hop_nt(hipStream_t s, int epi, int red, const HopArgs& a, hipEvent_t e0, hipEvent_t e1)
{
    dim3 grid(hop_blocks_nt(a.g, NT, a.cgroup)), block(256);
    // with events, they are recorded by the dispatch itself (exact kernel time)
#define QCDW_HOP_KERNEL(E, D) hop_kernel<P, R, E, D, F, STG>
#define QCDW_TKERNEL(E, D) hop_tkernel<P, R, E, D, NT, F>
#define QCDW_HOP_CASE(E, D)                                                                            \
    if (epi == E && red == D) {                                                                       \
        if constexpr (NT == 1) {                                                                      \
            if (e0) hipExtLaunchKernelGGL((QCDW_HOP_KERNEL(E, D)), grid, block, 0, s, e0, e1, 0, a);    \
            else hipLaunchKernelGGL((QCDW_HOP_KERNEL(E, D)), grid, block, 0, s, a);                     \
        } else {                                                                                      \
            if (e0) hipExtLaunchKernelGGL((QCDW_TKERNEL(E, D)), grid, block, 0, s, e0, e1, 0, a);       \
            else hipLaunchKernelGGL((QCDW_TKERNEL(E, D)), grid, block, 0, s, a);                        \
        }                                                                                             \
        return hipGetLastError();                                                                     \
    }
    QCDW_HOP_CASE(EPI_NONE, RED_NONE)
    QCDW_HOP_CASE(EPI_CLOV, RED_NONE)
    QCDW_HOP_CASE(EPI_CLOV_XPAY, RED_NONE)
    QCDW_HOP_CASE(EPI_CLOV_XPAY, RED_WDOT)
    QCDW_HOP_CASE(EPI_CLOV_XPAY, RED_TS)
    QCDW_HOP_CASE(EPI_XPAY_CLOVY, RED_NONE)
#undef QCDW_HOP_CASE
#undef QCDW_TKERNEL
#undef QCDW_HOP_KERNEL
    return hipErrorInvalidValue;
}

template <class P, int R, bool F>
static hipError_t launch_hop_prf(hipStream_t s, int epi, int red, const HopArgs& a, hipEvent_t e0, hipEvent_t e1)
{
    if (a.fma & 2) {  // LDS-staged t-neighbours: slice groups, one site per thread group
        if (a.cgroup <= 0 || a.nt > 1) return hipErrorInvalidValue;
        return launch_hop_nt<P, R, 1, F, true>(s, epi, red, a, e0, e1);
    }
    switch (a.nt) {
    case 2: return launch_hop_nt<P, R, 2, F>(s, epi, red, a, e0, e1);
    case 4: return launch_hop_nt<P, R, 4, F>(s, epi, red, a, e0, e1);
    case 8: return launch_hop_nt<P, R, 8, F>(s, epi, red, a, e0, e1);
    default: return launch_hop_nt<P, R, 1, F>(s, epi, red, a, e0, e1);
    }
}

template <class P, int R>
static hipError_t launch_hop_pr(hipStream_t s, int epi, int red, const HopArgs& a, hipEvent_t e0, hipEvent_t e1)
{
    if (!hop_nt_fits(a.g, a.nt) || !hop_cgroup_fits(a.g, a.cgroup)) return hipErrorInvalidValue;
    return (a.fma & 1) ? launch_hop_prf<P, R, true>(s, epi, red, a, e0, e1)
                       : launch_hop_prf<P, R, false>(s, epi, red, a, e0, e1);
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
