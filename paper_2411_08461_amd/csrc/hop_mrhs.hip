// Multi-right-hand-side parity hop (a propagator is 12 solves, paper Sec. III.B;
// the paper names a multi-source solve as the next step).  Same four-lane site
// decomposition as hop.hip, but each lane loads its four reconstruct-12 links
// and its clover window once and applies them to every right-hand side in a
// register-resident loop, so link and clover bytes are paid once per site for
// all RHS.  RHS k of a field lives at offset k * 12 * Vh complex (a stack of
// single-RHS fields), and RHS whose solver flag is set are skipped.  With
// cgroup > 0 the tiles follow the slice-group order of the single-RHS hop.
#include <hip/hip_ext.h>

#include "hop_common.h"

// right-hand sides processed together per loop step (their neighbour loads in flight together); two
// per step were measured 1.5x slower at 24^3x64 (the doubled accumulators push the kernel to 256 VGPRs)
#ifndef QCDW_MRHS_STEP
#define QCDW_MRHS_STEP 1
#endif

namespace qcdw {

template <class P, int EPI, int RED>
__global__ __launch_bounds__(256) void hop_mrhs_kernel(HopArgs a, const Scal* S)
{
    using T = typename P::real;
    const Geom g = a.g;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int nblk = gridDim.x;
    const int q = threadIdx.x & 3;
    int site;
    bool valid;
    if (a.cgroup > 0) {  // slice-group order, as in the single-RHS hop_kernel
        const int G = a.cgroup, St = g.Lxh * g.Ly * g.Lz;
        const int grp = tile / (G * g.Lt), rr = tile - grp * G * g.Lt;
        const int t = rr / G, ct = grp * G + (rr - t * G);
        const int c = ct * HOP_SITES_PER_BLOCK + (threadIdx.x >> 2);
        site = t * St + c;
        valid = c < St;
    } else {
        site = tile * HOP_SITES_PER_BLOCK + (threadIdx.x >> 2);
        valid = site < g.Vh;
    }
    const int gq = q >> 1, k = q & 1;
    const long Vh = g.Vh;
    const long field = 12L * Vh;  // complex per RHS
    const int lane = threadIdx.x & 63;
    const int src = (lane & ~3) + (q < 2 ? q + 2 : 3 - q);  // in-quad partner finishing the other spin
    const int su = k, sl = gq == 0 ? 3 - k : 2 + k;

    // per-lane hop geometry, links (row 2 rebuilt once) and clover window, shared by all RHS
    LaneHops<T, 6> L;
    cx<T> ur[4][9];
    T win[27];
#pragma unroll
    for (int h = 0; h < 4; h++) {
        L.nbh[h] = 0;
        L.loff[h] = 0;
        L.cs[h] = T(0);
        L.fsg[h] = T(1);
#pragma unroll
        for (int e = 0; e < 9; e++) ur[h][e] = {T(0), T(0)};
    }
#pragma unroll
    for (int e = 0; e < 27; e++) win[e] = T(0);
    if (valid) {
        lane_hops<T, 6, link_soa_for(P::cbytes)>(g, site, a.parity, q, L);
#pragma unroll
        for (int h = 0; h < 4; h++) load_link<P, 6>(a.gauge, L.loff[h], L.lstr, ur[h]);
        if constexpr (EPI != EPI_NONE) load_window<P>(a.clov, Vh, site, q, win);
    }

    // right-hand sides in groups of QCDW_MRHS_STEP, so that their neighbour loads are in flight together
    constexpr int RS = QCDW_MRHS_STEP;
    for (int r0 = 0; r0 < a.nrhs; r0 += RS) {
        bool act[RS];
#pragma unroll
        for (int j = 0; j < RS; j++)  // uniform: every thread reads the same flags
            act[j] = r0 + j < a.nrhs && !(S && S[r0 + j].flags);
        bool any = false;
#pragma unroll
        for (int j = 0; j < RS; j++) any = any || act[j];
        if (!any) continue;
        cx<T> acc2_u[RS][3], acc2_l[RS][3];
#pragma unroll
        for (int j = 0; j < RS; j++)
#pragma unroll
            for (int c = 0; c < 3; c++) acc2_u[j][c] = acc2_l[j][c] = {T(0), T(0)};
        if (valid) {
#pragma unroll
            for (int h = 0; h < 4; h++) {
                cx<T> hv[RS][3];
#pragma unroll
                for (int j = 0; j < RS; j++) {
                    cx<T> pu[3], pl[3];
                    if (act[j]) {
                        load_pair<P>((const char*)a.psi + (long)(r0 + j) * field * P::cbytes, Vh, su, sl, L.nbh[h],
                                     pu, pl);
                    } else {
#pragma unroll
                        for (int c = 0; c < 3; c++) pu[c] = pl[c] = {T(0), T(0)};
                    }
                    project<true>(pu, pl, L.cs[h], h < 2, hv[j]);
                }
#pragma unroll
                for (int j = 0; j < RS; j++)
                    hop_rows<true>(ur[h], h & 1, h < 2, L.fsg[h], L.cs[h], hv[j], acc2_u[j], acc2_l[j]);
            }
        }
#pragma unroll
        for (int j = 0; j < RS; j++) {
        if (!act[j]) continue;
        const int r = r0 + j;
        const long off = (long)r * field;
        const cx<T>(&acc_u)[3] = acc2_u[j];
        const cx<T>(&acc_l)[3] = acc2_l[j];
        cx<T> res[3];
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const cx<T> mine = gq == 0 ? acc_u[c] : acc_l[c];
            const cx<T> theirs = gq == 0 ? acc_l[c] : acc_u[c];
            res[c] = mine + shfl_cx(theirs, src);
        }
        cx<T> outv[3], yv[3];
        if constexpr (EPI == EPI_CLOV_XPAY || RED == RED_TS) {
#pragma unroll
            for (int c = 0; c < 3; c++)
                yv[c] = valid ? P::ld(a.y, off + sp_idx(q, site, c, Vh)) : cx<T>{T(0), T(0)};
        }
        if constexpr (EPI == EPI_NONE) {
#pragma unroll
            for (int c = 0; c < 3; c++) outv[c] = res[c];
        } else {
            cx<T> ox[3], br[3];
#pragma unroll
            for (int c = 0; c < 3; c++) ox[c] = shfl_xor_cx(res[c], 1);
            herm_rows<true>(win, q & 1, res, ox, br);
            const T aa = (T)a.a;
#pragma unroll
            for (int c = 0; c < 3; c++) outv[c] = (EPI == EPI_CLOV) ? br[c] : yv[c] - aa * br[c];
        }
#pragma unroll
        for (int c = 0; c < 3; c++) outv[c] = P::rt(outv[c]);
        if (valid) {
#pragma unroll
            for (int c = 0; c < 3; c++) P::st(a.out, off + sp_idx(q, site, c, Vh), outv[c]);
        }
        if constexpr (RED != RED_NONE) {
            double v[3] = {0.0, 0.0, 0.0};
            if (valid) {
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    const cx<T> o = outv[c];
                    if constexpr (RED == RED_WDOT) {
                        const cx<T> wv = P::ld(a.w, off + sp_idx(q, site, c, Vh));
                        v[0] += (double)wv.re * o.re + (double)wv.im * o.im;
                        v[1] += (double)wv.re * o.im - (double)wv.im * o.re;
                    } else {
                        v[0] += (double)o.re * yv[c].re + (double)o.im * yv[c].im;
                        v[1] += (double)o.re * yv[c].im - (double)o.im * yv[c].re;
                        v[2] += (double)o.re * o.re + (double)o.im * o.im;
                    }
                }
            }
            block_sum_store<3>(v, a.partials + 3 * ((long)r * nblk + tile));
            __syncthreads();  // the block reduction's shared buffer is reused for the next RHS
        }
        }
    }
}

template <class P>
static hipError_t launch_mrhs_p(hipStream_t s, int epi, int red, const HopArgs& a, const Scal* S, hipEvent_t e0,
                                hipEvent_t e1)
{
    dim3 grid(a.cgroup > 0 ? hop_ctiles(a.g) * a.g.Lt : hop_blocks(a.g.Vh)), block(256);
#define QCDW_MRHS_CASE(E, D)                                                                     \
    if (epi == E && red == D) {                                                                 \
        if (e0)                                                                                 \
            hipExtLaunchKernelGGL((hop_mrhs_kernel<P, E, D>), grid, block, 0, s, e0, e1, 0, a, S); \
        else                                                                                    \
            hipLaunchKernelGGL((hop_mrhs_kernel<P, E, D>), grid, block, 0, s, a, S);             \
        return hipGetLastError();                                                               \
    }
    QCDW_MRHS_CASE(EPI_CLOV, RED_NONE)
    QCDW_MRHS_CASE(EPI_CLOV_XPAY, RED_NONE)
    QCDW_MRHS_CASE(EPI_CLOV_XPAY, RED_WDOT)
    QCDW_MRHS_CASE(EPI_CLOV_XPAY, RED_TS)
#undef QCDW_MRHS_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_hop_mrhs(hipStream_t s, int prec, int epi, int red, const HopArgs& a, const Scal* S,
                           hipEvent_t e0, hipEvent_t e1)
{
    if (a.g.Vh <= 0 || a.nrhs <= 0) return hipSuccess;
    switch (prec) {
    case F64: return launch_mrhs_p<P64>(s, epi, red, a, S, e0, e1);
    case F32: return launch_mrhs_p<P32>(s, epi, red, a, S, e0, e1);
    case BF16: return launch_mrhs_p<PBF16>(s, epi, red, a, S, e0, e1);
    case F16: return launch_mrhs_p<PF16>(s, epi, red, a, S, e0, e1);
    }
    return hipErrorInvalidValue;
}

}  // namespace qcdw
