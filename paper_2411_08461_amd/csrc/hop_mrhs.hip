// Multi-right-hand-side parity hop (a propagator is 12 solves, paper Sec. III.B;
// the paper names a multi-source solve as the next step).  Same four-lane site
// decomposition as hop.hip, but each lane loads its four reconstruct-12 links
// and its clover window once and applies them to every right-hand side in a
// register-resident loop, so link and clover bytes are paid once per site for
// all RHS.  RHS k of a field lives at offset k * 12 * Vh complex (a stack of
// single-RHS fields), and RHS whose solver flag is set are skipped.
#include <hip/hip_ext.h>

#include "internal.h"

namespace qcdw {

template <typename T>
__device__ __forceinline__ cx<T> mshfl(cx<T> v, int src)
{
    return {__shfl(v.re, src, 64), __shfl(v.im, src, 64)};
}
template <typename T>
__device__ __forceinline__ cx<T> mshfl_xor(cx<T> v, int m)
{
    return {__shfl_xor(v.re, m, 64), __shfl_xor(v.im, m, 64)};
}

// rows 3h..3h+2 of the Hermitian block times (own | other); window layout as in hop.hip
template <typename T>
__device__ __forceinline__ void mrhs_herm_rows(const T (&win)[27], int h, const cx<T> (&vo)[3], const cx<T> (&vx)[3],
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
            cx<T> cb = h ? cx<T>{Xr[3 * a + b], Xi[3 * a + b]} : cx<T>{Xr[3 * b + a], -Xi[3 * b + a]};
            s = s + cb * vx[b];
        }
        out[a] = s;
    }
}

template <class P, int EPI, int RED>
__global__ __launch_bounds__(256) void hop_mrhs_kernel(HopArgs a, const Scal* S)
{
    using T = typename P::real;
    const Geom g = a.g;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int nblk = gridDim.x;
    const int q = threadIdx.x & 3;
    const int site = tile * HOP_SITES_PER_BLOCK + (threadIdx.x >> 2);
    const bool valid = site < g.Vh;
    const int gq = q >> 1, k = q & 1;
    const int p = a.parity;
    const long Vh = g.Vh;
    const long field = 12L * Vh;  // complex per RHS
    const int lane = threadIdx.x & 63;
    const int src = (lane & ~3) + (q < 2 ? q + 2 : 3 - q);

    // per-lane hop geometry, raw links and clover window (loaded once for all RHS)
    int nbh[4] = {0, 0, 0, 0};
    T cre[4], cim[4], fsg[4];
    cx<T> ur[4][6];
    T win[27];
    const int su = k, sl = gq == 0 ? 3 - k : 2 + k;
#pragma unroll
    for (int h = 0; h < 4; h++) {
        cre[h] = cim[h] = T(0);
        fsg[h] = T(1);
#pragma unroll
        for (int e = 0; e < 6; e++) ur[h][e] = {T(0), T(0)};
    }
#pragma unroll
    for (int e = 0; e < 27; e++) win[e] = T(0);
    if (valid) {
        int x, y, z, t;
        site_coords(g, site, p, x, y, z, t);
        const int xh = site % g.Lxh;
        const int Sy = g.Lxh, Sz = g.Lxh * g.Ly, St = g.Lxh * g.Ly * g.Lz;
#pragma unroll
        for (int j = 0; j < 2; j++) {
            const int mu = 2 * gq + j;
            int fwd, bwd;
            bool fcross = false, bcross = false;
            T c_re, c_im;
            if (j == 0) {
                if (gq == 0) {
                    const int row = site - xh;
                    const int xp = (x + 1 == g.Lx) ? 0 : x + 1;
                    const int xm = (x == 0) ? g.Lx - 1 : x - 1;
                    fwd = row + (xp >> 1);
                    bwd = row + (xm >> 1);
                    c_re = T(0);
                    c_im = T(-1);
                } else {
                    fwd = (z + 1 == g.Lz) ? site - (g.Lz - 1) * Sz : site + Sz;
                    bwd = (z == 0) ? site + (g.Lz - 1) * Sz : site - Sz;
                    c_re = T(0);
                    c_im = k == 0 ? T(-1) : T(1);
                }
            } else {
                if (gq == 0) {
                    fwd = (y + 1 == g.Ly) ? site - (g.Ly - 1) * Sy : site + Sy;
                    bwd = (y == 0) ? site + (g.Ly - 1) * Sy : site - Sy;
                    c_re = k == 0 ? T(1) : T(-1);
                    c_im = T(0);
                } else {
                    fwd = (t + 1 == g.Lt) ? site - (g.Lt - 1) * St : site + St;
                    bwd = (t == 0) ? site + (g.Lt - 1) * St : site - St;
                    fcross = (t + 1 == g.Lt);
                    bcross = (t == 0);
                    c_re = T(-1);
                    c_im = T(0);
                }
            }
            nbh[2 * j] = fwd;
            nbh[2 * j + 1] = bwd;
            const long lf = ((long)(mu * 2 + p) * Vh + site) * 6;
            const long lb = ((long)(mu * 2 + (1 - p)) * Vh + bwd) * 6;
#pragma unroll
            for (int e = 0; e < 6; e++) {
                ur[2 * j][e] = P::ld(a.gauge, lf + e);
                ur[2 * j + 1][e] = P::ld(a.gauge, lb + e);
            }
            cre[2 * j] = c_re;
            cim[2 * j] = c_im;
            cre[2 * j + 1] = -c_re;
            cim[2 * j + 1] = -c_im;
            fsg[2 * j] = (g.t_bc < 0 && fcross) ? T(-1) : T(1);
            fsg[2 * j + 1] = (g.t_bc < 0 && bcross) ? T(-1) : T(1);
        }
        if constexpr (EPI != EPI_NONE) {
            const long base = clov_index(site, q >> 1, 9 * (q & 1));
#pragma unroll
            for (int e = 0; e < 27; e++) win[e] = P::ldr(a.clov, base + (long)e * CLOV_STRIDE);
        }
    }

    for (int r = 0; r < a.nrhs; r++) {
        if (S && S[r].flags) continue;  // uniform: every thread reads the same flag
        const long off = (long)r * field;
        cx<T> acc_u[3], acc_l[3];
#pragma unroll
        for (int c = 0; c < 3; c++) acc_u[c] = acc_l[c] = {T(0), T(0)};
        if (valid) {
#pragma unroll
            for (int h = 0; h < 4; h++) {
                const int dir = h & 1;
                const cx<T> cc = {cre[h], cim[h]};
                cx<T> u[9];
#pragma unroll
                for (int e = 0; e < 6; e++) u[e] = ur[h][e];
                u[6] = conj(u[1] * u[5] - u[2] * u[4]);
                u[7] = conj(u[2] * u[3] - u[0] * u[5]);
                u[8] = conj(u[0] * u[4] - u[1] * u[3]);
                cx<T> hv[3];
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    const cx<T> pu = P::ld(a.psi, off + ((long)su * Vh + nbh[h]) * 3 + c);
                    const cx<T> pl = P::ld(a.psi, off + ((long)sl * Vh + nbh[h]) * 3 + c);
                    hv[c] = pu + cc * pl;
                }
                const cx<T> cd = conj(cc);
#pragma unroll
                for (int rr = 0; rr < 3; rr++) {
                    cx<T> sacc = {T(0), T(0)};
#pragma unroll
                    for (int c = 0; c < 3; c++)
                        sacc = dir == 0 ? sacc + u[3 * rr + c] * hv[c] : sacc + cmul_conj(u[3 * c + rr], hv[c]);
                    const cx<T> wr = fsg[h] * sacc;
                    acc_u[rr] = acc_u[rr] + wr;
                    acc_l[rr] = acc_l[rr] + cd * wr;
                }
            }
        }
        cx<T> res[3];
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const cx<T> mine = gq == 0 ? acc_u[c] : acc_l[c];
            const cx<T> theirs = gq == 0 ? acc_l[c] : acc_u[c];
            res[c] = mine + mshfl(theirs, src);
        }
        cx<T> outv[3], yv[3];
        if constexpr (EPI == EPI_CLOV_XPAY || RED == RED_TS) {
#pragma unroll
            for (int c = 0; c < 3; c++)
                yv[c] = valid ? P::ld(a.y, off + ((long)q * Vh + site) * 3 + c) : cx<T>{T(0), T(0)};
        }
        if constexpr (EPI == EPI_NONE) {
#pragma unroll
            for (int c = 0; c < 3; c++) outv[c] = res[c];
        } else {
            cx<T> ox[3], br[3];
#pragma unroll
            for (int c = 0; c < 3; c++) ox[c] = mshfl_xor(res[c], 1);
            mrhs_herm_rows(win, q & 1, res, ox, br);
            const T aa = (T)a.a;
#pragma unroll
            for (int c = 0; c < 3; c++) outv[c] = (EPI == EPI_CLOV) ? br[c] : yv[c] - aa * br[c];
        }
#pragma unroll
        for (int c = 0; c < 3; c++) outv[c] = P::rt(outv[c]);
        if (valid) {
#pragma unroll
            for (int c = 0; c < 3; c++) P::st(a.out, off + ((long)q * Vh + site) * 3 + c, outv[c]);
        }
        if constexpr (RED != RED_NONE) {
            double v[3] = {0.0, 0.0, 0.0};
            if (valid) {
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    const cx<T> o = outv[c];
                    if constexpr (RED == RED_WDOT) {
                        const cx<T> wv = P::ld(a.w, off + ((long)q * Vh + site) * 3 + c);
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

template <class P>
static hipError_t launch_mrhs_p(hipStream_t s, int epi, int red, const HopArgs& a, const Scal* S, hipEvent_t e0,
                                hipEvent_t e1)
{
    dim3 grid(hop_blocks(a.g.Vh)), block(256);
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
