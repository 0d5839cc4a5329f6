// Device helpers shared by the parity-hop kernels (single-RHS forms, multi-RHS
// and batched): link reconstruction, the lane geometry of the four-lanes-per-site
// decomposition, the projected hop, and the Hermitian clover rows.
//
// Lane q = 2 gq + k of a site handles directions mu = 2 gq and 2 gq + 1
// (forward and backward) and only row k of the half-spinor that (1 -/+ g_mu)
// projects onto: in the DeGrand-Rossi basis h_k = psi_k + c psi_l with a unit
// coefficient c and l = 3 - k (mu = x, y) or 2 + k (mu = z, t); W h_k adds to
// spin k and conj(c) W h_k to spin l (paper Sec. III.B, Eq. "clover", the
// Wilson hopping term written out).
#pragma once
#include "internal.h"

namespace qcdw {

// link at element offset off (link_base), entries `stride` apart (link_stride)
template <class P, int R>
__device__ __forceinline__ void load_link(const void* gauge, long off, long stride, cx<typename P::real> (&u)[9])
{
    if constexpr (R == 9) {
#pragma unroll
        for (int e = 0; e < 9; e++) u[e] = P::ld(gauge, off + e * stride);
    } else {
#pragma unroll
        for (int e = 0; e < 6; e++) u[e] = P::ld(gauge, off + e * stride);
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
// FMA: every complex multiply-add as four real multiply-adds (fewer instructions; used by the
// multi-RHS hop, whose loop is bound by vector ALU issue); else the plain complex products.
template <bool FMA, typename T>
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
        cx<T> s;
        if constexpr (FMA) {
            // diagonal entry (real) first, then the rest of the own block
            s = {own[a][a].re * vo[a].re, own[a][a].re * vo[a].im};
#pragma unroll
            for (int b = 0; b < 3; b++)
                if (b != a) cmac(s, own[a][b], vo[b]);
        } else {
            s = {T(0), T(0)};
#pragma unroll
            for (int b = 0; b < 3; b++) s = s + own[a][b] * vo[b];
        }
#pragma unroll
        for (int b = 0; b < 3; b++) {
            // cross block: rows of this half, columns of the other half
            cx<T> cb = h ? cx<T>{Xr[3 * a + b], Xi[3 * a + b]} : cx<T>{Xr[3 * b + a], -Xi[3 * b + a]};
            if constexpr (FMA)
                cmac(s, cb, vx[b]);
            else
                s = s + cb * vx[b];
        }
        out[a] = s;
    }
}

// lane q's 27-entry window: chirality q >> 1, entries 9 (q & 1) .. 9 (q & 1) + 26
template <class P>
__device__ __forceinline__ void load_window(const void* clov, long Vh, int site, int q, typename P::real (&win)[27])
{
    const long base = clov_index(site, q >> 1, 9 * (q & 1));
#pragma unroll
    for (int e = 0; e < 27; e++) win[e] = P::ldr(clov, base + (long)e * CLOV_STRIDE);
}

// The same window with each of the two lanes of a chirality block reading half of the block: lane h loads
// the 18 contiguous entries 18 h .. 18 h + 17 (its own 9 and half of the shared 18) and takes the other 9 of its
// window from its partner lane (q ^ 1) by DPP.  All four lanes of the quad must be active; invalid lanes
// (valid = false) load nothing and pass zeros.  The single-RHS hop uses it (QCDW_WIN_SHARE = 1): at 24^3x64
// the FP64 hop issues 57 instead of 62 loads per lane (178 -> 177 us), and the 16-bit window, which now starts
// on a 4-byte boundary, is read by a few wide loads instead of 16-bit ones (BF16 hop 52 -> 45 us).
#ifndef QCDW_WIN_SHARE
#define QCDW_WIN_SHARE 1
#endif
template <class P>
__device__ __forceinline__ void load_window_shared(const void* clov, long Vh, int site, int q, bool valid,
                                                   typename P::real (&win)[27]);

// In-quad permutations through DPP (a VALU operand modifier, no trip through the LDS crossbar): lane
// 4 b + i receives the value of lane 4 b + sel_i, CTRL = sel_0 | sel_1 << 2 | sel_2 << 4 | sel_3 << 6.
// Every lane of the quad must be active.
constexpr int QUAD_XOR1 = 0xB1;      // (1, 0, 3, 2): the partner spin of a chirality block
constexpr int QUAD_PARTNER = 0x1E;   // (2, 3, 1, 0): the lane holding the other half of a spin's hops
template <int CTRL>
__device__ __forceinline__ float quad_dpp(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ double quad_dpp(double v)
{
    const uint2 u = __builtin_bit_cast(uint2, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)u.x, CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)u.y, CTRL, 0xf, 0xf, true);
    return __builtin_bit_cast(double, make_uint2((unsigned)lo, (unsigned)hi));
}
template <int CTRL, typename T>
__device__ __forceinline__ cx<T> quad_dpp_cx(cx<T> v)
{
    return {quad_dpp<CTRL>(v.re), quad_dpp<CTRL>(v.im)};
}

// The four hops of one lane at one site: neighbour indices (input parity), link
// offsets, projection coefficients and time-boundary signs.  Hop h = 2 j + dir,
// mu = 2 gq + j, dir 0 forward / 1 backward.  The projection coefficient c is a
// unit number, imaginary for j = 0 (mu = x, z) and real for j = 1 (mu = y, t), so
// only its nonzero part cs is kept: c = i cs (h < 2) or c = cs (h >= 2).
template <typename T, int R>
struct LaneHops {
    int nbh[4];
    long loff[4];  // link_base of each hop's link
    long lstr;     // link_stride
    T cs[4], fsg[4];
};

template <typename T, int R, bool SOA>
__device__ __forceinline__ void lane_hops(const Geom& g, int site, int p, int q, LaneHops<T, R>& L)
{
    const int gq = q >> 1, k = q & 1;
    const long Vh = g.Vh;
    L.lstr = link_stride(Vh, SOA);
    int x, y, z, t;
    site_coords(g, site, p, x, y, z, t);
    const int xh = site % g.Lxh;
    const int Sy = g.Lxh, Sz = g.Lxh * g.Ly, St = g.Lxh * g.Ly * g.Lz;
#pragma unroll
    for (int j = 0; j < 2; j++) {
        const int mu = 2 * gq + j;
        int fwd, bwd;
        bool fcross = false, bcross = false;
        T c_s;  // projection coefficient of the forward hop: i c_s (x, z) or c_s (y, t)
        if (j == 0) {
            if (gq == 0) {  // x: the neighbour lies in the same row of the other parity
                const int row = site - xh;
                const int xp = (x + 1 == g.Lx) ? 0 : x + 1;
                const int xm = (x == 0) ? g.Lx - 1 : x - 1;
                fwd = row + (xp >> 1);
                bwd = row + (xm >> 1);
                c_s = T(-1);
            } else {  // z
                fwd = (z + 1 == g.Lz) ? site - (g.Lz - 1) * Sz : site + Sz;
                bwd = (z == 0) ? site + (g.Lz - 1) * Sz : site - Sz;
                c_s = k == 0 ? T(-1) : T(1);
            }
        } else {
            if (gq == 0) {  // y
                fwd = (y + 1 == g.Ly) ? site - (g.Ly - 1) * Sy : site + Sy;
                bwd = (y == 0) ? site + (g.Ly - 1) * Sy : site - Sy;
                c_s = k == 0 ? T(1) : T(-1);
            } else {  // t
                fwd = (t + 1 == g.Lt) ? site - (g.Lt - 1) * St : site + St;
                bwd = (t == 0) ? site + (g.Lt - 1) * St : site - St;
                fcross = (t + 1 == g.Lt);
                bcross = (t == 0);
                c_s = T(-1);
            }
        }
        // forward: U_mu(x) psi(x+mu) with (1 - g_mu); backward: U_mu(x-mu)^+ psi(x-mu)
        // with (1 + g_mu), which flips the projection coefficient
        L.nbh[2 * j] = fwd;
        L.nbh[2 * j + 1] = bwd;
        L.loff[2 * j] = link_base(mu, p, site, Vh, R, SOA);
        L.loff[2 * j + 1] = link_base(mu, 1 - p, bwd, Vh, R, SOA);
        L.cs[2 * j] = c_s;
        L.cs[2 * j + 1] = -c_s;
        // boundary sign times the direction's weight (spatial hops: g.xs)
        const T wgt = (j == 1 && gq == 1) ? T(1) : T(g.xs);
        L.fsg[2 * j] = (g.t_bc < 0 && fcross) ? -wgt : wgt;
        L.fsg[2 * j + 1] = (g.t_bc < 0 && bcross) ? -wgt : wgt;
    }
}

template <class P>
__device__ __forceinline__ void load_window_shared(const void* clov, long Vh, int site, int q, bool valid,
                                                   typename P::real (&win)[27])
{
    using T = typename P::real;
    const int h = q & 1;
    T own[18];
#pragma unroll
    for (int e = 0; e < 18; e++) own[e] = T(0);
    if (valid) {
        const long base = clov_index(site, q >> 1, 18 * h);
#pragma unroll
        for (int e = 0; e < 18; e++) own[e] = P::ldr(clov, base + (long)e * CLOV_STRIDE);
    }
    // half 0 needs entries 18..26 (the partner's own[0..8]), half 1 entries 9..17 (the partner's own[9..17])
    T rcv[9];
#pragma unroll
    for (int j = 0; j < 9; j++) rcv[j] = quad_dpp<QUAD_XOR1>(h ? own[j] : own[9 + j]);
#pragma unroll
    for (int e = 0; e < 27; e++) win[e] = h ? (e < 9 ? rcv[e] : own[e - 9]) : (e < 18 ? own[e] : rcv[e - 18]);
}

// the two spins (su, sl) of neighbour nb that this lane's row of the projection needs
template <class P>
__device__ __forceinline__ void load_pair(const void* psi, long Vh, int su, int sl, int nb,
                                          cx<typename P::real> (&pu)[3], cx<typename P::real> (&pl)[3])
{
#pragma unroll
    for (int c = 0; c < 3; c++) {
        pu[c] = P::ld(psi, sp_idx(su, nb, c, Vh));
        pl[c] = P::ld(psi, sp_idx(sl, nb, c, Vh));
    }
}

// w = W hv with W = U (dir 0) or U^+ (dir 1); acc_u += s w and acc_l += conj(c) s w for the hop's
// boundary sign s and projection coefficient c (imag: c = i cs, else c = cs).  FMA: written out so
// that every update is one multiply-add and no product with a zero coefficient is formed; else the
// plain complex products (the compiler keeps the products with zero, which IEEE arithmetic needs).
template <bool FMA, typename T>
__device__ __forceinline__ void hop_rows(const cx<T> (&u)[9], int dir, bool imag, T s, T cs, const cx<T> (&hv)[3],
                                         cx<T> (&acc_u)[3], cx<T> (&acc_l)[3])
{
#pragma unroll
    for (int r = 0; r < 3; r++) {
        if constexpr (FMA) {
            cx<T> w = dir == 0 ? u[3 * r] * hv[0] : cmul_conj(u[r], hv[0]);
#pragma unroll
            for (int c = 1; c < 3; c++) {
                if (dir == 0)
                    cmac(w, u[3 * r + c], hv[c]);
                else
                    cmac_conj(w, u[3 * c + r], hv[c]);
            }
            const T cf = cs * s;
            acc_u[r] = {acc_u[r].re + s * w.re, acc_u[r].im + s * w.im};
            acc_l[r] = imag ? cx<T>{acc_l[r].re + cf * w.im, acc_l[r].im - cf * w.re}
                            : cx<T>{acc_l[r].re + cf * w.re, acc_l[r].im + cf * w.im};
        } else {
            cx<T> w = {T(0), T(0)};
#pragma unroll
            for (int c = 0; c < 3; c++) w = dir == 0 ? w + u[3 * r + c] * hv[c] : w + cmul_conj(u[3 * c + r], hv[c]);
            const cx<T> cd = imag ? cx<T>{T(0), -cs} : cx<T>{cs, T(0)};  // conj(c)
            const cx<T> wr = s * w;
            acc_u[r] = acc_u[r] + wr;
            acc_l[r] = acc_l[r] + cd * wr;
        }
    }
}

// W h for hop h with the projected row hv, accumulated into the two output spins
template <bool FMA, class P, int R>
__device__ __forceinline__ void hop_apply(const void* gauge, const LaneHops<typename P::real, R>& L, int h,
                                          const cx<typename P::real> (&hv)[3], cx<typename P::real> (&acc_u)[3],
                                          cx<typename P::real> (&acc_l)[3])
{
    using T = typename P::real;
    cx<T> u[9];
    load_link<P, R>(gauge, L.loff[h], L.lstr, u);
    hop_rows<FMA>(u, h & 1, h < 2, L.fsg[h], L.cs[h], hv, acc_u, acc_l);
}

// hv = pu + c pl with c = i cs (imag) or cs
template <bool FMA, typename T>
__device__ __forceinline__ void project(const cx<T> (&pu)[3], const cx<T> (&pl)[3], T cs, bool imag, cx<T> (&hv)[3])
{
#pragma unroll
    for (int c = 0; c < 3; c++) {
        if constexpr (FMA)
            hv[c] = imag ? cx<T>{pu[c].re - cs * pl[c].im, pu[c].im + cs * pl[c].re}
                         : cx<T>{pu[c].re + cs * pl[c].re, pu[c].im + cs * pl[c].im};
        else
            hv[c] = pu[c] + (imag ? cx<T>{T(0), cs} : cx<T>{cs, T(0)}) * pl[c];
    }
}


}  // namespace qcdw
