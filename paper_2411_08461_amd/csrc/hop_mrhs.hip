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
        // lanes past the last site run too (their neighbour offsets point at site 0 and their links are
        // zero) and store nothing: no divergent branch around the loads
#pragma unroll
        for (int h = 0; h < 4; h++) {
            cx<T> hv[RS][3];
#pragma unroll
            for (int j = 0; j < RS; j++) {
                cx<T> pu[3], pl[3];
                if (act[j]) {
                    load_pair<P>((const char*)a.psi + (long)(r0 + j) * field * P::cbytes, Vh, su, sl, L.nbh[h], pu,
                                 pl);
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
            res[c] = mine + quad_dpp_cx<QUAD_PARTNER>(theirs);
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
            for (int c = 0; c < 3; c++) ox[c] = quad_dpp_cx<QUAD_XOR1>(res[c]);
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

// ---------------------------------------------------------------------------
// Matrix-core form (16-bit storage): the SU(3) products of the hop on v_mfma_f32_4x4x4 (16 blocks of
// 4x4x4 per wave, FP32 accumulation).  Block b of an instruction is the quad of lanes 4b..4b+3, one site:
// lane 4b+i supplies row i of the A operand (K = 4 entries), lane 4b+j column j of B, and receives column j
// of D = A B in its four accumulator elements.  With A the hop's link W (rows: colour i, K: colour k, row and
// column 3 zero) and column j of B the neighbour's spin j, D holds (W psi_j)[i] in lane j: the lane of the
// output spin.  The spin projector is not formed: (1 -/+ gamma_mu) psi = psi_j + e_j psi_perm(j) with e_j a
// unit number (+-1 or +-i), so each direction adds W psi_j and W (e_j psi_perm(j)); the partner's spin comes
// from the quad by a DPP permutation, e_j by swapping re/im and flipping sign bits, both exact in 16 bits.
// Complex products take four real instructions (Re: Wr Br - Wi Bi, Im: Wr Bi + Wi Br).  Row 2 of the link
// is rebuilt in FP32 and rounded to 16 bits once per site (the only rounding the vector form does not have);
// the products are exact in FP32 and all eight directions accumulate there (the spatial ones first, their sum
// then scaled by the spatial weight).  Link operands are built once per site and kept in registers for all
// right-hand sides; the clover epilogue is the vector form's.  Measured at 24^3x64 with 12 RHS (BF16): 370 us
// against 306 us for the vector register loop, with a third fewer vector instructions: the vector form keeps
// its SIMDs issuing 74 % of the time and its address unit 86 % busy, while this form waits on its loads with
// less work in flight.  The multi-RHS tuner times this form beside the others.
// ---------------------------------------------------------------------------
typedef float mf4 __attribute__((ext_vector_type(4)));
typedef short ms4 __attribute__((ext_vector_type(4)));
typedef _Float16 mh4 __attribute__((ext_vector_type(4)));

template <class P>
struct Mfma16;
template <>
struct Mfma16<PBF16> {
    __device__ static uint32_t bits(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
    __device__ static float val(uint32_t b) { return bf_bits2f(b & 0xffffu); }
    __device__ static mf4 mma(ms4 a, ms4 b, mf4 c) { return __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(a, b, c, 0, 0, 0); }
};
template <>
struct Mfma16<PF16> {
    __device__ static uint32_t bits(float f) { return __builtin_bit_cast(uint16_t, (_Float16)f); }
    __device__ static float val(uint32_t b) { return (float)__builtin_bit_cast(_Float16, (uint16_t)(b & 0xffffu)); }
    __device__ static mf4 mma(ms4 a, ms4 b, mf4 c)
    {
        return __builtin_amdgcn_mfma_f32_4x4x4f16(__builtin_bit_cast(mh4, a), __builtin_bit_cast(mh4, b), c, 0, 0, 0);
    }
};

__device__ __forceinline__ ms4 ms4_of(uint32_t lo, uint32_t hi) { return __builtin_bit_cast(ms4, make_uint2(lo, hi)); }

// quad permutations of the partner spin: 3 - s (x, y) and s + 2 mod 4 (z, t)
template <int CTRL>
__device__ __forceinline__ uint32_t quad_dpp(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xf, 0xf, true);
}

template <class P, int EPI, int RED>
__global__ __launch_bounds__(256) void hop_mrhs_mfma_kernel(HopArgs a, const Scal* S)
{
    static_assert(QCDW_SPINOR_SOA == 0, "the matrix-core form reads a spin's three colours as one run");
    using M = Mfma16<P>;
    constexpr uint32_t SGN = 0x80008000u;
    const Geom g = a.g;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int nblk = gridDim.x;
    const int q = threadIdx.x & 3;
    int site;
    bool valid;
    if (a.cgroup > 0) {
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
    const long Vh = g.Vh;
    const long field = 12L * Vh;

    // the eight hops of the site: group G = 0 (x, y) and 1 (z, t), hop h = 2 j + dir (mu = 2 G + j);
    // nb: the lane's spin of each neighbour (complex offset within one right-hand side)
    int nb[8];
    ms4 Ar[8], Ai[8];
#pragma unroll
    for (int G = 0; G < 2; G++) {
        LaneHops<float, 6> L;
        L.lstr = 1;
#pragma unroll
        for (int h = 0; h < 4; h++) {
            L.nbh[h] = 0;
            L.loff[h] = 0;
            L.fsg[h] = 1.f;
        }
        if (valid) lane_hops<float, 6, link_soa_for(P::cbytes)>(g, site, a.parity, 2 * G, L);
#pragma unroll
        for (int h = 0; h < 4; h++) {
            nb[4 * G + h] = (int)sp_idx(q, L.nbh[h], 0, Vh);  // site 0 when invalid: read, results dropped
            cx<float> u[9];
#pragma unroll
            for (int e = 0; e < 6; e++) u[e] = P::ld(a.gauge, L.loff[h] + e * L.lstr);
            u[6] = conj(u[1] * u[5] - u[2] * u[4]);
            u[7] = conj(u[2] * u[3] - u[0] * u[5]);
            u[8] = conj(u[0] * u[4] - u[1] * u[3]);
            // row q of W = U (forward) or U^+ (backward), times the time-boundary sign; the spatial weight
            // is applied to the accumulated sum
            const float sg = (G == 1 && (h >> 1) == 1) ? L.fsg[h] : 1.f;
            uint32_t wr[3], wi[3];
#pragma unroll
            for (int k = 0; k < 3; k++) {
                // entries selected as scalars (a select of whole structs would select their addresses and
                // keep u in scratch memory)
                const int e0 = (h & 1) == 0 ? k : 3 * k, e1 = (h & 1) == 0 ? 3 + k : 3 * k + 1,
                          e2 = (h & 1) == 0 ? 6 + k : 3 * k + 2;
                const float re = q == 0 ? u[e0].re : q == 1 ? u[e1].re : u[e2].re;
                const float im = q == 0 ? u[e0].im : q == 1 ? u[e1].im : u[e2].im;
                wr[k] = q == 3 ? 0u : M::bits(sg * re);
                wi[k] = q == 3 ? 0u : M::bits((h & 1) == 0 ? sg * im : -sg * im);
            }
            Ar[4 * G + h] = ms4_of(wr[0] | (wr[1] << 16), wr[2]);
            Ai[4 * G + h] = ms4_of(wi[0] | (wi[1] << 16), wi[2]);
        }
    }
    float win[27];
#pragma unroll
    for (int e = 0; e < 27; e++) win[e] = 0.f;
    if constexpr (EPI != EPI_NONE)
        if (valid) load_window<P>(a.clov, Vh, site, q, win);

    // sign bits of e_j psi_perm(j) per direction (forward hop; the backward hop has the opposite sign):
    // x: e = -i, -i, +i, +i;  y: +1, -1, -1, +1;  z: -i, +i, +i, -i;  t: -1 for every spin
    const uint32_t sx = q < 2 ? SGN : 0u;                // sigma = -1 where e = -i (x)
    const uint32_t sy = (q == 1 || q == 2) ? SGN : 0u;  // sigma = -1 where e = -1 (y)
    const uint32_t sz = (q == 0 || q == 3) ? SGN : 0u;  // sigma = -1 where e = -i (z)
    const float xs = (float)g.xs;
    const uint32_t* psi = reinterpret_cast<const uint32_t*>(a.psi);

    // the lane's spin of the eight neighbours of right-hand side r (three colours, re/im interleaved)
    auto fetch = [&](int r, uint32_t (&d)[8][3]) {
        const uint32_t* base = psi + (long)r * field;
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const uint32_t* pp = base + nb[k];
            d[k][0] = pp[0];
            d[k][1] = pp[1];
            d[k][2] = pp[2];
        }
    };
    auto next_rhs = [&](int r) {  // uniform: every thread reads the same flags
        while (r < a.nrhs && S && S[r].flags) r++;
        return r;
    };
    auto compute = [&](int r, const uint32_t (&d)[8][3]) {
        const long off = (long)r * field;
        mf4 dr = {0.f, 0.f, 0.f, 0.f}, di = dr;
        // spatial directions first (x, y, then z), the sum scaled by the spatial weight, then t
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const int G = k >> 2, h = k & 3;
            if (k == 6) {
                dr *= xs;
                di *= xs;
            }
            const uint32_t d0 = d[k][0], d1 = d[k][1], d2 = d[k][2];
            // own spin: re and im planes of the three colours
            const uint32_t br0 = __builtin_amdgcn_perm(d1, d0, 0x05040100u), br1 = d2 & 0xffffu;
            const uint32_t bi0 = __builtin_amdgcn_perm(d1, d0, 0x07060302u), bi1 = d2 >> 16;
            // partner spin from the quad
            uint32_t pr0, pr1, pi0, pi1;
            if (G == 0) {
                pr0 = quad_dpp<0x1b>(br0);
                pr1 = quad_dpp<0x1b>(br1);
                pi0 = quad_dpp<0x1b>(bi0);
                pi1 = quad_dpp<0x1b>(bi1);
            } else {
                pr0 = quad_dpp<0x4e>(br0);
                pr1 = quad_dpp<0x4e>(br1);
                pi0 = quad_dpp<0x4e>(bi0);
                pi1 = quad_dpp<0x4e>(bi1);
            }
            const uint32_t flip = (h & 1) ? SGN : 0u;  // backward hop: -e
            ms4 b2r, b2i;
            if ((h >> 1) == 0) {  // x or z: e = i sigma, e psi = (-sigma psi_i, sigma psi_r)
                const uint32_t m = (G == 0 ? sx : sz) ^ flip;
                b2r = ms4_of(pi0 ^ m ^ SGN, pi1 ^ ((m ^ SGN) & 0xffffu));
                b2i = ms4_of(pr0 ^ m, pr1 ^ (m & 0xffffu));
            } else {  // y or t: e = sigma
                const uint32_t m = (G == 0 ? sy : SGN) ^ flip;
                b2r = ms4_of(pr0 ^ m, pr1 ^ (m & 0xffffu));
                b2i = ms4_of(pi0 ^ m, pi1 ^ (m & 0xffffu));
            }
            const ms4 b1r = ms4_of(br0, br1), b1i = ms4_of(bi0, bi1);
            const uint2 ai = __builtin_bit_cast(uint2, Ai[k]);
            const ms4 nai = ms4_of(ai.x ^ SGN, ai.y ^ SGN);
            dr = M::mma(Ar[k], b1r, dr);
            dr = M::mma(nai, b1i, dr);
            di = M::mma(Ar[k], b1i, di);
            di = M::mma(Ai[k], b1r, di);
            dr = M::mma(Ar[k], b2r, dr);
            dr = M::mma(nai, b2i, dr);
            di = M::mma(Ar[k], b2i, di);
            di = M::mma(Ai[k], b2r, di);
        }
        cx<float> res[3];
#pragma unroll
        for (int c = 0; c < 3; c++) res[c] = {dr[c], di[c]};
        cx<float> outv[3], yv[3];
        if constexpr (EPI == EPI_CLOV_XPAY || RED == RED_TS) {
#pragma unroll
            for (int c = 0; c < 3; c++) yv[c] = valid ? P::ld(a.y, off + sp_idx(q, site, c, Vh)) : cx<float>{0.f, 0.f};
        }
        if constexpr (EPI == EPI_NONE) {
#pragma unroll
            for (int c = 0; c < 3; c++) outv[c] = res[c];
        } else {
            cx<float> ox[3], br[3];
#pragma unroll
            for (int c = 0; c < 3; c++) ox[c] = quad_dpp_cx<QUAD_XOR1>(res[c]);
            herm_rows<true>(win, q & 1, res, ox, br);
            const float aa = (float)a.a;
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
                    const cx<float> o = outv[c];
                    if constexpr (RED == RED_WDOT) {
                        const cx<float> wv = P::ld(a.w, off + sp_idx(q, site, c, Vh));
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
    };

    // right-hand sides in a register double buffer: the neighbours of the next active RHS are in flight
    // while the current one is computed
    // (a register double buffer that fetches the next RHS during the current one was measured slower: the
    // extra 24 VGPRs cost a wave per SIMD)
    uint32_t da[8][3];
    for (int r = next_rhs(0); r < a.nrhs; r = next_rhs(r + 1)) {
        fetch(r, da);
        compute(r, da);
    }
}

template <class P>
static hipError_t launch_mrhs_mfma_p(hipStream_t s, int epi, int red, const HopArgs& a, const Scal* S, hipEvent_t e0,
                                     hipEvent_t e1)
{
    dim3 grid(a.cgroup > 0 ? hop_ctiles(a.g) * a.g.Lt : hop_blocks(a.g.Vh)), block(256);
#define QCDW_MRHS_CASE(E, D)                                                                          \
    if (epi == E && red == D) {                                                                      \
        if (e0)                                                                                      \
            hipExtLaunchKernelGGL((hop_mrhs_mfma_kernel<P, E, D>), grid, block, 0, s, e0, e1, 0, a, S); \
        else                                                                                         \
            hipLaunchKernelGGL((hop_mrhs_mfma_kernel<P, E, D>), grid, block, 0, s, a, S);             \
        return hipGetLastError();                                                                    \
    }
    QCDW_MRHS_CASE(EPI_CLOV, RED_NONE)
    QCDW_MRHS_CASE(EPI_CLOV_XPAY, RED_NONE)
    QCDW_MRHS_CASE(EPI_CLOV_XPAY, RED_WDOT)
    QCDW_MRHS_CASE(EPI_CLOV_XPAY, RED_TS)
#undef QCDW_MRHS_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_hop_mrhs_mfma(hipStream_t s, int prec, int epi, int red, const HopArgs& a, const Scal* S,
                                hipEvent_t e0, hipEvent_t e1)
{
    if (a.g.Vh <= 0 || a.nrhs <= 0) return hipSuccess;
    if (12L * a.g.Vh > 0x7fffffffL) return hipErrorInvalidValue;  // 32-bit neighbour offsets
    switch (prec) {
    case BF16: return launch_mrhs_mfma_p<PBF16>(s, epi, red, a, S, e0, e1);
    case F16: return launch_mrhs_mfma_p<PF16>(s, epi, red, a, S, e0, e1);
    }
    return hipErrorInvalidValue;  // FP64 and FP32 storage use the vector forms
}

}  // namespace qcdw
