// Kernels of the learned gauge-covariant preconditioner (the published idea of
// gauge-equivariant convolutions: Favoni et al. 2022, Lehner and Wettig 2023;
// the paper's own accelerator for clover solves is multigrid, Sec. II.E).
//
// A layer maps CIN channels phi_c (colour 3-vector fields on the full lattice)
// to COUT channels:  out_{c'}(x) = sum_a sum_c W_a[c', c] (T_a phi_c)(x),
// a in {0, +-mu}: T_0 = 1, (T_{+mu} phi)(x) = U_mu(x) phi(x+mu),
// (T_{-mu} phi)(x) = U_mu(x-mu)^+ phi(x-mu).  Hop index a = 1 + 2 mu + back.
// Activation layout [parity][channel][Vh][3] complex: with 4 channels it is two
// internal spinor fields (even, odd), so spins are the input/output channels.
// Links: the operator's reconstruct-12 internal layout, FP32.  Arithmetic FP32.
#include "internal.h"

namespace qcdw {

struct NetArgs {
    const void* in;
    void* out;
    const void* gauge;  // reconstruct-12 links in FP32, in the layout of the FP64 links (link_base, link_stride)
    const float2* W;    // [9][COUT][CIN]
    Geom g;
};

// link (mu, p, site) of an FP32 reconstruct-12 internal gauge field (two rows stored)
__device__ __forceinline__ void su3_row3(const void* gauge, int mu, int p, int site, long Vh, cx<float> (&u)[9])
{
    constexpr bool soa = link_soa_for(P64::cbytes);  // an element-wise FP32 copy of the operator's FP64 links
    const long off = link_base(mu, p, site, Vh, 6, soa), st = link_stride(Vh, soa);
#pragma unroll
    for (int e = 0; e < 6; e++) u[e] = P32::ld(gauge, off + e * st);
    u[6] = conj(u[1] * u[5] - u[2] * u[4]);
    u[7] = conj(u[2] * u[3] - u[0] * u[5]);
    u[8] = conj(u[0] * u[4] - u[1] * u[3]);
}

// neighbour (parity 1 - p) of site i of parity p one step along mu (dir 0 forward, 1 backward)
__device__ __forceinline__ int nbr_index(const Geom& g, int i, int x, int y, int z, int t, int mu, int dir)
{
    const int xh = i % g.Lxh;
    switch (mu) {
    case 0: {
        const int row = i - xh;
        const int xn = dir == 0 ? ((x + 1 == g.Lx) ? 0 : x + 1) : ((x == 0) ? g.Lx - 1 : x - 1);
        return row + (xn >> 1);
    }
    case 1: {
        const int S = g.Lxh;
        return dir == 0 ? ((y + 1 == g.Ly) ? i - (g.Ly - 1) * S : i + S) : ((y == 0) ? i + (g.Ly - 1) * S : i - S);
    }
    case 2: {
        const int S = g.Lxh * g.Ly;
        return dir == 0 ? ((z + 1 == g.Lz) ? i - (g.Lz - 1) * S : i + S) : ((z == 0) ? i + (g.Lz - 1) * S : i - S);
    }
    default: {
        const int S = g.Lxh * g.Ly * g.Lz;
        return dir == 0 ? ((t + 1 == g.Lt) ? i - (g.Lt - 1) * S : i + S) : ((t == 0) ? i + (g.Lt - 1) * S : i - S);
    }
    }
}

// Y[c] = (T_a phi_c)(x) for the site (p, i)
template <class PI, int CIN>
__device__ __forceinline__ void transport(const void* in, const void* gauge, const Geom& g, int p, int i, int x,
                                          int y, int z, int t, int a, cx<float> (&Y)[CIN][3])
{
    const long Vh = g.Vh;
    if (a == 0) {
#pragma unroll
        for (int c = 0; c < CIN; c++)
#pragma unroll
            for (int k = 0; k < 3; k++) {
                const auto v = PI::ld(in, sp_idx((long)p * CIN + c, i, k, Vh));
                Y[c][k] = {(float)v.re, (float)v.im};
            }
        return;
    }
    const int mu = (a - 1) >> 1, back = (a - 1) & 1;
    const int j = nbr_index(g, i, x, y, z, t, mu, back);
    cx<float> u[9];
    su3_row3(gauge, mu, back == 0 ? p : 1 - p, back == 0 ? i : j, Vh, u);
#pragma unroll
    for (int c = 0; c < CIN; c++) {
        cx<float> v[3];
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const auto w = PI::ld(in, sp_idx((long)(1 - p) * CIN + c, j, k, Vh));
            v[k] = {(float)w.re, (float)w.im};
        }
#pragma unroll
        for (int r = 0; r < 3; r++) {
            cx<float> s = {0.f, 0.f};
#pragma unroll
            for (int k = 0; k < 3; k++) s = back == 0 ? s + u[3 * r + k] * v[k] : s + cmul_conj(u[3 * k + r], v[k]);
            Y[c][r] = s;
        }
    }
}

typedef float mfma_f4 __attribute__((ext_vector_type(4)));
typedef short mfma_s4 __attribute__((ext_vector_type(4)));

// two floats rounded to BF16 (nearest even) and packed low, high
__device__ __forceinline__ uint32_t pk_bf16(float lo, float hi)
{
    return __builtin_bit_cast(uint32_t, f2bf2(lo, hi));
}
__device__ __forceinline__ mfma_s4 s4_of(uint32_t lo, uint32_t hi) { return __builtin_bit_cast(mfma_s4, make_uint2(lo, hi)); }

// The layers with their channel mixing on the matrix cores in BF16 (v_mfma_f32_16x16x16_bf16, FP32
// accumulation): the application path of the preconditioner.  For each colour k the mixing of hop a is the
// real product  D[m][n] = sum_kk A[m][kk] B[kk][n]  with the weights as A (rows m = 2 d + re/im of output
// channel d; K: kk = 2 c + re/im of input channel c; the real form [[Re W, -Im W], [Im W, Re W]]) and the
// sites of a wave as the 16 columns n.  The instruction takes A[m][kk] from lane m + 16 (kk / 4) and B[kk][n]
// from lane n + 16 (kk / 4), elements kk % 4, 16 kk per step, and leaves D[m][n] in lane n + 16 (m / 4),
// element m % 4: lane L = n + 16 g supplies input channels 2 g, 2 g + 1 (+ 8 per step) of site n and
// receives output channels 2 g, 2 g + 1 (+ 8 per row tile) of the same site, as whole complex numbers.
// Two orders of the same sum, chosen by the cheaper transport: CIN <= COUT transports the CIN inputs first
// (B = T_a phi, one accumulator over all hops); CIN > COUT mixes the neighbour's raw inputs first
// (B = phi(x + a), the 16-bit inputs taken as they are stored) and transports the COUT mixed channels.

// A operand of hop a, row tile t, K step s for this lane
template <int CIN, int COUT>
__device__ __forceinline__ mfma_s4 net_wop(const float2* __restrict__ W, int a, int t, int s, int lane)
{
    const int m = 16 * t + (lane & 15), d = m >> 1, rho = m & 1, grp = lane >> 4;
    uint32_t v[2];
#pragma unroll
    for (int h = 0; h < 2; h++) {
        const int c = 8 * s + 2 * grp + h;
        float x = 0.f, y = 0.f;
        if (d < COUT && c < CIN) {
            const float2 w = W[((long)a * COUT + d) * CIN + c];
            x = rho ? w.y : w.x;   // row re: (Re W, -Im W); row im: (Im W, Re W)
            y = rho ? w.x : -w.y;
        }
        v[h] = pk_bf16(x, y);
    }
    return s4_of(v[0], v[1]);
}

// B operand dword of input channel c (colour k) of site (p, i): a 16-bit complex as stored, or FP32 rounded
template <class PI>
__device__ __forceinline__ uint32_t net_in_bits(const void* in, long idx)
{
    if constexpr (PI::cbytes == 4) {
        return reinterpret_cast<const uint32_t*>(in)[idx];
    } else {
        const auto v = PI::ld(in, idx);
        return pk_bf16((float)v.re, (float)v.im);
    }
}

// W v with W = U (forward hop) or U^+ (backward hop)
__device__ __forceinline__ void net_link_mul(const cx<float> (&u)[9], int back, const cx<float> (&v)[3],
                                             cx<float> (&y)[3])
{
#pragma unroll
    for (int r = 0; r < 3; r++) {
        cx<float> sacc = {0.f, 0.f};
#pragma unroll
        for (int k = 0; k < 3; k++) sacc = back == 0 ? sacc + u[3 * r + k] * v[k] : sacc + cmul_conj(u[3 * k + r], v[k]);
        y[r] = sacc;
    }
}

template <class PI, class PO, int CIN, int COUT>
__global__ __launch_bounds__(256) void k_net_layer_mfma(NetArgs n)
{
    constexpr int NT = (2 * COUT + 15) / 16;  // row tiles of the output channels
    constexpr int NS = (2 * CIN + 15) / 16;   // K steps over the input channels
    constexpr bool TFIRST = CIN <= COUT;
    const Geom g = n.g;
    const long Vh = g.Vh;
    const int lane = threadIdx.x & 63, grp = lane >> 4;
    // the weight operands of every (hop, row tile, K step) for the 64 lane positions, built once per block
    __shared__ uint2 wop[9 * NT * NS][64];
    for (int e = threadIdx.x; e < 9 * NT * NS * 64; e += 256) {
        const int l = e & 63, q = e >> 6, s2 = q % NS, tl = (q / NS) % NT, a = q / (NS * NT);
        wop[q][l] = __builtin_bit_cast(uint2, net_wop<CIN, COUT>(n.W, a, tl, s2, l));
    }
    __syncthreads();
    const long wave = ((long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long gsite = wave * 16 + (lane & 15);
    const bool valid = gsite < 2 * Vh;  // other lanes compute on site 0 and store nothing
    const int p = valid ? (int)(gsite / Vh) : 0, i = valid ? (int)(gsite % Vh) : 0;
    int x, y, z, t;
    site_coords(g, i, p, x, y, z, t);
    using TO = typename PO::real;
    if constexpr (TFIRST) {
        mfma_f4 acc[3][NT];
#pragma unroll
        for (int k = 0; k < 3; k++)
#pragma unroll
            for (int tl = 0; tl < NT; tl++) acc[k][tl] = mfma_f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int a = 0; a < 9; a++) {
            const int mu = (a - 1) >> 1, back = (a - 1) & 1;
            const int j = a == 0 ? i : nbr_index(g, i, x, y, z, t, mu, back);
            const int pj = a == 0 ? p : 1 - p;
            cx<float> u[9];
            const bool link = a > 0 && 2 * grp < CIN;
            if (link) su3_row3(n.gauge, mu, back == 0 ? p : 1 - p, back == 0 ? i : j, Vh, u);
            mfma_s4 B[NS][3];
#pragma unroll
            for (int s2 = 0; s2 < NS; s2++) {
                const int c0 = 8 * s2 + 2 * grp;
                uint32_t bw[2][3];
#pragma unroll
                for (int h = 0; h < 2; h++) {
                    const int c = c0 + h;
                    cx<float> v[3], yv[3] = {{0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}};
                    if (c < CIN) {  // (u is loaded only by lanes with input channels)
#pragma unroll
                        for (int k = 0; k < 3; k++) {
                            const auto w = PI::ld(n.in, sp_idx((long)pj * CIN + c, j, k, Vh));
                            v[k] = {(float)w.re, (float)w.im};
                        }
                        if (a > 0)
                            net_link_mul(u, back, v, yv);
                        else
#pragma unroll
                            for (int k = 0; k < 3; k++) yv[k] = v[k];
                    }
#pragma unroll
                    for (int k = 0; k < 3; k++) bw[h][k] = pk_bf16(yv[k].re, yv[k].im);
                }
#pragma unroll
                for (int k = 0; k < 3; k++) B[s2][k] = s4_of(bw[0][k], bw[1][k]);
            }
#pragma unroll
            for (int tl = 0; tl < NT; tl++)
#pragma unroll
                for (int s2 = 0; s2 < NS; s2++) {
                    const mfma_s4 A = __builtin_bit_cast(mfma_s4, wop[(a * NT + tl) * NS + s2][lane]);
#pragma unroll
                    for (int k = 0; k < 3; k++)
                        acc[k][tl] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, B[s2][k], acc[k][tl], 0, 0, 0);
                }
        }
#pragma unroll
        for (int tl = 0; tl < NT; tl++)
#pragma unroll
            for (int h = 0; h < 2; h++) {
                const int d = 8 * tl + 2 * grp + h;
                if (valid && d < COUT) {
#pragma unroll
                    for (int k = 0; k < 3; k++)
                        PO::st(n.out, sp_idx((long)p * COUT + d, i, k, Vh),
                               cx<TO>{(TO)acc[k][tl][2 * h], (TO)acc[k][tl][2 * h + 1]});
                }
            }
    } else {
        static_assert(NT == 1, "the mix-first order keeps one row tile");
        cx<float> o[2][3];
#pragma unroll
        for (int h = 0; h < 2; h++)
#pragma unroll
            for (int k = 0; k < 3; k++) o[h][k] = {0.f, 0.f};
#pragma unroll
        for (int a = 0; a < 9; a++) {
            const int mu = (a - 1) >> 1, back = (a - 1) & 1;
            const int j = a == 0 ? i : nbr_index(g, i, x, y, z, t, mu, back);
            const int pj = a == 0 ? p : 1 - p;
            cx<float> u[9];
            if (a > 0 && 2 * grp < COUT) su3_row3(n.gauge, mu, back == 0 ? p : 1 - p, back == 0 ? i : j, Vh, u);
            mfma_f4 acc[3];
#pragma unroll
            for (int k = 0; k < 3; k++) acc[k] = mfma_f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s2 = 0; s2 < NS; s2++) {
                const int c0 = 8 * s2 + 2 * grp;
                mfma_s4 B[3];
#pragma unroll
                for (int k = 0; k < 3; k++) {
                    const uint32_t b0 = c0 < CIN ? net_in_bits<PI>(n.in, sp_idx((long)pj * CIN + c0, j, k, Vh)) : 0u;
                    const uint32_t b1 =
                        c0 + 1 < CIN ? net_in_bits<PI>(n.in, sp_idx((long)pj * CIN + c0 + 1, j, k, Vh)) : 0u;
                    B[k] = s4_of(b0, b1);
                }
                const mfma_s4 A = __builtin_bit_cast(mfma_s4, wop[a * NS + s2][lane]);
#pragma unroll
                for (int k = 0; k < 3; k++) acc[k] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, B[k], acc[k], 0, 0, 0);
            }
            // this lane's mixed channels d = 2 grp + h of the neighbour, then their transport
            if (2 * grp < COUT) {
#pragma unroll
                for (int h = 0; h < 2; h++) {
                    cx<float> v[3], yv[3];
#pragma unroll
                    for (int k = 0; k < 3; k++) v[k] = {acc[k][2 * h], acc[k][2 * h + 1]};
                    if (a > 0)
                        net_link_mul(u, back, v, yv);
                    else
#pragma unroll
                        for (int k = 0; k < 3; k++) yv[k] = v[k];
#pragma unroll
                    for (int k = 0; k < 3; k++) o[h][k] = o[h][k] + yv[k];
                }
            }
        }
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const int d = 2 * grp + h;
            if (valid && d < COUT) {
#pragma unroll
                for (int k = 0; k < 3; k++)
                    PO::st(n.out, sp_idx((long)p * COUT + d, i, k, Vh), cx<TO>{(TO)o[h][k].re, (TO)o[h][k].im});
            }
        }
    }
}

template <class PI, class PO, int CIN, int COUT>
__global__ __launch_bounds__(256) void k_net_layer(NetArgs n)
{
    const Geom g = n.g;
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= 2L * g.Vh) return;
    const int p = (int)(gid / g.Vh), i = (int)(gid % g.Vh);
    int x, y, z, t;
    site_coords(g, i, p, x, y, z, t);
    cx<float> acc[COUT][3];
#pragma unroll
    for (int d = 0; d < COUT; d++)
#pragma unroll
        for (int k = 0; k < 3; k++) acc[d][k] = {0.f, 0.f};
    for (int a = 0; a < 9; a++) {
        cx<float> Y[CIN][3];
        transport<PI, CIN>(n.in, n.gauge, g, p, i, x, y, z, t, a, Y);
        const float2* Wa = n.W + (long)a * COUT * CIN;
#pragma unroll
        for (int d = 0; d < COUT; d++)
#pragma unroll
            for (int c = 0; c < CIN; c++) {
                const float2 w = Wa[d * CIN + c];
                const cx<float> wc = {w.x, w.y};
#pragma unroll
                for (int k = 0; k < 3; k++) acc[d][k] = acc[d][k] + wc * Y[c][k];
            }
    }
    using TO = typename PO::real;
#pragma unroll
    for (int d = 0; d < COUT; d++)
#pragma unroll
        for (int k = 0; k < 3; k++)
            PO::st(n.out, sp_idx((long)p * COUT + d, i, k, g.Vh), cx<TO>{(TO)acc[d][k].re, (TO)acc[d][k].im});
}

// per-block partials of G_a[c', c] = sum_x sum_k g_{c'}(x)_k conj((T_a phi_c)(x)_k), one hop a per launch;
// reduced one output channel at a time to bound register use
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_net_wgrad(const void* phi, const void* gz, const void* gauge, Geom g, int a,
                                                   double* partials)
{
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = gid < 2L * g.Vh;
    const int p = valid ? (int)(gid / g.Vh) : 0, i = valid ? (int)(gid % g.Vh) : 0;
    cx<float> Y[CIN][3];
    if (valid) {
        int x, y, z, t;
        site_coords(g, i, p, x, y, z, t);
        transport<P32, CIN>(phi, gauge, g, p, i, x, y, z, t, a, Y);
    } else {
#pragma unroll
        for (int c = 0; c < CIN; c++)
#pragma unroll
            for (int k = 0; k < 3; k++) Y[c][k] = {0.f, 0.f};
    }
    double* base = partials + (long)blockIdx.x * 2 * CIN * COUT;
    for (int d = 0; d < COUT; d++) {
        cx<float> gd[3];
#pragma unroll
        for (int k = 0; k < 3; k++)
            gd[k] = valid ? P32::ld(gz, sp_idx((long)p * COUT + d, i, k, g.Vh)) : cx<float>{0.f, 0.f};
        double v[2 * CIN];
#pragma unroll
        for (int c = 0; c < CIN; c++) {
            cx<float> s = {0.f, 0.f};
#pragma unroll
            for (int k = 0; k < 3; k++) s = s + cmul_conj(Y[c][k], gd[k]);  // g conj(Y)
            v[2 * c] = s.re;
            v[2 * c + 1] = s.im;
        }
        block_sum_store<2 * CIN>(v, base + 2 * CIN * d);
        __syncthreads();  // the block reduction's shared buffer is reused for the next channel
    }
}

// out[e] (+)= sum over nb blocks of partials[b][e], e < K; one block per 64 entries
__global__ __launch_bounds__(256) void k_sum_columns(const double* partials, int nb, int K, double* out, int accumulate)
{
    const int e = blockIdx.x;
    if (e >= K) return;
    double v[1] = {0.0};
    for (int b = threadIdx.x; b < nb; b += 256) v[0] += partials[(long)b * K + e];
    __shared__ double res[1];
    block_sum_store<1>(v, res);
    __syncthreads();
    if (threadIdx.x == 0) out[e] = accumulate ? out[e] + res[0] : res[0];
}

// Wt[a'][c][d] = conj(W[a][d][c]), a' the reversed hop (T_a^+ = T_a'), for the adjoint layer
__global__ void k_net_adjoint_w(const float2* W, float2* Wt, int cout, int cin)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 9 * cout * cin) return;
    const int a = e / (cout * cin), r = e % (cout * cin), d = r / cin, c = r % cin;
    const int at = a == 0 ? 0 : (((a - 1) & 1) ? a - 1 : a + 1);
    const float2 w = W[e];
    Wt[(long)at * cin * cout + c * cout + d] = make_float2(w.x, -w.y);
}

// gz = coef * (FP64 even field) on even sites, zero on odd sites (4 channels)
__global__ void k_net_make_gz(const double2* diff, float2* gz, long n_half, double coef)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 2 * n_half) return;
    if (e < n_half) {
        const double2 d = diff[e];
        gz[e] = make_float2((float)(coef * d.x), (float)(coef * d.y));
    } else {
        gz[e] = make_float2(0.f, 0.f);
    }
}

// Adam (Kingma and Ba 2015) on the real and imaginary parts of the weights
__global__ void k_adam(float* W, const double* G, double* m, double* v, int n, double lr, double b1, double b2,
                       double eps, int step, double gscale)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const double g = G[e] * gscale;
    m[e] = b1 * m[e] + (1.0 - b1) * g;
    v[e] = b2 * v[e] + (1.0 - b2) * g * g;
    const double mh = m[e] / (1.0 - pow(b1, (double)step));
    const double vh = v[e] / (1.0 - pow(b2, (double)step));
    W[e] = (float)((double)W[e] - lr * mh / (sqrt(vh) + eps));
}

// Gaussian complex entries (re, im ~ N(0,1)) from a counter-based generator:
// splitmix64 of (seed, stream, element) feeds a Box-Muller transform, so the
// field depends only on (seed, stream), not on the launch shape.
__device__ __forceinline__ uint64_t splitmix64(uint64_t z)
{
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__global__ void k_gaussian(double2* out, long n, uint64_t seed, uint64_t stream)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const uint64_t k = splitmix64(seed ^ splitmix64(stream ^ splitmix64((uint64_t)e)));
    const uint64_t k2 = splitmix64(k);
    const double u1 = ((k >> 11) + 1.0) * (1.0 / 9007199254740993.0);  // (0, 1]
    const double u2 = (k2 >> 11) * (1.0 / 9007199254740992.0);          // [0, 1)
    const double rad = sqrt(-2.0 * log(u1)), th = 6.283185307179586 * u2;
    out[e] = make_double2(rad * cos(th), rad * sin(th));
}

static inline dim3 g256(long n) { return dim3((unsigned)((n + 255) / 256)); }

hipError_t launch_gaussian(hipStream_t s, void* out, long n, uint64_t seed, uint64_t stream)
{
    hipLaunchKernelGGL(k_gaussian, g256(n), dim3(256), 0, s, (double2*)out, n, seed, stream);
    return hipGetLastError();
}

hipError_t launch_net_layer(hipStream_t s, int pin, int pout, int cin, int cout, const void* in, void* out,
                            const void* gauge32, const void* W, const Geom& g, int mfma)
{
    NetArgs n{in, out, gauge32, (const float2*)W, g};
    const dim3 grid = g256(2L * g.Vh);
    const dim3 grid_mfma((unsigned)((2L * g.Vh + 63) / 64));  // 16 sites per wave, 4 waves per block
    // layers with a BF16 end (the preconditioner's application) mix channels on the matrix cores
#define QCDW_NET_MFMA_CASE(PI, PO, CI, CO, pi, po)                                                \
    if (pin == pi && pout == po && cin == CI && cout == CO) {                                     \
        hipLaunchKernelGGL((k_net_layer_mfma<PI, PO, CI, CO>), grid_mfma, dim3(256), 0, s, n);     \
        return hipGetLastError();                                                                 \
    }
#define QCDW_NET_CASE(PI, PO, CI, CO, pi, po)                                              \
    if (pin == pi && pout == po && cin == CI && cout == CO) {                              \
        hipLaunchKernelGGL((k_net_layer<PI, PO, CI, CO>), grid, dim3(256), 0, s, n);        \
        return hipGetLastError();                                                          \
    }
    if (mfma) {
        QCDW_NET_MFMA_CASE(P32, PBF16, 4, 12, F32, BF16)
        QCDW_NET_MFMA_CASE(PBF16, P32, 12, 4, BF16, F32)
        QCDW_NET_MFMA_CASE(P32, PBF16, 4, 4, F32, BF16)
        QCDW_NET_MFMA_CASE(PBF16, P32, 4, 4, BF16, F32)
    }
    QCDW_NET_CASE(P32, P32, 4, 12, F32, F32)
    QCDW_NET_CASE(P32, P32, 12, 4, F32, F32)
    QCDW_NET_CASE(P32, PBF16, 4, 12, F32, BF16)
    QCDW_NET_CASE(PBF16, P32, 12, 4, BF16, F32)
    QCDW_NET_CASE(P32, P32, 4, 4, F32, F32)
    QCDW_NET_CASE(P32, PBF16, 4, 4, F32, BF16)
    QCDW_NET_CASE(PBF16, P32, 4, 4, BF16, F32)
#undef QCDW_NET_CASE
#undef QCDW_NET_MFMA_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_net_wgrad(hipStream_t s, int cin, int cout, const void* phi, const void* gz, const void* gauge32,
                            const Geom& g, int a, double* partials, double* out, int accumulate)
{
    const dim3 grid = g256(2L * g.Vh);
    const int K = 2 * cin * cout;
    if (cin == 4 && cout == 12)
        hipLaunchKernelGGL((k_net_wgrad<4, 12>), grid, dim3(256), 0, s, phi, gz, gauge32, g, a, partials);
    else if (cin == 12 && cout == 4)
        hipLaunchKernelGGL((k_net_wgrad<12, 4>), grid, dim3(256), 0, s, phi, gz, gauge32, g, a, partials);
    else if (cin == 4 && cout == 4)
        hipLaunchKernelGGL((k_net_wgrad<4, 4>), grid, dim3(256), 0, s, phi, gz, gauge32, g, a, partials);
    else
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sum_columns, dim3(K), dim3(256), 0, s, partials, (int)grid.x, K, out, accumulate);
    return hipGetLastError();
}

hipError_t launch_net_adjoint_w(hipStream_t s, const void* W, void* Wt, int cout, int cin)
{
    hipLaunchKernelGGL(k_net_adjoint_w, g256(9L * cout * cin), dim3(256), 0, s, (const float2*)W, (float2*)Wt, cout,
                       cin);
    return hipGetLastError();
}

hipError_t launch_net_make_gz(hipStream_t s, const void* diff, void* gz, long n_half, double coef)
{
    hipLaunchKernelGGL(k_net_make_gz, g256(2 * n_half), dim3(256), 0, s, (const double2*)diff, (float2*)gz, n_half,
                       coef);
    return hipGetLastError();
}

hipError_t launch_adam(hipStream_t s, void* W, const double* G, double* m, double* v, int n, double lr, double b1,
                       double b2, double eps, int step, double gscale)
{
    hipLaunchKernelGGL(k_adam, g256(n), dim3(256), 0, s, (float*)W, G, m, v, n, lr, b1, b2, eps, step, gscale);
    return hipGetLastError();
}

}  // namespace qcdw
