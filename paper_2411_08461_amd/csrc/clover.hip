// Clover term kernels on the paper layouts (FP64):
//   build  : C(x) = sum_{mu<nu} sigma_{mu nu} F_{mu nu}(x)     (Sec. III.B, Eq. "clover")
//   apply  : out = (1 - kappa csw C) psi
//   invert : (1 - kappa csw C)^-1 per chirality block, by Cholesky
//   to_A   : packed A = 1 - kappa csw C (for the full-operator epilogue)
// Packed clover per site and chirality (Sec. II.A): 6 real diagonal entries,
// then the 15 strictly-lower complex entries in row-major order; block index
// j = 3 * (spin % 2) + colour, chirality 0 = spins {0,1}, 1 = spins {2,3}.
#include "internal.h"

namespace qcdw {

using cd = cx<double>;

struct M3 {
    cd m[9];
};

__device__ __forceinline__ M3 ld_link(const double2* U, long Vh, int mu, int parity, int site)
{
    M3 r;
    const double2* p = U + (((long)mu * 2 + parity) * Vh + site) * 9;
#pragma unroll
    for (int e = 0; e < 9; e++) r.m[e] = {p[e].x, p[e].y};
    return r;
}

__device__ __forceinline__ M3 mul(const M3& a, const M3& b)
{
    M3 r;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            cd s = a.m[3 * i] * b.m[j];
            s = s + a.m[3 * i + 1] * b.m[3 + j];
            s = s + a.m[3 * i + 2] * b.m[6 + j];
            r.m[3 * i + j] = s;
        }
    return r;
}

// a * b^+
__device__ __forceinline__ M3 mul_nd(const M3& a, const M3& b)
{
    M3 r;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            cd s = a.m[3 * i] * conj(b.m[3 * j]);
            s = s + a.m[3 * i + 1] * conj(b.m[3 * j + 1]);
            s = s + a.m[3 * i + 2] * conj(b.m[3 * j + 2]);
            r.m[3 * i + j] = s;
        }
    return r;
}

// a^+ * b
__device__ __forceinline__ M3 mul_dn(const M3& a, const M3& b)
{
    M3 r;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            cd s = cmul_conj(a.m[i], b.m[j]);
            s = s + cmul_conj(a.m[3 + i], b.m[3 + j]);
            s = s + cmul_conj(a.m[6 + i], b.m[6 + j]);
            r.m[3 * i + j] = s;
        }
    return r;
}

__device__ __forceinline__ void site_index_of(const Geom& g, const int (&c)[4], int& parity, int& cb)
{
    parity = (c[0] + c[1] + c[2] + c[3]) & 1;
    cb = ((c[3] * g.Lz + c[2]) * g.Ly + c[1]) * g.Lxh + (c[0] >> 1);
}

__device__ __forceinline__ M3 link_at(const double2* U, const Geom& g, int mu, const int (&c)[4])
{
    int par, cb;
    site_index_of(g, c, par, cb);
    return ld_link(U, g.Vh, mu, par, cb);
}

__device__ __forceinline__ void shifted(const Geom& g, const int (&c)[4], int mu, int dmu, int nu, int dnu,
                                        int (&o)[4])
{
    const int L[4] = {g.Lx, g.Ly, g.Lz, g.Lt};
#pragma unroll
    for (int i = 0; i < 4; i++) o[i] = c[i];
    o[mu] = (o[mu] + dmu + L[mu]) % L[mu];
    o[nu] = (o[nu] + dnu + L[nu]) % L[nu];
}

// F_{mu nu}(x): traceless part of (Q - Q^+)/8, Q = sum of the four
// counter-clockwise plaquettes in the (mu, nu) plane that touch x.
__device__ M3 field_strength(const double2* U, const Geom& g, const int (&c)[4], int mu, int nu)
{
    int xpm[4], xpn[4], xmm[4], xmn[4], xmm_pn[4], xmm_mn[4], xpm_mn[4];
    shifted(g, c, mu, 1, nu, 0, xpm);
    shifted(g, c, mu, 0, nu, 1, xpn);
    shifted(g, c, mu, -1, nu, 0, xmm);
    shifted(g, c, mu, 0, nu, -1, xmn);
    shifted(g, c, mu, -1, nu, 1, xmm_pn);
    shifted(g, c, mu, -1, nu, -1, xmm_mn);
    shifted(g, c, mu, 1, nu, -1, xpm_mn);

    const M3 umu_x = link_at(U, g, mu, c);
    const M3 unu_x = link_at(U, g, nu, c);
    // upper-right leaf: U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
    M3 q = mul_nd(mul_nd(mul(umu_x, link_at(U, g, nu, xpm)), link_at(U, g, mu, xpn)), unu_x);
    // upper-left leaf: U_nu(x) U_mu(x-mu+nu)^+ U_nu(x-mu)^+ U_mu(x-mu)
    const M3 umu_xmm = link_at(U, g, mu, xmm);
    M3 l2 = mul(mul_nd(mul_nd(unu_x, link_at(U, g, mu, xmm_pn)), link_at(U, g, nu, xmm)), umu_xmm);
    // lower-left leaf: U_mu(x-mu)^+ U_nu(x-mu-nu)^+ U_mu(x-mu-nu) U_nu(x-nu)
    const M3 unu_xmn = link_at(U, g, nu, xmn);
    const M3 l3a = mul_dn(link_at(U, g, nu, xmm_mn), link_at(U, g, mu, xmm_mn));  // U_nu(x-mu-nu)^+ U_mu(x-mu-nu)
    const M3 l3 = mul(mul_dn(umu_xmm, l3a), unu_xmn);
    // lower-right leaf: U_nu(x-nu)^+ U_mu(x-nu) U_nu(x+mu-nu) U_mu(x)^+
    M3 l4 = mul_nd(mul(mul_dn(unu_xmn, link_at(U, g, mu, xmn)), link_at(U, g, nu, xpm_mn)), umu_x);
#pragma unroll
    for (int e = 0; e < 9; e++) q.m[e] = q.m[e] + l2.m[e] + l3.m[e] + l4.m[e];
    M3 f;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) f.m[3 * i + j] = 0.125 * (q.m[3 * i + j] - conj(q.m[3 * j + i]));
    const cd tr = (1.0 / 3.0) * (f.m[0] + f.m[4] + f.m[8]);
    f.m[0] = f.m[0] - tr;
    f.m[4] = f.m[4] - tr;
    f.m[8] = f.m[8] - tr;
    return f;
}

// In the DeGrand-Rossi basis sigma_{mu nu} = [g_mu, g_nu]/2 is block-diagonal
// in chirality; its 2x2 spin blocks give, with F_{mu nu} (mu, nu = 0..3):
//   upper (spins 0,1): B00 = -iF01 + iF23   B11 = iF01 - iF23
//                      B01 = -F02 + iF03 - iF12 - F13   B10 = F02 + iF03 - iF12 + F13
//   lower (spins 2,3): B00 = -iF01 - iF23   B11 = iF01 + iF23
//                      B01 = -F02 - iF03 - iF12 + F13   B10 = F02 - iF03 - iF12 - F13
// and the 6x6 chirality block is [[B00, B01], [B10, B11]] in colour-inner order.
// wt weights the planes (i, t) and ws the spatial planes (the anisotropic action of Sec. III.B:
// wt = c_SW^t, ws = c_SW^r / xi_0; 1 and 1 for the isotropic C).
__device__ __forceinline__ M3 scaled(M3 f, double w)
{
#pragma unroll
    for (int e = 0; e < 9; e++) f.m[e] = {w * f.m[e].re, w * f.m[e].im};
    return f;
}

__global__ void k_clover_build(const double2* __restrict__ U, double* __restrict__ clover, Geom g, double wt,
                               double ws)
{
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= 2L * g.Vh) return;
    const int parity = (int)(gid / g.Vh), site = (int)(gid % g.Vh);
    int c[4];
    site_coords(g, site, parity, c[0], c[1], c[2], c[3]);
    const M3 F01 = scaled(field_strength(U, g, c, 0, 1), ws), F02 = scaled(field_strength(U, g, c, 0, 2), ws),
             F03 = scaled(field_strength(U, g, c, 0, 3), wt), F12 = scaled(field_strength(U, g, c, 1, 2), ws),
             F13 = scaled(field_strength(U, g, c, 1, 3), wt), F23 = scaled(field_strength(U, g, c, 2, 3), wt);
    const cd I = {0.0, 1.0};
    double* out = clover + gid * 72;
#pragma unroll
    for (int chi = 0; chi < 2; chi++) {
        const double s = chi == 0 ? 1.0 : -1.0;  // sign of the time-plane terms
        cd B[6][6];
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int b = 0; b < 3; b++) {
                const int e = 3 * a + b;
                const cd f01 = F01.m[e], f02 = F02.m[e], f03 = F03.m[e], f12 = F12.m[e], f13 = F13.m[e],
                         f23 = F23.m[e];
                B[a][b] = I * (s * f23 - f01);
                B[3 + a][3 + b] = I * (f01 - s * f23);
                B[a][3 + b] = ((-s) * f13 - f02) + I * (s * f03 - f12);
                B[3 + a][b] = (f02 + s * f13) + I * (s * f03 - f12);
            }
        double* o = out + chi * 36;
#pragma unroll
        for (int j = 0; j < 6; j++) o[j] = B[j][j].re;
        int slot = 0;
#pragma unroll
        for (int j = 1; j < 6; j++)
#pragma unroll
            for (int k = 0; k < j; k++) {
                o[6 + 2 * slot] = B[j][k].re;
                o[7 + 2 * slot] = B[j][k].im;
                slot++;
            }
    }
}

__device__ __forceinline__ void unpack6(const double* p, cd (&B)[6][6])
{
#pragma unroll
    for (int j = 0; j < 6; j++) B[j][j] = {p[j], 0.0};
    int slot = 0;
#pragma unroll
    for (int j = 1; j < 6; j++)
#pragma unroll
        for (int k = 0; k < j; k++) {
            B[j][k] = {p[6 + 2 * slot], p[7 + 2 * slot]};
            B[k][j] = conj(B[j][k]);
            slot++;
        }
}

__global__ void k_clover_apply(const double* __restrict__ clover, const double2* __restrict__ psi,
                               double2* __restrict__ out, long V, double kc)
{
    const long blk = (long)blockIdx.x * blockDim.x + threadIdx.x;  // site*2 + chirality
    if (blk >= 2 * V) return;
    cd B[6][6];
    unpack6(clover + blk * 36, B);
    cd v[6];
#pragma unroll
    for (int j = 0; j < 6; j++) v[j] = {psi[blk * 6 + j].x, psi[blk * 6 + j].y};
#pragma unroll
    for (int j = 0; j < 6; j++) {
        cd s = {0.0, 0.0};
#pragma unroll
        for (int k = 0; k < 6; k++) s = s + B[j][k] * v[k];
        out[blk * 6 + j] = make_double2(v[j].re - kc * s.re, v[j].im - kc * s.im);
    }
}

// A = 1 - kc C = L L^+ (Cholesky), A^-1 = L^-+ L^-1.
__global__ void k_clover_invert(const double* __restrict__ clover, double* __restrict__ inv, long V, double kc,
                                int* notpd)
{
    const long blk = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (blk >= 2 * V) return;
    cd A[6][6];
    unpack6(clover + blk * 36, A);
#pragma unroll
    for (int j = 0; j < 6; j++)
#pragma unroll
        for (int k = 0; k < 6; k++) A[j][k] = (j == k ? 1.0 : 0.0) * cd{1.0, 0.0} - kc * A[j][k];
    cd Lm[6][6];
    double dinv[6];
    bool ok = true;
#pragma unroll
    for (int j = 0; j < 6; j++) {
        double d = A[j][j].re;
#pragma unroll
        for (int k = 0; k < j; k++) d -= norm2(Lm[j][k]);
        if (!(d > 0.0)) ok = false;
        const double lj = sqrt(d > 0.0 ? d : 1.0);
        dinv[j] = 1.0 / lj;
        Lm[j][j] = {lj, 0.0};
#pragma unroll
        for (int i = j + 1; i < 6; i++) {
            cd s = A[i][j];
#pragma unroll
            for (int k = 0; k < j; k++) s = s - Lm[i][k] * conj(Lm[j][k]);
            Lm[i][j] = dinv[j] * s;
        }
    }
    // W = L^-1 (lower triangular) by forward substitution
    cd W[6][6];
#pragma unroll
    for (int j = 0; j < 6; j++) {
#pragma unroll
        for (int i = 0; i < 6; i++) W[i][j] = {0.0, 0.0};
        W[j][j] = {dinv[j], 0.0};
#pragma unroll
        for (int i = j + 1; i < 6; i++) {
            cd s = {0.0, 0.0};
#pragma unroll
            for (int k = j; k < i; k++) s = s + Lm[i][k] * W[k][j];
            W[i][j] = (-dinv[i]) * s;
        }
    }
    // A^-1 = W^+ W ; entry (j,k) = sum_{m >= max(j,k)} conj(W[m][j]) W[m][k]
    double* o = inv + blk * 36;
#pragma unroll
    for (int j = 0; j < 6; j++) {
        double s = 0.0;
#pragma unroll
        for (int m = j; m < 6; m++) s += norm2(W[m][j]);
        o[j] = s;
    }
    int slot = 0;
#pragma unroll
    for (int j = 1; j < 6; j++)
#pragma unroll
        for (int k = 0; k < j; k++) {
            cd s = {0.0, 0.0};
#pragma unroll
            for (int m = j; m < 6; m++) s = s + cmul_conj(W[m][j], W[m][k]);
            o[6 + 2 * slot] = s.re;
            o[7 + 2 * slot] = s.im;
            slot++;
        }
    if (!ok) atomicAdd(notpd, 1);
}

__global__ void k_clover_to_A(const double* __restrict__ clover, double* __restrict__ A, long n36, double kc)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n36) return;
    const int m = (int)(e % 36);
    A[e] = (m < 6 ? 1.0 : 0.0) - kc * clover[e];
}

static inline dim3 grid_for(long n) { return dim3((unsigned)((n + 255) / 256)); }

hipError_t launch_clover_build(hipStream_t s, const Geom& g, const void* U, void* clover, double wt, double ws)
{
    const long n = 2L * g.Vh;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_clover_build, grid_for(n), dim3(256), 0, s, (const double2*)U, (double*)clover, g, wt, ws);
    return hipGetLastError();
}

hipError_t launch_clover_apply(hipStream_t s, const Geom& g, const void* clover, const void* psi, void* out,
                               double kappa, double csw)
{
    const long V = 2L * g.Vh;
    if (V == 0) return hipSuccess;
    hipLaunchKernelGGL(k_clover_apply, grid_for(2 * V), dim3(256), 0, s, (const double*)clover, (const double2*)psi,
                       (double2*)out, V, kappa * csw);
    return hipGetLastError();
}

hipError_t launch_clover_invert(hipStream_t s, const Geom& g, const void* clover, double kappa, double csw, void* inv,
                                int* notpd_count)
{
    const long V = 2L * g.Vh;
    if (V == 0) return hipSuccess;
    hipLaunchKernelGGL(k_clover_invert, grid_for(2 * V), dim3(256), 0, s, (const double*)clover, (double*)inv, V,
                       kappa * csw, notpd_count);
    return hipGetLastError();
}

hipError_t launch_clover_to_A(hipStream_t s, const Geom& g, const void* clover, double kappa, double csw, void* A)
{
    const long n = 2L * g.Vh * 72;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_clover_to_A, grid_for(n), dim3(256), 0, s, (const double*)clover, (double*)A, n, kappa * csw);
    return hipGetLastError();
}

}  // namespace qcdw
