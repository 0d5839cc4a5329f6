// Clover fermion force: the derivative of the bilinear 2 Re(Y^+ M X) with respect to every link.
//
// HMC with clover fermions (paper Sec. IV) moves the links along the derivative of the pseudo-fermion
// action; for S = phi^+ (M^+ M)^-1 phi with X = (M^+ M)^-1 phi and Y = M X the change of S is
// -2 Re(Y^+ dM X).  For a link variation U_mu(x) -> exp(i w T^a) U_mu(x) the derivative of
// 2 Re(Y^+ M X) is F^a = 2 Tr(T^a H_mu(x)), and this file computes the Hermitian traceless H_mu(x):
//
//   hop term (M = A - kappa H):  K = kappa s (B - B^+) / (2i),  B = U A1 - A2 U^+,
//     A1 = sum_s [(1 - g_mu) X(x+mu)]_s Y(x)_s^+,  A2 = sum_s [(1 + g_mu) X(x)]_s Y(x+mu)_s^+,
//     s the time-boundary sign of the link;
//   clover term (A = 1 - kappa csw sum_{mu<nu} sigma_{mu nu} F_{mu nu}, F = traceless (Q - Q^+)/8):
//     with Gam_{mu nu}(x) = the traceless part of (L - L^+), L = sum_s (sigma_{mu nu} X(x))_s Y(x)_s^+,
//     every leaf through the link contributes +-(kappa csw / 8)(G - G^+)/(2i), G the leaf's loop started
//     at x along the link (leaves that run the link forward, +) or ended along it backward (-), with
//     Gam inserted at the leaf's base corner.  For the link in direction rho and a plane (rho, sig), the
//     forward leaves are the four corners of the plaquette on the +sig side when rho is the plane's first
//     direction (on the -sig side when it is the second), the backward leaves the four corners of the
//     other plaquette.
// Fields in the paper layouts (Sec. II.A), FP64: one thread per site computes Gam for the six planes,
// then one thread per link the force (prefix and suffix products of each plaquette share the work of its
// four corners).
#include "host.h"

namespace qcdw {

namespace {

using c3 = cx<double>[3][3];

struct FGeom {
    int L[4];
    int Lxh, Vh;
    int t_bc;
};

// eo index (parity * Vh + site) of full coordinates, periodic
__device__ __forceinline__ int eo_of(const FGeom& g, int x, int y, int z, int t)
{
    const int p = (x + y + z + t) & 1;
    return p * g.Vh + ((t * g.L[2] + z) * g.L[1] + y) * g.Lxh + (x >> 1);
}
__device__ __forceinline__ void coords_of(const FGeom& g, int e, int (&c)[4])
{
    const int p = e >= g.Vh, i = e - p * g.Vh;
    const int xh = i % g.Lxh;
    int r = i / g.Lxh;
    c[1] = r % g.L[1];
    r /= g.L[1];
    c[2] = r % g.L[2];
    c[3] = r / g.L[2];
    c[0] = 2 * xh + ((p + c[1] + c[2] + c[3]) & 1);
}
__device__ __forceinline__ int shifted(const FGeom& g, const int (&c)[4], int mu, int d)
{
    int q[4] = {c[0], c[1], c[2], c[3]};
    q[mu] = (q[mu] + d + g.L[mu]) % g.L[mu];
    return eo_of(g, q[0], q[1], q[2], q[3]);
}

// DeGrand-Rossi gamma_mu: one nonzero per row, gamma_mu[s][perm] = ph
__device__ __forceinline__ int gperm(int mu, int s) { return mu < 2 ? 3 - s : (s + 2) & 3; }
__device__ __forceinline__ cx<double> gph(int mu, int s)
{
    switch (mu) {
    case 0: return s < 2 ? cx<double>{0.0, 1.0} : cx<double>{0.0, -1.0};
    case 1: return (s == 0 || s == 3) ? cx<double>{-1.0, 0.0} : cx<double>{1.0, 0.0};
    case 2: return (s == 0 || s == 3) ? cx<double>{0.0, 1.0} : cx<double>{0.0, -1.0};
    default: return {1.0, 0.0};
    }
}

__device__ __forceinline__ void ld3(const double2* p, c3& m)
{
#pragma unroll
    for (int i = 0; i < 9; i++) m[i / 3][i % 3] = {p[i].x, p[i].y};
}
__device__ __forceinline__ void dag(const c3& a, c3& o)
{
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) o[i][j] = conj(a[j][i]);
}
__device__ __forceinline__ void mul(const c3& a, const c3& b, c3& o)
{
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            cx<double> s = a[i][0] * b[0][j];
            s = s + a[i][1] * b[1][j];
            s = s + a[i][2] * b[2][j];
            o[i][j] = s;
        }
}
__device__ __forceinline__ void addto(c3& o, const c3& a)
{
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) o[i][j] = o[i][j] + a[i][j];
}
// o += w (G - G^+) / (2i)
__device__ __forceinline__ void add_herm(c3& o, const c3& G, double w)
{
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            const cx<double> d = G[i][j] - conj(G[j][i]);  // G - G^+
            o[i][j] = o[i][j] + cx<double>{w * d.im * 0.5, -w * d.re * 0.5};  // d / (2i)
        }
}

// plane index of (mu, nu), mu < nu: (0,1) (0,2) (0,3) (1,2) (1,3) (2,3)
__device__ __forceinline__ int plane_of(int mu, int nu)
{
    return mu == 0 ? nu - 1 : (mu == 1 ? nu + 1 : 5);
}

}  // namespace

// Gam[p][e] (6 planes, V sites in eo order) = traceless part of (L - L^+), L = sum_s (sigma X)_s Y_s^+,
// sigma_{mu nu} = g_mu g_nu (mu != nu, the DeGrand-Rossi gammas anticommute)
__global__ __launch_bounds__(256) void k_force_gamma(FGeom g, const double2* __restrict__ X,
                                                     const double2* __restrict__ Y, double2* Gam)
{
    const int V = 2 * g.Vh;
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= V) return;
    cx<double> xs[4][3], ys[4][3];
#pragma unroll
    for (int s = 0; s < 4; s++)
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const double2 a = X[(long)e * 12 + 3 * s + c], b = Y[(long)e * 12 + 3 * s + c];
            xs[s][c] = {a.x, a.y};
            ys[s][c] = {b.x, b.y};
        }
#pragma unroll
    for (int mu = 0; mu < 4; mu++)
#pragma unroll
        for (int nu = mu + 1; nu < 4; nu++) {
            c3 Lm;
#pragma unroll
            for (int i = 0; i < 3; i++)
#pragma unroll
                for (int j = 0; j < 3; j++) Lm[i][j] = {0.0, 0.0};
#pragma unroll
            for (int s = 0; s < 4; s++) {
                const int s1 = gperm(mu, s), s2 = gperm(nu, s1);
                const cx<double> ph = gph(mu, s) * gph(nu, s1);  // (g_mu g_nu)[s][s2]
#pragma unroll
                for (int i = 0; i < 3; i++) {
                    const cx<double> sx = ph * xs[s2][i];
#pragma unroll
                    for (int j = 0; j < 3; j++) Lm[i][j] = Lm[i][j] + sx * conj(ys[s][j]);
                }
            }
            c3 Gm;
#pragma unroll
            for (int i = 0; i < 3; i++)
#pragma unroll
                for (int j = 0; j < 3; j++) Gm[i][j] = Lm[i][j] - conj(Lm[j][i]);
            const cx<double> tr3 = {(Gm[0][0].re + Gm[1][1].re + Gm[2][2].re) / 3.0,
                                    (Gm[0][0].im + Gm[1][1].im + Gm[2][2].im) / 3.0};
#pragma unroll
            for (int i = 0; i < 3; i++) Gm[i][i] = Gm[i][i] - tr3;
            double2* o = Gam + ((long)plane_of(mu, nu) * V + e) * 9;
#pragma unroll
            for (int i = 0; i < 9; i++) o[i] = make_double2(Gm[i / 3][i % 3].re, Gm[i / 3][i % 3].im);
        }
}

// H for every link (rho, e), one thread per link; U, H: paper gauge layout [4][V][3][3]
__global__ __launch_bounds__(256) void k_force_link(FGeom g, const double2* __restrict__ U,
                                                    const double2* __restrict__ X, const double2* __restrict__ Y,
                                                    const double2* __restrict__ Gam, double kappa, double csw,
                                                    double2* H)
{
    const int V = 2 * g.Vh;
    const long tid = (long)blockIdx.x * 256 + threadIdx.x;
    if (tid >= 4L * V) return;
    const int rho = (int)(tid / V), e = (int)(tid - (long)rho * V);
    int c[4];
    coords_of(g, e, c);
    const int ep = shifted(g, c, rho, 1);
    auto link = [&](int mu, int site, c3& m) { ld3(U + ((long)mu * V + site) * 9, m); };
    auto gam = [&](int p, int site, c3& m) { ld3(Gam + ((long)p * V + site) * 9, m); };
    c3 u, ud, K;
    link(rho, e, u);
    dag(u, ud);
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) K[i][j] = {0.0, 0.0};

    // hop term: B = s (U A1 - A2 U^+)
    {
        c3 A1, A2;
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) A1[i][j] = A2[i][j] = {0.0, 0.0};
        for (int s = 0; s < 4; s++) {
            const int so = gperm(rho, s);
            const cx<double> ph = gph(rho, s);
            for (int i = 0; i < 3; i++) {
                const double2 xa = X[(long)ep * 12 + 3 * s + i], xb = X[(long)ep * 12 + 3 * so + i];
                const double2 xc = X[(long)e * 12 + 3 * s + i], xd = X[(long)e * 12 + 3 * so + i];
                const cx<double> w1 = cx<double>{xa.x, xa.y} - ph * cx<double>{xb.x, xb.y};  // (1 - g) X(x+rho)
                const cx<double> w2 = cx<double>{xc.x, xc.y} + ph * cx<double>{xd.x, xd.y};  // (1 + g) X(x)
                for (int j = 0; j < 3; j++) {
                    const double2 ya = Y[(long)e * 12 + 3 * s + j], yb = Y[(long)ep * 12 + 3 * s + j];
                    A1[i][j] = A1[i][j] + w1 * cx<double>{ya.x, -ya.y};
                    A2[i][j] = A2[i][j] + w2 * cx<double>{yb.x, -yb.y};
                }
            }
        }
        c3 B, T;
        mul(u, A1, B);
        mul(A2, ud, T);
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) B[i][j] = B[i][j] - T[i][j];
        const double sgn = (rho == 3 && g.t_bc < 0 && c[3] == g.L[3] - 1) ? -1.0 : 1.0;
        add_herm(K, B, kappa * sgn);
    }

    // clover term: the two plaquettes through the link in each plane (rho, sig)
    const double wcl = kappa * csw / 8.0;
    for (int sig = 0; sig < 4; sig++) {
        if (sig == rho) continue;
        const int p = rho < sig ? plane_of(rho, sig) : plane_of(sig, rho);
        const int dfw = rho < sig ? 1 : -1;  // side of the plaquette run forward
        for (int side = 0; side < 2; side++) {
            const int d = side == 0 ? dfw : -dfw;  // plaquette on the d sig side of the link
            const int e_d = shifted(g, c, sig, d);  // y + d sig
            int cd[4] = {c[0], c[1], c[2], c[3]};
            cd[sig] = (cd[sig] + d + g.L[sig]) % g.L[sig];
            const int e_dr = shifted(g, cd, rho, 1);  // y + d sig + rho
            const int e_dmr = d > 0 ? ep : shifted(g, cd, rho, 1);  // base of the sig link on the y+rho side
            c3 a, b, G0, G1, G2, G3;
            if (side == 0) {
                // forward: G = U U2 U3 U4 with Gam at y+rho, y+rho+d, y+d, y (after U, U2, U3, U4)
                c3 U2, U3, U4, t1;
                if (d > 0) {
                    link(sig, ep, U2);                  // U_sig(y+rho)
                } else {
                    link(sig, e_dmr, t1);               // U_sig(y+rho-sig)^+
                    dag(t1, U2);
                }
                link(rho, e_d, t1);                     // U_rho(y+d)^+
                dag(t1, U3);
                if (d > 0) {
                    link(sig, e, t1);                   // U_sig(y)^+
                    dag(t1, U4);
                } else {
                    link(sig, e_d, U4);                 // U_sig(y-sig)
                }
                c3 S34, S234, P12, P123, P1234;
                mul(U3, U4, S34);
                mul(U2, S34, S234);
                mul(u, U2, P12);
                mul(P12, U3, P123);
                mul(P123, U4, P1234);
                c3 G;
                gam(p, ep, G0);
                mul(G0, S234, a);
                mul(u, a, G);
                gam(p, e_dr, G1);
                mul(G1, S34, a);
                mul(P12, a, b);
                addto(G, b);
                gam(p, e_d, G2);
                mul(G2, U4, a);
                mul(P123, a, b);
                addto(G, b);
                gam(p, e, G3);
                mul(P1234, G3, b);
                addto(G, b);
                add_herm(K, G, wcl);
            } else {
                // backward: G' = V1 V2 V3 U^+ with Gam at y, y+d, y+d+rho, y+rho (before V1, V2, V3, U^+)
                c3 V1, V2, V3, t1;
                if (d > 0) {
                    link(sig, e, V1);                   // U_sig(y)
                } else {
                    link(sig, e_d, t1);                 // U_sig(y-sig)^+
                    dag(t1, V1);
                }
                link(rho, e_d, V2);                     // U_rho(y+d)
                if (d > 0) {
                    link(sig, ep, t1);                  // U_sig(y+rho)^+
                    dag(t1, V3);
                } else {
                    link(sig, e_dmr, V3);               // U_sig(y+rho-sig)
                }
                c3 R3, R23, R123, Q12, Q123;
                mul(V3, ud, R3);
                mul(V2, R3, R23);
                mul(V1, R23, R123);
                mul(V1, V2, Q12);
                mul(Q12, V3, Q123);
                c3 G;
                gam(p, e, G0);
                mul(G0, R123, G);
                gam(p, e_d, G1);
                mul(G1, R23, a);
                mul(V1, a, b);
                addto(G, b);
                gam(p, e_dr, G2);
                mul(G2, R3, a);
                mul(Q12, a, b);
                addto(G, b);
                gam(p, ep, G3);
                mul(G3, ud, a);
                mul(Q123, a, b);
                addto(G, b);
                add_herm(K, G, -wcl);
            }
        }
    }
    // traceless part
    const double tr = (K[0][0].re + K[1][1].re + K[2][2].re) / 3.0;
    double2* o = H + tid * 9;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            const cx<double> v = K[i][j];
            o[3 * i + j] = make_double2(i == j ? v.re - tr : v.re, i == j ? 0.0 : v.im);
        }
}

hipError_t launch_clover_force(hipStream_t s, const Geom& g, const void* U, const void* X, const void* Y,
                               double kappa, double csw, void* Gam, void* H)
{
    FGeom f{{g.Lx, g.Ly, g.Lz, g.Lt}, g.Lxh, g.Vh, g.t_bc};
    const int V = 2 * g.Vh;
    hipLaunchKernelGGL(k_force_gamma, dim3((V + 255) / 256), dim3(256), 0, s, f, (const double2*)X,
                       (const double2*)Y, (double2*)Gam);
    hipLaunchKernelGGL(k_force_link, dim3((unsigned)((4L * V + 255) / 256)), dim3(256), 0, s, f, (const double2*)U,
                       (const double2*)X, (const double2*)Y, (const double2*)Gam, kappa, csw, (double2*)H);
    return hipGetLastError();
}

}  // namespace qcdw

extern "C" qcdw_status qcdw_clover_force(qcdw_ctx* ctx, const qcdw_lattice* lat, const void* U, const void* X,
                                         const void* Y, double kappa, double csw, void* H)
{
    if (!ctx) return QCDW_EINVAL;
    DeviceGuard dg(ctx->device);
    Geom g;
    CHK(check_lattice(ctx, lat, g));
    CHK(check_dev(ctx, U, "U"));
    CHK(check_dev(ctx, X, "X"));
    CHK(check_dev(ctx, Y, "Y"));
    CHK(check_dev(ctx, H, "H"));
    if (H == U || H == X || H == Y) return fail(ctx, QCDW_EINVAL, "H must not alias U, X or Y");
    if (!std::isfinite(kappa) || !std::isfinite(csw)) return fail(ctx, QCDW_EINVAL, "kappa and csw must be finite");
    PoolBuf gam;  // Gam for the six planes, [6][V][3][3] complex; the stream is drained before it goes back
    HIPCHK(ctx, gam.alloc(6UL * 2 * g.Vh * 9 * 16));
    const hipError_t launched = launch_clover_force(ctx->stream, g, U, X, Y, kappa, csw, gam.p, H);
    const hipError_t drained = hipStreamSynchronize(ctx->stream);
    HIPCHK(ctx, launched);
    HIPCHK(ctx, drained);
    return QCDW_OK;
}
