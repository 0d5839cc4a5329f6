// Wall sources, sequential sources and meson contractions: the steps on either
// side of the solves in the paper's propagator workflow (Sec. III.B).  Conventions: a
// propagator is 12 fields S_k (k = 3 s0 + c0) in the paper's fermion layout,
// S(x)[3 s + c][k] = S_k(x)[s][c]; the wall source of component k on slice t0
// with momentum n is e^{+i p.x} on that slice (p_i = 2 pi n_i / L_i); and
//   C(t) = sum_{x: x_t = t} e^{-i p.x} Tr[G_snk S(x) G_src g5 S(x)^+ g5]
// for the bitmask gammas Gamma(n) = g1^(n&1) g2^(n>>1&1) g3^(n>>2&1) g4^(n>>3&1); with a
// second propagator T in place of S in the backward leg (T = M^-1 of the sequential sources
// delta(x_t, t_f) e^{+i p.x} g5 Gamma_f^+ g5 S) the same trace is the three-point function.
//
// Every Gamma(n) in the DeGrand-Rossi basis has one nonzero entry per row,
// G[s][perm(s)] = ph(s) with ph a power of i, so with A = G_snk, B = G_src:
//   Tr[...] = sum_{s, s0} ph_A(s) ph_B(s0) g5(s) g5(perm_B(s0))
//             sum_{c, c0} S_{3 s0 + c0}[perm_A(s)][c] conj(T_{3 perm_B(s0) + c0}[s][c]).
// One lane per (s, s0) pair (16 per site) forms its colour sum; the lanes of a
// site are summed by shuffles, and the sites of a slice in a fixed order.
#include "internal.h"

namespace qcdw {

struct MesonArgs {
    const double2* S;  // 12 fields, [12][V][4][3]
    const double2* T;  // second propagator (T = S: the two-point function; a sequential one: three-point)
    double2* site;     // per-site contribution (phase included), [V]
    Geom g;
    int perm_a[4], perm_b[4];
    double2 ph_a[4], ph_b[4];
    double px, py, pz;  // momentum components 2 pi n_i / L_i
};

__device__ __forceinline__ void site_xyzt(const Geom& g, long x, int& X, int& Y, int& Z, int& T)
{
    const int parity = (int)(x / g.Vh), site = (int)(x % g.Vh);
    site_coords(g, site, parity, X, Y, Z, T);
}

__global__ __launch_bounds__(256) void k_wall_sources(double2* out, Geom g, int t0, double px, double py, double pz)
{
    const long V = 2L * g.Vh;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;  // element of the 12 fields
    if (e >= 12L * V * 12) return;
    const int sc = (int)(e % 12);
    const long x = (e / 12) % V;
    const int k = (int)(e / (12 * V));
    double2 v = make_double2(0.0, 0.0);
    if (sc == k) {
        int X, Y, Z, T;
        site_xyzt(g, x, X, Y, Z, T);
        if (T == t0) {
            double sn, cs;
            sincos(px * X + py * Y + pz * Z, &sn, &cs);
            v = make_double2(cs, sn);
        }
    }
    out[e] = v;
}

// One lane (s, s0) of a site's 16: the (s, s0) term of Tr[G_snk S(x) G_src g5 T(x)^+ g5] with the monomial
// gammas, summed over the site's lanes in a fixed order; lane 0 stores it with the momentum phase.
// f1(k, sp) / f2(k, sp) give the 3 colours of field k, spin sp at this site, from memory or LDS.
template <class F1, class F2>
__device__ __forceinline__ void meson_site(const MesonArgs& a, long V, long x, int lane, F1 f1, F2 f2)
{
    const int s = lane >> 2, s0 = lane & 3;
    double re = 0.0, im = 0.0;
    if (x < V) {
        const int sa = a.perm_a[s], sb = a.perm_b[s0];
#pragma unroll
        for (int c0 = 0; c0 < 3; c0++) {
            const double2* u3 = f1(3 * s0 + c0, sa);  // S_{3 s0 + c0}[perm_A(s)]
            const double2* w3 = f2(3 * sb + c0, s);   // T_{3 perm_B(s0) + c0}[s]
#pragma unroll
            for (int c = 0; c < 3; c++) {
                const double2 u = u3[c], w = w3[c];  // u conj(w)
                re += u.x * w.x + u.y * w.y;
                im += u.y * w.x - u.x * w.y;
            }
        }
        // ph_A(s) ph_B(s0) g5(s) g5(perm_B(s0))
        const double2 pa = a.ph_a[s], pb = a.ph_b[s0];
        double cr = pa.x * pb.x - pa.y * pb.y, ci = pa.x * pb.y + pa.y * pb.x;
        const double sg = ((s < 2) == (sb < 2)) ? 1.0 : -1.0;
        cr *= sg;
        ci *= sg;
        const double tr = cr * re - ci * im, ti = cr * im + ci * re;
        re = tr;
        im = ti;
    }
    // sum over the 16 lanes of the site, fixed order
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) {
        re += __shfl_xor(re, off, 16);
        im += __shfl_xor(im, off, 16);
    }
    if (lane == 0 && x < V) {
        int X, Y, Z, T;
        site_xyzt(a.g, x, X, Y, Z, T);
        double sn, cs;
        sincos(-(a.px * X + a.py * Y + a.pz * Z), &sn, &cs);
        a.site[x] = make_double2(cs * re - sn * im, cs * im + sn * re);
    }
}

// The 12 x 12 matrices of a block's SITES sites (of S, and of T unless SAME) are staged in LDS with coalesced
// loads (for each field the sites' 12 SITES complex numbers are contiguous), so every element is read from HBM
// once; each thread issues all its loads before its first LDS store, so they are in flight together.  The lanes
// then take their rows and columns from LDS.  SAME (T = S, the two-point function): 16 sites per 256-thread
// block; otherwise 8 sites per 128-thread block.  Either way the block holds 36 KB of LDS.
template <int SITES, bool SAME>
__global__ __launch_bounds__(SITES * 16) void k_meson_sites(MesonArgs a)
{
    constexpr int NT = SITES * 16, TILE = SITES * 12, NB = SAME ? 1 : 2;
    constexpr int FIELDS = 12 * TILE;             // complex numbers of one propagator per block
    constexpr int LOADS = NB * FIELDS / NT;       // per thread: 9 (SAME) or 18
    static_assert(LOADS * NT == NB * FIELDS, "staging loop must tile the block's matrices exactly");
    __shared__ double2 sm[NB * FIELDS];
    const long V = 2L * a.g.Vh;
    const long x0 = (long)blockIdx.x * SITES;
    double2 v[LOADS];
#pragma unroll
    for (int j = 0; j < LOADS; j++) {
        const int idx = j * NT + threadIdx.x;
        const int b = idx / FIELDS, rem = idx - b * FIELDS;
        const int k = rem / TILE, r = rem - k * TILE;  // r = 12 site + (3 spin + colour)
        const double2* src = b ? a.T : a.S;
        v[j] = x0 + r / 12 < V ? src[((long)k * V + x0) * 12 + r] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int j = 0; j < LOADS; j++) sm[j * NT + threadIdx.x] = v[j];
    __syncthreads();
    const int sl = threadIdx.x >> 4;
    auto fS = [&](int k, int sp) { return (const double2*)sm + k * TILE + sl * 12 + sp * 3; };
    auto fT = [&](int k, int sp) { return (const double2*)sm + (NB - 1) * FIELDS + k * TILE + sl * 12 + sp * 3; };
    meson_site(a, V, x0 + sl, threadIdx.x & 15, fS, fT);
}

// Sequential sources: out_k(x)[s][c] = delta(x_t, t_f) e^{+i p.x} G[s][perm(s)] S_k(x)[perm(s)][c] with the
// monomial spin matrix G = g5 Gamma_f^+ g5 (perm, ph); one thread per output element
__global__ __launch_bounds__(256) void k_seq_sources(const double2* S, double2* out, Geom g, int t_f, double px,
                                                     double py, double pz, int4 perm, double4 ph_re, double4 ph_im)
{
    const long V = 2L * g.Vh;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 12L * V * 12) return;
    const int c = (int)(e % 3), s = (int)((e / 3) % 4);
    const long x = (e / 12) % V;
    const int k = (int)(e / (12 * V));
    double2 v = make_double2(0.0, 0.0);
    int X, Y, Z, T;
    site_xyzt(g, x, X, Y, Z, T);
    if (T == t_f) {
        const int ps = s == 0 ? perm.x : s == 1 ? perm.y : s == 2 ? perm.z : perm.w;
        const double gr = s == 0 ? ph_re.x : s == 1 ? ph_re.y : s == 2 ? ph_re.z : ph_re.w;
        const double gi = s == 0 ? ph_im.x : s == 1 ? ph_im.y : s == 2 ? ph_im.z : ph_im.w;
        const double2 u = S[(((long)k * V + x) * 4 + ps) * 3 + c];
        double sn, cs;
        sincos(px * X + py * Y + pz * Z, &sn, &cs);
        const double wr = cs * gr - sn * gi, wi = cs * gi + sn * gr;  // phase times G entry
        v = make_double2(wr * u.x - wi * u.y, wr * u.y + wi * u.x);
    }
    out[e] = v;
}

// out[t] = sum of the per-site values of slice t (both parities, eo order t St + c), one block per t
__global__ __launch_bounds__(256) void k_slice_sum(const double2* site, double2* out, Geom g)
{
    const int t = blockIdx.x;
    const int St = g.Vh / g.Lt;  // sites of one parity on a time slice, contiguous in the eo order
    double v[2] = {0.0, 0.0};
    for (int par = 0; par < 2; par++) {
        const double2* slice = site + (long)par * g.Vh + (long)t * St;
        for (int i = threadIdx.x; i < St; i += 256) {
            const double2 z = slice[i];
            v[0] += z.x;
            v[1] += z.y;
        }
    }
    __shared__ double res[2];
    block_sum_store<2>(v, res);
    __syncthreads();
    if (threadIdx.x == 0) out[t] = make_double2(res[0], res[1]);
}

static inline double mom_comp(int n, int L) { return 2.0 * 3.14159265358979323846 * n / L; }

hipError_t launch_wall_sources(hipStream_t s, const Geom& g, int t0, const int mom[3], void* out)
{
    const long n = 12L * 2L * g.Vh * 12;
    hipLaunchKernelGGL(k_wall_sources, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (double2*)out, g, t0,
                       mom_comp(mom[0], g.Lx), mom_comp(mom[1], g.Ly), mom_comp(mom[2], g.Lz));
    return hipGetLastError();
}

// Gamma(n) of the DeGrand-Rossi basis as (perm, phase) rows
namespace {
struct C4 {
    double re[4][4], im[4][4];
};
C4 gamma_dr(int mu)
{
    // g1..g4 in the DeGrand-Rossi basis, entries (row, col, re, im)
    static const int nz[4][4][4] = {
        {{0, 3, 0, 1}, {1, 2, 0, 1}, {2, 1, 0, -1}, {3, 0, 0, -1}},
        {{0, 3, -1, 0}, {1, 2, 1, 0}, {2, 1, 1, 0}, {3, 0, -1, 0}},
        {{0, 2, 0, 1}, {1, 3, 0, -1}, {2, 0, 0, -1}, {3, 1, 0, 1}},
        {{0, 2, 1, 0}, {1, 3, 1, 0}, {2, 0, 1, 0}, {3, 1, 1, 0}},
    };
    C4 m{};
    for (const auto& e : nz[mu]) {
        m.re[e[0]][e[1]] = e[2];
        m.im[e[0]][e[1]] = e[3];
    }
    return m;
}
C4 mul(const C4& a, const C4& b)
{
    C4 c{};
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++)
            for (int k = 0; k < 4; k++) {
                c.re[i][j] += a.re[i][k] * b.re[k][j] - a.im[i][k] * b.im[k][j];
                c.im[i][j] += a.re[i][k] * b.im[k][j] + a.im[i][k] * b.re[k][j];
            }
    return c;
}
void monomial(int n, int perm[4], double2 ph[4])
{
    C4 m{};
    for (int i = 0; i < 4; i++) m.re[i][i] = 1.0;
    for (int mu = 0; mu < 4; mu++)
        if ((n >> mu) & 1) m = mul(m, gamma_dr(mu));
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++)
            if (m.re[i][j] != 0.0 || m.im[i][j] != 0.0) {
                perm[i] = j;
                ph[i] = make_double2(m.re[i][j], m.im[i][j]);
            }
}
}  // namespace

hipError_t launch_seq_sources(hipStream_t s, const Geom& g, const void* S, int t_f, int g_f, const int mom[3],
                              void* out)
{
    // G = g5 Gamma_f^+ g5: row i has its entry at column perm_f(i)^{-1}... built as a matrix, then read by rows
    int pf[4];
    double2 phf[4];
    monomial(g_f, pf, phf);
    C4 G{};
    for (int i = 0; i < 4; i++) {  // (Gamma^+)[perm(i)][i] = conj(ph(i)); g5 on both sides: sign g5(row) g5(col)
        const int r = pf[i], col = i;
        const double sg = ((r < 2) == (col < 2)) ? 1.0 : -1.0;
        G.re[r][col] = sg * phf[i].x;
        G.im[r][col] = -sg * phf[i].y;
    }
    int perm[4];
    double2 ph[4];
    for (int r = 0; r < 4; r++)
        for (int col = 0; col < 4; col++)
            if (G.re[r][col] != 0.0 || G.im[r][col] != 0.0) {
                perm[r] = col;
                ph[r] = make_double2(G.re[r][col], G.im[r][col]);
            }
    const long n = 12L * 2L * g.Vh * 12;
    hipLaunchKernelGGL(k_seq_sources, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (const double2*)S,
                       (double2*)out, g, t_f, mom_comp(mom[0], g.Lx), mom_comp(mom[1], g.Ly), mom_comp(mom[2], g.Lz),
                       make_int4(perm[0], perm[1], perm[2], perm[3]), make_double4(ph[0].x, ph[1].x, ph[2].x, ph[3].x),
                       make_double4(ph[0].y, ph[1].y, ph[2].y, ph[3].y));
    return hipGetLastError();
}

hipError_t launch_meson_2pt(hipStream_t s, const Geom& g, const void* S, const void* T, int g_snk, int g_src,
                            const int mom[3], void* site_scratch, void* out)
{
    MesonArgs a{};
    a.S = (const double2*)S;
    a.T = (const double2*)T;
    a.site = (double2*)site_scratch;
    a.g = g;
    monomial(g_snk, a.perm_a, a.ph_a);
    monomial(g_src, a.perm_b, a.ph_b);
    a.px = mom_comp(mom[0], g.Lx);
    a.py = mom_comp(mom[1], g.Ly);
    a.pz = mom_comp(mom[2], g.Lz);
    const long V = 2L * g.Vh;  // 16 lanes per site
    if (S == T)
        hipLaunchKernelGGL((k_meson_sites<16, true>), dim3((unsigned)((V + 15) / 16)), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((k_meson_sites<8, false>), dim3((unsigned)((V + 7) / 8)), dim3(128), 0, s, a);
    hipLaunchKernelGGL(k_slice_sum, dim3(g.Lt), dim3(256), 0, s, (const double2*)site_scratch, (double2*)out, g);
    return hipGetLastError();
}

}  // namespace qcdw
