/*
 * Plain FP64 CPU oracle for the even-odd Wilson-clover inversion.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or helper
 * with the HIP library.
 *
 * Everything here is written for obviousness, not speed: full 4x4 spin
 * matrices instead of half-spinor projection, full 3x3 links (no
 * compression), dense 6x6 Gauss-Jordan inversion, textbook BiCGStab on the
 * full (unpreconditioned) system.  OpenMP parallel-for over sites is the only
 * concession to run time.
 *
 * Conventions (paper, Sec. II.A "Convention"):
 *   - lattice [Lx, Ly, Lz, Lt]; even-odd ("cb2") site order
 *     [2, Lt, Lz, Ly, Lx/2], parity = (x+y+z+t) mod 2, x fastest;
 *   - gauge   [Nd, 2, Lt, Lz, Ly, Lx/2, Nc, Nc], row-column colour order;
 *   - fermion [2, Lt, Lz, Ly, Lx/2, Ns, Nc];
 *   - clover  [2, Lt, Lz, Ly, Lx/2, 2, 36] reals: per chirality block
 *     (upper = spins 0,1; lower = spins 2,3) 6 real diagonal entries
 *     followed by the 15 complex strictly-lower entries in row-major order;
 *   - Dirac matrices in the DeGrand-Rossi basis.
 * Operator (paper, Sec. III.B, Eq. "clover", isotropic limit xi0 = nu = 1):
 *   M psi = A psi - kappa H psi,   A = 1 - kappa csw sum_{mu<nu} sigma F,
 *   H psi(x) = sum_mu (1-g_mu) U_mu(x) psi(x+mu) + (1+g_mu) U_mu(x-mu)^+ psi(x-mu).
 * The solver (paper, Sec. II.E: BiCGStab is the default for clover) is the
 * van der Vorst (1992) iteration.
 *
 * Parity pinning of every function lives in tests/test_oracle_*.py.
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* ------------------------------------------------------------------ */
/* Geometry (Sec. II.A)                                                */
/* ------------------------------------------------------------------ */

static long volume(const int L[4]) { return (long)L[0] * L[1] * L[2] * L[3]; }

/* eo index of the site with coordinates c = (x, y, z, t). */
static long site_index(const int L[4], const int c[4])
{
    long V = volume(L);
    int parity = (c[0] + c[1] + c[2] + c[3]) & 1;
    long within = (((long)c[3] * L[2] + c[2]) * L[1] + c[1]) * (L[0] / 2) + c[0] / 2;
    return parity * (V / 2) + within;
}

/* Inverse of site_index. */
static void site_coords(const int L[4], long i, int c[4])
{
    long Vh = volume(L) / 2;
    int parity = (int)(i / Vh);
    long r = i % Vh;
    int xh = (int)(r % (L[0] / 2));
    r /= (L[0] / 2);
    c[1] = (int)(r % L[1]);
    r /= L[1];
    c[2] = (int)(r % L[2]);
    c[3] = (int)(r / L[2]);
    c[0] = 2 * xh + ((parity + c[1] + c[2] + c[3]) & 1);
}

/* Site reached from c by one step of `step` (+1 or -1) along mu, periodic. */
static long neighbour(const int L[4], const int c[4], int mu, int step)
{
    int d[4] = {c[0], c[1], c[2], c[3]};
    d[mu] = (d[mu] + step + L[mu]) % L[mu];
    return site_index(L, d);
}

long orc_site_index(const int L[4], const int c[4]) { return site_index(L, c); }
int orc_num_threads(void) { return omp_get_max_threads(); }
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
void orc_site_coords(const int L[4], long i, int c[4]) { site_coords(L, i, c); }

/* ------------------------------------------------------------------ */
/* Dirac matrices, DeGrand-Rossi basis (Sec. II.A)                    */
/* ------------------------------------------------------------------ */

static void gamma_matrix(int mu, cplx g[4][4])
{
    memset(g, 0, sizeof(cplx) * 16);
    switch (mu) {
    case 0: /* gamma_1 */
        g[0][3] = I; g[1][2] = I; g[2][1] = -I; g[3][0] = -I;
        break;
    case 1: /* gamma_2 */
        g[0][3] = -1; g[1][2] = 1; g[2][1] = 1; g[3][0] = -1;
        break;
    case 2: /* gamma_3 */
        g[0][2] = I; g[1][3] = -I; g[2][0] = -I; g[3][1] = I;
        break;
    case 3: /* gamma_4 */
        g[0][2] = 1; g[1][3] = 1; g[2][0] = 1; g[3][1] = 1;
        break;
    }
}

/* Exported as 16 (re, im) pairs, row-major. */
void orc_gamma(int mu, double *out)
{
    cplx g[4][4];
    gamma_matrix(mu, g);
    for (int i = 0; i < 16; i++) {
        out[2 * i] = creal(g[i / 4][i % 4]);
        out[2 * i + 1] = cimag(g[i / 4][i % 4]);
    }
}

/* ------------------------------------------------------------------ */
/* Small complex matrix helpers                                        */
/* ------------------------------------------------------------------ */

static void mat3_mul(const cplx a[9], const cplx b[9], cplx out[9])
{
    cplx r[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            cplx s = 0;
            for (int k = 0; k < 3; k++) s += a[3 * i + k] * b[3 * k + j];
            r[3 * i + j] = s;
        }
    memcpy(out, r, sizeof r);
}

static void mat3_dagger(const cplx a[9], cplx out[9])
{
    cplx r[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) r[3 * i + j] = conj(a[3 * j + i]);
    memcpy(out, r, sizeof r);
}

static const cplx *link(const cplx *U, long V, int mu, long site) { return U + ((long)mu * V + site) * 9; }

/* ------------------------------------------------------------------ */
/* Hopping term H (Sec. III.B, Eq. "clover"; Wilson term written out)  */
/* ------------------------------------------------------------------ */

/*
 * out = H psi on every site whose parity equals out_parity (or on all sites
 * when out_parity < 0); other output sites are set to zero.  t_bc multiplies
 * every link that crosses the t = Lt-1 -> 0 boundary.  w[mu] weights the two
 * hops of direction mu (the anisotropic operator of Sec. III.B weights the
 * spatial ones by nu / xi_0); w = NULL means all weights 1.
 */
void orc_hop_w(const int L[4], int t_bc, const double *U_, const double *psi_, double *out_, int out_parity,
               const double *w)
{
    const cplx *U = (const cplx *)U_;
    const cplx *psi = (const cplx *)psi_;
    cplx *out = (cplx *)out_;
    long V = volume(L);
    cplx gam[4][4][4];
    for (int mu = 0; mu < 4; mu++) gamma_matrix(mu, gam[mu]);

#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; i++) {
        int c[4];
        site_coords(L, i, c);
        int parity = (int)(i / (V / 2));
        cplx acc[4][3];
        memset(acc, 0, sizeof acc);
        if (out_parity < 0 || parity == out_parity) {
            for (int mu = 0; mu < 4; mu++) {
                for (int dir = 0; dir < 2; dir++) {
                    /* dir 0: forward, (1 - g) U(x) psi(x+mu)
                       dir 1: backward, (1 + g) U(x-mu)^+ psi(x-mu) */
                    int step = dir == 0 ? +1 : -1;
                    long j = neighbour(L, c, mu, step);
                    cplx u[9];
                    if (dir == 0) {
                        memcpy(u, link(U, V, mu, i), sizeof u);
                    } else {
                        mat3_dagger(link(U, V, mu, j), u);
                    }
                    double sign = w ? w[mu] : 1.0;
                    if (mu == 3 && t_bc < 0) {
                        if (dir == 0 && c[3] == L[3] - 1) sign = -sign;
                        if (dir == 1 && c[3] == 0) sign = -sign;
                    }
                    /* colour: chi[s][a] = sum_b u[a][b] psi_j[s][b] */
                    cplx chi[4][3];
                    for (int s = 0; s < 4; s++)
                        for (int a = 0; a < 3; a++) {
                            cplx v = 0;
                            for (int b = 0; b < 3; b++) v += u[3 * a + b] * psi[j * 12 + s * 3 + b];
                            chi[s][a] = sign * v;
                        }
                    /* spin: (1 -/+ gamma_mu) */
                    double pm = dir == 0 ? -1.0 : +1.0;
                    for (int s = 0; s < 4; s++)
                        for (int a = 0; a < 3; a++) {
                            cplx v = chi[s][a];
                            for (int r = 0; r < 4; r++) v += pm * gam[mu][s][r] * chi[r][a];
                            acc[s][a] += v;
                        }
                }
            }
        }
        for (int s = 0; s < 4; s++)
            for (int a = 0; a < 3; a++) out[i * 12 + s * 3 + a] = acc[s][a];
    }
}

void orc_hop(const int L[4], int t_bc, const double *U_, const double *psi_, double *out_, int out_parity)
{
    orc_hop_w(L, t_bc, U_, psi_, out_, out_parity, NULL);
}

/* ------------------------------------------------------------------ */
/* Clover field (Sec. II.A clover layout; Sec. III.B Eq. "clover")     */
/* ------------------------------------------------------------------ */

/*
 * Clover-leaf sum Q_{mu nu}(x) of the four plaquettes in the (mu, nu) plane
 * that touch x, each traversed counter-clockwise and starting at x.
 */
static void clover_leaves(const int L[4], const cplx *U, long V, const int c[4], int mu, int nu, cplx Q[9])
{
    /* sites x, x+mu, x+nu, x-mu, x-nu, x-mu+nu, x-mu-nu, x+mu-nu */
    long s_x = site_index(L, c);
    long s_pm = neighbour(L, c, mu, +1);
    long s_pn = neighbour(L, c, nu, +1);
    long s_mm = neighbour(L, c, mu, -1);
    long s_mn = neighbour(L, c, nu, -1);
    int d[4];
    memcpy(d, c, sizeof d);
    d[mu] = (d[mu] - 1 + L[mu]) % L[mu];
    d[nu] = (d[nu] + 1) % L[nu];
    long s_mm_pn = site_index(L, d);
    memcpy(d, c, sizeof d);
    d[mu] = (d[mu] - 1 + L[mu]) % L[mu];
    d[nu] = (d[nu] - 1 + L[nu]) % L[nu];
    long s_mm_mn = site_index(L, d);
    memcpy(d, c, sizeof d);
    d[mu] = (d[mu] + 1) % L[mu];
    d[nu] = (d[nu] - 1 + L[nu]) % L[nu];
    long s_pm_mn = site_index(L, d);

    cplx t1[9], t2[9], leaf[9];
    memset(Q, 0, sizeof(cplx) * 9);

    /* leaf 1: U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+ */
    mat3_mul(link(U, V, mu, s_x), link(U, V, nu, s_pm), t1);
    mat3_dagger(link(U, V, mu, s_pn), t2);
    mat3_mul(t1, t2, t1);
    mat3_dagger(link(U, V, nu, s_x), t2);
    mat3_mul(t1, t2, leaf);
    for (int k = 0; k < 9; k++) Q[k] += leaf[k];

    /* leaf 2: U_nu(x) U_mu(x-mu+nu)^+ U_nu(x-mu)^+ U_mu(x-mu) */
    mat3_dagger(link(U, V, mu, s_mm_pn), t2);
    mat3_mul(link(U, V, nu, s_x), t2, t1);
    mat3_dagger(link(U, V, nu, s_mm), t2);
    mat3_mul(t1, t2, t1);
    mat3_mul(t1, link(U, V, mu, s_mm), leaf);
    for (int k = 0; k < 9; k++) Q[k] += leaf[k];

    /* leaf 3: U_mu(x-mu)^+ U_nu(x-mu-nu)^+ U_mu(x-mu-nu) U_nu(x-nu) */
    mat3_dagger(link(U, V, mu, s_mm), t1);
    mat3_dagger(link(U, V, nu, s_mm_mn), t2);
    mat3_mul(t1, t2, t1);
    mat3_mul(t1, link(U, V, mu, s_mm_mn), t1);
    mat3_mul(t1, link(U, V, nu, s_mn), leaf);
    for (int k = 0; k < 9; k++) Q[k] += leaf[k];

    /* leaf 4: U_nu(x-nu)^+ U_mu(x-nu) U_nu(x+mu-nu) U_mu(x)^+ */
    mat3_dagger(link(U, V, nu, s_mn), t1);
    mat3_mul(t1, link(U, V, mu, s_mn), t1);
    mat3_mul(t1, link(U, V, nu, s_pm_mn), t1);
    mat3_dagger(link(U, V, mu, s_x), t2);
    mat3_mul(t1, t2, leaf);
    for (int k = 0; k < 9; k++) Q[k] += leaf[k];
}

/* Field strength F_{mu nu}(x) = (Q - Q^+)/8 with its trace removed. */
static void field_strength(const int L[4], const cplx *U, long V, const int c[4], int mu, int nu, cplx F[9])
{
    cplx Q[9], Qd[9];
    clover_leaves(L, U, V, c, mu, nu, Q);
    mat3_dagger(Q, Qd);
    for (int k = 0; k < 9; k++) F[k] = (Q[k] - Qd[k]) / 8.0;
    cplx tr = (F[0] + F[4] + F[8]) / 3.0;
    F[0] -= tr;
    F[4] -= tr;
    F[8] -= tr;
}

/* Index of the packed 6x6 entry (j, k), j > k, in the 15 lower entries. */
static int lower_slot(int j, int k) { return j * (j - 1) / 2 + k; }

/* Pack one 6x6 Hermitian block into 36 reals (diag re, then lower re/im). */
static void pack_block(const cplx B[6][6], double *p)
{
    for (int j = 0; j < 6; j++) p[j] = creal(B[j][j]);
    for (int j = 1; j < 6; j++)
        for (int k = 0; k < j; k++) {
            int s = lower_slot(j, k);
            p[6 + 2 * s] = creal(B[j][k]);
            p[6 + 2 * s + 1] = cimag(B[j][k]);
        }
}

/* Unpack 36 reals into the full Hermitian 6x6 block. */
static void unpack_block(const double *p, cplx B[6][6])
{
    for (int j = 0; j < 6; j++) B[j][j] = p[j];
    for (int j = 1; j < 6; j++)
        for (int k = 0; k < j; k++) {
            int s = lower_slot(j, k);
            cplx v = p[6 + 2 * s] + I * p[6 + 2 * s + 1];
            B[j][k] = v;
            B[k][j] = conj(v);
        }
}

/*
 * clover = C = sum_{mu<nu} sigma_{mu nu} (x) F_{mu nu} with
 * sigma_{mu nu} = [gamma_mu, gamma_nu] / 2, packed per chirality block.
 * Returns the largest magnitude found in the off-chirality blocks (which a
 * chiral basis makes exactly zero) so tests can check it.
 */
double orc_clover_build_w(const int L[4], const double *U_, double *clover, double wt, double ws);
double orc_clover_build(const int L[4], const double *U_, double *clover)
{
    return orc_clover_build_w(L, U_, clover, 1.0, 1.0);
}

/*
 * The same with the planes weighted: wt for the three planes (i, t) and ws for
 * the three spatial planes (i, j) -- the anisotropic clover term of Sec. III.B
 * has wt = c_SW^t and ws = c_SW^r / xi_0 (with the overall c_SW then 1).
 */
double orc_clover_build_w(const int L[4], const double *U_, double *clover, double wt, double ws)
{
    const cplx *U = (const cplx *)U_;
    long V = volume(L);
    cplx gam[4][4][4], sigma[4][4][4][4];
    for (int mu = 0; mu < 4; mu++) gamma_matrix(mu, gam[mu]);
    for (int mu = 0; mu < 4; mu++)
        for (int nu = 0; nu < 4; nu++)
            for (int a = 0; a < 4; a++)
                for (int b = 0; b < 4; b++) {
                    cplx s = 0;
                    for (int k = 0; k < 4; k++) s += gam[mu][a][k] * gam[nu][k][b] - gam[nu][a][k] * gam[mu][k][b];
                    sigma[mu][nu][a][b] = 0.5 * s;
                }
    double offmax = 0.0;
#pragma omp parallel for schedule(static) reduction(max : offmax)
    for (long i = 0; i < V; i++) {
        int c[4];
        site_coords(L, i, c);
        cplx C[12][12];
        memset(C, 0, sizeof C);
        for (int mu = 0; mu < 4; mu++)
            for (int nu = mu + 1; nu < 4; nu++) {
                cplx F[9];
                field_strength(L, U, V, c, mu, nu, F);
                const double wgt = nu == 3 ? wt : ws;
                for (int s = 0; s < 4; s++)
                    for (int sp = 0; sp < 4; sp++)
                        for (int a = 0; a < 3; a++)
                            for (int b = 0; b < 3; b++)
                                C[3 * s + a][3 * sp + b] += wgt * sigma[mu][nu][s][sp] * F[3 * a + b];
            }
        for (int r = 0; r < 12; r++)
            for (int q = 0; q < 12; q++)
                if ((r < 6) != (q < 6) && cabs(C[r][q]) > offmax) offmax = cabs(C[r][q]);
        for (int chi = 0; chi < 2; chi++) {
            cplx B[6][6];
            for (int j = 0; j < 6; j++)
                for (int k = 0; k < 6; k++) B[j][k] = C[6 * chi + j][6 * chi + k];
            pack_block(B, clover + (i * 2 + chi) * 36);
        }
    }
    return offmax;
}

/* Apply packed Hermitian blocks: out(x) = B(x) psi(x) per chirality. */
void orc_packed_apply(const int L[4], const double *packed, const double *psi_, double *out_)
{
    const cplx *psi = (const cplx *)psi_;
    cplx *out = (cplx *)out_;
    long V = volume(L);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; i++) {
        cplx res[12];
        for (int chi = 0; chi < 2; chi++) {
            cplx B[6][6];
            unpack_block(packed + (i * 2 + chi) * 36, B);
            for (int j = 0; j < 6; j++) {
                cplx v = 0;
                for (int k = 0; k < 6; k++) v += B[j][k] * psi[i * 12 + 6 * chi + k];
                res[6 * chi + j] = v;
            }
        }
        for (int k = 0; k < 12; k++) out[i * 12 + k] = res[k];
    }
}

/* out = A psi, A = 1 - kappa csw C. */
void orc_clover_apply(const int L[4], const double *clover, const double *psi_, double *out_, double kappa, double csw)
{
    const cplx *psi = (const cplx *)psi_;
    cplx *out = (cplx *)out_;
    long V = volume(L);
    orc_packed_apply(L, clover, psi_, out_);
#pragma omp parallel for schedule(static)
    for (long k = 0; k < V * 12; k++) out[k] = psi[k] - kappa * csw * out[k];
}

/*
 * Inverse of A = 1 - kappa csw C on every block by Gauss-Jordan elimination
 * with partial pivoting, packed like the clover.  Returns the number of
 * blocks whose pivot vanished (singular A).
 */
long orc_clover_invert(const int L[4], const double *clover, double kappa, double csw, double *clover_inv)
{
    long V = volume(L);
    long bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (long blk = 0; blk < 2 * V; blk++) {
        cplx C[6][6], a[6][12];
        unpack_block(clover + blk * 36, C);
        for (int j = 0; j < 6; j++)
            for (int k = 0; k < 6; k++) {
                a[j][k] = (j == k ? 1.0 : 0.0) - kappa * csw * C[j][k];
                a[j][6 + k] = (j == k) ? 1.0 : 0.0;
            }
        int singular = 0;
        for (int col = 0; col < 6; col++) {
            int piv = col;
            for (int r = col + 1; r < 6; r++)
                if (cabs(a[r][col]) > cabs(a[piv][col])) piv = r;
            if (cabs(a[piv][col]) == 0.0) {
                singular = 1;
                break;
            }
            if (piv != col)
                for (int k = 0; k < 12; k++) {
                    cplx tmp = a[col][k];
                    a[col][k] = a[piv][k];
                    a[piv][k] = tmp;
                }
            cplx d = a[col][col];
            for (int k = 0; k < 12; k++) a[col][k] /= d;
            for (int r = 0; r < 6; r++) {
                if (r == col) continue;
                cplx f = a[r][col];
                for (int k = 0; k < 12; k++) a[r][k] -= f * a[col][k];
            }
        }
        if (singular) {
            bad++;
            memset(clover_inv + blk * 36, 0, 36 * sizeof(double));
            continue;
        }
        cplx B[6][6];
        for (int j = 0; j < 6; j++)
            for (int k = 0; k < 6; k++) B[j][k] = a[j][6 + k];
        pack_block(B, clover_inv + blk * 36);
    }
    return bad;
}

/* ------------------------------------------------------------------ */
/* Full Wilson-clover operator                                        */
/* ------------------------------------------------------------------ */

/* out = M psi = A psi - kappa H psi on the full lattice (w: hop weights per direction, or NULL). */
void orc_dirac_w(const int L[4], int t_bc, const double *U, const double *clover, const double *psi, double *out_,
                 double kappa, double csw, const double *w)
{
    long V = volume(L);
    cplx *out = (cplx *)out_;
    cplx *h = malloc(sizeof(cplx) * V * 12);
    orc_hop_w(L, t_bc, U, psi, (double *)h, -1, w);
    orc_clover_apply(L, clover, psi, out_, kappa, csw);
#pragma omp parallel for schedule(static)
    for (long k = 0; k < V * 12; k++) out[k] -= kappa * h[k];
    free(h);
}

void orc_dirac(const int L[4], int t_bc, const double *U, const double *clover, const double *psi, double *out_,
               double kappa, double csw)
{
    orc_dirac_w(L, t_bc, U, clover, psi, out_, kappa, csw, NULL);
}

/* ------------------------------------------------------------------ */
/* BiCGStab on the full system (van der Vorst 1992)                    */
/* ------------------------------------------------------------------ */

static cplx dot(long n, const cplx *a, const cplx *b)
{
    cplx s = 0;
    for (long k = 0; k < n; k++) s += conj(a[k]) * b[k];
    return s;
}

static double norm2(long n, const cplx *a)
{
    double s = 0;
    for (long k = 0; k < n; k++) s += creal(a[k]) * creal(a[k]) + cimag(a[k]) * cimag(a[k]);
    return s;
}

/* Status values shared in meaning (not in code) with the product library. */
enum { ORC_OK = 0, ORC_ENOCONV = -4, ORC_ENAN = -6 };

/*
 * Solve M x = b to ||b - M x|| / ||b|| <= tol.  x holds the initial guess on
 * entry and the solution on exit.  res_hist (maxiter+1 entries, may be NULL)
 * receives the recursive relative residual after each iteration, entry 0 the
 * initial one.  out[0] = iterations, out[1] = true relative residual,
 * out[2] = number of restarts after breakdown.
 */
int orc_bicgstab(const int L[4], int t_bc, const double *U, const double *clover, double kappa, double csw,
                 const double *b_, double *x_, double tol, int maxiter, double *res_hist, double *out)
{
    long V = volume(L);
    long n = V * 12;
    const cplx *b = (const cplx *)b_;
    cplx *x = (cplx *)x_;
    cplx *r = malloc(sizeof(cplx) * n), *rh = malloc(sizeof(cplx) * n), *p = calloc(n, sizeof(cplx)),
         *v = calloc(n, sizeof(cplx)), *s = malloc(sizeof(cplx) * n), *t = malloc(sizeof(cplx) * n);
    double bnorm = sqrt(norm2(n, b));
    int status = ORC_ENOCONV, it = 0, restarts = 0;
    if (!isfinite(bnorm)) {
        status = ORC_ENAN;
        goto done;
    }
    if (bnorm == 0.0) {
        memset(x, 0, sizeof(cplx) * n);
        status = ORC_OK;
        goto done;
    }

restart:
    orc_dirac(L, t_bc, U, clover, x_, (double *)r, kappa, csw);
    for (long k = 0; k < n; k++) r[k] = b[k] - r[k];
    memcpy(rh, r, sizeof(cplx) * n);
    memset(p, 0, sizeof(cplx) * n);
    memset(v, 0, sizeof(cplx) * n);
    {
        cplx rho = 1, alpha = 1, omega = 1;
        double rn = sqrt(norm2(n, r)) / bnorm;
        if (res_hist && it == 0) res_hist[0] = rn;
        if (rn <= tol) {
            status = ORC_OK;
            goto done;
        }
        double rhnorm = sqrt(norm2(n, rh));
        while (it < maxiter) {
            cplx rho_new = dot(n, rh, r);
            if (cabs(rho_new) < 1e-30 * rhnorm * sqrt(norm2(n, r))) {
                restarts++;
                goto restart;
            }
            cplx beta = (rho_new / rho) * (alpha / omega);
            for (long k = 0; k < n; k++) p[k] = r[k] + beta * (p[k] - omega * v[k]);
            orc_dirac(L, t_bc, U, clover, (double *)p, (double *)v, kappa, csw);
            cplx rv = dot(n, rh, v);
            if (cabs(rv) < 1e-30 * rhnorm * sqrt(norm2(n, v))) {
                restarts++;
                goto restart;
            }
            alpha = rho_new / rv;
            for (long k = 0; k < n; k++) s[k] = r[k] - alpha * v[k];
            orc_dirac(L, t_bc, U, clover, (double *)s, (double *)t, kappa, csw);
            double tt = norm2(n, t);
            it++;
            if (tt == 0.0) {
                /* s = 0 exactly: x + alpha p is the solution. */
                for (long k = 0; k < n; k++) x[k] += alpha * p[k];
                for (long k = 0; k < n; k++) r[k] = s[k];
                rn = sqrt(norm2(n, r)) / bnorm;
                if (res_hist) res_hist[it] = rn;
                status = ORC_OK;
                break;
            }
            omega = dot(n, t, s) / tt;
            for (long k = 0; k < n; k++) {
                x[k] += alpha * p[k] + omega * s[k];
                r[k] = s[k] - omega * t[k];
            }
            rho = rho_new;
            rn = sqrt(norm2(n, r)) / bnorm;
            if (res_hist) res_hist[it] = rn;
            if (!isfinite(rn)) {
                status = ORC_ENAN;
                break;
            }
            if (rn <= tol) {
                status = ORC_OK;
                break;
            }
        }
    }
done:
    if (out) {
        double tr = NAN;
        if (status != ORC_ENAN && bnorm > 0) {
            orc_dirac(L, t_bc, U, clover, x_, (double *)t, kappa, csw);
            for (long k = 0; k < n; k++) t[k] = b[k] - t[k];
            tr = sqrt(norm2(n, t)) / bnorm;
            if (status == ORC_OK && !(tr <= tol)) status = ORC_ENOCONV;
        } else if (bnorm == 0) {
            tr = 0.0;
        }
        out[0] = it;
        out[1] = tr;
        out[2] = restarts;
    }
    free(r);
    free(rh);
    free(p);
    free(v);
    free(s);
    free(t);
    return status;
}
