// BLAS-1 kernels of the Krylov solver with fused, deterministic reductions,
// and the small single-block kernels that turn reduction partials into the
// BiCGStab scalars on the device (van der Vorst 1992; paper Sec. II.E names
// BiCGStab as the clover solver).  Every reduction sums in a fixed order
// (fixed grid, lane-ordered wave sums, wave-ordered block sums, block-ordered
// final sum), so results are bitwise reproducible.
#include "internal.h"

namespace qcdw {

#define QCDW_GRID_LOOP(e, n) \
    for (long e = (long)blockIdx.x * BLAS_THREADS + threadIdx.x; e < (n); e += (long)gridDim.x * BLAS_THREADS)

// Vector y of a launch (blockIdx.y) covers elements [off, off + len): with a map
// (offset, length per vector: problems of different sizes) or uniformly y n, n.
#define QCDW_VEC_RANGE(n, map)                                            \
    const long off = (map) ? (map)[blockIdx.y].x : (long)blockIdx.y * (n); \
    const long nn = (map) ? (map)[blockIdx.y].y : (n);

// ---------------------------------------------------------------------------
// generic vector kernels
// ---------------------------------------------------------------------------
// one RHS per blockIdx.y: elements [y n, (y+1) n)
template <class P>
__global__ __launch_bounds__(256) void k_norm2(const void* x, long n, double* partials, const long2* map)
{
    double v[1] = {0.0};
    QCDW_VEC_RANGE(n, map)
    QCDW_GRID_LOOP(e, nn)
    {
        const auto a = P::ld(x, off + e);
        v[0] += (double)a.re * a.re + (double)a.im * a.im;
    }
    block_sum_store<1>(v, partials + (long)blockIdx.y * gridDim.x + blockIdx.x);
}

template <class PB, class PY>
__global__ __launch_bounds__(256) void k_xmy_norm2(const void* b, const void* y, double2* r, long n,
                                                   double* partials, const long2* map)
{
    double v[1] = {0.0};
    QCDW_VEC_RANGE(n, map)
    QCDW_GRID_LOOP(e, nn)
    {
        const auto bb = PB::ld(b, off + e);
        const auto yy = PY::ld(y, off + e);
        const double re = (double)bb.re - (double)yy.re, im = (double)bb.im - (double)yy.im;
        if (r) r[off + e] = make_double2(re, im);
        v[0] += re * re + im * im;
    }
    block_sum_store<1>(v, partials + (long)blockIdx.y * gridDim.x + blockIdx.x);
}

// one block per RHS: out[K x] = sum over the nb partials of RHS x
template <int K>
__global__ __launch_bounds__(256) void k_sum_partials(const double* partials, int nb, double* out)
{
    double v[K];
    const double* pp = partials + (long)blockIdx.x * nb * K;
#pragma unroll
    for (int k = 0; k < K; k++) v[k] = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256)
#pragma unroll
        for (int k = 0; k < K; k++) v[k] += pp[(long)b * K + k];
    block_sum_store<K>(v, out + (long)blockIdx.x * K);
}

// out = scale_y in for RHS y (scales: per-RHS device array, or nullptr for `scale`)
template <class PI, class PO>
__global__ __launch_bounds__(256) void k_convert(const void* in, void* out, long n, double scale,
                                                 const double* scales, const long2* map)
{
    using T = typename PO::real;
    QCDW_VEC_RANGE(n, map)
    const double sc = scales ? scales[blockIdx.y] : scale;
    QCDW_GRID_LOOP(e, nn)
    {
        const auto a = PI::ld(in, off + e);
        PO::st(out, off + e, cx<T>{(T)(sc * (double)a.re), (T)(sc * (double)a.im)});
    }
}

// y += a_y x for RHS y (coefs: per-RHS device array, or nullptr for `a`)
template <class PX>
__global__ __launch_bounds__(256) void k_axpy_hi(double a, const double* coefs, const void* x, double2* y, long n,
                                                 const long2* map)
{
    QCDW_VEC_RANGE(n, map)
    const double c = coefs ? coefs[blockIdx.y] : a;
    QCDW_GRID_LOOP(e, nn)
    {
        const auto xv = PX::ld(x, off + e);
        double2 yv = y[off + e];
        yv.x += c * (double)xv.re;
        yv.y += c * (double)xv.im;
        y[off + e] = yv;
    }
}

// out = B in, B the packed Hermitian clover-type matrix of each site (internal
// reordered packing, see hop.hip); one thread per (site, chirality, row half).
template <class P>
__global__ __launch_bounds__(256) void k_clov_apply(const void* clov, const void* in, void* out, int Vh)
{
    using T = typename P::real;
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= 4L * Vh) return;
    const int site = (int)(gid >> 2), q = (int)(gid & 3);  // q = spin
    const int h = q & 1, partner = q ^ 1;
    T win[27];
    const long base = clov_index(site, q >> 1, 9 * h);
#pragma unroll
    for (int e = 0; e < 27; e++) win[e] = P::ldr(clov, base + (long)e * CLOV_STRIDE);
    cx<T> vo[3], vx[3];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        vo[c] = P::ld(in, sp_idx(q, site, c, Vh));
        vx[c] = P::ld(in, sp_idx(partner, site, c, Vh));
    }
    // same row formula as the hop epilogue
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
        P::st(out, sp_idx(q, site, a, Vh), s);
    }
}

// ---------------------------------------------------------------------------
// BiCGStab pieces
// ---------------------------------------------------------------------------
__device__ __forceinline__ cx<double> cdiv(cx<double> a, cx<double> b)
{
    const double d = b.re * b.re + b.im * b.im;
    return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}
__device__ __forceinline__ cx<double> ld2(const double* p) { return {p[0], p[1]}; }
__device__ __forceinline__ void st2(double* p, cx<double> v)
{
    p[0] = v.re;
    p[1] = v.im;
}

// fixed-order sum of nb x 3 partials, result in every thread of the block (all threads must call it).
// Four rows per thread are loaded before they are added, so the loads overlap.
__device__ __forceinline__ void sum3(const double* partials, int nb, double (&v)[3])
{
    __shared__ double res[3];
    v[0] = v[1] = v[2] = 0.0;
    for (int b0 = threadIdx.x; b0 < nb; b0 += 4 * 256) {
        double t[4][3];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int b = b0 + u * 256;
#pragma unroll
            for (int k = 0; k < 3; k++) t[u][k] = b < nb ? partials[3L * b + k] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; u++)
#pragma unroll
            for (int k = 0; k < 3; k++) v[k] += t[u][k];
    }
    block_sum_store<3>(v, res);
    __syncthreads();
    v[0] = res[0];
    v[1] = res[1];
    v[2] = res[2];
}

// The three scalar steps of a BiCGStab iteration.  Each one turns the summed reduction partials v
// into the next scalar (or a flag), and a matching record step writes it to the problem's S.  A
// single-block kernel runs step and record back to back; a fused vector kernel runs the step in
// every block (same partials, same order: the same value everywhere) and block 0 of each problem
// records it.  Block 0 writes the flags only when its step sets one, and then every block's step
// sets the same one, so a block that reads the flags while they change leaves all the same.  A step
// reads only fields of S that no block writes in the same launch:
//   alpha step reads rho, r0n2, rr         records alpha, rho_prev (= rho), flags
//   omega step reads nothing               records omega, iter (+1), flags
//   beta  step reads rho_prev, alpha,      records beta, rho, rr, history, flags
//              omega, iter, r0n2, stop_rr, fault_iter
// alpha = rho / (r0, v) with v = M p; v holds ((r0, v), -)
__device__ __forceinline__ int alpha_step(const Scal* S, const double (&v)[3], cx<double>& alpha)
{
    const cx<double> rv = {v[0], v[1]};
    const double arv = sqrt(rv.re * rv.re + rv.im * rv.im);
    if (!isfinite(arv)) return FLAG_NAN;
    if (arv <= 1e-30 * sqrt(S->r0n2 * S->rr)) return FLAG_BREAK;
    alpha = cdiv(ld2(S->rho), rv);
    return 0;
}
__device__ __forceinline__ void alpha_record(Scal* S, int flag, cx<double> alpha)
{
    if (flag) {
        S->flags = flag;
        return;
    }
    st2(S->alpha, alpha);
    st2(S->rho_prev, ld2(S->rho));
}

// omega = (t, s) / (t, t) with t = M s; v holds ((t, s), ||t||^2).  s = 0 gives omega = 0: x + alpha p
// is then exact and the beta step flags the breakdown unless the residual has converged.
__device__ __forceinline__ int omega_step(const double (&v)[3], cx<double>& omega)
{
    const double tt = v[2];
    if (!isfinite(tt) || !isfinite(v[0]) || !isfinite(v[1])) return FLAG_NAN;
    omega = tt == 0.0 ? cx<double>{0.0, 0.0} : cx<double>{v[0] / tt, v[1] / tt};
    return 0;
}
__device__ __forceinline__ void omega_record(Scal* S, int flag, cx<double> omega)
{
    if (flag) {
        S->flags = flag;
        return;
    }
    st2(S->omega, omega);
    S->iter = S->iter + 1;
}

// rho' = (r0, r), beta = (rho' / rho)(alpha / omega); v holds ((r0, r), ||r||^2) of the new residual
__device__ __forceinline__ int beta_step(const Scal* S, const double (&v)[3], cx<double>& beta)
{
    const cx<double> rho_new = {v[0], v[1]};
    const double rr = v[2];
    const int it = S->iter;
    const cx<double> omega = ld2(S->omega);
    if (!isfinite(rr) || !isfinite(rho_new.re) || !isfinite(rho_new.im) ||
        (S->fault_iter < 0 && it == -S->fault_iter))
        return FLAG_NAN;
    if (rr <= S->stop_rr) return FLAG_CONV;
    if (omega.re == 0.0 && omega.im == 0.0) return FLAG_BREAK;
    if (sqrt(rho_new.re * rho_new.re + rho_new.im * rho_new.im) <= 1e-30 * sqrt(S->r0n2 * rr)) return FLAG_BREAK;
    if (S->fault_iter > 0 && it == S->fault_iter) return FLAG_BREAK;
    beta = cdiv(rho_new, ld2(S->rho_prev)) * cdiv(ld2(S->alpha), omega);
    return 0;
}
// hist: the problem's residual history (or nullptr)
__device__ __forceinline__ void beta_record(Scal* S, const double (&v)[3], int flag, cx<double> beta, double* hist)
{
    const int it = S->iter;
    S->rr = v[2];
    if (hist && it < S->hist_len) hist[it] = sqrt(v[2]) * S->hist_norm;
    if (flag) {
        S->flags = flag;
        return;
    }
    st2(S->beta, beta);
    st2(S->rho, cx<double>{v[0], v[1]});
}

// Fused scalar input of a vector kernel: fin[y][nb][3] reduction partials of problem y (nbs: per-problem
// counts, or nullptr for nb).  With fin == nullptr the scalar was recorded in S by a finaliser kernel.
struct Fin {
    const double* fin;
    int nb;
    const int* nbs;
    double* hist;  // beta step only
};
__device__ __forceinline__ void fin_sum(const Fin& f, double (&v)[3])
{
    sum3(f.fin + 3L * f.nb * blockIdx.y, f.nbs ? f.nbs[blockIdx.y] : f.nb, v);
}
__device__ __forceinline__ bool records() { return blockIdx.x == 0 && threadIdx.x == 0; }

// p = r + beta (p - omega v)
// blockIdx.y selects the right-hand side: its scalars S[y] and elements [y n, (y+1) n)
template <class P>
__global__ __launch_bounds__(256) void k_bicg_p(void* p, const void* r, const void* v, long n, Scal* S,
                                                const long2* map, Fin f)
{
    S += blockIdx.y;
    const int f0 = S->flags;  // issued together with the partials' loads
    cx<double> beta;
    if (f.fin) {
        double acc[3];
        fin_sum(f, acc);  // every thread takes part (block barriers)
        const int fl = f0 ? f0 : beta_step(S, acc, beta);
        if (records() && !f0) beta_record(S, acc, fl, beta, f.hist ? f.hist + (long)blockIdx.y * S->hist_len : nullptr);
        if (fl) return;
    } else {
        if (f0) return;
        beta = ld2(S->beta);
    }
    using T = typename P::real;
    QCDW_VEC_RANGE(n, map)
    const cx<T> bt = {(T)beta.re, (T)beta.im}, omega = {(T)S->omega[0], (T)S->omega[1]};
    QCDW_GRID_LOOP(e, nn)
    {
        const auto pv = P::ld(p, off + e), rv = P::ld(r, off + e), vv = P::ld(v, off + e);
        P::st(p, off + e, rv + bt * (pv - omega * vv));
    }
}

// s = r - alpha v
template <class P>
__global__ __launch_bounds__(256) void k_bicg_s(void* sv, const void* r, const void* v, long n, Scal* S,
                                                const long2* map, Fin f)
{
    S += blockIdx.y;
    const int f0 = S->flags;  // issued together with the partials' loads
    cx<double> alpha;
    if (f.fin) {
        double acc[3];
        fin_sum(f, acc);  // every thread takes part (block barriers)
        const int fl = f0 ? f0 : alpha_step(S, acc, alpha);
        if (records() && !f0) alpha_record(S, fl, alpha);
        if (fl) return;
    } else {
        if (f0) return;
        alpha = ld2(S->alpha);
    }
    using T = typename P::real;
    QCDW_VEC_RANGE(n, map)
    const cx<T> al = {(T)alpha.re, (T)alpha.im};
    QCDW_GRID_LOOP(e, nn)
    {
        const auto rv = P::ld(r, off + e), vv = P::ld(v, off + e);
        P::st(sv, off + e, rv - al * vv);
    }
}

// x += alpha p + omega s ; r = s - omega t ; partials (r0, r), ||r||^2 (must not overlap f.fin)
template <class P, class PX>
__global__ __launch_bounds__(256) void k_bicg_xr(void* x, const void* p, const void* sv, void* r, const void* t,
                                                 const void* r0, long n, Scal* S, double* partials,
                                                 const long2* map, Fin f)
{
    S += blockIdx.y;
    const int f0 = S->flags;  // issued together with the partials' loads
    cx<double> om;
    if (f.fin) {
        double acc[3];
        fin_sum(f, acc);  // every thread takes part (block barriers)
        const int fl = f0 ? f0 : omega_step(acc, om);
        if (records() && !f0) omega_record(S, fl, om);
        if (fl) return;
    } else {
        if (f0) return;
        om = ld2(S->omega);
    }
    using T = typename P::real;
    using TX = typename PX::real;
    QCDW_VEC_RANGE(n, map)
    const cx<TX> alpha = {(TX)S->alpha[0], (TX)S->alpha[1]}, omega_x = {(TX)om.re, (TX)om.im};
    const cx<T> omega = {(T)om.re, (T)om.im};
    double acc[3] = {0.0, 0.0, 0.0};
    QCDW_GRID_LOOP(e, nn)
    {
        const auto pv = P::ld(p, off + e), sv_ = P::ld(sv, off + e), tv = P::ld(t, off + e), w = P::ld(r0, off + e);
        const cx<TX> xv = PX::ld(x, off + e);
        const cx<TX> pX = {(TX)pv.re, (TX)pv.im}, sX = {(TX)sv_.re, (TX)sv_.im};
        PX::st(x, off + e, xv + alpha * pX + omega_x * sX);
        const auto rn = P::rt(sv_ - omega * tv);
        P::st(r, off + e, rn);
        acc[0] += (double)w.re * rn.re + (double)w.im * rn.im;
        acc[1] += (double)w.re * rn.im - (double)w.im * rn.re;
        acc[2] += (double)rn.re * rn.re + (double)rn.im * rn.im;
    }
    block_sum_store<3>(acc, partials + 3L * ((long)blockIdx.y * gridDim.x + blockIdx.x));
}

// partials ((w, r), ||r||^2) per vector of a launch
template <class P>
__global__ __launch_bounds__(256) void k_wdot_norm2(const void* w, const void* r, long n, double* partials,
                                                    const long2* map)
{
    double acc[3] = {0.0, 0.0, 0.0};
    QCDW_VEC_RANGE(n, map)
    QCDW_GRID_LOOP(e, nn)
    {
        const auto wv = P::ld(w, off + e), rv = P::ld(r, off + e);
        acc[0] += (double)wv.re * rv.re + (double)wv.im * rv.im;
        acc[1] += (double)wv.re * rv.im - (double)wv.im * rv.re;
        acc[2] += (double)rv.re * rv.re + (double)rv.im * rv.im;
    }
    block_sum_store<3>(acc, partials + 3L * ((long)blockIdx.y * gridDim.x + blockIdx.x));
}

// Continue the recurrence after a reliable update that replaced r by the (rescaled) true residual:
// rho' = (r0, r), beta = (rho' / rho)(alpha / omega) with the last step's alpha and omega, then the
// usual p = r + beta (p - omega v).  Any rescaling of r cancels in beta (p, v and rho carry the old
// scale together).  A near-zero rho' is a breakdown (the caller restarts).  The last step ended in
// convergence, so rho is still the value its alpha step used.
__global__ __launch_bounds__(256) void k_bicg_resume(Scal* S, const double* partials, int nb)
{
    S += blockIdx.x;
    if (S->flags) return;
    double v[3];
    sum3(partials + 3L * nb * blockIdx.x, nb, v);
    if (threadIdx.x == 0) {
        const cx<double> rho_new = {v[0], v[1]};
        const double rr = v[2];
        const cx<double> omega = ld2(S->omega);
        S->rr = rr;
        if (!isfinite(rr) || !isfinite(rho_new.re) || !isfinite(rho_new.im)) {
            S->flags = FLAG_NAN;
        } else if (rr <= S->stop_rr) {
            S->flags = FLAG_CONV;
        } else if ((omega.re == 0.0 && omega.im == 0.0) ||
                   sqrt(rho_new.re * rho_new.re + rho_new.im * rho_new.im) <= 1e-30 * sqrt(S->r0n2 * rr)) {
            S->flags = FLAG_BREAK;
        } else {
            st2(S->beta, cdiv(rho_new, ld2(S->rho)) * cdiv(ld2(S->alpha), omega));
            st2(S->rho, rho_new);
        }
    }
}

// Start of a Krylov cycle from the FP64 residual rhi of every problem: r = scale_y rhi rounded to
// the Krylov precision; without `resume` also r0 = p = r and partials of ||r||^2 (of the rounded
// r, as the iteration sees it); x_lo = 0 when given (the FP32 correction of a mixed cycle).
template <class P>
__global__ __launch_bounds__(256) void k_cycle_start(const double2* rhi, void* r, void* r0, void* p, float2* xlo,
                                                     long n, const double* scales, double* partials,
                                                     const long2* map, int resume)
{
    using T = typename P::real;
    QCDW_VEC_RANGE(n, map)
    const double sc = scales[blockIdx.y];
    double acc[1] = {0.0};
    QCDW_GRID_LOOP(e, nn)
    {
        const double2 a = rhi[off + e];
        const cx<T> v = P::rt(cx<T>{(T)(sc * a.x), (T)(sc * a.y)});
        P::st(r, off + e, v);
        if (!resume) {
            P::st(r0, off + e, v);
            P::st(p, off + e, v);
            acc[0] += (double)v.re * v.re + (double)v.im * v.im;
        }
        if (xlo) xlo[off + e] = make_float2(0.f, 0.f);
    }
    if (!resume) block_sum_store<1>(acc, partials + (long)blockIdx.y * gridDim.x + blockIdx.x);
}

// start (or restart) from the residual r with r0 = r: rho = (r0, r) = ||r||^2, summed from the nb
// partials of each problem (one block per problem)
__global__ __launch_bounds__(256) void k_bicg_init(Scal* S, const double* partials, int nb)
{
    S += blockIdx.x;
    double v[1] = {0.0};
    for (int b = threadIdx.x; b < nb; b += 256) v[0] += partials[(long)blockIdx.x * nb + b];
    __shared__ double res;
    block_sum_store<1>(v, &res);
    __syncthreads();
    if (threadIdx.x) return;
    const double rr = res;
    S->rho[0] = rr;
    S->rho[1] = 0.0;
    S->rho_prev[0] = rr;
    S->rho_prev[1] = 0.0;
    S->rr = rr;
    S->r0n2 = rr;
    S->alpha[0] = 1.0;
    S->alpha[1] = 0.0;
    S->omega[0] = 1.0;
    S->omega[1] = 0.0;
    S->beta[0] = 0.0;
    S->beta[1] = 0.0;
    S->flags = (rr <= S->stop_rr) ? FLAG_CONV : 0;
    if (!isfinite(rr)) S->flags = FLAG_NAN;
}

// single-block finalisers: one block per problem (blockIdx.x), partials [problem][nb][3]
__global__ __launch_bounds__(256) void k_fin_alpha(Scal* S, const double* partials, int nb, const int* nbs)
{
    S += blockIdx.x;
    if (S->flags) return;  // no other block of this launch writes them
    double v[3];
    sum3(partials + 3L * nb * blockIdx.x, nbs ? nbs[blockIdx.x] : nb, v);
    cx<double> alpha;
    const int fl = alpha_step(S, v, alpha);
    if (threadIdx.x == 0) alpha_record(S, fl, alpha);
}

__global__ __launch_bounds__(256) void k_fin_omega(Scal* S, const double* partials, int nb, const int* nbs)
{
    S += blockIdx.x;
    if (S->flags) return;  // no other block of this launch writes them
    double v[3];
    sum3(partials + 3L * nb * blockIdx.x, nbs ? nbs[blockIdx.x] : nb, v);
    cx<double> omega;
    const int fl = omega_step(v, omega);
    if (threadIdx.x == 0) omega_record(S, fl, omega);
}

__global__ __launch_bounds__(256) void k_fin_beta(Scal* S, const double* partials, int nb, double* hist)
{
    S += blockIdx.x;
    if (S->flags) return;  // no other block of this launch writes them
    double v[3];
    sum3(partials + 3L * nb * blockIdx.x, nb, v);
    cx<double> beta;
    const int fl = beta_step(S, v, beta);
    if (threadIdx.x == 0) beta_record(S, v, fl, beta, hist ? hist + (long)blockIdx.x * S->hist_len : nullptr);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
#define QCDW_DISPATCH1(prec, KERNEL, ...)                                              \
    switch (prec) {                                                                    \
    case F64: hipLaunchKernelGGL(KERNEL<P64>, __VA_ARGS__); break;                     \
    case F32: hipLaunchKernelGGL(KERNEL<P32>, __VA_ARGS__); break;                     \
    case BF16: hipLaunchKernelGGL(KERNEL<PBF16>, __VA_ARGS__); break;                  \
    case F16: hipLaunchKernelGGL(KERNEL<PF16>, __VA_ARGS__); break;                    \
    default: return hipErrorInvalidValue;                                              \
    }

// grid.x covers the longest vector of the launch (nmax); blocks past a shorter
// vector's end contribute zero partials
hipError_t launch_norm2(hipStream_t s, int prec, const void* x, long n, double* partials, double* out, int nrhs,
                        const long2* map, long nmax)
{
    const int nb = blas_blocks(map ? nmax : n);
    QCDW_DISPATCH1(prec, k_norm2, dim3(nb, nrhs), dim3(256), 0, s, x, n, partials, map)
    hipLaunchKernelGGL(k_sum_partials<1>, dim3(nrhs), dim3(256), 0, s, partials, nb, out);
    return hipGetLastError();
}

template <class PB>
static hipError_t xmy_b(hipStream_t s, int prec_y, const void* b, const void* y, void* r, long n, double* partials,
                        int nrhs, const long2* map, int nb)
{
    const dim3 grid(nb, nrhs);
    switch (prec_y) {
    case F64: hipLaunchKernelGGL((k_xmy_norm2<PB, P64>), grid, dim3(256), 0, s, b, y, (double2*)r, n, partials, map); break;
    case F32: hipLaunchKernelGGL((k_xmy_norm2<PB, P32>), grid, dim3(256), 0, s, b, y, (double2*)r, n, partials, map); break;
    default: return hipErrorInvalidValue;
    }
    return hipSuccess;
}

hipError_t launch_xmy_norm2(hipStream_t s, int prec_b, int prec_y, const void* b, const void* y, void* r, long n,
                            double* partials, double* out, int nrhs, const long2* map, long nmax)
{
    const int nb = blas_blocks(map ? nmax : n);
    hipError_t e;
    if (prec_b == F64) e = xmy_b<P64>(s, prec_y, b, y, r, n, partials, nrhs, map, nb);
    else if (prec_b == F32) e = xmy_b<P32>(s, prec_y, b, y, r, n, partials, nrhs, map, nb);
    else return hipErrorInvalidValue;
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sum_partials<1>, dim3(nrhs), dim3(256), 0, s, partials, nb, out);
    return hipGetLastError();
}

template <class PI>
static hipError_t convert_in(hipStream_t s, int prec_out, const void* in, void* out, long n, double scale,
                             const double* scales, int nrhs, const long2* map, int nb)
{
    const dim3 grid(nb, nrhs);
    switch (prec_out) {
    case F64: hipLaunchKernelGGL((k_convert<PI, P64>), grid, dim3(256), 0, s, in, out, n, scale, scales, map); break;
    case F32: hipLaunchKernelGGL((k_convert<PI, P32>), grid, dim3(256), 0, s, in, out, n, scale, scales, map); break;
    case BF16: hipLaunchKernelGGL((k_convert<PI, PBF16>), grid, dim3(256), 0, s, in, out, n, scale, scales, map); break;
    case F16: hipLaunchKernelGGL((k_convert<PI, PF16>), grid, dim3(256), 0, s, in, out, n, scale, scales, map); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_convert(hipStream_t s, int prec_in, int prec_out, const void* in, void* out, long n, double scale,
                          const double* scales, int nrhs, const long2* map, long nmax)
{
    const int nb = blas_blocks(map ? nmax : n);
    switch (prec_in) {
    case F64: return convert_in<P64>(s, prec_out, in, out, n, scale, scales, nrhs, map, nb);
    case F32: return convert_in<P32>(s, prec_out, in, out, n, scale, scales, nrhs, map, nb);
    case BF16: return convert_in<PBF16>(s, prec_out, in, out, n, scale, scales, nrhs, map, nb);
    case F16: return convert_in<PF16>(s, prec_out, in, out, n, scale, scales, nrhs, map, nb);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_axpy_hi(hipStream_t s, int prec_x, double a, const double* coefs, const void* x, void* y, long n,
                          int nrhs, const long2* map, long nmax)
{
    QCDW_DISPATCH1(prec_x, k_axpy_hi, dim3(blas_blocks(map ? nmax : n), nrhs), dim3(256), 0, s, a, coefs, x,
                   (double2*)y, n, map)
    return hipGetLastError();
}

hipError_t launch_clov_apply_internal(hipStream_t s, int prec, const Geom& g, const void* clov, const void* in,
                                      void* out)
{
    const long n = 4L * g.Vh;
    if (n == 0) return hipSuccess;
    QCDW_DISPATCH1(prec, k_clov_apply, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, clov, in, out, g.Vh)
    return hipGetLastError();
}

hipError_t launch_cycle_start(hipStream_t s, int prec, const void* rhi, void* r, void* r0, void* p, void* xlo, long n,
                              const double* scales, Scal* S, double* partials, int nrhs, const long2* map, long nmax,
                              bool resume)
{
    const int nb = blas_blocks(map ? nmax : n);
    QCDW_DISPATCH1(prec, k_cycle_start, dim3(nb, nrhs), dim3(256), 0, s, (const double2*)rhi, r, r0, p, (float2*)xlo,
                   n, scales, partials, map, resume ? 1 : 0)
    if (!resume) hipLaunchKernelGGL(k_bicg_init, dim3(nrhs), dim3(256), 0, s, S, partials, nb);
    return hipGetLastError();
}

hipError_t launch_bicg_resume(hipStream_t s, int prec, const void* r0, const void* r, long n, Scal* S,
                              double* partials, int nrhs, const long2* map, long nmax)
{
    const int nb = blas_blocks(map ? nmax : n);
    QCDW_DISPATCH1(prec, k_wdot_norm2, dim3(nb, nrhs), dim3(256), 0, s, r0, r, n, partials, map)
    hipLaunchKernelGGL(k_bicg_resume, dim3(nrhs), dim3(256), 0, s, S, partials, nb);
    return hipGetLastError();
}

hipError_t launch_bicg_p(hipStream_t s, int prec, void* p, const void* r, const void* v, long n, Scal* S,
                         int nrhs, const long2* map, long nmax, const double* fin, int fin_nb, double* hist)
{
    const Fin f{fin, fin_nb, nullptr, hist};
    QCDW_DISPATCH1(prec, k_bicg_p, dim3(blas_blocks(map ? nmax : n), nrhs), dim3(256), 0, s, p, r, v, n, S, map, f)
    return hipGetLastError();
}

hipError_t launch_bicg_s(hipStream_t s, int prec, void* sv, const void* r, const void* v, long n, Scal* S,
                         int nrhs, const long2* map, long nmax, const double* fin, int fin_nb, const int* fin_nbs)
{
    const Fin f{fin, fin_nb, fin_nbs, nullptr};
    QCDW_DISPATCH1(prec, k_bicg_s, dim3(blas_blocks(map ? nmax : n), nrhs), dim3(256), 0, s, sv, r, v, n, S, map, f)
    return hipGetLastError();
}

template <class PX>
static hipError_t bicg_xr_x(hipStream_t s, int prec, void* x, const void* p, const void* sv, void* r, const void* t,
                            const void* r0, long n, Scal* S, double* partials, int nrhs, const long2* map, int nb,
                            const Fin& f)
{
    const dim3 grid(nb, nrhs);
    switch (prec) {
    case F64: hipLaunchKernelGGL((k_bicg_xr<P64, PX>), grid, dim3(256), 0, s, x, p, sv, r, t, r0, n, S, partials, map, f); break;
    case F32: hipLaunchKernelGGL((k_bicg_xr<P32, PX>), grid, dim3(256), 0, s, x, p, sv, r, t, r0, n, S, partials, map, f); break;
    case BF16: hipLaunchKernelGGL((k_bicg_xr<PBF16, PX>), grid, dim3(256), 0, s, x, p, sv, r, t, r0, n, S, partials, map, f); break;
    case F16: hipLaunchKernelGGL((k_bicg_xr<PF16, PX>), grid, dim3(256), 0, s, x, p, sv, r, t, r0, n, S, partials, map, f); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_bicg_xr(hipStream_t s, int prec, int prec_x, void* x, const void* p, const void* sv, void* r,
                          const void* t, const void* r0, long n, Scal* S, double* partials, int nrhs,
                          const long2* map, long nmax, const double* fin, int fin_nb, const int* fin_nbs)
{
    const int nb = blas_blocks(map ? nmax : n);
    // the fused omega step reads fin while the blocks write their own partials
    if (fin && partials < fin + 3L * fin_nb * nrhs && fin < partials + 3L * nb * nrhs) return hipErrorInvalidValue;
    const Fin f{fin, fin_nb, fin_nbs, nullptr};
    if (prec_x == F64) return bicg_xr_x<P64>(s, prec, x, p, sv, r, t, r0, n, S, partials, nrhs, map, nb, f);
    if (prec_x == F32) return bicg_xr_x<P32>(s, prec, x, p, sv, r, t, r0, n, S, partials, nrhs, map, nb, f);
    return hipErrorInvalidValue;
}

hipError_t launch_fin_alpha(hipStream_t s, Scal* S, const double* partials, int nb, int nrhs, const int* nbs)
{
    hipLaunchKernelGGL(k_fin_alpha, dim3(nrhs), dim3(256), 0, s, S, partials, nb, nbs);
    return hipGetLastError();
}
hipError_t launch_fin_omega(hipStream_t s, Scal* S, const double* partials, int nb, int nrhs, const int* nbs)
{
    hipLaunchKernelGGL(k_fin_omega, dim3(nrhs), dim3(256), 0, s, S, partials, nb, nbs);
    return hipGetLastError();
}
hipError_t launch_fin_beta(hipStream_t s, Scal* S, const double* partials, int nb, double* hist, int nrhs)
{
    hipLaunchKernelGGL(k_fin_beta, dim3(nrhs), dim3(256), 0, s, S, partials, nb, hist);
    return hipGetLastError();
}

}  // namespace qcdw
