// Multi-shift CG on the normal even-odd operator, (M_hat^+ M_hat + sigma_i) x_i = b for several
// shifts at the cost of one Krylov space: the solves of a rational approximation in RHMC (paper
// Sec. IV uses RHMC; the multi-shift solver is the part of it that reuses the hot path).
// Shifted CG as in Jegerlehner (1996): the residuals of all shifted systems are collinear with the
// base residual, r_i = zeta_i r, and the zeta_i follow a scalar recurrence; every shift costs one
// axpy pair per iteration, the operator is applied once.  M_hat^+ needs no kernel of its own: with
// M^+ = g5 M g5 on the full lattice and A commuting with g5, the Schur complement S = A_ee M_hat
// satisfies S^+ = g5 S g5, so M_hat^+ psi = g5 A_ee M_hat (g5 A_ee^-1 psi).  FP64 throughout; the
// scalars live on the device (two one-block step kernels per iteration), shifts that have converged
// drop out of the vector updates, and the host synchronises only to read the done flag.
#include <cstddef>

#include "host.h"

namespace {

constexpr int MS_MAX = 64;  // shifts per solve

// Solver state on the device; wave 0 of the two step kernels owns it, every other kernel reads it.
struct MsState {
    double rr;            // (r, r) of the base system
    double a;             // alpha of the current iteration (0 once done: r stays put)
    double a_old, b_old;  // alpha and beta of the previous iteration
    double stop;          // tol^2 (b, b)
    int it, done, status, pad;  // status: 1 breakdown, 2 non-finite residual
    double z[MS_MAX], z_old[MS_MAX], z_new[MS_MAX], d[MS_MAX], res2[MS_MAX];
    int act[MS_MAX];            // shift still iterating
    double c[4 * MS_MAX + 1];   // per shift [alpha_i, zeta_i', beta_i, active], then beta
};

// Sum the per-block partials of a dot product over a 256-thread block; every thread gets the sum.
__device__ double sum_partials(const double* partials, int nb)
{
    double v[1] = {0.0};
    for (int b = threadIdx.x; b < nb; b += 256) v[0] += partials[b];
    __shared__ double tot[1];
    block_sum_store<1>(v, tot);
    __syncthreads();
    return tot[0];
}

// partials of (r, r), and their total
__global__ __launch_bounds__(256) void k_ms_norm(const double2* r, long n, double* partials)
{
    double acc[1] = {0.0};
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long)gridDim.x * 256) {
        const double2 rv = r[e];
        acc[0] += rv.x * rv.x + rv.y * rv.y;
    }
    block_sum_store<1>(acc, partials + blockIdx.x);
}

__global__ __launch_bounds__(256) void k_ms_total(const double* partials, int nb, double* out)
{
    const double v = sum_partials(partials, nb);
    if (threadIdx.x == 0) *out = v;
}

// w = g5 w + s0 p (g5 negates the elements from `half` on: spins 2 and 3) and the partials of (p, w)
__global__ __launch_bounds__(256) void k_ms_w_dot(double2* w, const double2* p, long n, long half, double s0,
                                                  double* partials)
{
    double acc[1] = {0.0};
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long)gridDim.x * 256) {
        const double2 pv = p[e];
        double2 v = w[e];
        const double sg = e < half ? 1.0 : -1.0;
        v.x = sg * v.x + s0 * pv.x;
        v.y = sg * v.y + s0 * pv.y;
        w[e] = v;
        acc[0] += pv.x * v.x + pv.y * v.y;
    }
    block_sum_store<1>(acc, partials + blockIdx.x);
}

// r -= alpha w and the partials of (r, r)
__global__ __launch_bounds__(256) void k_ms_axpy_norm(double2* r, const double2* w, const MsState* st, long n,
                                                      double* partials)
{
    const double a = st->a;
    double acc[1] = {0.0};
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long)gridDim.x * 256) {
        const double2 wv = w[e];
        double2 rv = r[e];
        rv.x -= a * wv.x;
        rv.y -= a * wv.y;
        r[e] = rv;
        acc[0] += rv.x * rv.x + rv.y * rv.y;
    }
    block_sum_store<1>(acc, partials + blockIdx.x);
}

// alpha = (r, r) / (p, N p) and the next zeta of every live shift (Jegerlehner's recurrence with the
// shift relative to the base shift, d_i = sigma_i - sigma_0)
__global__ __launch_bounds__(256) void k_ms_alpha(MsState* st, const double* partials, int nb, int nshift)
{
    const double pw = sum_partials(partials, nb);
    const int t = threadIdx.x;
    if (t >= 64) return;
    const int done = st->done;
    double a = 0.0;
    bool brk = false;
    if (!done) {
        if (!(pw > 0.0) || !isfinite(pw))
            brk = true;
        else
            a = st->rr / pw;
    }
    if (t < nshift && !done && !brk && st->act[t]) {
        const double z = st->z[t], zo = st->z_old[t], d = st->d[t];
        const double ao = st->a_old, bo = st->b_old;
        st->z_new[t] = z * zo * ao / (a * bo * (zo - z) + zo * ao * (1.0 + d * a));
    }
    if (t == 0) {
        st->a = a;
        if (brk) {
            st->status = 1;
            st->done = 1;
        }
    }
}

// beta = (r', r') / (r, r), the update coefficients of every shift, the shifted residuals |zeta_i'| |r'|;
// a shift whose residual reaches the stopping value takes this last update and then stays put
__global__ __launch_bounds__(256) void k_ms_beta(MsState* st, const double* partials, int nb, int nshift)
{
    const double rn = sum_partials(partials, nb);
    const int t = threadIdx.x;
    if (t >= 64) return;
    double* c = st->c + 4 * t;
    if (st->done) {
        if (t < nshift) c[0] = c[1] = c[2] = c[3] = 0.0;
        if (t == 0) st->c[4 * nshift] = 0.0;
        return;
    }
    const double a = st->a;
    bool bad = !isfinite(rn);
    const double beta = bad ? 0.0 : rn / st->rr;
    bool live = false;
    if (t < nshift) {
        bool upd = false;  // this shift takes an update in this iteration
        if (st->act[t] && !bad) {
            const double zn = st->z_new[t], z = st->z[t];
            const double q = zn / z;
            if (!isfinite(q)) {
                bad = true;
            } else {
                c[0] = a * q;
                c[1] = zn;
                c[2] = beta * q * q;
                c[3] = 1.0;
                upd = true;
                st->z_old[t] = z;
                st->z[t] = zn;
                const double r2 = zn * zn * rn;
                if (r2 <= st->stop) {
                    st->act[t] = 0;
                    st->res2[t] = r2;
                } else {
                    live = true;
                }
            }
        }
        if (!upd) c[0] = c[1] = c[2] = c[3] = 0.0;  // converged earlier (or failed): x_i and p_i stay put
    }
    const unsigned long long any_live = __ballot(live), any_bad = __ballot(bad);
    if (t == 0) {
        st->c[4 * nshift] = beta;
        if (any_bad) {
            st->status = 2;
            st->done = 1;
        } else {
            st->a_old = a;
            st->b_old = beta;
            st->rr = rn;
            st->it += 1;
            if (!any_live) st->done = 1;
        }
    }
}

// All shifted updates of one iteration in one pass, reading each old p_i once:
//   x_i += alpha_i p_i,  p_i = zeta_i' r + beta_i p_i  (live shifts only),  p = r + beta p.
// c = [alpha_i, zeta_i', beta_i, active] per shift, then beta; vectors X_i, P_i at stride n (complex).
__global__ __launch_bounds__(256) void k_shift_update(double2* X, double2* P, double2* p, const double2* r, long n,
                                                      int nshift, const double* c)
{
    const double beta = c[4 * nshift];
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long)gridDim.x * 256) {
        const double2 rv = r[e];
        for (int i = 0; i < nshift; i++) {
            if (c[4 * i + 3] == 0.0) continue;
            const double a = c[4 * i], z = c[4 * i + 1], b = c[4 * i + 2];
            const double2 pv = P[(long)i * n + e];
            double2 xv = X[(long)i * n + e];
            xv.x += a * pv.x;
            xv.y += a * pv.y;
            X[(long)i * n + e] = xv;
            P[(long)i * n + e] = make_double2(z * rv.x + b * pv.x, z * rv.y + b * pv.y);
        }
        const double2 pb = p[e];
        p[e] = make_double2(rv.x + beta * pb.x, rv.y + beta * pb.y);
    }
}

// g5 in the internal layout [4 spin][Vh][3]: negate spins 2 and 3 (the second half)
hipError_t apply_g5(hipStream_t s, void* v, const Geom& g)
{
    void* hi = (char*)v + 6L * g.Vh * 16;
    return launch_convert(s, F64, F64, hi, hi, 6L * g.Vh, -1.0, nullptr);
}

// r = b - w and the partials of (r, r): the true residual of a shifted system
__global__ __launch_bounds__(256) void k_ms_resid(double2* r, const double2* b, const double2* w, long n,
                                                  double* partials)
{
    double acc[1] = {0.0};
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long)gridDim.x * 256) {
        const double2 bv = b[e], wv = w[e];
        const double2 rv = make_double2(bv.x - wv.x, bv.y - wv.y);
        r[e] = rv;
        acc[0] += rv.x * rv.x + rv.y * rv.y;
    }
    block_sum_store<1>(acc, partials + blockIdx.x);
}

// x += c (a refinement's correction)
__global__ __launch_bounds__(256) void k_ms_add(double2* x, const double2* c, long n)
{
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long)gridDim.x * 256) {
        const double2 cv = c[e];
        double2 xv = x[e];
        xv.x += cv.x;
        xv.y += cv.y;
        x[e] = xv;
    }
}

// Drains the stream when the solve returns, so pooled buffers go back to the cache idle.
struct DrainOnExit {
    hipStream_t s;
    ~DrainOnExit() { (void)hipStreamSynchronize(s); }
};

// Device buffers of one solve (internal layout, n complex each) and the per-block dot partials.
struct MsBufs {
    void *r, *p, *w, *t1, *t2, *tmpo;
    double* part;
    int nb;
    MsState* st;
};

// w = (M_hat^+ M_hat + sigma) x with M_hat^+ = g5 A_ee M_hat g5 A_ee^-1; the partials of (x, w) land in
// B.part.  Uses t1, t2 and tmpo.
hipError_t apply_normal(hipStream_t s, const qcdw_op* op, const PrecView& v, const MsBufs& B, const void* x, void* w,
                        long n, double sigma)
{
    const Geom& g = op->g;
    hipError_t e = matpc(s, op, v, x, B.t1, B.tmpo, RED_NONE, nullptr, nullptr, nullptr);
    if (e == hipSuccess) e = launch_clov_apply_internal(s, F64, g, op->Ainv64[0].p, B.t1, B.t2);
    if (e == hipSuccess) e = apply_g5(s, B.t2, g);
    if (e == hipSuccess) e = matpc(s, op, v, B.t2, B.t1, B.tmpo, RED_NONE, nullptr, nullptr, nullptr);
    if (e == hipSuccess) e = launch_clov_apply_internal(s, F64, g, op->A64[0].p, B.t1, w);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ms_w_dot, dim3(B.nb), dim3(256), 0, s, (double2*)w, (const double2*)x, n, 6L * g.Vh, sigma,
                       B.part);
    return hipGetLastError();
}

// Shifted CG from x_i = 0 on the source held in B.r (overwritten), for ns shifts, solutions into X
// (ns fields at stride n) with search directions in P.  Runs until every shifted residual tracked by
// the recurrence is <= sqrt(stop2), or maxiter iterations; h returns the final state.
qcdw_status ms_cg(qcdw_ctx* ctx, qcdw_op* op, const PrecView& v, const MsBufs& B, void* X, void* P, long n, int ns,
                  const double* shifts, double stop2, int maxiter, MsState& h)
{
    hipStream_t s = ctx->stream;
    const size_t vb = (size_t)n * 16;
    double s0 = shifts[0];
    for (int i = 1; i < ns; i++) s0 = std::min(s0, shifts[i]);
    HIPCHK(ctx, launch_convert(s, F64, F64, B.r, B.p, n, 1.0, nullptr));
    for (int i = 0; i < ns; i++) {
        HIPCHK(ctx, launch_convert(s, F64, F64, B.r, (char*)P + i * vb, n, 1.0, nullptr));
        HIPCHK(ctx, hipMemsetAsync((char*)X + i * vb, 0, vb, s));
    }
    double* hd = ctx->host_d;  // pinned
    hipLaunchKernelGGL(k_ms_norm, dim3(B.nb), dim3(256), 0, s, (const double2*)B.r, n, B.part);
    hipLaunchKernelGGL(k_ms_total, dim3(1), dim3(256), 0, s, (const double*)B.part, B.nb, (double*)B.t1);
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, hipMemcpyAsync(hd, B.t1, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    const double rr0 = hd[0];
    if (!std::isfinite(rr0)) return fail(ctx, QCDW_ENAN, "multi-shift CG: non-finite source norm");
    h = MsState{};
    h.rr = rr0;
    h.a_old = 1.0;
    h.stop = stop2;
    h.done = rr0 <= stop2;
    for (int i = 0; i < ns; i++) {
        h.z[i] = h.z_old[i] = 1.0;
        h.d[i] = shifts[i] - s0;
        h.act[i] = !h.done;
        h.res2[i] = rr0;
    }
    MsState* st = B.st;
    HIPCHK(ctx, hipMemcpyAsync(st, &h, sizeof(MsState), hipMemcpyHostToDevice, s));
    // The scalars stay on the device: the host enqueues iterations and reads the done flag every
    // CHECK iterations; iterations enqueued after convergence change nothing (alpha = 0, no live shift).
    constexpr int CHECK = 4;
    const size_t flags_off = offsetof(MsState, it);
    for (int k = 0; k < maxiter && !h.done; k++) {
        HIPCHK(ctx, apply_normal(s, op, v, B, B.p, B.w, n, s0));
        hipLaunchKernelGGL(k_ms_alpha, dim3(1), dim3(256), 0, s, st, (const double*)B.part, B.nb, ns);
        hipLaunchKernelGGL(k_ms_axpy_norm, dim3(B.nb), dim3(256), 0, s, (double2*)B.r, (const double2*)B.w,
                           (const MsState*)st, n, B.part);
        hipLaunchKernelGGL(k_ms_beta, dim3(1), dim3(256), 0, s, st, (const double*)B.part, B.nb, ns);
        hipLaunchKernelGGL(k_shift_update, dim3(B.nb), dim3(256), 0, s, (double2*)X, (double2*)P, (double2*)B.p,
                           (const double2*)B.r, n, ns, (const double*)st->c);
        HIPCHK(ctx, hipGetLastError());
        if ((k + 1) % CHECK == 0 || k + 1 == maxiter) {
            HIPCHK(ctx, hipMemcpyAsync(hd, (char*)st + flags_off, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
            HIPCHK(ctx, hipStreamSynchronize(s));
            std::memcpy(&h.it, hd, 4 * sizeof(int));
        }
    }
    HIPCHK(ctx, hipMemcpyAsync(&h, st, sizeof(MsState), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    if (h.status == 1) return fail(ctx, QCDW_EBREAKDOWN, "multi-shift CG: (p, N p) is not positive");
    if (h.status == 2) return fail(ctx, QCDW_ENAN, "multi-shift CG: non-finite residual");
    return QCDW_OK;
}

// ||b - (N + sigma) x||^2 on the GPU in FP64 (b, x internal layout); the residual itself is left in B.r.
qcdw_status true_res2(qcdw_ctx* ctx, qcdw_op* op, const PrecView& v, const MsBufs& B, const void* bint, const void* x,
                      long n, double sigma, double& r2)
{
    hipStream_t s = ctx->stream;
    HIPCHK(ctx, apply_normal(s, op, v, B, x, B.w, n, sigma));
    hipLaunchKernelGGL(k_ms_resid, dim3(B.nb), dim3(256), 0, s, (double2*)B.r, (const double2*)bint,
                       (const double2*)B.w, n, B.part);
    hipLaunchKernelGGL(k_ms_total, dim3(1), dim3(256), 0, s, (const double*)B.part, B.nb, (double*)B.t1);
    HIPCHK(ctx, hipGetLastError());
    CHK(read_double(ctx, (const double*)B.t1, r2));
    if (!std::isfinite(r2)) return fail(ctx, QCDW_ENAN, "multi-shift CG: non-finite true residual");
    return QCDW_OK;
}

}  // namespace

extern "C" qcdw_status qcdw_invert_multishift(qcdw_op* op, const void* b_e, void* const* x_e, const double* shifts,
                                              int n_shifts, double tol, int maxiter, int* iters, double* res)
{
    if (!op) return QCDW_EINVAL;
    qcdw_ctx* ctx = op->ctx;
    DeviceGuard dg(ctx->device);
    if (!x_e || !shifts || !iters || !res) return fail(ctx, QCDW_EINVAL, "x_e, shifts, iters and res must not be NULL");
    if (n_shifts < 1 || n_shifts > MS_MAX) return fail(ctx, QCDW_EINVAL, "n_shifts must lie in [1, 64], got %d", n_shifts);
    if (!(tol > 0.0) || !std::isfinite(tol)) return fail(ctx, QCDW_EINVAL, "tol must be positive");
    if (maxiter < 0) return fail(ctx, QCDW_EINVAL, "maxiter must be >= 0");
    CHK(check_dev(ctx, b_e, "b_e"));
    for (int i = 0; i < n_shifts; i++) {
        if (!(shifts[i] >= 0.0) || !std::isfinite(shifts[i]))
            return fail(ctx, QCDW_EINVAL, "shift %d must be finite and >= 0", i);
        CHK(check_dev(ctx, x_e[i], "x_e[i]"));
        if (x_e[i] == b_e) return fail(ctx, QCDW_EINVAL, "x_e[%d] must not alias b_e", i);
    }
    *iters = 0;
    const Geom& g = op->g;
    const long n = 12L * g.Vh;  // complex elements of an even-site field
    const size_t vb = (size_t)n * 16;
    const PrecView v = view(op, F64);
    hipStream_t s = ctx->stream;
    const int nb = blas_blocks(n);
    // r, p, w, t1, t2, tmp_o, the packed b, a refinement's correction and direction, then X_i, P_i;
    // the partials of one dot product; the solver state
    PoolBuf buf, part, state;
    HIPCHK(ctx, buf.alloc(vb * (9 + 2 * (size_t)n_shifts)));
    HIPCHK(ctx, part.alloc((size_t)nb * sizeof(double)));
    HIPCHK(ctx, state.alloc(sizeof(MsState)));
    DrainOnExit drain{s};
    char* base = (char*)buf.p;
    MsBufs B{base, base + vb, base + 2 * vb, base + 3 * vb, base + 4 * vb, base + 5 * vb, (double*)part.p, nb,
             (MsState*)state.p};
    void *bint = base + 6 * vb, *xc = base + 7 * vb, *pc = base + 8 * vb;
    auto X = [&](int i) { return (void*)(base + (9 + i) * vb); };
    auto P = [&](int i) { return (void*)(base + (9 + n_shifts + i) * vb); };

    HIPCHK(ctx, launch_pack_spinor(s, F64, g, b_e, 0, bint, 1.0));
    HIPCHK(ctx, launch_convert(s, F64, F64, bint, B.r, n, 1.0, nullptr));
    // The recurrence runs to half the tolerance, so that the true residuals (which drift from the
    // recurrence's by rounding) normally pass without refinement.
    MsState h;
    {
        hipLaunchKernelGGL(k_ms_norm, dim3(nb), dim3(256), 0, s, (const double2*)bint, n, B.part);
        hipLaunchKernelGGL(k_ms_total, dim3(1), dim3(256), 0, s, (const double*)B.part, nb, (double*)B.t1);
        HIPCHK(ctx, hipGetLastError());
    }
    double bb = 0.0;
    CHK(read_double(ctx, (const double*)B.t1, bb));
    if (!std::isfinite(bb)) return fail(ctx, QCDW_ENAN, "multi-shift CG: non-finite source norm");
    const double half2 = 0.25 * tol * tol * bb;
    CHK(ms_cg(ctx, op, v, B, X(0), P(0), n, n_shifts, shifts, half2, maxiter, h));
    int used = h.it;
    *iters = used;
    for (int i = 0; i < n_shifts; i++) HIPCHK(ctx, launch_unpack_spinor(s, F64, g, X(i), 0, x_e[i], 1.0));
    if (!h.done) {
        for (int i = 0; i < n_shifts; i++) {
            const double r2 = h.act[i] ? h.z[i] * h.z[i] * h.rr : h.res2[i];
            res[i] = bb > 0.0 ? std::sqrt(r2 / bb) : 0.0;
        }
        HIPCHK(ctx, hipStreamSynchronize(s));
        return fail(ctx, QCDW_ENOCONV, "multi-shift CG did not converge within %d iterations", maxiter);
    }
    // True residuals, recomputed from each x_i in FP64; a shift above tol is refined by a
    // single-shift CG on its residual, x_i += c (at most three times, within the iteration budget).
    constexpr int MAX_REFINE = 3;
    bool all_ok = true;
    for (int i = 0; i < n_shifts; i++) {
        double r2 = 0.0;
        CHK(true_res2(ctx, op, v, B, bint, X(i), n, shifts[i], r2));
        for (int k = 0; k < MAX_REFINE && r2 > tol * tol * bb && used < maxiter; k++) {
            MsState hr;
            CHK(ms_cg(ctx, op, v, B, xc, pc, n, 1, shifts + i, half2, maxiter - used, hr));
            used += hr.it;
            hipLaunchKernelGGL(k_ms_add, dim3(nb), dim3(256), 0, s, (double2*)X(i), (const double2*)xc, n);
            HIPCHK(ctx, hipGetLastError());
            CHK(true_res2(ctx, op, v, B, bint, X(i), n, shifts[i], r2));
            HIPCHK(ctx, launch_unpack_spinor(s, F64, g, X(i), 0, x_e[i], 1.0));
        }
        res[i] = bb > 0.0 ? std::sqrt(r2 / bb) : 0.0;
        if (r2 > tol * tol * bb) all_ok = false;
    }
    *iters = used;
    HIPCHK(ctx, hipStreamSynchronize(s));
    if (!all_ok) return fail(ctx, QCDW_ENOCONV, "multi-shift CG: a true shifted residual stays above tol");
    return QCDW_OK;
}
