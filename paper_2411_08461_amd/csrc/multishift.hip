// Multi-shift CG on the normal even-odd operator, (M_hat^+ M_hat + sigma_i) x_i = b for several
// shifts at the cost of one Krylov space: the solves of a rational approximation in RHMC (paper
// Sec. IV uses RHMC; the multi-shift solver is the part of it that reuses the hot path).
// Shifted CG as in Jegerlehner (1996): the residuals of all shifted systems are collinear with the
// base residual, r_i = zeta_i r, and the zeta_i follow a scalar recurrence; every shift costs one
// axpy pair per iteration, the operator is applied once.  M_hat^+ needs no kernel of its own: with
// M^+ = g5 M g5 on the full lattice and A commuting with g5, the Schur complement S = A_ee M_hat
// satisfies S^+ = g5 S g5, so M_hat^+ psi = g5 A_ee M_hat (g5 A_ee^-1 psi).  FP64 throughout; the
// scalars are formed on the host (one synchronisation per dot product).
#include "host.h"

namespace {

// All shifted updates of one iteration in one pass, reading each old p_i once:
//   x_i += alpha_i p_i,  p_i = zeta_i' r + beta_i p_i  (i < nshift),  p = r + beta p.
// c = [alpha_i, zeta_i', beta_i] per shift, then beta; vectors X_i, P_i at stride n (complex elements).
__global__ __launch_bounds__(256) void k_shift_update(double2* X, double2* P, double2* p, const double2* r, long n,
                                                      int nshift, const double* c)
{
    const double beta = c[3 * nshift];
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long)gridDim.x * 256) {
        const double2 rv = r[e];
        for (int i = 0; i < nshift; i++) {
            const double a = c[3 * i], z = c[3 * i + 1], b = c[3 * i + 2];
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

}  // namespace

extern "C" qcdw_status qcdw_invert_multishift(qcdw_op* op, const void* b_e, void* const* x_e, const double* shifts,
                                              int n_shifts, double tol, int maxiter, int* iters, double* res)
{
    if (!op) return QCDW_EINVAL;
    qcdw_ctx* ctx = op->ctx;
    DeviceGuard dg(ctx->device);
    if (!x_e || !shifts || !iters || !res) return fail(ctx, QCDW_EINVAL, "x_e, shifts, iters and res must not be NULL");
    if (n_shifts < 1 || n_shifts > 64) return fail(ctx, QCDW_EINVAL, "n_shifts must lie in [1, 64], got %d", n_shifts);
    if (!(tol > 0.0) || !std::isfinite(tol)) return fail(ctx, QCDW_EINVAL, "tol must be positive");
    if (maxiter < 0) return fail(ctx, QCDW_EINVAL, "maxiter must be >= 0");
    CHK(check_dev(ctx, b_e, "b_e"));
    for (int i = 0; i < n_shifts; i++) {
        if (!(shifts[i] >= 0.0) || !std::isfinite(shifts[i]))
            return fail(ctx, QCDW_EINVAL, "shift %d must be finite and >= 0", i);
        CHK(check_dev(ctx, x_e[i], "x_e[i]"));
        if (x_e[i] == b_e) return fail(ctx, QCDW_EINVAL, "x_e[%d] must not alias b_e", i);
    }
    const Geom& g = op->g;
    const long n = 12L * g.Vh;  // complex elements of an even-site field
    const size_t vb = (size_t)n * 16;
    const PrecView v = view(op, F64);
    hipStream_t s = ctx->stream;
    // r, p, w, t1, t2, tmp_o, then X_i, P_i
    DevBuf buf, part, dev;
    HIPCHK(ctx, buf.alloc(vb * (6 + 2 * (size_t)n_shifts)));
    HIPCHK(ctx, part.alloc(16UL * 2048 * sizeof(double)));
    // device scalars: [0, 2) a dot product; [2, 4) the base shift and [4, 6) alpha as complex pairs for
    // the axpys; [6, 7 + 3n) the shifted-update coefficients [alpha_i, zeta_i', beta_i] and beta.  Each
    // block is staged at the same offset of the pinned host buffer and copied once, after the
    // synchronisation that precedes it, so no staged value is overwritten before its copy has run.
    const int nsc = 7 + 3 * n_shifts;
    static_assert(HOST_D_N >= 7 + 3 * 64, "pinned host staging too small for 64 shifts");
    HIPCHK(ctx, dev.alloc(nsc * sizeof(double)));
    char* base = (char*)buf.p;
    void *r = base, *p = base + vb, *w = base + 2 * vb, *t1 = base + 3 * vb, *t2 = base + 4 * vb, *tmpo = base + 5 * vb;
    auto X = [&](int i) { return (void*)(base + (6 + i) * vb); };
    auto P = [&](int i) { return (void*)(base + (6 + n_shifts + i) * vb); };
    double* dd = (double*)dev.p;  // device scalars
    double* hd = ctx->host_d;     // pinned staging, same offsets
    const int c_s0 = 2, c_a = 4, c_up = 6;
    double s0 = shifts[0];
    for (int i = 1; i < n_shifts; i++) s0 = std::min(s0, shifts[i]);
    auto stage = [&](int off, int count) -> qcdw_status {  // copy hd[off, off + count) to the device
        HIPCHK(ctx, hipMemcpyAsync(dd + off, hd + off, count * sizeof(double), hipMemcpyHostToDevice, s));
        return QCDW_OK;
    };
    auto read_dot = [&](const void* a, const void* b_, double& re) -> qcdw_status {
        HIPCHK(ctx, launch_multidot(s, a, 0, 1, b_, n, (double*)part.p, dd));
        HIPCHK(ctx, hipMemcpyAsync(hd, dd, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(ctx, hipStreamSynchronize(s));
        re = hd[0];
        return QCDW_OK;
    };

    HIPCHK(ctx, launch_pack_spinor(s, F64, g, b_e, 0, r, 1.0));
    HIPCHK(ctx, launch_convert(s, F64, F64, r, p, n, 1.0, nullptr));
    for (int i = 0; i < n_shifts; i++) {
        HIPCHK(ctx, launch_convert(s, F64, F64, r, P(i), n, 1.0, nullptr));
        HIPCHK(ctx, hipMemsetAsync(X(i), 0, vb, s));
    }
    hd[c_s0] = s0;
    hd[c_s0 + 1] = 0.0;
    CHK(stage(c_s0, 2));
    double bb;
    CHK(read_dot(r, r, bb));  // synchronises: the staged constants are on the device
    std::vector<double> z(n_shifts, 1.0), z_old(n_shifts, 1.0), z_new(n_shifts);
    double a_old = 1.0, b_old = 0.0, rr = bb;
    const double stop = tol * tol * bb;
    int it = 0;
    bool conv = bb == 0.0;
    while (!conv && it < maxiter) {
        // w = (M_hat^+ M_hat + s0) p
        HIPCHK(ctx, matpc(s, op, v, p, t1, tmpo, RED_NONE, nullptr, nullptr, nullptr));
        HIPCHK(ctx, launch_clov_apply_internal(s, F64, g, op->Ainv64[0].p, t1, t2));
        HIPCHK(ctx, apply_g5(s, t2, g));
        HIPCHK(ctx, matpc(s, op, v, t2, t1, tmpo, RED_NONE, nullptr, nullptr, nullptr));
        HIPCHK(ctx, launch_clov_apply_internal(s, F64, g, op->A64[0].p, t1, w));
        HIPCHK(ctx, apply_g5(s, w, g));
        if (s0 != 0.0) HIPCHK(ctx, launch_multiaxpy(s, p, 0, 1, dd + c_s0, w, n, 1.0));
        double pw;
        CHK(read_dot(p, w, pw));
        if (!(pw > 0.0) || !std::isfinite(pw)) return fail(ctx, QCDW_EBREAKDOWN, "multi-shift CG: (p, N p) = %g", pw);
        const double a = rr / pw;
        for (int i = 0; i < n_shifts; i++) {
            const double d = shifts[i] - s0;
            z_new[i] = z[i] * z_old[i] * a_old / (a * b_old * (z_old[i] - z[i]) + z_old[i] * a_old * (1.0 + d * a));
        }
        hd[c_a] = a;
        hd[c_a + 1] = 0.0;
        CHK(stage(c_a, 2));
        HIPCHK(ctx, launch_multiaxpy(s, w, 0, 1, dd + c_a, r, n, -1.0));  // r -= alpha w
        double rr_new;
        CHK(read_dot(r, r, rr_new));
        const double beta = rr_new / rr;
        for (int i = 0; i < n_shifts; i++) {
            hd[c_up + 3 * i] = a * z_new[i] / z[i];                                    // alpha_i
            hd[c_up + 3 * i + 1] = z_new[i];                                           // zeta_i'
            hd[c_up + 3 * i + 2] = beta * (z_new[i] / z[i]) * (z_new[i] / z[i]);      // beta_i
        }
        hd[c_up + 3 * n_shifts] = beta;
        CHK(stage(c_up, 3 * n_shifts + 1));
        hipLaunchKernelGGL(k_shift_update, dim3(blas_blocks(n)), dim3(256), 0, s, (double2*)X(0), (double2*)P(0),
                           (double2*)p, (const double2*)r, n, n_shifts, dd + c_up);
        HIPCHK(ctx, hipGetLastError());
        z_old = z;
        z = z_new;
        a_old = a;
        b_old = beta;
        rr = rr_new;
        it++;
        if (!std::isfinite(rr)) return fail(ctx, QCDW_ENAN, "multi-shift CG: non-finite residual");
        conv = true;  // residual of shift i: |zeta_i| |r|
        for (int i = 0; i < n_shifts; i++)
            if (z[i] * z[i] * rr > stop) conv = false;
    }
    for (int i = 0; i < n_shifts; i++) {
        HIPCHK(ctx, launch_unpack_spinor(s, F64, g, X(i), 0, x_e[i], 1.0));
        res[i] = bb > 0.0 ? std::fabs(z[i]) * std::sqrt(rr / bb) : 0.0;
    }
    HIPCHK(ctx, hipStreamSynchronize(s));
    *iters = it;
    if (!conv) return fail(ctx, QCDW_ENOCONV, "multi-shift CG did not converge within %d iterations", maxiter);
    return QCDW_OK;
}
