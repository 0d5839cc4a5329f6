// C-ABI of libqcdw (declared in include/qcdw.h): argument checking, device
// workspaces, and the host side of the even-odd preconditioned BiCGStab solver
// whose iterations run entirely on the device (scalars never leave the GPU
// except for the periodic convergence poll).
#include <algorithm>

#include "host.h"

namespace {

// multi-RHS hop forms (tuning-cache value of "mrhs_hop/..."): bit 0 set: one block per (tile, RHS), links
// re-read from L2; else the register loop, in slice-group order of (v & 1023) / 2 c-tiles when nonzero, on
// the matrix cores when MRHS_MFMA is set (16-bit storage)
constexpr int MRHS_MFMA = 1024;

bool mrhs_variant_fits(const qcdw::Geom& g, int prec, int v)
{
    if (v == 1) return true;
    if ((v & 1) || (v & ~(MRHS_MFMA | 1023))) return false;
    // the matrix-core form keeps its neighbour offsets (complex index within one RHS) in 32 bits
    if ((v & MRHS_MFMA) && ((prec != qcdw::BF16 && prec != qcdw::F16) || 12L * g.Vh > 0x7fffffffL)) return false;
    const int cg = (v & 1023) >> 1;
    return cg == 0 || hop_cgroup_fits(g, cg);
}

int mrhs_blocks(const qcdw::Geom& g, int v)
{
    const int cg = (v & 1) ? 0 : (v & 1023) >> 1;
    return cg > 0 ? hop_ctiles(g) * g.Lt : hop_blocks(g.Vh);
}

hipError_t launch_mrhs_variant(hipStream_t st, int prec, int epi, int red, qcdw::HopArgs a, const qcdw::Scal* S,
                               int v, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr)
{
    a.cgroup = (v & 1) ? 0 : (v & 1023) >> 1;
    if (v & 1) return qcdw::launch_hop_rhs(st, prec, epi, red, a, S, e0, e1);
    if (v & MRHS_MFMA) return qcdw::launch_hop_mrhs_mfma(st, prec, epi, red, a, S, e0, e1);
    return qcdw::launch_hop_mrhs(st, prec, epi, red, a, S, e0, e1);
}

}  // namespace

extern "C" {

void qcdw_solver_params_default(qcdw_solver_params* p)
{
    if (!p) return;
    p->tol = 1e-10;
    p->maxiter = 10000;
    p->inner = QCDW_F64;
    p->delta = 0.1;
    p->check_every = 8;
    p->max_restarts = 8;
    p->collect_timing = 0;
    p->fault_inject = 0;
    p->use_graph = 1;
    p->gmres_restart = 32;
    p->gmres_fallback = 1;
    p->inner_resume = 0;
}

qcdw_status qcdw_ctx_create(qcdw_ctx** ctx, int device, void* hip_stream)
{
    if (!ctx) return QCDW_EINVAL;
    *ctx = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return QCDW_EHIP;
    if (device < 0 || device >= ndev) return QCDW_EINVAL;
    DeviceGuard dg(device);
    qcdw_ctx* c = new qcdw_ctx;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    if (hipHostMalloc((void**)&c->host_scal, HOST_SCAL_N * sizeof(Scal)) != hipSuccess ||
        hipHostMalloc((void**)&c->host_d, HOST_D_N * sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&c->dev_int, 64 * sizeof(int)) != hipSuccess ||
        hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        qcdw_ctx_destroy(c);
        return QCDW_ENOMEM;
    }
    if (noalloc_scratch_init(device) != hipSuccess) {  // device address of the fixed no-alloc workspace
        qcdw_ctx_destroy(c);
        return QCDW_EHIP;
    }
    c->tune_load();
    *ctx = c;
    return QCDW_OK;
}

void qcdw_ctx_destroy(qcdw_ctx* ctx)
{
    if (!ctx) return;
    DeviceGuard dg(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    if (ctx->host_scal) (void)hipHostFree(ctx->host_scal);
    if (ctx->host_d) (void)hipHostFree(ctx->host_d);
    if (ctx->dev_int) (void)hipFree(ctx->dev_int);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    block_cache().trim(ctx->device);
    delete ctx;
}

const char* qcdw_last_error(const qcdw_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

qcdw_status qcdw_ctx_set_stream(qcdw_ctx* ctx, void* hip_stream)
{
    if (!ctx) return QCDW_EINVAL;
    ctx->stream = (hipStream_t)hip_stream;
    return QCDW_OK;
}

qcdw_status qcdw_ctx_tuned(const qcdw_ctx* ctx, const char* key, int* value)
{
    if (!ctx || !key || !value) return QCDW_EINVAL;
    const auto it = ctx->tune.find(key);
    if (it == ctx->tune.end()) return QCDW_EINVAL;
    *value = it->second;
    return QCDW_OK;
}

qcdw_status qcdw_wall_sources(qcdw_ctx* ctx, const qcdw_lattice* lat, int t0, const int* mom, void* out)
{
    if (!ctx) return QCDW_EINVAL;
    DeviceGuard dg(ctx->device);
    Geom g;
    CHK(check_lattice(ctx, lat, g));
    if (!mom) return fail(ctx, QCDW_EINVAL, "mom is NULL");
    if (t0 < 0 || t0 >= g.Lt) return fail(ctx, QCDW_EINVAL, "t0 = %d outside [0, %d)", t0, g.Lt);
    CHK(check_dev(ctx, out, "out"));
    HIPCHK(ctx, launch_wall_sources(ctx->stream, g, t0, mom, out));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return QCDW_OK;
}

qcdw_status qcdw_meson_contract(qcdw_ctx* ctx, const qcdw_lattice* lat, const void* S, const void* T, int gamma_snk,
                                int gamma_src, const int* mom, void* out)
{
    if (!ctx) return QCDW_EINVAL;
    DeviceGuard dg(ctx->device);
    Geom g;
    CHK(check_lattice(ctx, lat, g));
    if (!mom) return fail(ctx, QCDW_EINVAL, "mom is NULL");
    if (gamma_snk < 0 || gamma_snk > 15 || gamma_src < 0 || gamma_src > 15)
        return fail(ctx, QCDW_EINVAL, "gamma bitmasks must lie in [0, 15], got %d and %d", gamma_snk, gamma_src);
    CHK(check_dev(ctx, S, "S"));
    CHK(check_dev(ctx, T, "T"));
    CHK(check_dev(ctx, out, "out"));
    PoolBuf site;  // per-site contributions, from the block cache; the stream is drained before it goes back
    HIPCHK(ctx, site.alloc(2UL * g.Vh * 16));
    const hipError_t launched = launch_meson_2pt(ctx->stream, g, S, T, gamma_snk, gamma_src, mom, site.p, out);
    const hipError_t drained = hipStreamSynchronize(ctx->stream);
    HIPCHK(ctx, launched);
    HIPCHK(ctx, drained);
    return QCDW_OK;
}

qcdw_status qcdw_meson_2pt(qcdw_ctx* ctx, const qcdw_lattice* lat, const void* S, int gamma_snk, int gamma_src,
                           const int* mom, void* out)
{
    return qcdw_meson_contract(ctx, lat, S, S, gamma_snk, gamma_src, mom, out);
}

qcdw_status qcdw_seq_sources(qcdw_ctx* ctx, const qcdw_lattice* lat, const void* S, int t_f, int gamma_f,
                             const int* mom, void* out)
{
    if (!ctx) return QCDW_EINVAL;
    DeviceGuard dg(ctx->device);
    Geom g;
    CHK(check_lattice(ctx, lat, g));
    if (!mom) return fail(ctx, QCDW_EINVAL, "mom is NULL");
    if (t_f < 0 || t_f >= g.Lt) return fail(ctx, QCDW_EINVAL, "t_f = %d outside [0, %d)", t_f, g.Lt);
    if (gamma_f < 0 || gamma_f > 15) return fail(ctx, QCDW_EINVAL, "gamma bitmask must lie in [0, 15], got %d", gamma_f);
    CHK(check_dev(ctx, S, "S"));
    CHK(check_dev(ctx, out, "out"));
    if (S == out) return fail(ctx, QCDW_EINVAL, "out must not alias S");
    HIPCHK(ctx, launch_seq_sources(ctx->stream, g, S, t_f, gamma_f, mom, out));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return QCDW_OK;
}

qcdw_status qcdw_clover_build(qcdw_ctx* ctx, const qcdw_lattice* lat, const void* U, void* clover)
{
    if (!ctx) return QCDW_EINVAL;
    DeviceGuard dg(ctx->device);
    Geom g;
    CHK(check_lattice(ctx, lat, g));
    CHK(check_dev(ctx, U, "U"));
    CHK(check_dev(ctx, clover, "clover"));
    HIPCHK(ctx, launch_clover_build(ctx->stream, g, U, clover));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return QCDW_OK;
}

qcdw_status qcdw_clover_apply(qcdw_ctx* ctx, const qcdw_lattice* lat, const void* clover, const void* psi, void* out,
                              double kappa, double csw)
{
    if (!ctx) return QCDW_EINVAL;
    DeviceGuard dg(ctx->device);
    Geom g;
    CHK(check_lattice(ctx, lat, g));
    CHK(check_dev(ctx, clover, "clover"));
    CHK(check_dev(ctx, psi, "psi"));
    CHK(check_dev(ctx, out, "out"));
    if (psi == out) return fail(ctx, QCDW_EINVAL, "out must not alias psi");
    HIPCHK(ctx, launch_clover_apply(ctx->stream, g, clover, psi, out, kappa, csw));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return QCDW_OK;
}

qcdw_status qcdw_clover_invert(qcdw_ctx* ctx, const qcdw_lattice* lat, const void* clover, double kappa, double csw,
                               void* clover_inv)
{
    if (!ctx) return QCDW_EINVAL;
    DeviceGuard dg(ctx->device);
    Geom g;
    CHK(check_lattice(ctx, lat, g));
    CHK(check_dev(ctx, clover, "clover"));
    CHK(check_dev(ctx, clover_inv, "clover_inv"));
    HIPCHK(ctx, hipMemsetAsync(ctx->dev_int, 0, sizeof(int), ctx->stream));
    HIPCHK(ctx, launch_clover_invert(ctx->stream, g, clover, kappa, csw, clover_inv, ctx->dev_int));
    HIPCHK(ctx, hipMemcpyAsync(ctx->host_d, ctx->dev_int, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    int bad;
    memcpy(&bad, ctx->host_d, sizeof(int));
    if (bad) return fail(ctx, QCDW_ENOTPD, "%d clover blocks are not positive definite", bad);
    return QCDW_OK;
}

qcdw_status qcdw_hop(qcdw_ctx* ctx, const qcdw_lattice* lat, const void* U, const void* psi, void* out, int out_parity)
{
    if (!ctx) return QCDW_EINVAL;
    DeviceGuard dg(ctx->device);
    Geom g;
    CHK(check_lattice(ctx, lat, g));
    CHK(check_dev(ctx, U, "U"));
    CHK(check_dev(ctx, psi, "psi"));
    CHK(check_dev(ctx, out, "out"));
    if (out_parity != 0 && out_parity != 1) return fail(ctx, QCDW_EINVAL, "out_parity must be 0 or 1");
    if (psi == out) return fail(ctx, QCDW_EINVAL, "out must not alias psi");
    const size_t vb = 12UL * g.Vh * 16;
    DevBuf gauge, in, res;
    HIPCHK(ctx, gauge.alloc(8UL * g.Vh * 9 * 16));
    HIPCHK(ctx, in.alloc(vb));
    HIPCHK(ctx, res.alloc(vb));
    hipStream_t s = ctx->stream;
    HIPCHK(ctx, launch_pack_gauge(s, F64, 18, g, U, gauge.p));
    HIPCHK(ctx, launch_pack_spinor(s, F64, g, psi, 1 - out_parity, in.p, 1.0));
    HopArgs a = hop_args(g, out_parity);
    a.psi = in.p;
    a.out = res.p;
    a.gauge = gauge.p;
    HIPCHK(ctx, launch_hop(s, F64, 18, EPI_NONE, RED_NONE, a));
    HIPCHK(ctx, launch_unpack_spinor(s, F64, g, res.p, out_parity, out, 1.0));
    HIPCHK(ctx, hipMemsetAsync((char*)out + (size_t)(1 - out_parity) * vb, 0, vb, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    return QCDW_OK;
}

qcdw_status qcdw_dslash(qcdw_ctx* ctx, const qcdw_lattice* lat, const void* U, const void* clover, const void* psi,
                        void* out, double kappa, double csw)
{
    if (!ctx) return QCDW_EINVAL;
    DeviceGuard dg(ctx->device);
    Geom g;
    CHK(check_lattice(ctx, lat, g));
    CHK(check_dev(ctx, U, "U"));
    if (clover) CHK(check_dev(ctx, clover, "clover"));
    CHK(check_dev(ctx, psi, "psi"));
    CHK(check_dev(ctx, out, "out"));
    if (psi == out) return fail(ctx, QCDW_EINVAL, "out must not alias psi");
    hipStream_t s = ctx->stream;
    const size_t vb = 12UL * g.Vh * 16;
    DevBuf gauge, clov, Apaper, A[2], in[2], res;
    HIPCHK(ctx, gauge.alloc(8UL * g.Vh * 9 * 16));
    HIPCHK(ctx, Apaper.alloc(144UL * g.Vh * 8));
    for (int p = 0; p < 2; p++) {
        HIPCHK(ctx, A[p].alloc(clov_reals(g.Vh) * 8));
        HIPCHK(ctx, in[p].alloc(vb));
    }
    HIPCHK(ctx, res.alloc(vb));
    HIPCHK(ctx, launch_pack_gauge(s, F64, 18, g, U, gauge.p));
    if (!clover) {
        HIPCHK(ctx, clov.alloc(144UL * g.Vh * 8));
        HIPCHK(ctx, launch_clover_build(s, g, U, clov.p));
        clover = clov.p;
    }
    HIPCHK(ctx, launch_clover_to_A(s, g, clover, kappa, csw, Apaper.p));
    for (int p = 0; p < 2; p++) {
        HIPCHK(ctx, launch_pack_clover(s, F64, g, Apaper.p, p, A[p].p));
        HIPCHK(ctx, launch_pack_spinor(s, F64, g, psi, p, in[p].p, 1.0));
    }
    for (int p = 0; p < 2; p++) {
        HopArgs a = hop_args(g, p);
        a.psi = in[1 - p].p;
        a.out = res.p;
        a.gauge = gauge.p;
        a.clov = A[p].p;
        a.y = in[p].p;
        a.a = kappa;
        HIPCHK(ctx, launch_hop(s, F64, 18, EPI_XPAY_CLOVY, RED_NONE, a));
        HIPCHK(ctx, launch_unpack_spinor(s, F64, g, res.p, p, out, 1.0));
    }
    HIPCHK(ctx, hipStreamSynchronize(s));
    return QCDW_OK;
}

// Form of the operator's single-RHS hop in precision prec: sites per thread along t (nt), c-tiles
// per group swept along t (cg) and the arithmetic form (fma).  The cached choice for this lattice
// (code nt + 16 cg + 4096 fma), else the fastest candidate timed on scratch vectors.
static qcdw_status tune_op_hop(qcdw_op* op, int prec)
{
    qcdw_ctx* ctx = op->ctx;
    const Geom& g = op->g;
    char key[96];
    snprintf(key, sizeof key, "hop_nt/p%d/L%dx%dx%dx%d", prec, g.Lx, g.Ly, g.Lz, g.Lt);
    const int nct = hop_ctiles(g);
    auto divisor_upto = [&](int m) {  // largest divisor of nct in [4, m], below nct; 0 if none
        for (int d = std::min(m, nct - 1); d >= 4; d--)
            if (nct % d == 0) return d;
        return 0;
    };
    std::vector<int> cand;  // codes nt + 16 cg + 4096 fma (fma: bit 0 multiply-add form, bit 1 LDS staging)
    auto add = [&](int nt, int cg) {
        for (int f : {0, 1, 2, 3}) {
            if ((f & 2) && !(nt == 1 && cg > 0)) continue;  // staging needs slice groups, one site per thread group
            const int code = nt + 16 * cg + 4096 * f;
            if (hop_nt_fits(g, nt) && hop_cgroup_fits(g, cg) && std::find(cand.begin(), cand.end(), code) == cand.end())
                cand.push_back(code);
        }
    };
    add(1, 0);
    for (int m : {8, 16, 32})
        if (int d = divisor_upto(m)) add(1, d);
    for (int nt : {2, 4}) {
        add(nt, 0);
        if (int d = divisor_upto(16)) add(nt, d);
    }
    auto apply = [&](int code) {
        op->hop_nt[prec] = code % 16;
        op->hop_cg[prec] = (code / 16) % 256;
        op->hop_fma[prec] = code / 4096;
    };
    auto it = ctx->tune.find(key);
    if (it != ctx->tune.end()) {
        const int nt = it->second % 16, cg = (it->second / 16) % 256, f = it->second / 4096;
        if (hop_nt_fits(g, nt) && hop_cgroup_fits(g, cg) && f >= 0 && f <= 3 && (!(f & 2) || (nt == 1 && cg > 0))) {
            apply(it->second);
            return QCDW_OK;
        }
    }
    apply(1);
    if (cand.size() == 1) return QCDW_OK;
    const PrecView v = view(op, prec);
    const size_t vb = 12UL * g.Vh * cplx_bytes(prec);
    DevBuf in, out;
    HIPCHK(ctx, in.alloc(vb));
    HIPCHK(ctx, out.alloc(vb));
    hipStream_t s = ctx->stream;
    HIPCHK(ctx, hipMemsetAsync(in.p, 0, vb, s));
    hipEvent_t e0, e1;
    HIPCHK(ctx, hipEventCreate(&e0));
    HIPCHK(ctx, hipEventCreate(&e1));
    float best = 1e30f;
    int best_c = 1;
    hipError_t e = hipSuccess;
    for (int code : cand) {
        HopArgs a = hop_args(g, 1);
        a.nt = code % 16;
        a.cgroup = (code / 16) % 256;
        a.fma = code / 4096;
        a.psi = in.p;
        a.out = out.p;
        a.gauge = v.gauge;
        a.clov = v.Ainv[1];
        for (int rep = 0; rep < 2 && e == hipSuccess; rep++) e = launch_hop(s, prec, v.recon, EPI_CLOV, RED_NONE, a);
        if (e == hipSuccess) e = hipEventRecord(e0, s);
        for (int rep = 0; rep < 20 && e == hipSuccess; rep++) e = launch_hop(s, prec, v.recon, EPI_CLOV, RED_NONE, a);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) break;
        // the plain form (first candidate) is kept unless another is more than 3 % faster, so
        // that timing noise does not flip the choice between runs
        const float t = code == cand[0] ? ms : ms * 1.03f;
        if (t < best) {
            best = t;
            best_c = code;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(ctx, QCDW_EHIP, "hop tuning failed: %s", hipGetErrorString(e));
    apply(best_c);
    ctx->tune_store(key, best_c);
    return QCDW_OK;
}

// The operator M = A - kappa H with A = 1 - kappa csw C, C = wt sum_i sigma_i4 F_i4 + ws sum_{i<j}
// sigma_ij F_ij and the spatial hops of H weighted by xs (isotropic: wt = ws = xs = 1).
static qcdw_status op_create(qcdw_ctx* ctx, const qcdw_lattice* lat, const void* U, double kappa, double csw,
                             double wt, double ws, double xs, qcdw_prec inner, int recon, qcdw_op** op_out)
{
    if (!ctx) return QCDW_EINVAL;
    if (!op_out) return fail(ctx, QCDW_EINVAL, "op pointer is NULL");
    *op_out = nullptr;
    DeviceGuard dg(ctx->device);
    Geom g;
    CHK(check_lattice(ctx, lat, g));
    CHK(check_dev(ctx, U, "U"));
    if (!(xs > 0.0) || !std::isfinite(xs) || !std::isfinite(wt) || !std::isfinite(ws))
        return fail(ctx, QCDW_EINVAL, "anisotropy coefficients must be finite (and nu / xi_0 positive)");
    g.xs = xs;
    if (recon != 12 && recon != 18) return fail(ctx, QCDW_EINVAL, "recon must be 12 or 18, got %d", recon);
    if (inner < QCDW_F64 || inner > QCDW_F16) return fail(ctx, QCDW_EINVAL, "bad inner precision %d", (int)inner);
    if (!(kappa > 0.0) || !std::isfinite(kappa) || !std::isfinite(csw))
        return fail(ctx, QCDW_EINVAL, "kappa must be positive and finite");
    hipStream_t s = ctx->stream;
    qcdw_op* op = new qcdw_op;
    op->ctx = ctx;
    op->g = g;
    op->kappa = kappa;
    op->csw = csw;
    op->inner = inner;
    op->recon = recon;
    auto cleanup = [&](qcdw_status st) {
        (void)hipStreamSynchronize(s);  // before the blocks return to the cache
        delete op;
        return st;
    };
    const int R = recon == 18 ? 9 : 6;
    PoolBuf clov, inv, Ap;  // released after the stream synchronisation below (or in cleanup)
    if (op->gauge64.alloc(8UL * g.Vh * R * 16) != hipSuccess || clov.alloc(144UL * g.Vh * 8) != hipSuccess ||
        inv.alloc(144UL * g.Vh * 8) != hipSuccess || Ap.alloc(144UL * g.Vh * 8) != hipSuccess)
        return cleanup(fail(ctx, QCDW_ENOMEM, "out of device memory creating the operator"));
    for (int p = 0; p < 2; p++)
        if (op->Ainv64[p].alloc(clov_reals(g.Vh) * 8) != hipSuccess || op->A64[p].alloc(clov_reals(g.Vh) * 8) != hipSuccess)
            return cleanup(fail(ctx, QCDW_ENOMEM, "out of device memory creating the operator"));
    hipError_t e = launch_pack_gauge(s, F64, recon, g, U, op->gauge64.p);
    if (e == hipSuccess) e = launch_clover_build(s, g, U, clov.p, wt, ws);
    if (e == hipSuccess) e = hipMemsetAsync(ctx->dev_int, 0, sizeof(int), s);
    if (e == hipSuccess) e = launch_clover_invert(s, g, clov.p, kappa, csw, inv.p, ctx->dev_int);
    if (e == hipSuccess) e = launch_clover_to_A(s, g, clov.p, kappa, csw, Ap.p);
    for (int p = 0; p < 2 && e == hipSuccess; p++) {
        e = launch_pack_clover(s, F64, g, inv.p, p, op->Ainv64[p].p);
        if (e == hipSuccess) e = launch_pack_clover(s, F64, g, Ap.p, p, op->A64[p].p);
    }
    if (e == hipSuccess && inner != QCDW_F64) {
        const int lrecon = (inner == QCDW_F32) ? recon : 12;
        const int lR = lrecon == 18 ? 9 : 6;
        if (op->gauge_lo.alloc(8UL * g.Vh * lR * cplx_bytes(inner)) != hipSuccess)
            return cleanup(fail(ctx, QCDW_ENOMEM, "out of device memory creating the operator"));
        e = launch_pack_gauge(s, inner, lrecon, g, U, op->gauge_lo.p);
        for (int p = 0; p < 2 && e == hipSuccess; p++) {
            if (op->Ainv_lo[p].alloc(clov_reals(g.Vh) * real_bytes(inner)) != hipSuccess)
                return cleanup(fail(ctx, QCDW_ENOMEM, "out of device memory creating the operator"));
            e = launch_pack_clover(s, inner, g, inv.p, p, op->Ainv_lo[p].p);
        }
    }
    if (e == hipSuccess) e = hipMemcpyAsync(ctx->host_d, ctx->dev_int, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return cleanup(fail(ctx, QCDW_EHIP, "operator setup failed: %s", hipGetErrorString(e)));
    int bad;
    memcpy(&bad, ctx->host_d, sizeof(int));
    if (bad) return cleanup(fail(ctx, QCDW_ENOTPD, "%d clover blocks are not positive definite", bad));
    for (int prec : {(int)F64, (int)inner}) {
        const qcdw_status st = tune_op_hop(op, prec);
        if (st != QCDW_OK) return cleanup(st);
    }
    *op_out = op;
    return QCDW_OK;
}

qcdw_status qcdw_op_create(qcdw_ctx* ctx, const qcdw_lattice* lat, const void* U, double kappa, double csw,
                           qcdw_prec inner, int recon, qcdw_op** op_out)
{
    return op_create(ctx, lat, U, kappa, csw, 1.0, 1.0, 1.0, inner, recon, op_out);
}

qcdw_status qcdw_op_create_aniso(qcdw_ctx* ctx, const qcdw_lattice* lat, const void* U, double kappa, double xi_0,
                                 double nu, double csw_t, double csw_r, qcdw_prec inner, int recon, qcdw_op** op_out)
{
    if (!(xi_0 > 0.0) || !(nu > 0.0) || !std::isfinite(xi_0) || !std::isfinite(nu))
        return ctx ? fail(ctx, QCDW_EINVAL, "xi_0 and nu must be positive and finite") : QCDW_EINVAL;
    return op_create(ctx, lat, U, kappa, 1.0, csw_t, csw_r / xi_0, nu / xi_0, inner, recon, op_out);
}

void qcdw_op_destroy(qcdw_op* op)
{
    if (!op) return;
    DeviceGuard dg(op->ctx->device);
    (void)hipStreamSynchronize(op->ctx->stream);
    delete op;
}

qcdw_status qcdw_op_hop_form(const qcdw_op* op, qcdw_prec prec, int* nt, int* cgroup, int* fma)
{
    if (!op) return QCDW_EINVAL;
    if (!nt || !cgroup) return fail(op->ctx, QCDW_EINVAL, "nt and cgroup must not be NULL");
    if (prec != QCDW_F64 && prec != (qcdw_prec)op->inner)
        return fail(op->ctx, QCDW_EINVAL, "prec must be F64 or the operator's inner precision");
    *nt = op->hop_nt[prec];
    *cgroup = op->hop_cg[prec];
    if (fma) *fma = op->hop_fma[prec];
    return QCDW_OK;
}

qcdw_status qcdw_op_matpc(qcdw_op* op, qcdw_prec prec, const void* in_e, void* out_e)
{
    if (!op) return QCDW_EINVAL;
    qcdw_ctx* ctx = op->ctx;
    DeviceGuard dg(ctx->device);
    CHK(check_dev(ctx, in_e, "in_e"));
    CHK(check_dev(ctx, out_e, "out_e"));
    if (prec != QCDW_F64 && prec != (qcdw_prec)op->inner)
        return fail(ctx, QCDW_EINVAL, "prec must be F64 or the operator's inner precision");
    const Geom& g = op->g;
    const long n = 12L * g.Vh;
    DevBuf in, out, tmp;
    HIPCHK(ctx, in.alloc(n * cplx_bytes(prec)));
    HIPCHK(ctx, out.alloc(n * cplx_bytes(prec)));
    HIPCHK(ctx, tmp.alloc(n * cplx_bytes(prec)));
    hipStream_t s = ctx->stream;
    const PrecView v = view(op, prec);
    HIPCHK(ctx, launch_pack_spinor(s, prec, g, in_e, 0, in.p, 1.0));
    HIPCHK(ctx, matpc(s, op, v, in.p, out.p, tmp.p, RED_NONE, nullptr, nullptr, nullptr));
    HIPCHK(ctx, launch_unpack_spinor(s, prec, g, out.p, 0, out_e, 1.0));
    HIPCHK(ctx, hipStreamSynchronize(s));
    return QCDW_OK;
}

qcdw_status qcdw_op_matpc_multi(qcdw_op* op, qcdw_prec prec, int nrhs, const void* in_e, void* out_e)
{
    if (!op) return QCDW_EINVAL;
    qcdw_ctx* ctx = op->ctx;
    DeviceGuard dg(ctx->device);
    CHK(check_dev(ctx, in_e, "in_e"));
    CHK(check_dev(ctx, out_e, "out_e"));
    if (nrhs < 1 || nrhs > 16) return fail(ctx, QCDW_EINVAL, "nrhs must lie in [1, 16]");
    if (prec != QCDW_F64 && prec != (qcdw_prec)op->inner)
        return fail(ctx, QCDW_EINVAL, "prec must be F64 or the operator's inner precision");
    if (op->recon != 12 && prec == QCDW_F64)
        return fail(ctx, QCDW_EINVAL, "the multi-RHS kernel uses reconstruct-12 links");
    const Geom& g = op->g;
    const long n = 12L * g.Vh;
    const size_t half = (size_t)n * 16;  // bytes of one even-site FP64 field
    DevBuf in, out, tmp;
    HIPCHK(ctx, in.alloc(nrhs * n * cplx_bytes(prec)));
    HIPCHK(ctx, out.alloc(nrhs * n * cplx_bytes(prec)));
    HIPCHK(ctx, tmp.alloc(nrhs * n * cplx_bytes(prec)));
    hipStream_t s = ctx->stream;
    const PrecView v = view(op, prec);
    for (int k = 0; k < nrhs; k++)
        HIPCHK(ctx, launch_pack_spinor(s, prec, g, (const char*)in_e + k * half, 0,
                                       (char*)in.p + (size_t)k * n * cplx_bytes(prec), 1.0));
    // the kernel form cached for this shape by a multi-RHS solve (or a tuning file), else the register loop
    int form = 0;
    char key[96];
    snprintf(key, sizeof key, "mrhs_hop/p%d/L%dx%dx%dx%d/n%d", (int)prec, g.Lx, g.Ly, g.Lz, g.Lt, nrhs);
    const auto it = ctx->tune.find(key);
    if (it != ctx->tune.end() && mrhs_variant_fits(g, prec, it->second)) form = it->second;
    HopArgs a = hop_args(g, 1);
    a.psi = in.p;
    a.out = tmp.p;
    a.gauge = v.gauge;
    a.clov = v.Ainv[1];
    a.nrhs = nrhs;
    HIPCHK(ctx, launch_mrhs_variant(s, prec, EPI_CLOV, RED_NONE, a, nullptr, form));
    HopArgs b2 = hop_args(g, 0);
    b2.psi = tmp.p;
    b2.out = out.p;
    b2.gauge = v.gauge;
    b2.clov = v.Ainv[0];
    b2.y = in.p;
    b2.a = op->kappa * op->kappa;
    b2.nrhs = nrhs;
    HIPCHK(ctx, launch_mrhs_variant(s, prec, EPI_CLOV_XPAY, RED_NONE, b2, nullptr, form));
    for (int k = 0; k < nrhs; k++)
        HIPCHK(ctx, launch_unpack_spinor(s, prec, g, (const char*)out.p + (size_t)k * n * cplx_bytes(prec), 0,
                                         (char*)out_e + k * half, 1.0));
    HIPCHK(ctx, hipStreamSynchronize(s));
    return QCDW_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// solver
// ---------------------------------------------------------------------------
namespace {

struct Timing {
    bool on = false;
    std::vector<hipEvent_t> ev;  // start/stop pairs in launch order
    std::vector<int> kind;       // hop kind of each pair
    size_t used = 0;
    double ms[3] = {0, 0, 0};
    long launches[3] = {0, 0, 0};
    ~Timing()
    {
        for (auto e : ev) (void)hipEventDestroy(e);
    }
    hipEvent_t get()
    {
        if (used == ev.size()) {
            hipEvent_t e;
            (void)hipEventCreate(&e);
            ev.push_back(e);
        }
        return ev[used++];
    }
    // accumulate the first n_pairs recorded pairs, then start over
    void collect(size_t n_pairs)
    {
        for (size_t k = 0; k < n_pairs && 2 * k + 1 < used; k++) {
            float t = 0;
            if (hipEventElapsedTime(&t, ev[2 * k], ev[2 * k + 1]) == hipSuccess) {
                ms[kind[k]] += t;
                launches[kind[k]]++;
            } else {
                (void)hipGetLastError();
            }
        }
        used = 0;
        kind.clear();
    }
};

constexpr int MAX_RHS = 16;
constexpr int MAX_BATCH = 64;
static_assert(HOST_SCAL_N >= MAX_BATCH && HOST_D_N >= 2 * MAX_BATCH && MAX_RHS <= MAX_BATCH,
              "pinned staging buffers must hold every problem of a solve");

// The problems of one solve: nprob right-hand sides of one operator (multi-RHS,
// batch == nullptr) or the operators of a batch (one RHS each).
struct Solver {
    qcdw_ctx* ctx;
    Workspace& W;
    std::vector<qcdw_op*> ops;  // per problem
    qcdw_batch* batch;          // non-null for batched solves
    hipStream_t s;
    int nprob;
    std::vector<long> off, len;  // element offsets / lengths (complex) of each problem
    long nmax;                   // longest problem
    int nb_hop;                  // hop partials stride per problem (set by the hop form in use)
    int nb_hop_cap;              // largest stride any hop form of these problems can need
    int nb_blas;                 // BLAS partials per problem
    const long2* map;            // device (off, len) per problem (batch) or nullptr (uniform)
    const int* nbs;              // device hop tiles per problem (batch) or nullptr
    int variant = 0;             // multi-RHS kernel form (mrhs_variant_fits), batch grid, or the single-RHS
                                 // hop form
    int nt = 1, cg = 0, fma = 0;  // single-RHS hop: sites per thread along t, c-tile group, arithmetic form
    int fuse_nb;                 // largest partials count (all problems of a launch) whose scalars are
                                 // formed in the vector kernels
    Timing tm;

    Solver(qcdw_ctx* c, Workspace& w, std::vector<qcdw_op*> o, qcdw_batch* b)
        : ctx(c), W(w), ops(std::move(o)), batch(b), s(c->stream), nprob((int)ops.size())
    {
        if (batch) {
            off = batch->off;
            len = batch->len;
            nmax = batch->nmax;
            nb_hop = nb_hop_cap = batch->nbmax;
            map = (const long2*)batch->map.p;
            nbs = (const int*)batch->nbs.p;
        } else {
            const long n = 12L * ops[0]->g.Vh;
            for (int k = 0; k < nprob; k++) {
                off.push_back(k * n);
                len.push_back(n);
            }
            nmax = n;
            nb_hop = hop_blocks(ops[0]->g.Vh);
            // slice-group forms launch one block per (c-tile, t), t-stepping forms fewer
            nb_hop_cap = std::max(nb_hop, hop_ctiles(ops[0]->g) * ops[0]->g.Lt);
            map = nullptr;
            nbs = nullptr;
        }
        nb_blas = blas_blocks(nmax);
        const char* f = getenv("QCDW_FUSE_NB");
        fuse_nb = f && *f ? atoi(f) : 2048;
    }
    long n0() const { return len[0]; }  // uniform length (multi-RHS)
    // partials per problem in each of the two regions of W.partials (hop or vector reductions, then
    // the x/r update's own)
    long part_stride() const { return std::max<long>(std::max<long>(nb_blas, nb_hop_cap), 1); }

    void* at(const DevBuf& b, int k) const { return (char*)b.p + (size_t)off[k] * 16; }

    hipError_t hop(hipStream_t st, int prec, int epi, int red, const void* psi, void* out, const void* y,
                   const void* w, double* partials, const Scal* S, int parity)
    {
        const int kind = epi == EPI_CLOV ? 0 : (red == RED_WDOT ? 1 : 2);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (tm.on) {
            tm.kind.push_back(kind);
            e0 = tm.get();
            e1 = tm.get();
        }
        if (batch) {
            BatchHopArgs b{};
            b.tab = (const BatchEntry*)(prec == F64 ? batch->tab64.p : batch->tablo.p);
            b.nprob = nprob;
            b.total_tiles = batch->total_tiles;
            b.parity = parity;
            b.nbmax = batch->nbmax;
            b.use_kappa2 = epi == EPI_CLOV_XPAY;
            b.psi = psi;
            b.out = out;
            b.y = y;
            b.w = w;
            b.partials = partials;
            b.S = S;
            return launch_hop_batch(st, prec, epi, red, b, variant, e0, e1);
        }
        const qcdw_op* op = ops[0];
        const PrecView v = view(op, prec);
        HopArgs a = hop_args(op->g, parity);
        a.psi = psi;
        a.out = out;
        a.gauge = v.gauge;
        a.clov = v.Ainv[parity];
        a.y = y;
        a.w = w;
        a.a = op->kappa * op->kappa;
        a.partials = partials;
        a.stop = S ? &S->flags : nullptr;
        a.nrhs = nprob;
        a.nt = nprob == 1 ? nt : 1;
        a.cgroup = nprob == 1 ? cg : 0;
        a.fma = nprob == 1 ? fma : 0;
        // the reduction partials of this form must fit the workspace sized for nb_hop_cap
        if (red != RED_NONE && nprob == 1 && hop_blocks_nt(op->g, a.nt, a.cgroup) > nb_hop_cap)
            return hipErrorInvalidValue;
        if (nprob > 1) return launch_mrhs_variant(st, prec, epi, red, a, S, variant, e0, e1);
        return launch_hop(st, prec, v.recon, epi, red, a, e0, e1);
    }

    // one BiCGStab iteration on M_hat for every problem in the Krylov precision (van der Vorst 1992):
    //   v = M p, alpha = rho / (r0, v), s = r - alpha v, t = M s, omega = (t, s) / (t, t),
    //   x += alpha p + omega s, r = s - omega t, beta = (rho'/rho)(alpha/omega), p = r + beta (p - omega v)
    hipError_t enqueue_iters(hipStream_t st, int nit, int kprec, int xprec, void* xk)
    {
        void *r = W.kr[0].p, *r0 = W.kr[1].p, *p = W.kr[2].p, *vv = W.kr[3].p, *sv = W.kr[4].p, *t = W.kr[5].p,
             *tmpo = W.kr[6].p;
        Scal* dS = (Scal*)W.scal.p;
        double* dpart = (double*)W.partials.p;
        double* dpart2 = dpart + 3L * nprob * part_stride();  // partials of the x/r update
        double* hist = (double*)W.hist.p;
        const long n = n0();
        // a scalar is formed inside the vector kernel that uses it when the launch's partials are few
        // (every block of that kernel sums its problem's partials, so the reads grow with problems x
        // partials), else by a single-block kernel in between
        const bool fh = (long)nprob * nb_hop <= fuse_nb, fb = (long)nprob * nb_blas <= fuse_nb;
        hipError_t e = hipSuccess;
        for (int i = 0; i < nit && e == hipSuccess; i++) {
            e = hop(st, kprec, EPI_CLOV, RED_NONE, p, tmpo, nullptr, nullptr, nullptr, dS, 1);
            if (e == hipSuccess) e = hop(st, kprec, EPI_CLOV_XPAY, RED_WDOT, tmpo, vv, p, r0, dpart, dS, 0);
            if (e == hipSuccess && !fh) e = launch_fin_alpha(st, dS, dpart, nb_hop, nprob, nbs);
            if (e == hipSuccess)
                e = launch_bicg_s(st, kprec, sv, r, vv, n, dS, nprob, map, nmax, fh ? dpart : nullptr, nb_hop, nbs);
            if (e == hipSuccess) e = hop(st, kprec, EPI_CLOV, RED_NONE, sv, tmpo, nullptr, nullptr, nullptr, dS, 1);
            if (e == hipSuccess) e = hop(st, kprec, EPI_CLOV_XPAY, RED_TS, tmpo, t, sv, nullptr, dpart, dS, 0);
            if (e == hipSuccess && !fh) e = launch_fin_omega(st, dS, dpart, nb_hop, nprob, nbs);
            if (e == hipSuccess)
                e = launch_bicg_xr(st, kprec, xprec, xk, p, sv, r, t, r0, n, dS, dpart2, nprob, map, nmax,
                                   fh ? dpart : nullptr, nb_hop, nbs);
            if (e == hipSuccess && !fb) e = launch_fin_beta(st, dS, dpart2, nb_blas, hist, nprob);
            if (e == hipSuccess)
                e = launch_bicg_p(st, kprec, p, r, vv, n, dS, nprob, map, nmax, fb ? dpart2 : nullptr, nb_blas, hist);
        }
        return e;
    }

    // pick the multi-RHS kernel form or the batched grid by timing the candidates once
    // (result cached on the context, keyed by problem shape)
    qcdw_status tune(int kprec)
    {
        std::vector<int> cand;
        char key[160];
        if (nprob == 1) {  // the operator's own choice (tuned when it was created)
            nt = ops[0]->hop_nt[kprec];
            cg = ops[0]->hop_cg[kprec];
            fma = ops[0]->hop_fma[kprec];
            variant = nt + 16 * cg + 4096 * fma;
            nb_hop = hop_blocks_nt(ops[0]->g, nt, cg);
            return QCDW_OK;
        }
        if (batch) {
            snprintf(key, sizeof key, "batch_hop/p%d/tiles%d/n%d", kprec, batch->total_tiles, nprob);
            for (int gsz : {256, 512, 1024, 2048, 4096})
                if (gsz < batch->total_tiles) cand.push_back(gsz);
            cand.push_back(batch->total_tiles);
        } else {
            const Geom& g = ops[0]->g;
            snprintf(key, sizeof key, "mrhs_hop/p%d/L%dx%dx%dx%d/n%d", kprec, g.Lx, g.Ly, g.Lz, g.Lt, nprob);
            cand = {0, 1};
            const int nct = hop_ctiles(g);
            for (int m : {8, 16})  // register loop in slice-group order: largest divisor of nct in [4, m]
                for (int d = std::min(m, nct - 1); d >= 4; d--)
                    if (nct % d == 0) {
                        if (std::find(cand.begin(), cand.end(), 2 * d) == cand.end()) cand.push_back(2 * d);
                        break;
                    }
            if (kprec == BF16 || kprec == F16) {  // the matrix-core form, in both tile orders
                const size_t n = cand.size();
                for (size_t c = 0; c < n; c++)
                    if ((cand[c] & 1) == 0 && mrhs_variant_fits(g, kprec, MRHS_MFMA | cand[c]))
                        cand.push_back(MRHS_MFMA | cand[c]);
            }
        }
        auto choose = [&](int v) {
            variant = v;
            // multi-RHS register loop in slice-group order: one block per (c-tile, t)
            if (!batch && nprob > 1) nb_hop = mrhs_blocks(ops[0]->g, v);
        };
        auto it = ctx->tune.find(key);
        if (it != ctx->tune.end()) {
            const int v = it->second;
            const bool fits = batch ? std::find(cand.begin(), cand.end(), v) != cand.end()
                                    : mrhs_variant_fits(ops[0]->g, kprec, v);
            if (fits) {
                choose(v);
                return QCDW_OK;
            }
        }
        hipEvent_t e0, e1;
        HIPCHK(ctx, hipEventCreate(&e0));
        HIPCHK(ctx, hipEventCreate(&e1));
        float best = 1e30f;
        int best_v = cand[0];
        const bool was_on = tm.on;
        tm.on = false;
        for (int c : cand) {
            choose(c);
            // hop into odd sites from the (scratch) Krylov vectors; no solver state is touched
            hipError_t e = hop(s, kprec, EPI_CLOV, RED_NONE, W.kr[2].p, W.kr[6].p, nullptr, nullptr, nullptr,
                               nullptr, 1);
            if (e == hipSuccess) e = hipEventRecord(e0, s);
            for (int rep = 0; rep < 3 && e == hipSuccess; rep++)
                e = hop(s, kprec, EPI_CLOV, RED_NONE, W.kr[2].p, W.kr[6].p, nullptr, nullptr, nullptr, nullptr, 1);
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                (void)hipEventDestroy(e0);
                (void)hipEventDestroy(e1);
                return fail(ctx, QCDW_EHIP, "tuning launch failed: %s", hipGetErrorString(e));
            }
            if (ms < best) {
                best = ms;
                best_v = c;
            }
        }
        tm.on = was_on;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        choose(best_v);
        ctx->tune_store(key, best_v);
        return QCDW_OK;
    }

    // run nit iterations: eagerly, or by replaying a captured graph of exactly nit iterations
    qcdw_status run_chunk(int nit, int kprec, int xprec, void* xk, bool graph)
    {
        if (!graph) {
            HIPCHK(ctx, enqueue_iters(s, nit, kprec, xprec, xk));
            return QCDW_OK;
        }
        Workspace::Graph* gr = nullptr;
        for (auto& c : W.graphs)
            if (c.kprec == kprec && c.chunk == nit && c.nprob == nprob && c.variant == variant && c.gen == W.ws_gen &&
                c.fuse_nb == fuse_nb)
                gr = &c;
        if (!gr) {
            W.graphs.emplace_back();
            gr = &W.graphs.back();
            gr->kprec = kprec;
            gr->chunk = nit;
            gr->nprob = nprob;
            gr->variant = variant;
            gr->gen = W.ws_gen;
            gr->fuse_nb = fuse_nb;
            hipStream_t cs = ctx->cap_stream;
            HIPCHK(ctx, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            hipError_t e = enqueue_iters(cs, nit, kprec, xprec, xk);
            hipGraph_t g = nullptr;
            hipError_t e2 = hipStreamEndCapture(cs, &g);
            HIPCHK(ctx, e);
            HIPCHK(ctx, e2);
            gr->graph = g;
            HIPCHK(ctx, hipGraphInstantiate(&gr->exec, g, nullptr, nullptr, 0));
        }
        HIPCHK(ctx, hipGraphLaunch(gr->exec, s));
        return QCDW_OK;
    }

    qcdw_status read_doubles(std::vector<double>& out)
    {
        HIPCHK(ctx, hipMemcpyAsync(ctx->host_d, W.dres.p, nprob * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(ctx, hipStreamSynchronize(s));
        out.assign(ctx->host_d, ctx->host_d + nprob);
        return QCDW_OK;
    }

    // rhi = bhat - M_hat xhi in FP64 for every problem; rr[k] = ||rhi_k||^2
    qcdw_status true_schur_residual(std::vector<double>& rr)
    {
        for (int k = 0; k < nprob; k++) {
            const qcdw_op* op = ops[k];
            HIPCHK(ctx, matpc(s, op, view(op, F64), at(W.xhi, k), at(W.tmp64, k), W.tmpo64.p, RED_NONE, nullptr,
                              nullptr, nullptr));
        }
        HIPCHK(ctx, launch_xmy_norm2(s, F64, F64, W.bhat.p, W.tmp64.p, W.rhi.p, n0(), (double*)W.partials.p,
                                     (double*)W.dres.p, nprob, map, nmax));
        return read_doubles(rr);
    }

    // x_o = A_oo^-1 b_o + kappa A_oo^-1 H_oe x_e for problem k into tmpo64, then the FP64
    // full-lattice residual ||b - M x||^2 of that problem
    qcdw_status full_residual(int k, double& r2)
    {
        const qcdw_op* op = ops[k];
        const PrecView v64 = view(op, F64);
        const Geom& g = op->g;
        HopArgs a = hop_args(g, 1);
        a.psi = at(W.xhi, k);
        a.out = W.tmpo64.p;
        a.gauge = v64.gauge;
        a.clov = v64.Ainv[1];
        a.y = at(W.yo, k);
        a.a = -op->kappa;
        HIPCHK(ctx, launch_hop(s, F64, v64.recon, EPI_CLOV_XPAY, RED_NONE, a));
        r2 = 0;
        for (int p = 0; p < 2; p++) {
            HopArgs m = hop_args(g, p);  // (M x)_p = A_pp x_p - kappa H x_{1-p}
            m.psi = p == 0 ? W.tmpo64.p : at(W.xhi, k);
            m.out = W.tmp64.p;
            m.gauge = v64.gauge;
            m.clov = op->A64[p].p;
            m.y = p == 0 ? at(W.xhi, k) : W.tmpo64.p;
            m.a = op->kappa;
            HIPCHK(ctx, launch_hop(s, F64, v64.recon, EPI_XPAY_CLOVY, RED_NONE, m));
            HIPCHK(ctx, launch_xmy_norm2(s, F64, F64, p == 0 ? at(W.be, k) : at(W.bo, k), W.tmp64.p, nullptr, len[k],
                                         (double*)W.partials.p, (double*)W.dres.p + p));
        }
        HIPCHK(ctx, hipMemcpyAsync(ctx->host_d, W.dres.p, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(ctx, hipStreamSynchronize(s));
        r2 = ctx->host_d[0] + ctx->host_d[1];
        return QCDW_OK;
    }

    qcdw_status ensure_workspace(int kprec, int maxiter)
    {
        long total = 0;
        for (int k = 0; k < nprob; k++) total += len[k];
        std::vector<void*> before;
        DevBuf* all[] = {&W.kr[0], &W.kr[1], &W.kr[2], &W.kr[3], &W.kr[4], &W.kr[5], &W.kr[6], &W.xlo,
                         &W.xhi, &W.partials, &W.scal, &W.dres, &W.hist, &W.coef};
        for (DevBuf* b : all) before.push_back(b->p);
        DevBuf* stacked64[] = {&W.be, &W.bo, &W.yo, &W.ye, &W.bhat, &W.xhi, &W.rhi, &W.tmp64};
        for (DevBuf* b : stacked64) HIPCHK(ctx, b->alloc((size_t)total * 16));
        HIPCHK(ctx, W.tmpo64.alloc((size_t)nmax * 16));
        for (auto& b : W.kr) HIPCHK(ctx, b.alloc((size_t)total * cplx_bytes(kprec)));
        if (kprec != F64) HIPCHK(ctx, W.xlo.alloc((size_t)total * 8));
        HIPCHK(ctx, W.partials.alloc(2 * 3UL * nprob * part_stride() * sizeof(double)));
        HIPCHK(ctx, W.scal.alloc(MAX_BATCH * sizeof(Scal)));
        HIPCHK(ctx, W.dres.alloc(MAX_BATCH * sizeof(double)));
        HIPCHK(ctx, W.coef.alloc(2 * MAX_BATCH * sizeof(double)));
        HIPCHK(ctx, W.hist.alloc((size_t)nprob * ((size_t)maxiter + 2) * sizeof(double)));
        for (size_t i = 0; i < before.size(); i++)
            if (all[i]->p != before[i]) {
                W.ws_gen++;
                W.drop_graphs();
                break;
            }
        return QCDW_OK;
    }
};

// Solve M_k x_k = b_k for every problem of S (b, x: one full fermion field each).
// The problems share every launch of the iteration but keep their own scalars,
// targets and convergence flags; finished problems are masked.
qcdw_status solve(Solver& S, const void* const* bs, void* const* xs, const qcdw_solver_params* params,
                  qcdw_solve_info* infos)
{
    qcdw_ctx* ctx = S.ctx;
    Workspace& W = S.W;
    const int nprob = S.nprob;
    DeviceGuard dg(ctx->device);
    const auto t_start = std::chrono::steady_clock::now();
    qcdw_solver_params prm;
    if (params) prm = *params;
    else qcdw_solver_params_default(&prm);
    std::vector<double*> user_hist(nprob);
    std::vector<int> user_hist_len(nprob);
    for (int k = 0; k < nprob; k++) {
        user_hist[k] = infos[k].res_hist;
        user_hist_len[k] = infos[k].hist_len;
        infos[k] = qcdw_solve_info{};
        infos[k].res_hist = user_hist[k];
        infos[k].hist_len = user_hist_len[k];
        infos[k].status = QCDW_EINVAL;
    }
    for (int k = 0; k < nprob; k++) {
        CHK(check_dev(ctx, bs[k], "b"));
        CHK(check_dev(ctx, xs[k], "x"));
        if (bs[k] == xs[k]) return fail(ctx, QCDW_EINVAL, "x must not alias b");
    }
    if (!(prm.tol > 0.0) || !std::isfinite(prm.tol)) return fail(ctx, QCDW_EINVAL, "tol must be positive");
    if (prm.maxiter < 0) return fail(ctx, QCDW_EINVAL, "maxiter must be >= 0");
    if (prm.check_every < 1) prm.check_every = 1;
    int kprec = (int)prm.inner;  // raised to F64 if the low-precision cycles stop reducing the residual
    for (auto* op : S.ops)
        if (kprec != F64 && kprec != op->inner)
            return fail(ctx, QCDW_EINVAL, "inner precision %d not prepared by the operator (has %d)", kprec,
                        op->inner);
    if (kprec != F64 && !(prm.delta > 0.0 && prm.delta < 1.0))
        return fail(ctx, QCDW_EINVAL, "delta must lie in (0, 1)");
    CHK(S.ensure_workspace(kprec, prm.maxiter));
    S.tm.on = prm.collect_timing != 0;
    const bool use_graph = prm.use_graph != 0 && !S.tm.on;  // per-launch timing needs eager launches
    hipStream_t s = S.s;
    Scal* dS = (Scal*)W.scal.p;
    double* dhist = (double*)W.hist.p;
    double* dpart = (double*)W.partials.p;
    double* dres = (double*)W.dres.p;
    double* dcoef = (double*)W.coef.p;
    const int hist_len = prm.maxiter + 2;
    std::vector<std::vector<double>> hist_host(nprob);
    const long n0 = S.n0();

    // ---- source preparation (FP64) --------------------------------------
    for (int k = 0; k < nprob; k++) {
        const Geom& g = S.ops[k]->g;
        HIPCHK(ctx, launch_pack_spinor(s, F64, g, bs[k], 0, S.at(W.be, k), 1.0));
        HIPCHK(ctx, launch_pack_spinor(s, F64, g, bs[k], 1, S.at(W.bo, k), 1.0));
        HIPCHK(ctx, launch_pack_spinor(s, F64, g, xs[k], 0, S.at(W.xhi, k), 1.0));
    }
    std::vector<double> bn2e(nprob), bn2o(nprob), bnorm(nprob);
    {
        // ||b_e||^2 into dres[0, nprob), ||b_o||^2 into coef[0, nprob) (both sized for MAX_BATCH), one read
        HIPCHK(ctx, launch_norm2(s, F64, W.be.p, n0, dpart, dres, nprob, S.map, S.nmax));
        HIPCHK(ctx, launch_norm2(s, F64, W.bo.p, n0, dpart + 3L * nprob * S.part_stride(), dcoef, nprob, S.map,
                                 S.nmax));
        HIPCHK(ctx, hipMemcpyAsync(ctx->host_d, dres, nprob * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(ctx, hipMemcpyAsync(ctx->host_d + nprob, dcoef, nprob * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(ctx, hipStreamSynchronize(s));
        for (int k = 0; k < nprob; k++) {
            bn2e[k] = ctx->host_d[k];
            bn2o[k] = ctx->host_d[nprob + k];
        }
    }
    std::vector<int> status(nprob, QCDW_ENOCONV), done(nprob, 0), restarts(nprob, 0), iters(nprob, 0);
    std::vector<double> true_res(nprob, NAN), target(nprob), iter_res(nprob, NAN);
    for (int k = 0; k < nprob; k++) {
        const qcdw_op* op = S.ops[k];
        const Geom& g = op->g;
        const PrecView v64 = view(op, F64);
        const size_t fbytes = 24UL * g.Vh * 16;
        bnorm[k] = std::sqrt(bn2e[k] + bn2o[k]);
        if (!std::isfinite(bnorm[k])) {
            status[k] = QCDW_ENAN;
            done[k] = 1;
        } else if (bnorm[k] == 0.0) {
            status[k] = QCDW_OK;
            true_res[k] = 0.0;
            done[k] = 1;
            HIPCHK(ctx, hipMemsetAsync(S.at(W.xhi, k), 0, S.len[k] * 16, s));
            HIPCHK(ctx, hipMemsetAsync(xs[k], 0, fbytes, s));
        }
        target[k] = 0.5 * prm.tol * bnorm[k];  // on ||bhat - M_hat x_e||
        // y_o = A_oo^-1 b_o ; y_e = A_ee^-1 b_e ; bhat = y_e + kappa A_ee^-1 H_eo y_o
        HIPCHK(ctx, launch_clov_apply_internal(s, F64, g, v64.Ainv[1], S.at(W.bo, k), S.at(W.yo, k)));
        HIPCHK(ctx, launch_clov_apply_internal(s, F64, g, v64.Ainv[0], S.at(W.be, k), S.at(W.ye, k)));
        HopArgs a = hop_args(g, 0);
        a.psi = S.at(W.yo, k);
        a.out = S.at(W.bhat, k);
        a.gauge = v64.gauge;
        a.clov = v64.Ainv[0];
        a.y = S.at(W.ye, k);
        a.a = -op->kappa;
        HIPCHK(ctx, launch_hop(s, F64, v64.recon, EPI_CLOV_XPAY, RED_NONE, a));
    }
    CHK(S.tune(kprec));

    // ---- outer loop: Krylov cycles with FP64 residual recomputation -----
    std::vector<double> rr_hi;
    CHK(S.true_schur_residual(rr_hi));
    for (int k = 0; k < nprob; k++)
        if (!done[k]) hist_host[k].push_back(std::sqrt(rr_hi[k]) / bnorm[k]);
    int lock_iters = 0, reliable = 0, fault = prm.fault_inject, cycles = 0;
    const int maxiter = prm.maxiter;
    bool mixed = kprec != F64;
    void *r = W.kr[0].p, *r0 = W.kr[1].p, *p = W.kr[2].p;
    void* xk = mixed ? W.xlo.p : W.xhi.p;
    int xprec = mixed ? F32 : F64;
    // precision escalation: a healthy low-precision cycle cuts the FP64 residual by about delta; when
    // ESCALATE_CYCLES cycles in a row fail to halve it (the rounded operator is too far from the true
    // one, as near the critical kappa), or the inner iteration overflows, the remaining cycles run
    // in FP64
    constexpr int ESCALATE_CYCLES = 3;
    std::vector<double> progress_rr(rr_hi);
    std::vector<int> stalls(nprob, 0), iters_at_escalation(nprob, -1);
    auto escalate = [&]() -> qcdw_status {
        kprec = F64;
        mixed = false;
        xprec = F64;
        CHK(S.ensure_workspace(F64, prm.maxiter));
        CHK(S.tune(F64));
        dS = (Scal*)W.scal.p;
        dhist = (double*)W.hist.p;
        dpart = (double*)W.partials.p;
        dres = (double*)W.dres.p;
        dcoef = (double*)W.coef.p;
        r = W.kr[0].p;
        r0 = W.kr[1].p;
        p = W.kr[2].p;
        xk = W.xhi.p;
        cycles = 0;
        for (int k = 0; k < nprob; k++) iters_at_escalation[k] = iters[k];
        return QCDW_OK;
    };

    while (true) {
        bool pending = false;
        for (int k = 0; k < nprob; k++) {
            if (done[k]) continue;
            if (!std::isfinite(rr_hi[k])) {
                status[k] = QCDW_ENAN;
                done[k] = 1;
                continue;
            }
            if (std::sqrt(rr_hi[k]) <= target[k]) {
                double r2;
                CHK(S.full_residual(k, r2));
                true_res[k] = std::sqrt(r2) / bnorm[k];
                if (true_res[k] <= prm.tol) {
                    status[k] = QCDW_OK;
                    done[k] = 1;
                    const Geom& g = S.ops[k]->g;
                    HIPCHK(ctx, launch_unpack_spinor(s, F64, g, S.at(W.xhi, k), 0, xs[k], 1.0));
                    HIPCHK(ctx, launch_unpack_spinor(s, F64, g, W.tmpo64.p, 1, xs[k], 1.0));
                    continue;
                }
                target[k] *= 0.5 * prm.tol / true_res[k];  // tighten and keep iterating
            }
            pending = true;
        }
        if (!pending || lock_iters >= maxiter) break;

        // --- one Krylov cycle on M_hat c = rhi for the pending problems -----
        // with inner_resume a low-precision cycle continues the previous one's recurrence if every pending
        // problem's last cycle ended by convergence of its iterated residual; else (first cycle,
        // breakdown, overflow, stagnation stop, FP64) it restarts from the true residual
        bool resume = mixed && prm.inner_resume != 0 && cycles > 0;
        for (int k = 0; k < nprob && resume; k++)
            if (!done[k] && ctx->host_scal[k].flags != FLAG_CONV) resume = false;
        cycles++;
        double* hc = ctx->host_d;  // [0, nprob): scales, [nprob, 2 nprob): coefficients of the x update
        std::vector<double> scale(nprob, 1.0);
        for (int k = 0; k < nprob; k++) {
            scale[k] = (mixed && !done[k] && rr_hi[k] > 0) ? std::sqrt((double)S.len[k] / rr_hi[k]) : 1.0;
            hc[k] = scale[k];
            hc[nprob + k] = done[k] ? 0.0 : 1.0 / scale[k];
        }
        HIPCHK(ctx, hipMemcpyAsync(dcoef, hc, 2 * nprob * sizeof(double), hipMemcpyHostToDevice, s));
        Scal* hs = ctx->host_scal;  // a resumed cycle keeps the last cycle's rho, alpha, omega, r0 norm
        if (!resume) memset(hs, 0, nprob * sizeof(Scal));
        for (int k = 0; k < nprob; k++) {
            double cycle_stop = target[k] * scale[k];
            if (mixed) cycle_stop = std::max(cycle_stop, prm.delta * std::sqrt((double)S.len[k]));
            hs[k].stop_rr = done[k] ? INFINITY : cycle_stop * cycle_stop;  // finished problems start converged
            hs[k].hist_norm = 1.0 / (scale[k] * bnorm[k]);
            hs[k].iter = iters[k];
            hs[k].fault_iter = fault;
            hs[k].hist_len = hist_len;
            if (resume) hs[k].flags = done[k] ? FLAG_CONV : 0;
        }
        HIPCHK(ctx, hipMemcpyAsync(dS, hs, nprob * sizeof(Scal), hipMemcpyHostToDevice, s));
        // r = scale rhi; restart: r0 = p = r, rho = ||r||^2; the FP32 correction starts at zero
        HIPCHK(ctx, launch_cycle_start(s, kprec, W.rhi.p, r, r0, p, mixed ? W.xlo.p : nullptr, n0, dcoef, dS, dpart,
                                       nprob, S.map, S.nmax, resume));
        if (resume) {
            // reliable update without restart: r is the rescaled true residual, r0, p, v and the scalars
            // carry on (Sleijpen and van der Vorst 1996)
            HIPCHK(ctx, launch_bicg_resume(s, kprec, r0, r, n0, dS, dpart, nprob, S.map, S.nmax));
            HIPCHK(ctx, launch_bicg_p(s, kprec, p, r, W.kr[3].p, n0, dS, nprob, S.map, S.nmax));
        }
        int all_flags = 0;
        // stagnation of a low-precision cycle: no new minimum of the iterated residual for
        // STAG_ITERS iterations ends the cycle (a reliable update follows)
        constexpr int STAG_ITERS = 96;
        std::vector<double> cyc_min(nprob, INFINITY);
        std::vector<int> cyc_min_it(iters);
        while (true) {
            const int chunk = std::min(prm.check_every, maxiter - lock_iters);
            if (chunk <= 0) break;
            CHK(S.run_chunk(chunk, kprec, xprec, xk, use_graph));
            HIPCHK(ctx, hipMemcpyAsync(hs, dS, nprob * sizeof(Scal), hipMemcpyDeviceToHost, s));
            HIPCHK(ctx, hipStreamSynchronize(s));
            int advanced = 0;
            bool all_set = true;
            for (int k = 0; k < nprob; k++) {
                advanced = std::max(advanced, hs[k].iter - iters[k]);
                iters[k] = hs[k].iter;
                if (mixed && !done[k] && !hs[k].flags) {
                    if (hs[k].rr < cyc_min[k]) {
                        cyc_min[k] = hs[k].rr;
                        cyc_min_it[k] = iters[k];
                    } else if (iters[k] - cyc_min_it[k] >= STAG_ITERS) {
                        hs[k].flags = FLAG_STOP;
                        HIPCHK(ctx, hipMemcpyAsync(&dS[k].flags, &hs[k].flags, sizeof(int), hipMemcpyHostToDevice, s));
                    }
                }
                if (!hs[k].flags) all_set = false;
            }
            if (S.tm.on) S.tm.collect((size_t)4 * advanced);
            lock_iters += chunk;
            if (all_set) break;
        }
        for (int k = 0; k < nprob; k++) {
            all_flags |= hs[k].flags;
            if (!done[k]) iter_res[k] = std::sqrt(hs[k].rr) / (scale[k] * bnorm[k]);
        }
        bool raise = false;
        if (mixed) {
            // a low-precision cycle that overflowed contributes no correction; the problem escalates
            bool dropped = false;
            for (int k = 0; k < nprob; k++)
                if (!done[k] && (hs[k].flags & FLAG_NAN)) {
                    hc[nprob + k] = 0.0;
                    dropped = raise = true;
                }
            if (dropped)
                HIPCHK(ctx, hipMemcpyAsync(dcoef + nprob, hc + nprob, nprob * sizeof(double), hipMemcpyHostToDevice,
                                           s));
            HIPCHK(ctx, launch_axpy_hi(s, F32, 0.0, dcoef + nprob, W.xlo.p, W.xhi.p, n0, nprob, S.map, S.nmax));
        }
        for (int k = 0; k < nprob; k++) {
            if (done[k]) continue;
            if (hs[k].flags & FLAG_NAN) {
                if (mixed) continue;
                status[k] = QCDW_ENAN;
                done[k] = 1;
            } else if ((hs[k].flags & FLAG_BREAK) && ++restarts[k] > prm.max_restarts) {
                if (mixed) {
                    restarts[k] = 0;
                    raise = true;
                    continue;
                }
                status[k] = QCDW_EBREAKDOWN;
                done[k] = 2;
            }
        }
        if (all_flags & (FLAG_BREAK | FLAG_NAN)) fault = 0;
        CHK(S.true_schur_residual(rr_hi));
        reliable++;
        if (mixed) {
            for (int k = 0; k < nprob; k++) {
                if (done[k]) continue;
                if (rr_hi[k] < 0.25 * progress_rr[k]) {
                    progress_rr[k] = rr_hi[k];
                    stalls[k] = 0;
                } else if (++stalls[k] >= ESCALATE_CYCLES) {
                    raise = true;
                }
            }
            if (raise) CHK(escalate());
        }
    }

    // ---- unfinished problems: best iterate and its true residual ----------
    for (int k = 0; k < nprob; k++) {
        if (status[k] == QCDW_OK || status[k] == QCDW_ENAN) continue;
        double r2;
        CHK(S.full_residual(k, r2));
        true_res[k] = std::sqrt(r2) / bnorm[k];
        const Geom& g = S.ops[k]->g;
        HIPCHK(ctx, launch_unpack_spinor(s, F64, g, S.at(W.xhi, k), 0, xs[k], 1.0));
        HIPCHK(ctx, launch_unpack_spinor(s, F64, g, W.tmpo64.p, 1, xs[k], 1.0));
    }
    HIPCHK(ctx, hipStreamSynchronize(s));
    // the iterated-residual history of each problem, written by the device at iterations 1..iters
    for (int k = 0; k < nprob; k++) {
        const int m = std::min(iters[k], hist_len - 1);
        if (!user_hist[k] || user_hist_len[k] <= 0 || m <= 0) continue;
        const size_t at = hist_host[k].size();
        hist_host[k].resize(at + m);
        HIPCHK(ctx, hipMemcpy(hist_host[k].data() + at, dhist + (size_t)k * hist_len + 1, m * sizeof(double),
                              hipMemcpyDeviceToHost));
    }

    const double wall = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    qcdw_status worst = QCDW_OK;
    for (int k = 0; k < nprob; k++) {
        qcdw_solve_info* inf = infos + k;
        inf->status = status[k];
        inf->iters = iters[k];
        inf->n_reliable = reliable;
        inf->n_restarts = restarts[k];
        inf->true_res = true_res[k];
        inf->iter_res = iter_res[k];
        inf->time_ms = wall;
        inf->fallback = iters_at_escalation[k] >= 0;
        inf->fallback_iters = iters_at_escalation[k] >= 0 ? iters[k] - iters_at_escalation[k] : 0;
        for (int j = 0; j < 3; j++) {
            inf->hop_ms[j] = S.tm.ms[j];
            inf->n_hop[j] = (int32_t)S.tm.launches[j];
        }
        if (user_hist[k] && user_hist_len[k] > 0) {
            const int m = std::min<int>(user_hist_len[k], (int)hist_host[k].size());
            memcpy(user_hist[k], hist_host[k].data(), m * sizeof(double));
            inf->hist_count = m;
        }
        if (status[k] != QCDW_OK && worst == QCDW_OK) worst = (qcdw_status)status[k];
    }
    if (worst != QCDW_OK) {
        const char* what = worst == QCDW_ENOCONV      ? "did not converge within maxiter"
                           : worst == QCDW_ENAN       ? "NaN or Inf in the source or the iteration"
                           : worst == QCDW_EBREAKDOWN ? "BiCGStab breakdown persisted after restarts"
                                                      : "solver failed";
        int k0 = 0;
        while (k0 < nprob && status[k0] == QCDW_OK) k0++;
        return fail(ctx, worst, "%s (problem %d: iters %d, true residual %.3e)", what, k0, iters[k0], true_res[k0]);
    }
    return QCDW_OK;
}

}  // namespace

extern "C" qcdw_status qcdw_invert(qcdw_op* op, const void* b, void* x, const qcdw_solver_params* params,
                                   qcdw_solve_info* info)
{
    if (!op) return QCDW_EINVAL;
    qcdw_solve_info dummy{};
    Solver S(op->ctx, op->ws, {op}, nullptr);
    return solve(S, &b, &x, params, info ? info : &dummy);
}

extern "C" qcdw_status qcdw_invert_multi(qcdw_op* op, int nrhs, const void* b, void* x,
                                         const qcdw_solver_params* params, qcdw_solve_info* info)
{
    if (!op) return QCDW_EINVAL;
    if (nrhs < 1 || nrhs > MAX_RHS || !info)
        return fail(op->ctx, QCDW_EINVAL, "nrhs must lie in [1, %d] and info must not be NULL", MAX_RHS);
    const size_t fb = 24UL * op->g.Vh * 16;
    std::vector<const void*> bs(nrhs);
    std::vector<void*> xs(nrhs);
    for (int k = 0; k < nrhs; k++) {
        bs[k] = (const char*)b + k * fb;
        xs[k] = (char*)x + k * fb;
    }
    Solver S(op->ctx, op->ws, std::vector<qcdw_op*>(nrhs, op), nullptr);
    return solve(S, bs.data(), xs.data(), params, info);
}

extern "C" qcdw_status qcdw_batch_create(qcdw_ctx* ctx, int n, qcdw_op* const ops[], qcdw_batch** out)
{
    if (!ctx) return QCDW_EINVAL;
    if (!out || !ops || n < 1 || n > MAX_BATCH)
        return fail(ctx, QCDW_EINVAL, "need 1..%d operators and an output pointer", MAX_BATCH);
    *out = nullptr;
    DeviceGuard dg(ctx->device);
    for (int k = 0; k < n; k++) {
        if (!ops[k] || ops[k]->ctx != ctx) return fail(ctx, QCDW_EINVAL, "operator %d is NULL or of another context", k);
        if (ops[k]->inner != ops[0]->inner)
            return fail(ctx, QCDW_EINVAL, "all operators of a batch need the same inner precision");
        if (ops[k]->recon != 12) return fail(ctx, QCDW_EINVAL, "batched solves use reconstruct-12 operators");
    }
    qcdw_batch* b = new qcdw_batch;
    b->ctx = ctx;
    b->ops.assign(ops, ops + n);
    b->inner = ops[0]->inner;
    std::vector<long2> map(n);
    std::vector<int> tiles(n);
    std::vector<BatchEntry> t64(n), tlo(n);
    int tile0 = 0;
    for (int k = 0; k < n; k++) {
        const qcdw_op* op = ops[k];
        const long len = 12L * op->g.Vh;
        b->off.push_back(b->total);
        b->len.push_back(len);
        map[k] = make_long2(b->total, len);
        tiles[k] = hop_blocks(op->g.Vh);
        for (int pr = 0; pr < 2; pr++) {
            BatchEntry& e = pr == 0 ? t64[k] : tlo[k];
            const PrecView v = view(op, pr == 0 ? F64 : op->inner);
            e.g = op->g;
            e.kappa2 = op->kappa * op->kappa;
            e.gauge = v.gauge;
            e.clov[0] = v.Ainv[0];
            e.clov[1] = v.Ainv[1];
            e.off = b->total;
            e.n = len;
            e.tile0 = tile0;
            e.ntiles = tiles[k];
        }
        tile0 += tiles[k];
        b->total += len;
        b->nmax = std::max(b->nmax, len);
        b->nbmax = std::max(b->nbmax, tiles[k]);
    }
    b->total_tiles = tile0;
    hipStream_t s = ctx->stream;
    hipError_t e = b->map.alloc(n * sizeof(long2));
    if (e == hipSuccess) e = b->nbs.alloc(n * sizeof(int));
    if (e == hipSuccess) e = b->tab64.alloc(n * sizeof(BatchEntry));
    if (e == hipSuccess) e = b->tablo.alloc(n * sizeof(BatchEntry));
    if (e == hipSuccess) e = hipMemcpyAsync(b->map.p, map.data(), n * sizeof(long2), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(b->nbs.p, tiles.data(), n * sizeof(int), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(b->tab64.p, t64.data(), n * sizeof(BatchEntry), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(b->tablo.p, tlo.data(), n * sizeof(BatchEntry), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        delete b;
        return fail(ctx, e == hipErrorOutOfMemory ? QCDW_ENOMEM : QCDW_EHIP, "batch setup: %s", hipGetErrorString(e));
    }
    *out = b;
    return QCDW_OK;
}

extern "C" void qcdw_batch_destroy(qcdw_batch* b)
{
    if (!b) return;
    DeviceGuard dg(b->ctx->device);
    (void)hipStreamSynchronize(b->ctx->stream);
    delete b;
}

extern "C" qcdw_status qcdw_invert_batch(qcdw_batch* b, const void* const bs[], void* const xs[],
                                         const qcdw_solver_params* params, qcdw_solve_info* infos)
{
    if (!b) return QCDW_EINVAL;
    if (!bs || !xs || !infos) return fail(b->ctx, QCDW_EINVAL, "b, x and info arrays must not be NULL");
    Solver S(b->ctx, b->ws, b->ops, b);
    return solve(S, bs, xs, params, infos);
}
