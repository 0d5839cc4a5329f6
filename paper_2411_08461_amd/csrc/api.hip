// C-ABI of libqcdw (declared in include/qcdw.h): argument checking, device
// workspaces, and the host side of the even-odd preconditioned BiCGStab solver
// whose iterations run entirely on the device (scalars never leave the GPU
// except for the periodic convergence poll).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"
#include "qcdw.h"

using namespace qcdw;

struct qcdw_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;  // private stream used only to capture graphs
    std::string err;
    Scal* host_scal = nullptr;  // pinned
    double* host_d = nullptr;   // pinned, 64 doubles
    int* dev_int = nullptr;
};

namespace {

struct DevBuf {
    void* p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
    hipError_t alloc(size_t bytes)
    {
        if (p && n >= bytes) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
        if (bytes == 0) bytes = 16;
        hipError_t e = hipMalloc(&p, bytes);
        if (e == hipSuccess) n = bytes;
        return e;
    }
};

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

qcdw_status fail(qcdw_ctx* ctx, qcdw_status st, const char* fmt, ...)
{
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return st;
}

#define HIPCHK(ctx, expr)                                                                                   \
    do {                                                                                                    \
        hipError_t e_ = (expr);                                                                             \
        if (e_ != hipSuccess)                                                                               \
            return fail((ctx), e_ == hipErrorOutOfMemory ? QCDW_ENOMEM : QCDW_EHIP, "%s: %s (%s:%d)", #expr, \
                        hipGetErrorString(e_), __FILE__, __LINE__);                                         \
    } while (0)

qcdw_status check_lattice(qcdw_ctx* ctx, const qcdw_lattice* lat, Geom& g)
{
    if (!lat) return fail(ctx, QCDW_EINVAL, "lattice descriptor is NULL");
    for (int i = 0; i < 4; i++)
        if (lat->L[i] < 2 || lat->L[i] % 2)
            return fail(ctx, QCDW_EINVAL, "lattice extent L[%d] = %d must be even and >= 2", i, lat->L[i]);
    if (lat->t_bc != 1 && lat->t_bc != -1) return fail(ctx, QCDW_EINVAL, "t_bc must be +1 or -1, got %d", lat->t_bc);
    const long V = (long)lat->L[0] * lat->L[1] * lat->L[2] * lat->L[3];
    if (V / 2 > (1L << 28)) return fail(ctx, QCDW_EINVAL, "lattice too large (V = %ld)", V);
    g.Lx = lat->L[0];
    g.Ly = lat->L[1];
    g.Lz = lat->L[2];
    g.Lt = lat->L[3];
    g.Lxh = g.Lx / 2;
    g.Vh = (int)(V / 2);
    g.t_bc = lat->t_bc;
    return QCDW_OK;
}

qcdw_status check_dev(qcdw_ctx* ctx, const void* p, const char* name)
{
    if (!p) return fail(ctx, QCDW_EINVAL, "%s is NULL", name);
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, QCDW_EINVAL, "%s is not a device pointer", name);
    }
    if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged)
        return fail(ctx, QCDW_EINVAL, "%s is not device memory", name);
    return QCDW_OK;
}

#define CHK(expr)                          \
    do {                                   \
        qcdw_status s_ = (expr);           \
        if (s_ != QCDW_OK) return s_;      \
    } while (0)

}  // namespace

// ---------------------------------------------------------------------------
// operator object
// ---------------------------------------------------------------------------
struct qcdw_op {
    qcdw_ctx* ctx = nullptr;
    Geom g{};
    double kappa = 0, csw = 0;
    int inner = F64;
    int recon = 12;
    DevBuf gauge64, gauge_lo;
    DevBuf Ainv64[2], Ainv_lo[2], A64[2];
    // solver workspace (allocated on first use)
    DevBuf be, bo, yo, ye, bhat, xhi, rhi, tmp64, tmpo64;
    DevBuf kr[7];  // r, r0, p, v, s, t, tmp_o in the Krylov precision
    DevBuf xlo;    // FP32 correction (mixed precision)
    DevBuf partials, scal, dres, hist;
    int kr_prec = -1;
    int ws_gen = 0;  // bumped whenever a workspace buffer is (re)allocated
    // captured iteration chunks, replayed by the solver
    struct Graph {
        int kprec, chunk, gen;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
    };
    std::vector<Graph> graphs;
    void drop_graphs()
    {
        for (auto& gr : graphs) {
            if (gr.exec) (void)hipGraphExecDestroy(gr.exec);
            if (gr.graph) (void)hipGraphDestroy(gr.graph);
        }
        graphs.clear();
    }
    ~qcdw_op() { drop_graphs(); }
};

namespace {

constexpr long MAX_PARTIALS = 4096;  // >= blas_blocks(); hop partials are sized per lattice

struct PrecView {
    int prec;
    int recon;
    const void* gauge;
    const void* Ainv[2];
};

PrecView view(const qcdw_op* op, int prec)
{
    if (prec == F64) return {F64, op->recon, op->gauge64.p, {op->Ainv64[0].p, op->Ainv64[1].p}};
    return {op->inner, op->inner == F64 ? op->recon : (op->inner == F32 ? op->recon : 12), op->gauge_lo.p,
            {op->Ainv_lo[0].p, op->Ainv_lo[1].p}};
}

HopArgs hop_args(const Geom& g, int parity)
{
    HopArgs a{};
    a.g = g;
    a.parity = parity;
    a.nrhs = 1;
    return a;
}

// out_e = M_hat in_e = in_e - kappa^2 A_ee^-1 H_eo A_oo^-1 H_oe in_e, with an optional fused reduction
hipError_t matpc(hipStream_t s, const qcdw_op* op, const PrecView& v, const void* in, void* out, void* tmp_o, int red,
                 const void* w, double* partials, const int* stop)
{
    HopArgs a = hop_args(op->g, 1);
    a.psi = in;
    a.out = tmp_o;
    a.gauge = v.gauge;
    a.clov = v.Ainv[1];
    a.stop = stop;
    hipError_t e = launch_hop(s, v.prec, v.recon, EPI_CLOV, RED_NONE, a);
    if (e != hipSuccess) return e;
    HopArgs b = hop_args(op->g, 0);
    b.psi = tmp_o;
    b.out = out;
    b.gauge = v.gauge;
    b.clov = v.Ainv[0];
    b.y = in;
    b.w = w;
    b.a = op->kappa * op->kappa;
    b.partials = partials;
    b.stop = stop;
    return launch_hop(s, v.prec, v.recon, EPI_CLOV_XPAY, red, b);
}

qcdw_status read_double(qcdw_ctx* ctx, const double* dev, double& out)
{
    HIPCHK(ctx, hipMemcpyAsync(ctx->host_d, dev, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    out = ctx->host_d[0];
    return QCDW_OK;
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
    p->pad_ = 0;
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
    if (hipHostMalloc((void**)&c->host_scal, sizeof(Scal)) != hipSuccess ||
        hipHostMalloc((void**)&c->host_d, 64 * sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&c->dev_int, 64 * sizeof(int)) != hipSuccess ||
        hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        qcdw_ctx_destroy(c);
        return QCDW_ENOMEM;
    }
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
    delete ctx;
}

const char* qcdw_last_error(const qcdw_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

qcdw_status qcdw_ctx_set_stream(qcdw_ctx* ctx, void* hip_stream)
{
    if (!ctx) return QCDW_EINVAL;
    ctx->stream = (hipStream_t)hip_stream;
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
        HIPCHK(ctx, A[p].alloc(72UL * g.Vh * 8));
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

qcdw_status qcdw_op_create(qcdw_ctx* ctx, const qcdw_lattice* lat, const void* U, double kappa, double csw,
                           qcdw_prec inner, int recon, qcdw_op** op_out)
{
    if (!ctx) return QCDW_EINVAL;
    if (!op_out) return fail(ctx, QCDW_EINVAL, "op pointer is NULL");
    *op_out = nullptr;
    DeviceGuard dg(ctx->device);
    Geom g;
    CHK(check_lattice(ctx, lat, g));
    CHK(check_dev(ctx, U, "U"));
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
        delete op;
        return st;
    };
    const int R = recon == 18 ? 9 : 6;
    DevBuf clov, inv, Ap;
    if (op->gauge64.alloc(8UL * g.Vh * R * 16) != hipSuccess || clov.alloc(144UL * g.Vh * 8) != hipSuccess ||
        inv.alloc(144UL * g.Vh * 8) != hipSuccess || Ap.alloc(144UL * g.Vh * 8) != hipSuccess)
        return cleanup(fail(ctx, QCDW_ENOMEM, "out of device memory creating the operator"));
    for (int p = 0; p < 2; p++)
        if (op->Ainv64[p].alloc(72UL * g.Vh * 8) != hipSuccess || op->A64[p].alloc(72UL * g.Vh * 8) != hipSuccess)
            return cleanup(fail(ctx, QCDW_ENOMEM, "out of device memory creating the operator"));
    hipError_t e = launch_pack_gauge(s, F64, recon, g, U, op->gauge64.p);
    if (e == hipSuccess) e = launch_clover_build(s, g, U, clov.p);
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
            if (op->Ainv_lo[p].alloc(72UL * g.Vh * real_bytes(inner)) != hipSuccess)
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
    *op_out = op;
    return QCDW_OK;
}

void qcdw_op_destroy(qcdw_op* op)
{
    if (!op) return;
    DeviceGuard dg(op->ctx->device);
    (void)hipStreamSynchronize(op->ctx->stream);
    delete op;
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

struct Solver {
    qcdw_op* op;
    qcdw_ctx* ctx;
    hipStream_t s;
    long n;  // complex elements of a half-lattice spinor
    int nb_hop, nb_blas;
    Timing tm;

    hipError_t timed_hop(hipStream_t st, int prec, int recon, int epi, int red, const HopArgs& a)
    {
        const int kind = epi == EPI_CLOV ? 0 : (red == RED_WDOT ? 1 : 2);
        if (!tm.on) return launch_hop(st, prec, recon, epi, red, a);
        tm.kind.push_back(kind);
        hipEvent_t e0 = tm.get(), e1 = tm.get();
        return launch_hop(st, prec, recon, epi, red, a, e0, e1);
    }

    hipError_t matpc_t(hipStream_t st, const PrecView& v, const void* in, void* out, void* tmp_o, int red,
                       const void* w, double* partials, const int* stop)
    {
        HopArgs a = hop_args(op->g, 1);
        a.psi = in;
        a.out = tmp_o;
        a.gauge = v.gauge;
        a.clov = v.Ainv[1];
        a.stop = stop;
        hipError_t e = timed_hop(st, v.prec, v.recon, EPI_CLOV, RED_NONE, a);
        if (e != hipSuccess) return e;
        HopArgs b = hop_args(op->g, 0);
        b.psi = tmp_o;
        b.out = out;
        b.gauge = v.gauge;
        b.clov = v.Ainv[0];
        b.y = in;
        b.w = w;
        b.a = op->kappa * op->kappa;
        b.partials = partials;
        b.stop = stop;
        return timed_hop(st, v.prec, v.recon, EPI_CLOV_XPAY, red, b);
    }

    // one BiCGStab iteration on M_hat in the Krylov precision (van der Vorst 1992):
    //   v = M p, alpha = rho / (r0, v), s = r - alpha v, t = M s, omega = (t, s) / (t, t),
    //   x += alpha p + omega s, r = s - omega t, beta = (rho'/rho)(alpha/omega), p = r + beta (p - omega v)
    hipError_t enqueue_iters(hipStream_t st, int nit, int kprec, int xprec, void* xk)
    {
        const PrecView vk = view(op, kprec);
        void *r = op->kr[0].p, *r0 = op->kr[1].p, *p = op->kr[2].p, *vv = op->kr[3].p, *sv = op->kr[4].p,
             *t = op->kr[5].p, *tmpo = op->kr[6].p;
        Scal* dS = (Scal*)op->scal.p;
        double* dpart = (double*)op->partials.p;
        const int* stop = &dS->flags;
        hipError_t e = hipSuccess;
        for (int i = 0; i < nit && e == hipSuccess; i++) {
            e = matpc_t(st, vk, p, vv, tmpo, RED_WDOT, r0, dpart, stop);
            if (e == hipSuccess) e = launch_fin_alpha(st, dS, dpart, nb_hop);
            if (e == hipSuccess) e = launch_bicg_s(st, kprec, sv, r, vv, n, dS);
            if (e == hipSuccess) e = matpc_t(st, vk, sv, t, tmpo, RED_TS, nullptr, dpart, stop);
            if (e == hipSuccess) e = launch_fin_omega(st, dS, dpart, nb_hop);
            if (e == hipSuccess) e = launch_bicg_xr(st, kprec, xprec, xk, p, sv, r, t, r0, n, dS, dpart);
            if (e == hipSuccess) e = launch_fin_beta(st, dS, dpart, nb_blas, (double*)op->hist.p);
            if (e == hipSuccess) e = launch_bicg_p(st, kprec, p, r, vv, n, dS);
        }
        return e;
    }

    // run nit iterations: eagerly, or by replaying a captured graph of exactly nit iterations
    qcdw_status run_chunk(int nit, int kprec, int xprec, void* xk, bool graph)
    {
        if (!graph) {
            HIPCHK(ctx, enqueue_iters(s, nit, kprec, xprec, xk));
            return QCDW_OK;
        }
        qcdw_op::Graph* gr = nullptr;
        for (auto& cand : op->graphs)
            if (cand.kprec == kprec && cand.chunk == nit && cand.gen == op->ws_gen)
                gr = &cand;
        if (!gr) {
            op->graphs.emplace_back();
            gr = &op->graphs.back();
            gr->kprec = kprec;
            gr->chunk = nit;
            gr->gen = op->ws_gen;
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

    // rhi = bhat - M_hat xhi in FP64; returns ||rhi||^2
    qcdw_status true_schur_residual(double& rr)
    {
        const PrecView v = view(op, F64);
        HIPCHK(ctx, matpc(s, op, v, op->xhi.p, op->tmp64.p, op->tmpo64.p, RED_NONE, nullptr, nullptr, nullptr));
        HIPCHK(ctx, launch_xmy_norm2(s, F64, F64, op->bhat.p, op->tmp64.p, op->rhi.p, n, (double*)op->partials.p,
                                     (double*)op->dres.p));
        return read_double(ctx, (double*)op->dres.p, rr);
    }
};

qcdw_status ensure_workspace(qcdw_op* op, int kprec, int maxiter)
{
    qcdw_ctx* ctx = op->ctx;
    const long n = 12L * op->g.Vh;
    const size_t b64 = n * 16;
    std::vector<void*> before;
    DevBuf* all[] = {&op->kr[0], &op->kr[1], &op->kr[2], &op->kr[3], &op->kr[4], &op->kr[5], &op->kr[6], &op->xlo,
                     &op->xhi, &op->partials, &op->scal, &op->dres, &op->hist};
    for (DevBuf* b : all) before.push_back(b->p);
    DevBuf* f64bufs[] = {&op->be, &op->bo, &op->yo, &op->ye, &op->bhat, &op->xhi, &op->rhi, &op->tmp64, &op->tmpo64};
    for (DevBuf* b : f64bufs) HIPCHK(ctx, b->alloc(b64));
    for (auto& b : op->kr) HIPCHK(ctx, b.alloc(n * cplx_bytes(kprec)));
    if (kprec != F64) HIPCHK(ctx, op->xlo.alloc(n * 8));
    HIPCHK(ctx, op->partials.alloc(3UL * std::max<long>(MAX_PARTIALS, hop_blocks(op->g.Vh)) * sizeof(double)));
    HIPCHK(ctx, op->scal.alloc(sizeof(Scal)));
    HIPCHK(ctx, op->dres.alloc(64 * sizeof(double)));
    HIPCHK(ctx, op->hist.alloc(((size_t)maxiter + 2) * sizeof(double)));
    op->kr_prec = kprec;
    for (size_t i = 0; i < before.size(); i++)
        if (all[i]->p != before[i]) {
            op->ws_gen++;
            op->drop_graphs();
            break;
        }
    return QCDW_OK;
}

}  // namespace

extern "C" qcdw_status qcdw_invert(qcdw_op* op, const void* b, void* x, const qcdw_solver_params* params,
                                   qcdw_solve_info* info)
{
    if (!op) return QCDW_EINVAL;
    qcdw_ctx* ctx = op->ctx;
    DeviceGuard dg(ctx->device);
    const auto t_start = std::chrono::steady_clock::now();
    qcdw_solver_params prm;
    if (params) prm = *params;
    else qcdw_solver_params_default(&prm);
    qcdw_solve_info dummy{};
    qcdw_solve_info* inf = info ? info : &dummy;
    double* user_hist = inf->res_hist;
    const int user_hist_len = inf->hist_len;
    *inf = qcdw_solve_info{};
    inf->res_hist = user_hist;
    inf->hist_len = user_hist_len;
    inf->status = QCDW_EINVAL;
    CHK(check_dev(ctx, b, "b"));
    CHK(check_dev(ctx, x, "x"));
    if (b == x) return fail(ctx, QCDW_EINVAL, "x must not alias b");
    if (!(prm.tol > 0.0) || !std::isfinite(prm.tol)) return fail(ctx, QCDW_EINVAL, "tol must be positive");
    if (prm.maxiter < 0) return fail(ctx, QCDW_EINVAL, "maxiter must be >= 0");
    if (prm.check_every < 1) prm.check_every = 1;
    const int kprec = (int)prm.inner;
    if (kprec != F64 && kprec != op->inner)
        return fail(ctx, QCDW_EINVAL, "inner precision %d not prepared by this operator (has %d)", kprec, op->inner);
    if (kprec != F64 && !(prm.delta > 0.0 && prm.delta < 1.0))
        return fail(ctx, QCDW_EINVAL, "delta must lie in (0, 1)");
    CHK(ensure_workspace(op, kprec, prm.maxiter));

    Solver S{op, ctx, ctx->stream, 12L * op->g.Vh, hop_blocks(op->g.Vh), blas_blocks(12L * op->g.Vh)};
    S.tm.on = prm.collect_timing != 0;
    const bool use_graph = prm.use_graph != 0 && !S.tm.on;  // per-launch timing needs eager launches
    hipStream_t s = ctx->stream;
    const Geom& g = op->g;
    const long n = S.n;
    const PrecView v64 = view(op, F64);
    Scal* dS = (Scal*)op->scal.p;
    double* dhist = (double*)op->hist.p;
    double* dpart = (double*)op->partials.p;
    double* dres = (double*)op->dres.p;
    std::vector<double> hist_host;
    hist_host.reserve(64);

    // ---- source preparation (FP64) --------------------------------------
    HIPCHK(ctx, launch_pack_spinor(s, F64, g, b, 0, op->be.p, 1.0));
    HIPCHK(ctx, launch_pack_spinor(s, F64, g, b, 1, op->bo.p, 1.0));
    double bn2e, bn2o;
    HIPCHK(ctx, launch_norm2(s, F64, op->be.p, n, dpart, dres));
    CHK(read_double(ctx, dres, bn2e));
    HIPCHK(ctx, launch_norm2(s, F64, op->bo.p, n, dpart, dres));
    CHK(read_double(ctx, dres, bn2o));
    const double bnorm = std::sqrt(bn2e + bn2o);
    if (!std::isfinite(bnorm)) {
        inf->status = QCDW_ENAN;
        inf->true_res = NAN;
        return fail(ctx, QCDW_ENAN, "source contains NaN or Inf");
    }
    if (bnorm == 0.0) {
        HIPCHK(ctx, hipMemsetAsync(x, 0, 2 * n * 16, s));
        HIPCHK(ctx, hipStreamSynchronize(s));
        inf->status = QCDW_OK;
        return QCDW_OK;
    }
    // y_o = A_oo^-1 b_o ; y_e = A_ee^-1 b_e ; bhat = y_e + kappa A_ee^-1 H_eo y_o
    HIPCHK(ctx, launch_clov_apply_internal(s, F64, g, v64.Ainv[1], op->bo.p, op->yo.p));
    HIPCHK(ctx, launch_clov_apply_internal(s, F64, g, v64.Ainv[0], op->be.p, op->ye.p));
    {
        HopArgs a = hop_args(g, 0);
        a.psi = op->yo.p;
        a.out = op->bhat.p;
        a.gauge = v64.gauge;
        a.clov = v64.Ainv[0];
        a.y = op->ye.p;
        a.a = -op->kappa;
        HIPCHK(ctx, launch_hop(s, F64, v64.recon, EPI_CLOV_XPAY, RED_NONE, a));
    }
    HIPCHK(ctx, launch_pack_spinor(s, F64, g, x, 0, op->xhi.p, 1.0));  // initial guess (even sites)

    // ---- outer loop: Krylov cycles with FP64 residual recomputation -----
    double target = 0.5 * prm.tol * bnorm;  // on ||bhat - M_hat x_e||
    double rr_hi;
    CHK(S.true_schur_residual(rr_hi));
    hist_host.push_back(std::sqrt(rr_hi) / bnorm);
    int iters = 0, restarts = 0, reliable = 0, fault = prm.fault_inject;
    qcdw_status status = QCDW_ENOCONV;
    double true_res = NAN;
    const int maxiter = prm.maxiter;

    while (true) {
        if (!std::isfinite(rr_hi)) {
            status = QCDW_ENAN;
            break;
        }
        if (std::sqrt(rr_hi) <= target) {
            // reconstruct and check the full-lattice residual
            HopArgs a = hop_args(g, 1);  // x_o = y_o + kappa A_oo^-1 H_oe x_e
            a.psi = op->xhi.p;
            a.out = op->tmpo64.p;
            a.gauge = v64.gauge;
            a.clov = v64.Ainv[1];
            a.y = op->yo.p;
            a.a = -op->kappa;
            HIPCHK(ctx, launch_hop(s, F64, v64.recon, EPI_CLOV_XPAY, RED_NONE, a));
            double r2 = 0;
            for (int p = 0; p < 2; p++) {
                HopArgs m = hop_args(g, p);  // (M x)_p = A_pp x_p - kappa H x_{1-p}
                m.psi = p == 0 ? op->tmpo64.p : op->xhi.p;
                m.out = op->tmp64.p;
                m.gauge = v64.gauge;
                m.clov = op->A64[p].p;
                m.y = p == 0 ? op->xhi.p : op->tmpo64.p;
                m.a = op->kappa;
                HIPCHK(ctx, launch_hop(s, F64, v64.recon, EPI_XPAY_CLOVY, RED_NONE, m));
                double rp;
                HIPCHK(ctx, launch_xmy_norm2(s, F64, F64, p == 0 ? op->be.p : op->bo.p, op->tmp64.p, nullptr, n,
                                             dpart, dres));
                CHK(read_double(ctx, dres, rp));
                r2 += rp;
            }
            true_res = std::sqrt(r2) / bnorm;
            if (true_res <= prm.tol) {
                status = QCDW_OK;
                break;
            }
            // tighten the Schur target and keep iterating
            target *= 0.5 * prm.tol / true_res;
            if (iters >= maxiter) break;
        }
        if (iters >= maxiter) break;

        // --- one Krylov cycle on M_hat c = rhi --------------------------
        const bool mixed = kprec != F64;
        const double rhi_norm = std::sqrt(rr_hi);
        const double scale = mixed ? std::sqrt((double)n) / rhi_norm : 1.0;
        void *r = op->kr[0].p, *r0 = op->kr[1].p, *p = op->kr[2].p;
        void* xk = mixed ? op->xlo.p : op->xhi.p;
        const int xprec = mixed ? F32 : F64;
        HIPCHK(ctx, launch_convert(s, F64, kprec, op->rhi.p, r, n, scale));
        HIPCHK(ctx, launch_convert(s, kprec, kprec, r, r0, n, 1.0));
        HIPCHK(ctx, launch_convert(s, kprec, kprec, r, p, n, 1.0));
        if (mixed) HIPCHK(ctx, hipMemsetAsync(op->xlo.p, 0, n * 8, s));
        HIPCHK(ctx, launch_norm2(s, kprec, r, n, dpart, dres));
        Scal* hs = ctx->host_scal;
        memset(hs, 0, sizeof(Scal));
        double cycle_stop = target * scale;
        if (mixed) cycle_stop = std::max(cycle_stop, prm.delta * std::sqrt((double)n));
        hs->stop_rr = cycle_stop * cycle_stop;
        hs->hist_norm = 1.0 / (scale * bnorm);
        hs->iter = iters;
        hs->fault_iter = fault;
        hs->hist_len = maxiter + 2;
        HIPCHK(ctx, hipMemcpyAsync(dS, hs, sizeof(Scal), hipMemcpyHostToDevice, s));
        HIPCHK(ctx, launch_bicg_init(s, dS, dres));
        int flags = 0;
        while (true) {
            const int chunk = std::min(prm.check_every, maxiter - iters);
            if (chunk <= 0) break;
            CHK(S.run_chunk(chunk, kprec, xprec, xk, use_graph));
            HIPCHK(ctx, hipMemcpyAsync(hs, dS, sizeof(Scal), hipMemcpyDeviceToHost, s));
            HIPCHK(ctx, hipStreamSynchronize(s));
            const int done_now = hs->iter - iters;
            if (S.tm.on) S.tm.collect((size_t)4 * done_now);
            if (done_now > 0) {
                std::vector<double> h(done_now);
                HIPCHK(ctx, hipMemcpy(h.data(), dhist + iters + 1, done_now * sizeof(double), hipMemcpyDeviceToHost));
                hist_host.insert(hist_host.end(), h.begin(), h.end());
            }
            iters = hs->iter;
            flags = hs->flags;
            if (flags) break;
        }
        inf->iter_res = std::sqrt(hs->rr) / (scale * bnorm);
        if (mixed) HIPCHK(ctx, launch_axpy_hi(s, F32, 1.0 / scale, op->xlo.p, op->xhi.p, n));
        if (flags & FLAG_NAN) {
            status = QCDW_ENAN;
            break;
        }
        if (flags & FLAG_BREAK) {
            fault = 0;
            if (++restarts > prm.max_restarts) {
                status = QCDW_EBREAKDOWN;
                CHK(S.true_schur_residual(rr_hi));
                break;
            }
        }
        CHK(S.true_schur_residual(rr_hi));
        reliable++;
    }

    // ---- write x (even sites from xhi, odd sites reconstructed) -----------
    if (status == QCDW_OK || status == QCDW_ENOCONV || status == QCDW_EBREAKDOWN) {
        if (status != QCDW_OK) {
            HopArgs a = hop_args(g, 1);
            a.psi = op->xhi.p;
            a.out = op->tmpo64.p;
            a.gauge = v64.gauge;
            a.clov = v64.Ainv[1];
            a.y = op->yo.p;
            a.a = -op->kappa;
            HIPCHK(ctx, launch_hop(s, F64, v64.recon, EPI_CLOV_XPAY, RED_NONE, a));
            double r2 = 0;
            for (int p = 0; p < 2; p++) {
                HopArgs m = hop_args(g, p);
                m.psi = p == 0 ? op->tmpo64.p : op->xhi.p;
                m.out = op->tmp64.p;
                m.gauge = v64.gauge;
                m.clov = op->A64[p].p;
                m.y = p == 0 ? op->xhi.p : op->tmpo64.p;
                m.a = op->kappa;
                HIPCHK(ctx, launch_hop(s, F64, v64.recon, EPI_XPAY_CLOVY, RED_NONE, m));
                double rp;
                HIPCHK(ctx, launch_xmy_norm2(s, F64, F64, p == 0 ? op->be.p : op->bo.p, op->tmp64.p, nullptr, n,
                                             dpart, dres));
                CHK(read_double(ctx, dres, rp));
                r2 += rp;
            }
            true_res = std::sqrt(r2) / bnorm;
        }
        HIPCHK(ctx, launch_unpack_spinor(s, F64, g, op->xhi.p, 0, x, 1.0));
        HIPCHK(ctx, launch_unpack_spinor(s, F64, g, op->tmpo64.p, 1, x, 1.0));
    }
    HIPCHK(ctx, hipStreamSynchronize(s));

    inf->status = status;
    inf->iters = iters;
    inf->n_reliable = reliable;
    inf->n_restarts = restarts;
    inf->true_res = true_res;
    for (int k = 0; k < 3; k++) {
        inf->hop_ms[k] = S.tm.ms[k];
        inf->n_hop[k] = (int32_t)S.tm.launches[k];
    }
    if (user_hist && user_hist_len > 0) {
        const int m = std::min<int>(user_hist_len, (int)hist_host.size());
        memcpy(user_hist, hist_host.data(), m * sizeof(double));
        inf->hist_count = m;
    }
    inf->time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    if (status != QCDW_OK) {
        const char* what = status == QCDW_ENOCONV   ? "did not converge within maxiter"
                           : status == QCDW_ENAN    ? "NaN or Inf in the iteration"
                           : status == QCDW_EBREAKDOWN ? "BiCGStab breakdown persisted after restarts"
                                                    : "solver failed";
        return fail(ctx, status, "%s (iters %d, true residual %.3e)", what, iters, true_res);
    }
    return QCDW_OK;
}

extern "C" qcdw_status qcdw_invert_multi(qcdw_op* op, int nrhs, const void* b, void* x,
                                         const qcdw_solver_params* params, qcdw_solve_info* info)
{
    if (!op) return QCDW_EINVAL;
    if (nrhs < 1 || !info) return fail(op->ctx, QCDW_EINVAL, "nrhs must be >= 1 and info non-NULL");
    const size_t fb = 24UL * op->g.Vh * 16;  // bytes of one full fermion field
    qcdw_status worst = QCDW_OK;
    for (int k = 0; k < nrhs; k++) {
        qcdw_status st = qcdw_invert(op, (const char*)b + k * fb, (char*)x + k * fb, params, info + k);
        if (st != QCDW_OK && worst == QCDW_OK) worst = st;
    }
    return worst;
}
