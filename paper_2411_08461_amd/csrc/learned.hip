// Host side of the learned gauge-covariant preconditioner and of flexible
// GMRES: the network object, forward / gradient / Adam training on the device,
// and FGMRES(m) on the even-odd system with a BiCGStab fallback.
#include <complex>
#include <numeric>
#include <random>

#include "host.h"

struct qcdw_net {
    qcdw_op* op = nullptr;
    qcdw_ctx* ctx = nullptr;
    int hidden = 12;
    long nw1 = 0, nw2 = 0;            // complex weights per layer
    PoolBuf gauge32;                   // FP32 reconstruct-12 links
    PoolBuf W1, W2, Wt;                // FP32 complex weights and the adjoint-layer scratch
    PoolBuf W1bf, W2bf;                // weights rounded to BF16 values (application)
    PoolBuf G1, G2, m1, v1, m2, v2;    // FP64 gradients and Adam moments
    PoolBuf act0, hid, z, gz, gh;      // activations [parity][channel][Vh][3] complex
    PoolBuf hid16;                     // BF16 hidden activations (application)
    PoolBuf diff, tmp64, partials, res;
    int adam_step = 0;
    bool bf_dirty = true;
    int mfma = 0;  // BF16 application layers on the matrix cores: bit 0 the first, bit 1 the second (timed)
};

namespace {

using cdbl = std::complex<double>;

qcdw_status net_ensure(qcdw_net* net)
{
    qcdw_ctx* ctx = net->ctx;
    const long Vh = net->op->g.Vh;
    const int h = net->hidden;
    HIPCHK(ctx, net->act0.alloc(2L * 4 * Vh * 3 * 8));
    HIPCHK(ctx, net->z.alloc(2L * 4 * Vh * 3 * 8));
    HIPCHK(ctx, net->gz.alloc(2L * 4 * Vh * 3 * 8));
    HIPCHK(ctx, net->hid.alloc(2L * h * Vh * 3 * 8));
    HIPCHK(ctx, net->gh.alloc(2L * h * Vh * 3 * 8));
    HIPCHK(ctx, net->hid16.alloc(2L * h * Vh * 3 * 4));
    HIPCHK(ctx, net->diff.alloc(12L * Vh * 16));
    HIPCHK(ctx, net->tmp64.alloc(12L * Vh * 16));
    const long nb = (2L * Vh + 255) / 256;
    HIPCHK(ctx, net->partials.alloc((size_t)std::max<long>(nb * 2 * 4 * h, 3 * 4096) * sizeof(double)));
    HIPCHK(ctx, net->res.alloc(64 * sizeof(double)));
    return QCDW_OK;
}

// weights rounded to BF16-representable FP32 values for the application path
qcdw_status net_refresh_bf16(qcdw_net* net)
{
    if (!net->bf_dirty) return QCDW_OK;
    qcdw_ctx* ctx = net->ctx;
    hipStream_t s = ctx->stream;
    HIPCHK(ctx, launch_convert(s, F32, BF16, net->W1.p, net->Wt.p, net->nw1, 1.0));
    HIPCHK(ctx, launch_convert(s, BF16, F32, net->Wt.p, net->W1bf.p, net->nw1, 1.0));
    HIPCHK(ctx, launch_convert(s, F32, BF16, net->W2.p, net->Wt.p, net->nw2, 1.0));
    HIPCHK(ctx, launch_convert(s, BF16, F32, net->Wt.p, net->W2bf.p, net->nw2, 1.0));
    net->bf_dirty = false;
    return QCDW_OK;
}

// out (internal FP64 even field) = P(in) (internal FP64 even field)
qcdw_status net_forward_internal(qcdw_net* net, int prec, const void* in_int, void* out_int)
{
    qcdw_ctx* ctx = net->ctx;
    hipStream_t s = ctx->stream;
    const Geom& g = net->op->g;
    const long n = 12L * g.Vh;
    const int h = net->hidden;
    HIPCHK(ctx, launch_convert(s, F64, F32, in_int, net->act0.p, n, 1.0));
    HIPCHK(ctx, hipMemsetAsync((char*)net->act0.p + n * 8, 0, n * 8, s));
    if (prec == BF16) {
        CHK(net_refresh_bf16(net));
        HIPCHK(ctx, launch_net_layer(s, F32, BF16, 4, h, net->act0.p, net->hid16.p, net->gauge32.p, net->W1bf.p, g,
                                     net->mfma & 1));
        HIPCHK(ctx, launch_net_layer(s, BF16, F32, h, 4, net->hid16.p, net->z.p, net->gauge32.p, net->W2bf.p, g,
                                     (net->mfma >> 1) & 1));
    } else {
        HIPCHK(ctx, launch_net_layer(s, F32, F32, 4, h, net->act0.p, net->hid.p, net->gauge32.p, net->W1.p, g));
        HIPCHK(ctx, launch_net_layer(s, F32, F32, h, 4, net->hid.p, net->z.p, net->gauge32.p, net->W2.p, g));
    }
    HIPCHK(ctx, launch_convert(s, F32, F64, net->z.p, out_int, n, 1.0));
    return QCDW_OK;
}

// Layer kernels of the BF16 application: each layer's channel mixing on the matrix cores or on vector FMA,
// whichever pair is fastest on this lattice (timed on zero fields; cached per lattice and width on the
// context and in the tuning file as "net_mfma/h<hidden>/L<Lx>x<Ly>x<Lz>x<Lt> m", bit 0 of m the first
// layer on the matrix cores, bit 1 the second).
qcdw_status net_tune_layers(qcdw_net* net)
{
    qcdw_ctx* ctx = net->ctx;
    const Geom& g = net->op->g;
    char key[96];
    snprintf(key, sizeof key, "net_mfma/h%d/L%dx%dx%dx%d", net->hidden, g.Lx, g.Ly, g.Lz, g.Lt);
    auto it = ctx->tune.find(key);
    if (it != ctx->tune.end() && it->second >= 0 && it->second <= 3) {
        net->mfma = it->second;
        return QCDW_OK;
    }
    hipStream_t s = ctx->stream;
    const long n = 12L * g.Vh;
    HIPCHK(ctx, hipMemsetAsync(net->tmp64.p, 0, n * 16, s));
    hipEvent_t e0, e1;
    HIPCHK(ctx, hipEventCreate(&e0));
    HIPCHK(ctx, hipEventCreate(&e1));
    float best = 1e30f;
    int best_m = 0;
    qcdw_status st = QCDW_OK;
    for (int m : {0, 1, 2, 3}) {
        net->mfma = m;
        st = net_forward_internal(net, BF16, net->tmp64.p, net->diff.p);  // warm-up
        hipError_t e = hipEventRecord(e0, s);
        for (int rep = 0; rep < 3 && st == QCDW_OK && e == hipSuccess; rep++)
            st = net_forward_internal(net, BF16, net->tmp64.p, net->diff.p);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (st == QCDW_OK && e != hipSuccess) st = fail(ctx, QCDW_EHIP, "net tuning failed: %s", hipGetErrorString(e));
        if (st != QCDW_OK) break;
        if (ms < best) {
            best = ms;
            best_m = m;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != QCDW_OK) return st;
    net->mfma = best_m;
    ctx->tune_store(key, best_m);
    return QCDW_OK;
}

// one training pair: loss_k = ||P(r) - e||^2 / ||e||^2, gradients accumulated into G1, G2
qcdw_status net_pair_grad(qcdw_net* net, const void* r_e, const void* e_e, double& loss)
{
    qcdw_ctx* ctx = net->ctx;
    hipStream_t s = ctx->stream;
    const Geom& g = net->op->g;
    const long n = 12L * g.Vh;
    const int h = net->hidden;
    double* part = (double*)net->partials.p;
    double* res = (double*)net->res.p;
    // forward in FP32, the input embedded on even sites
    HIPCHK(ctx, launch_pack_spinor(s, F32, g, r_e, 0, net->act0.p, 1.0));
    HIPCHK(ctx, hipMemsetAsync((char*)net->act0.p + n * 8, 0, n * 8, s));
    HIPCHK(ctx, launch_net_layer(s, F32, F32, 4, h, net->act0.p, net->hid.p, net->gauge32.p, net->W1.p, g));
    HIPCHK(ctx, launch_net_layer(s, F32, F32, h, 4, net->hid.p, net->z.p, net->gauge32.p, net->W2.p, g));
    // diff = P(r) - e on even sites
    HIPCHK(ctx, launch_pack_spinor(s, F64, g, e_e, 0, net->tmp64.p, 1.0));
    HIPCHK(ctx, launch_norm2(s, F64, net->tmp64.p, n, part, res));
    HIPCHK(ctx, launch_xmy_norm2(s, F32, F64, net->z.p, net->tmp64.p, net->diff.p, n, part, res + 1));
    HIPCHK(ctx, hipMemcpyAsync(ctx->host_d, res, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    const double en = ctx->host_d[0], dn = ctx->host_d[1];
    if (!(en > 0.0)) return fail(ctx, QCDW_EINVAL, "training pair with a zero error field");
    loss = dn / en;
    // gz = 2 (P(r) - e) / ||e||^2 on even sites, 0 on odd sites
    HIPCHK(ctx, launch_net_make_gz(s, net->diff.p, net->gz.p, n, 2.0 / en));
    for (int a = 0; a < 9; a++)
        HIPCHK(ctx, launch_net_wgrad(s, h, 4, net->hid.p, net->gz.p, net->gauge32.p, g, a, part,
                                     (double*)net->G2.p + (long)a * 2 * 4 * h, 1));
    // gh = adjoint of layer 2 applied to gz
    HIPCHK(ctx, launch_net_adjoint_w(s, net->W2.p, net->Wt.p, 4, h));
    HIPCHK(ctx, launch_net_layer(s, F32, F32, 4, h, net->gz.p, net->gh.p, net->gauge32.p, net->Wt.p, g));
    for (int a = 0; a < 9; a++)
        HIPCHK(ctx, launch_net_wgrad(s, 4, h, net->act0.p, net->gh.p, net->gauge32.p, g, a, part,
                                     (double*)net->G1.p + (long)a * 2 * 4 * h, 1));
    return QCDW_OK;
}

}  // namespace

extern "C" qcdw_status qcdw_net_create(qcdw_op* op, int hidden, uint64_t seed, double init_scale, qcdw_net** out)
{
    if (!op) return QCDW_EINVAL;
    qcdw_ctx* ctx = op->ctx;
    DeviceGuard dg(ctx->device);
    if (!out) return fail(ctx, QCDW_EINVAL, "net pointer is NULL");
    *out = nullptr;
    if (hidden != 4 && hidden != 12) return fail(ctx, QCDW_EINVAL, "hidden channels must be 4 or 12");
    if (op->recon != 12) return fail(ctx, QCDW_EINVAL, "the net needs a reconstruct-12 operator");
    qcdw_net* net = new qcdw_net;
    net->op = op;
    net->ctx = ctx;
    net->hidden = hidden;
    net->nw1 = 9L * hidden * 4;
    net->nw2 = 9L * 4 * hidden;
    auto bail = [&](qcdw_status st) {
        delete net;
        return st;
    };
    hipStream_t s = ctx->stream;
    const long nl = 8L * op->g.Vh * 6;
    if (net->gauge32.alloc(nl * 8) != hipSuccess || net->W1.alloc(net->nw1 * 8) != hipSuccess ||
        net->W2.alloc(net->nw2 * 8) != hipSuccess || net->Wt.alloc(std::max(net->nw1, net->nw2) * 8) != hipSuccess ||
        net->W1bf.alloc(net->nw1 * 8) != hipSuccess || net->W2bf.alloc(net->nw2 * 8) != hipSuccess ||
        net->G1.alloc(net->nw1 * 16) != hipSuccess || net->G2.alloc(net->nw2 * 16) != hipSuccess ||
        net->m1.alloc(net->nw1 * 16) != hipSuccess || net->v1.alloc(net->nw1 * 16) != hipSuccess ||
        net->m2.alloc(net->nw2 * 16) != hipSuccess || net->v2.alloc(net->nw2 * 16) != hipSuccess)
        return bail(fail(ctx, QCDW_ENOMEM, "out of device memory creating the net"));
    if (net_ensure(net) != QCDW_OK) return bail(QCDW_ENOMEM);
    // links: the operator's FP64 reconstruct-12 pack converted to FP32 (same layout)
    if (launch_convert(s, F64, F32, op->gauge64.p, net->gauge32.p, nl, 1.0) != hipSuccess)
        return bail(fail(ctx, QCDW_EHIP, "link conversion failed"));
    // initial weights: the identity map through the hidden layer plus seeded Gaussian noise
    std::mt19937_64 rng(seed);
    std::normal_distribution<double> nd(0.0, 1.0);
    std::vector<float> w1(2 * net->nw1), w2(2 * net->nw2);
    for (auto& v : w1) v = (float)(init_scale * nd(rng));
    for (auto& v : w2) v = (float)(init_scale * nd(rng));
    for (int c = 0; c < 4; c++) {
        w1[2 * (c * 4 + c)] += 1.0f;       // W1[0][c][c]
        w2[2 * (c * hidden + c)] += 1.0f;  // W2[0][c][c]
    }
    if (hipMemcpy(net->W1.p, w1.data(), w1.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(net->W2.p, w2.data(), w2.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(net->m1.p, 0, net->nw1 * 16) != hipSuccess || hipMemset(net->v1.p, 0, net->nw1 * 16) != hipSuccess ||
        hipMemset(net->m2.p, 0, net->nw2 * 16) != hipSuccess || hipMemset(net->v2.p, 0, net->nw2 * 16) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return bail(fail(ctx, QCDW_EHIP, "net initialisation failed"));
    const qcdw_status st = net_tune_layers(net);
    if (st != QCDW_OK) return bail(st);
    *out = net;
    return QCDW_OK;
}

extern "C" void qcdw_net_destroy(qcdw_net* net)
{
    if (!net) return;
    DeviceGuard dg(net->ctx->device);
    (void)hipStreamSynchronize(net->ctx->stream);
    delete net;
}

extern "C" qcdw_status qcdw_net_bind(qcdw_net* net, qcdw_op* op)
{
    if (!net || !op) return QCDW_EINVAL;
    qcdw_ctx* ctx = net->ctx;
    DeviceGuard dg(ctx->device);
    if (op->ctx != ctx) return fail(ctx, QCDW_EINVAL, "the operator belongs to another context");
    if (op->recon != 12) return fail(ctx, QCDW_EINVAL, "the net needs a reconstruct-12 operator");
    const Geom &a = op->g, &b = net->op->g;
    if (a.Lx != b.Lx || a.Ly != b.Ly || a.Lz != b.Lz || a.Lt != b.Lt)
        return fail(ctx, QCDW_EINVAL, "the operator's lattice differs from the net's");
    const long nl = 8L * op->g.Vh * 6;
    HIPCHK(ctx, launch_convert(ctx->stream, F64, F32, op->gauge64.p, net->gauge32.p, nl, 1.0));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    net->op = op;
    return QCDW_OK;
}

extern "C" qcdw_status qcdw_net_get_weights(qcdw_net* net, double* w1, double* w2)
{
    if (!net) return QCDW_EINVAL;
    qcdw_ctx* ctx = net->ctx;
    DeviceGuard dg(ctx->device);
    if (!w1 || !w2) return fail(ctx, QCDW_EINVAL, "weight arrays must not be NULL");
    std::vector<float> a(2 * net->nw1), b(2 * net->nw2);
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    HIPCHK(ctx, hipMemcpy(a.data(), net->W1.p, a.size() * 4, hipMemcpyDeviceToHost));
    HIPCHK(ctx, hipMemcpy(b.data(), net->W2.p, b.size() * 4, hipMemcpyDeviceToHost));
    for (size_t i = 0; i < a.size(); i++) w1[i] = a[i];
    for (size_t i = 0; i < b.size(); i++) w2[i] = b[i];
    return QCDW_OK;
}

extern "C" qcdw_status qcdw_net_set_weights(qcdw_net* net, const double* w1, const double* w2)
{
    if (!net) return QCDW_EINVAL;
    qcdw_ctx* ctx = net->ctx;
    DeviceGuard dg(ctx->device);
    if (!w1 || !w2) return fail(ctx, QCDW_EINVAL, "weight arrays must not be NULL");
    std::vector<float> a(2 * net->nw1), b(2 * net->nw2);
    for (size_t i = 0; i < a.size(); i++) a[i] = (float)w1[i];
    for (size_t i = 0; i < b.size(); i++) b[i] = (float)w2[i];
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    HIPCHK(ctx, hipMemcpy(net->W1.p, a.data(), a.size() * 4, hipMemcpyHostToDevice));
    HIPCHK(ctx, hipMemcpy(net->W2.p, b.data(), b.size() * 4, hipMemcpyHostToDevice));
    net->bf_dirty = true;
    return QCDW_OK;
}

extern "C" qcdw_status qcdw_net_apply(qcdw_net* net, qcdw_prec prec, const void* in_e, void* out_e)
{
    if (!net) return QCDW_EINVAL;
    qcdw_ctx* ctx = net->ctx;
    DeviceGuard dg(ctx->device);
    CHK(check_dev(ctx, in_e, "in_e"));
    CHK(check_dev(ctx, out_e, "out_e"));
    if (prec != QCDW_F32 && prec != QCDW_BF16) return fail(ctx, QCDW_EINVAL, "prec must be F32 or BF16");
    const Geom& g = net->op->g;
    hipStream_t s = ctx->stream;
    HIPCHK(ctx, launch_pack_spinor(s, F64, g, in_e, 0, net->tmp64.p, 1.0));
    CHK(net_forward_internal(net, prec, net->tmp64.p, net->diff.p));
    HIPCHK(ctx, launch_unpack_spinor(s, F64, g, net->diff.p, 0, out_e, 1.0));
    HIPCHK(ctx, hipStreamSynchronize(s));
    return QCDW_OK;
}

extern "C" qcdw_status qcdw_net_loss_grad(qcdw_net* net, int npairs, const void* const r_e[],
                                          const void* const e_e[], double* loss, double* g1, double* g2)
{
    if (!net) return QCDW_EINVAL;
    qcdw_ctx* ctx = net->ctx;
    DeviceGuard dg(ctx->device);
    if (npairs < 1 || !r_e || !e_e || !loss || !g1 || !g2) return fail(ctx, QCDW_EINVAL, "bad arguments");
    for (int k = 0; k < npairs; k++) {
        CHK(check_dev(ctx, r_e[k], "r_e"));
        CHK(check_dev(ctx, e_e[k], "e_e"));
    }
    hipStream_t s = ctx->stream;
    HIPCHK(ctx, hipMemsetAsync(net->G1.p, 0, net->nw1 * 16, s));
    HIPCHK(ctx, hipMemsetAsync(net->G2.p, 0, net->nw2 * 16, s));
    double L = 0;
    for (int k = 0; k < npairs; k++) {
        double lk;
        CHK(net_pair_grad(net, r_e[k], e_e[k], lk));
        L += lk;
    }
    HIPCHK(ctx, hipStreamSynchronize(s));
    HIPCHK(ctx, hipMemcpy(g1, net->G1.p, net->nw1 * 16, hipMemcpyDeviceToHost));
    HIPCHK(ctx, hipMemcpy(g2, net->G2.p, net->nw2 * 16, hipMemcpyDeviceToHost));
    *loss = L;
    return QCDW_OK;
}

extern "C" qcdw_status qcdw_net_train(qcdw_net* net, int npairs, const void* const r_e[], const void* const e_e[],
                                      int steps, int batch, double lr, uint64_t seed, double* loss_hist)
{
    if (!net) return QCDW_EINVAL;
    qcdw_ctx* ctx = net->ctx;
    DeviceGuard dg(ctx->device);
    if (npairs < 1 || !r_e || !e_e || steps < 0 || batch < 1 || !(lr > 0))
        return fail(ctx, QCDW_EINVAL, "bad training arguments");
    for (int k = 0; k < npairs; k++) {
        CHK(check_dev(ctx, r_e[k], "r_e"));
        CHK(check_dev(ctx, e_e[k], "e_e"));
    }
    hipStream_t s = ctx->stream;
    std::mt19937_64 rng(seed);
    std::vector<int> order(npairs);
    std::iota(order.begin(), order.end(), 0);
    std::shuffle(order.begin(), order.end(), rng);
    int pos = 0;
    for (int step = 0; step < steps; step++) {
        HIPCHK(ctx, hipMemsetAsync(net->G1.p, 0, net->nw1 * 16, s));
        HIPCHK(ctx, hipMemsetAsync(net->G2.p, 0, net->nw2 * 16, s));
        double L = 0;
        for (int b = 0; b < batch; b++) {
            if (pos == npairs) {
                std::shuffle(order.begin(), order.end(), rng);
                pos = 0;
            }
            const int k = order[pos++];
            double lk;
            CHK(net_pair_grad(net, r_e[k], e_e[k], lk));
            L += lk;
        }
        net->adam_step++;
        HIPCHK(ctx, launch_adam(s, net->W1.p, (const double*)net->G1.p, (double*)net->m1.p, (double*)net->v1.p,
                                (int)(2 * net->nw1), lr, 0.9, 0.999, 1e-8, net->adam_step, 1.0 / batch));
        HIPCHK(ctx, launch_adam(s, net->W2.p, (const double*)net->G2.p, (double*)net->m2.p, (double*)net->v2.p,
                                (int)(2 * net->nw2), lr, 0.9, 0.999, 1e-8, net->adam_step, 1.0 / batch));
        if (loss_hist) loss_hist[step] = L / batch;
    }
    net->bf_dirty = true;
    HIPCHK(ctx, hipStreamSynchronize(s));
    return QCDW_OK;
}

extern "C" qcdw_status qcdw_make_training_pairs(qcdw_op* op, const void* b, int npairs, int stride,
                                                void* const r_e[], void* const e_e[], int* made)
{
    if (stride == 0) return QCDW_EINVAL;
    if (stride < 0) {  // random errors: e_k from the seeded generator, r_k = M_hat e_k
        if (!op) return QCDW_EINVAL;
        qcdw_ctx* ctx = op->ctx;
        DeviceGuard dg(ctx->device);
        if (!made || npairs < 1 || !r_e || !e_e) return fail(ctx, QCDW_EINVAL, "bad arguments");
        *made = 0;
        const Geom& g = op->g;
        const long n = 12L * g.Vh;
        hipStream_t s = ctx->stream;
        DevBuf e, r, tmpo, part, res;
        HIPCHK(ctx, e.alloc(n * 16));
        HIPCHK(ctx, r.alloc(n * 16));
        HIPCHK(ctx, tmpo.alloc(n * 16));
        HIPCHK(ctx, part.alloc(4096 * sizeof(double)));
        HIPCHK(ctx, res.alloc(8 * sizeof(double)));
        for (int k = 0; k < npairs; k++) {
            CHK(check_dev(ctx, r_e[k], "r_e"));
            CHK(check_dev(ctx, e_e[k], "e_e"));
            HIPCHK(ctx, launch_gaussian(s, e.p, n, (uint64_t)(-stride), (uint64_t)k));
            HIPCHK(ctx, matpc(s, op, view(op, F64), e.p, r.p, tmpo.p, RED_NONE, nullptr, nullptr, nullptr));
            HIPCHK(ctx, launch_norm2(s, F64, r.p, n, (double*)part.p, (double*)res.p));
            double rn2;
            CHK(read_double(ctx, (double*)res.p, rn2));
            const double sc = 1.0 / std::sqrt(rn2);
            HIPCHK(ctx, launch_unpack_spinor(s, F64, g, r.p, 0, r_e[k], sc));
            HIPCHK(ctx, launch_unpack_spinor(s, F64, g, e.p, 0, e_e[k], sc));
            *made = k + 1;
        }
        HIPCHK(ctx, hipStreamSynchronize(s));
        return QCDW_OK;
    }
    if (!op) return QCDW_EINVAL;
    qcdw_ctx* ctx = op->ctx;
    DeviceGuard dg(ctx->device);
    if (!made || npairs < 1 || stride < 1 || !r_e || !e_e) return fail(ctx, QCDW_EINVAL, "bad arguments");
    *made = 0;
    CHK(check_dev(ctx, b, "b"));
    for (int k = 0; k < npairs; k++) {
        CHK(check_dev(ctx, r_e[k], "r_e"));
        CHK(check_dev(ctx, e_e[k], "e_e"));
    }
    const Geom& g = op->g;
    const long n = 12L * g.Vh;
    hipStream_t s = ctx->stream;
    DevBuf xs, xk, a, c, e, r, tmpo, part, res;
    HIPCHK(ctx, xs.alloc(2 * n * 16));
    HIPCHK(ctx, xk.alloc(2 * n * 16));
    HIPCHK(ctx, a.alloc(n * 16));
    HIPCHK(ctx, c.alloc(n * 16));
    HIPCHK(ctx, e.alloc(n * 16));
    HIPCHK(ctx, r.alloc(n * 16));
    HIPCHK(ctx, tmpo.alloc(n * 16));
    HIPCHK(ctx, part.alloc(4096 * sizeof(double)));
    HIPCHK(ctx, res.alloc(8 * sizeof(double)));
    qcdw_solver_params prm;
    qcdw_solver_params_default(&prm);
    prm.tol = 1e-12;
    prm.maxiter = 100000;
    qcdw_solve_info info{};
    HIPCHK(ctx, hipMemsetAsync(xs.p, 0, 2 * n * 16, s));
    const qcdw_status st = qcdw_invert(op, b, xs.p, &prm, &info);
    if (st != QCDW_OK) return st;
    HIPCHK(ctx, hipMemsetAsync(xk.p, 0, 2 * n * 16, s));
    HIPCHK(ctx, launch_pack_spinor(s, F64, g, xs.p, 0, a.p, 1.0));
    prm.maxiter = stride;
    for (int k = 0; k < npairs; k++) {
        qcdw_solve_info ik{};
        const qcdw_status sk = qcdw_invert(op, b, xk.p, &prm, &ik);  // resume from x_{k-1}
        if (sk == QCDW_OK) break;                                    // converged: no error left to learn
        if (sk != QCDW_ENOCONV) return sk;
        HIPCHK(ctx, launch_pack_spinor(s, F64, g, xk.p, 0, c.p, 1.0));
        HIPCHK(ctx, launch_xmy_norm2(s, F64, F64, a.p, c.p, e.p, n, (double*)part.p, (double*)res.p));
        HIPCHK(ctx, matpc(s, op, view(op, F64), e.p, r.p, tmpo.p, RED_NONE, nullptr, nullptr, nullptr));
        HIPCHK(ctx, launch_norm2(s, F64, r.p, n, (double*)part.p, (double*)res.p + 1));
        double rn2;
        CHK(read_double(ctx, (double*)res.p + 1, rn2));
        if (!(rn2 > 0)) break;
        const double sc = 1.0 / std::sqrt(rn2);
        HIPCHK(ctx, launch_unpack_spinor(s, F64, g, r.p, 0, r_e[k], sc));
        HIPCHK(ctx, launch_unpack_spinor(s, F64, g, e.p, 0, e_e[k], sc));
        *made = k + 1;
    }
    HIPCHK(ctx, hipStreamSynchronize(s));
    return QCDW_OK;
}

// ---------------------------------------------------------------------------
// flexible GMRES on the even-odd system
// ---------------------------------------------------------------------------
// FGMRES(m) on the even-odd system with right preconditioning z_j = precond(v_j) (FP64 even-site internal
// fields; nullptr: none), shared by the learned net and the multigrid preconditioner
qcdw_status qcdw_host::fgmres_run(qcdw_op* op, const Precond* precond, const void* b, void* x,
                                  const qcdw_solver_params* params, qcdw_solve_info* info)
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
    if (!(prm.tol > 0.0)) return fail(ctx, QCDW_EINVAL, "tol must be positive");
    const int m = prm.gmres_restart;
    if (m < 1 || m > 64) return fail(ctx, QCDW_EINVAL, "gmres_restart must lie in [1, 64]");
    const Geom& g = op->g;
    const long n = 12L * g.Vh;
    const size_t vb = (size_t)n * 16;
    hipStream_t s = ctx->stream;
    const PrecView v64 = view(op, F64);

    DevBuf be, bo, yo, ye, bhat, xe, xo, r, w, tmp, tmpo, V, Z, part, coef, dres;
    HIPCHK(ctx, be.alloc(vb));
    HIPCHK(ctx, bo.alloc(vb));
    HIPCHK(ctx, yo.alloc(vb));
    HIPCHK(ctx, ye.alloc(vb));
    HIPCHK(ctx, bhat.alloc(vb));
    HIPCHK(ctx, xe.alloc(vb));
    HIPCHK(ctx, xo.alloc(vb));
    HIPCHK(ctx, r.alloc(vb));
    HIPCHK(ctx, w.alloc(vb));
    HIPCHK(ctx, tmp.alloc(vb));
    HIPCHK(ctx, tmpo.alloc(vb));
    HIPCHK(ctx, V.alloc(vb * (m + 1)));
    if (precond) HIPCHK(ctx, Z.alloc(vb * m));
    const int ngroups = (m + 1 + 7) / 8;
    HIPCHK(ctx, part.alloc((size_t)16 * ngroups * blas_blocks(n) * sizeof(double) + 64));
    HIPCHK(ctx, coef.alloc(2 * 65 * sizeof(double)));
    HIPCHK(ctx, dres.alloc(HOST_D_N * sizeof(double)));
    static_assert(HOST_D_N >= 257, "FGMRES stages two Gram-Schmidt columns and a norm");
    double* dpart = (double*)part.p;
    double* dd = (double*)dres.p;
    auto Vk = [&](int k) { return (char*)V.p + (size_t)k * vb; };
    auto Zk = [&](int k) { return precond ? (char*)Z.p + (size_t)k * vb : Vk(k); };
    auto rd = [&](int cnt, double* out) -> qcdw_status {
        HIPCHK(ctx, hipMemcpyAsync(ctx->host_d, dd, cnt * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(ctx, hipStreamSynchronize(s));
        if (out != ctx->host_d) memcpy(out, ctx->host_d, cnt * sizeof(double));
        return QCDW_OK;
    };
    // r = bhat - M_hat xe, returns ||r||
    auto schur_residual = [&](double& rn) -> qcdw_status {
        HIPCHK(ctx, matpc(s, op, v64, xe.p, tmp.p, tmpo.p, RED_NONE, nullptr, nullptr, nullptr));
        HIPCHK(ctx, launch_xmy_norm2(s, F64, F64, bhat.p, tmp.p, r.p, n, dpart, dd));
        double v;
        CHK(rd(1, &v));
        rn = std::sqrt(v);
        return QCDW_OK;
    };
    // x_o from x_e and the FP64 full-lattice relative residual
    auto full_check = [&](double& tr, double bnorm) -> qcdw_status {
        HopArgs a = hop_args(g, 1);
        a.psi = xe.p;
        a.out = xo.p;
        a.gauge = v64.gauge;
        a.clov = v64.Ainv[1];
        a.y = yo.p;
        a.a = -op->kappa;
        HIPCHK(ctx, launch_hop(s, F64, v64.recon, EPI_CLOV_XPAY, RED_NONE, a));
        double r2 = 0;
        for (int p = 0; p < 2; p++) {
            HopArgs mm = hop_args(g, p);
            mm.psi = p == 0 ? xo.p : xe.p;
            mm.out = tmp.p;
            mm.gauge = v64.gauge;
            mm.clov = op->A64[p].p;
            mm.y = p == 0 ? xe.p : xo.p;
            mm.a = op->kappa;
            HIPCHK(ctx, launch_hop(s, F64, v64.recon, EPI_XPAY_CLOVY, RED_NONE, mm));
            HIPCHK(ctx, launch_xmy_norm2(s, F64, F64, p == 0 ? be.p : bo.p, tmp.p, nullptr, n, dpart, dd));
            double v;
            CHK(rd(1, &v));
            r2 += v;
        }
        tr = std::sqrt(r2) / bnorm;
        return QCDW_OK;
    };

    // ---- source preparation ------------------------------------------------
    HIPCHK(ctx, launch_pack_spinor(s, F64, g, b, 0, be.p, 1.0));
    HIPCHK(ctx, launch_pack_spinor(s, F64, g, b, 1, bo.p, 1.0));
    HIPCHK(ctx, launch_pack_spinor(s, F64, g, x, 0, xe.p, 1.0));
    double bn[2];
    HIPCHK(ctx, launch_norm2(s, F64, be.p, n, dpart, dd));
    HIPCHK(ctx, launch_norm2(s, F64, bo.p, n, dpart, dd + 1));
    CHK(rd(2, bn));
    const double bnorm = std::sqrt(bn[0] + bn[1]);
    if (!std::isfinite(bnorm)) {
        inf->status = QCDW_ENAN;
        return fail(ctx, QCDW_ENAN, "source contains NaN or Inf");
    }
    if (bnorm == 0.0) {
        HIPCHK(ctx, hipMemsetAsync(x, 0, 2 * vb, s));
        HIPCHK(ctx, hipStreamSynchronize(s));
        inf->status = QCDW_OK;
        inf->true_res = 0;
        return QCDW_OK;
    }
    HIPCHK(ctx, launch_clov_apply_internal(s, F64, g, v64.Ainv[1], bo.p, yo.p));
    HIPCHK(ctx, launch_clov_apply_internal(s, F64, g, v64.Ainv[0], be.p, ye.p));
    {
        HopArgs a = hop_args(g, 0);
        a.psi = yo.p;
        a.out = bhat.p;
        a.gauge = v64.gauge;
        a.clov = v64.Ainv[0];
        a.y = ye.p;
        a.a = -op->kappa;
        HIPCHK(ctx, launch_hop(s, F64, v64.recon, EPI_CLOV_XPAY, RED_NONE, a));
    }

    // ---- FGMRES(m) ----------------------------------------------------------
    double target = 0.5 * prm.tol * bnorm;
    std::vector<double> hist;
    double rn;
    CHK(schur_residual(rn));
    hist.push_back(rn / bnorm);
    int iters = 0, cycles = 0;
    qcdw_status status = QCDW_ENOCONV;
    double true_res = NAN;
    bool stalled = false;
    std::vector<cdbl> H((size_t)(m + 1) * m), cs(m), sn(m), gv(m + 1);
    auto Hij = [&](int i, int j) -> cdbl& { return H[(size_t)i * m + j]; };
    while (true) {
        if (!std::isfinite(rn)) {
            status = QCDW_ENAN;
            break;
        }
        if (rn <= target) {
            CHK(full_check(true_res, bnorm));
            if (true_res <= prm.tol) {
                status = QCDW_OK;
                break;
            }
            target *= 0.5 * prm.tol / true_res;
        }
        if (iters >= prm.maxiter) break;
        // v0 = r / ||r||
        HIPCHK(ctx, launch_convert(s, F64, F64, r.p, Vk(0), n, 1.0 / rn));
        std::fill(gv.begin(), gv.end(), cdbl(0));
        gv[0] = rn;
        int j = 0;
        for (; j < m && iters < prm.maxiter; j++) {
            // z_j = P(v_j), w = M_hat z_j
            if (precond) CHK((*precond)(Vk(j), Zk(j)));
            HIPCHK(ctx, matpc(s, op, v64, Zk(j), w.p, tmpo.p, RED_NONE, nullptr, nullptr, nullptr));
            // block classical Gram-Schmidt against v_0..v_j, twice; the coefficients stay on the
            // device (dd[0..], dd[128..]), ||w||^2 lands in dd[256] and v_{j+1} = w / ||w|| is
            // formed on the device, so the step needs one host synchronisation
            HIPCHK(ctx, launch_multidot(s, V.p, n, j + 1, w.p, n, dpart, dd));
            HIPCHK(ctx, launch_multiaxpy(s, V.p, n, j + 1, dd, w.p, n, -1.0));
            HIPCHK(ctx, launch_multidot(s, V.p, n, j + 1, w.p, n, dpart, dd + 128));
            HIPCHK(ctx, launch_multiaxpy(s, V.p, n, j + 1, dd + 128, w.p, n, -1.0));
            HIPCHK(ctx, launch_norm2(s, F64, w.p, n, dpart, dd + 256));
            HIPCHK(ctx, launch_scale_inv_norm(s, w.p, Vk(j + 1), n, dd + 256));
            CHK(rd(257, ctx->host_d));
            const double* hc = ctx->host_d;
            const double* hc2 = ctx->host_d + 128;
            const double hn = std::sqrt(ctx->host_d[256]);
            for (int i = 0; i <= j; i++) Hij(i, j) = cdbl(hc[2 * i] + hc2[2 * i], hc[2 * i + 1] + hc2[2 * i + 1]);
            Hij(j + 1, j) = hn;
            // Givens rotations: apply the previous ones, then zero H(j+1, j)
            for (int i = 0; i < j; i++) {
                const cdbl a = Hij(i, j), c = Hij(i + 1, j);
                Hij(i, j) = std::conj(cs[i]) * a + std::conj(sn[i]) * c;
                Hij(i + 1, j) = -sn[i] * a + cs[i] * c;
            }
            const cdbl a = Hij(j, j);
            const double bb = std::abs(Hij(j + 1, j)), na = std::abs(a), den = std::sqrt(na * na + bb * bb);
            if (den == 0.0) {
                cs[j] = 1.0;
                sn[j] = 0.0;
            } else {
                cs[j] = a / den;
                sn[j] = Hij(j + 1, j) / den;
            }
            Hij(j, j) = den;
            Hij(j + 1, j) = 0.0;
            gv[j + 1] = -sn[j] * gv[j];
            gv[j] = std::conj(cs[j]) * gv[j];
            iters++;
            const double est = std::abs(gv[j + 1]);
            hist.push_back(est / bnorm);
            if (est <= target || hn == 0.0 || !std::isfinite(est)) {
                j++;
                break;
            }
        }
        // y = R^-1 g (back substitution), x_e += Z y
        std::vector<cdbl> y(j);
        for (int i = j - 1; i >= 0; i--) {
            cdbl acc = gv[i];
            for (int k = i + 1; k < j; k++) acc -= Hij(i, k) * y[k];
            y[i] = Hij(i, i) != 0.0 ? acc / Hij(i, i) : 0.0;
        }
        double* hy = ctx->host_d;
        for (int i = 0; i < j; i++) {
            hy[2 * i] = y[i].real();
            hy[2 * i + 1] = y[i].imag();
        }
        HIPCHK(ctx, hipMemcpyAsync(coef.p, hy, 2 * j * sizeof(double), hipMemcpyHostToDevice, s));
        if (precond) HIPCHK(ctx, launch_multiaxpy(s, Z.p, n, j, (const double*)coef.p, xe.p, n, 1.0));
        else HIPCHK(ctx, launch_multiaxpy(s, V.p, n, j, (const double*)coef.p, xe.p, n, 1.0));
        cycles++;
        const double rn_prev = rn;
        CHK(schur_residual(rn));
        if (prm.gmres_fallback && rn > 0.9 * rn_prev && rn > target) {
            stalled = true;
            break;
        }
    }

    // ---- write x; BiCGStab finishes a stalled solve ----------------------------
    if (status != QCDW_ENAN) {
        if (status != QCDW_OK) CHK(full_check(true_res, bnorm));
        HIPCHK(ctx, launch_unpack_spinor(s, F64, g, xe.p, 0, x, 1.0));
        HIPCHK(ctx, launch_unpack_spinor(s, F64, g, xo.p, 1, x, 1.0));
    }
    HIPCHK(ctx, hipStreamSynchronize(s));
    inf->fallback = 0;
    if (stalled && status != QCDW_OK && status != QCDW_ENAN) {
        qcdw_solver_params fb = prm;
        fb.inner = (qcdw_prec)op->inner;
        fb.maxiter = std::max(0, prm.maxiter - iters);
        qcdw_solve_info finf{};
        std::vector<double> fh(std::max(1, fb.maxiter + 2));
        finf.res_hist = fh.data();
        finf.hist_len = (int)fh.size();
        const qcdw_status st = qcdw_invert(op, b, x, &fb, &finf);
        status = st;
        true_res = finf.true_res;
        inf->fallback = 1;
        inf->fallback_iters = finf.iters;
        iters += finf.iters;
        for (int k = 1; k < finf.hist_count; k++) hist.push_back(fh[k]);
    }
    inf->status = status;
    inf->iters = iters;
    inf->n_restarts = cycles;
    inf->true_res = true_res;
    inf->iter_res = rn / bnorm;
    if (user_hist && user_hist_len > 0) {
        const int cnt = std::min<int>(user_hist_len, (int)hist.size());
        memcpy(user_hist, hist.data(), cnt * sizeof(double));
        inf->hist_count = cnt;
    }
    inf->time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    if (status != QCDW_OK)
        return fail(ctx, status, "FGMRES did not reach tol (iters %d, true residual %.3e)", iters, true_res);
    return QCDW_OK;
}

extern "C" qcdw_status qcdw_invert_fgmres(qcdw_op* op, qcdw_net* net, const void* b, void* x,
                                          const qcdw_solver_params* params, qcdw_solve_info* info)
{
    if (!op) return QCDW_EINVAL;
    if (net && net->op != op) return fail(op->ctx, QCDW_EINVAL, "the net was built on another operator");
    const Precond pnet = [net](const void* v, void* z) { return net_forward_internal(net, BF16, v, z); };
    return fgmres_run(op, net ? &pnet : nullptr, b, x, params, info);
}
