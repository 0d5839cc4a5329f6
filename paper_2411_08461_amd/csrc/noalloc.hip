// qcdw_dslash_noalloc: the full Wilson-clover operator of qcdw_dslash with its workspace taken from a
// fixed device array instead of device allocations, for callers that cannot allocate.
//
// `scratch` is a file-scope device array; its host-side name is not a device address, so host code
// never passes it to a kernel or a copy.  qcdw_ctx_create calls noalloc_scratch_init with the device
// current, which looks the array's device address up once per device (each device holds its own copy)
// and keeps it in scratch_ptr[device]; every use below goes through that pointer.  Calls that overlap
// on one device share the array and race; the caller serialises them (one stream, or a wait between).
#include "host.h"

namespace {

constexpr size_t NOALLOC_BYTES = (size_t)QCDW_NOALLOC_MAX_BYTES;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void* scratch_ptr[MAX_DEVICES] = {};

size_t round256(size_t n) { return (n + 255) / 256 * 256; }

}  // namespace

namespace qcdw_host {

// device address of this device's copy of `scratch`; call with `device` current
hipError_t noalloc_scratch_init(int device)
{
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (scratch_ptr[device]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_ptr[device] = p;
    return hipSuccess;
}

// bytes of workspace qcdw_dslash_noalloc needs for a lattice of Vh sites per parity
size_t noalloc_dslash_bytes(long Vh, bool build_clover)
{
    const size_t vb = round256(12UL * Vh * 16);           // one internal spinor parity, FP64
    const size_t gauge = round256(8UL * Vh * 9 * 16);     // reconstruct-18 links, both parities
    const size_t cpaper = round256(144UL * Vh * 8);       // clover-layout field, both parities
    const size_t apar = round256(clov_reals(Vh) * 8);     // packed A of one parity
    return gauge + cpaper /* A */ + (build_clover ? cpaper : 0) + 2 * apar + 3 * vb;
}

}  // namespace qcdw_host

extern "C" qcdw_status qcdw_dslash_noalloc(qcdw_ctx* ctx, const qcdw_lattice* lat, const void* U, const void* clover,
                                           const void* psi, void* out, double kappa, double csw)
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
    const size_t need = noalloc_dslash_bytes(g.Vh, clover == nullptr);
    if (need > NOALLOC_BYTES)
        return fail(ctx, QCDW_EINVAL,
                    "qcdw_dslash_noalloc: lattice of %ld sites needs %zu bytes of workspace, above the fixed %zu",
                    2L * g.Vh, need, NOALLOC_BYTES);
    void* base;
    {
        std::lock_guard<std::mutex> lk(scratch_mu);
        base = (ctx->device >= 0 && ctx->device < MAX_DEVICES) ? scratch_ptr[ctx->device] : nullptr;
    }
    if (!base) return fail(ctx, QCDW_EHIP, "qcdw_dslash_noalloc: workspace of device %d not initialised", ctx->device);

    // carve the workspace: every region is fully written before it is read, so nothing is cleared
    char* w = (char*)base;
    auto take = [&](size_t n) {
        void* p = w;
        w += round256(n);
        return p;
    };
    const size_t vb = 12UL * g.Vh * 16;
    void* gauge = take(8UL * g.Vh * 9 * 16);
    void* Apaper = take(144UL * g.Vh * 8);
    void* A[2] = {take(clov_reals(g.Vh) * 8), take(clov_reals(g.Vh) * 8)};
    void* in[2] = {take(vb), take(vb)};
    void* res = take(vb);
    hipStream_t s = ctx->stream;
    HIPCHK(ctx, launch_pack_gauge(s, F64, 18, g, U, gauge));
    if (!clover) {
        void* clov = take(144UL * g.Vh * 8);
        HIPCHK(ctx, launch_clover_build(s, g, U, clov));
        clover = clov;
    }
    HIPCHK(ctx, launch_clover_to_A(s, g, clover, kappa, csw, Apaper));
    for (int p = 0; p < 2; p++) {
        HIPCHK(ctx, launch_pack_clover(s, F64, g, Apaper, p, A[p]));
        HIPCHK(ctx, launch_pack_spinor(s, F64, g, psi, p, in[p], 1.0));
    }
    for (int p = 0; p < 2; p++) {
        HopArgs a = hop_args(g, p);
        a.psi = in[1 - p];
        a.out = res;
        a.gauge = gauge;
        a.clov = A[p];
        a.y = in[p];
        a.a = kappa;
        HIPCHK(ctx, launch_hop(s, F64, 18, EPI_XPAY_CLOVY, RED_NONE, a));
        HIPCHK(ctx, launch_unpack_spinor(s, F64, g, res, p, out, 1.0));
    }
    HIPCHK(ctx, hipStreamSynchronize(s));
    return QCDW_OK;
}
