// Host-side objects of libqcdw shared by the C-ABI sources: the context, the
// operator and batch objects, device buffers, argument checks and small helpers.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"
#include "qcdw.h"

using namespace qcdw;

// pinned host staging sizes: a solve has at most 64 problems (batch) and needs
// one Scal and two doubles per problem
constexpr int HOST_SCAL_N = 64;
constexpr int HOST_D_N = 320;

struct qcdw_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;  // private stream used only to capture graphs
    std::string err;
    Scal* host_scal = nullptr;  // pinned, HOST_SCAL_N entries (one per problem of a solve)
    double* host_d = nullptr;   // pinned, HOST_D_N doubles (per-problem scalars, 2 per problem)
    int* dev_int = nullptr;
    // launch-parameter tuning cache (the role of the paper's resource_path):
    // "key value" lines, kept in memory and in $QCDW_TUNE_CACHE when set
    std::map<std::string, int> tune;
    std::string tune_path;
    void tune_load()
    {
        const char* p = getenv("QCDW_TUNE_CACHE");
        if (!p || !*p) return;
        tune_path = p;
        std::ifstream f(tune_path);
        std::string k;
        int v;
        while (f >> k >> v) tune[k] = v;
    }
    void tune_store(const std::string& k, int v)
    {
        tune[k] = v;
        if (tune_path.empty()) return;
        std::ofstream f(tune_path, std::ios::trunc);
        for (auto& kv : tune) f << kv.first << " " << kv.second << "\n";
    }
};

namespace qcdw_host {

// Device blocks of destroyed operators, batches and nets, kept per device and handed to the next
// allocation of about the same size: creating operators one after another (a new gauge field per
// solve) then costs no hipMalloc, and no hipFree, which also waits for the whole device.  Blocks
// enter the cache only once their owner's stream has drained (the destroy calls synchronise it).
struct BlockCache {
    std::mutex m;
    std::map<int, std::multimap<size_t, void*>> free;  // device -> (size, block)
    // smallest cached block of at least `bytes` and at most a quarter (plus 1 MiB) larger
    void* take(int dev, size_t bytes, size_t& got)
    {
        std::lock_guard<std::mutex> lk(m);
        auto& f = free[dev];
        auto it = f.lower_bound(bytes);
        if (it == f.end() || it->first > bytes + bytes / 4 + (1u << 20)) return nullptr;
        void* q = it->second;
        got = it->first;
        f.erase(it);
        return q;
    }
    void give(int dev, void* q, size_t n)
    {
        std::lock_guard<std::mutex> lk(m);
        free[dev].emplace(n, q);
    }
    // return every cached block of the device to the runtime (the current device must be dev)
    void trim(int dev)
    {
        std::lock_guard<std::mutex> lk(m);
        for (auto& kv : free[dev]) (void)hipFree(kv.second);
        free[dev].clear();
    }
};
inline BlockCache& block_cache()
{
    static BlockCache* c = new BlockCache;  // never destroyed: blocks live until the process ends or a trim
    return *c;
}

struct DevBuf {
    void* p = nullptr;
    size_t n = 0;
    int dev = 0;
    bool pooled = false;  // released into the block cache (only for owners that drain their stream first)
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf()
    {
        if (!p) return;
        if (pooled)
            block_cache().give(dev, p, n);
        else
            (void)hipFree(p);
    }
    hipError_t alloc(size_t bytes)
    {
        if (p && n >= bytes) return hipSuccess;
        if (p) (void)hipFree(p);  // growing: queued work may still use the old block
        p = nullptr;
        n = 0;
        if (bytes == 0) bytes = 16;
        if (hipGetDevice(&dev) != hipSuccess) dev = 0;
        if (pooled) {
            size_t got = 0;
            if ((p = block_cache().take(dev, bytes, got)) != nullptr) {
                n = got;
                return hipSuccess;
            }
        }
        hipError_t e = hipMalloc(&p, bytes);
        if (e == hipErrorOutOfMemory && pooled) {
            (void)hipGetLastError();
            block_cache().trim(dev);
            e = hipMalloc(&p, bytes);
        }
        if (e == hipSuccess)
            n = bytes;
        else
            p = nullptr;
        return e;
    }
};
// a DevBuf whose block goes back into the cache
struct PoolBuf : DevBuf {
    PoolBuf() { pooled = true; }
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

inline qcdw_status fail(qcdw_ctx* ctx, qcdw_status st, const char* fmt, ...)
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

inline qcdw_status check_lattice(qcdw_ctx* ctx, const qcdw_lattice* lat, Geom& g)
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

inline qcdw_status check_dev(qcdw_ctx* ctx, const void* p, const char* name)
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

}  // namespace qcdw_host
using namespace qcdw_host;

// ---------------------------------------------------------------------------
// operator object
// ---------------------------------------------------------------------------
// Solver workspace: stacked/concatenated vectors of all problems of a solve,
// scalars, partials, and the graphs captured over them.
struct Workspace {
    PoolBuf be, bo, yo, ye, bhat, xhi, rhi, tmp64, tmpo64;  // FP64, per problem
    PoolBuf kr[7];  // r, r0, p, v, s, t, tmp_o in the Krylov precision
    PoolBuf xlo;    // FP32 correction (mixed precision)
    PoolBuf partials, scal, dres, hist, coef;
    int ws_gen = 0;  // bumped whenever a buffer is (re)allocated
    struct Graph {
        int kprec, chunk, nprob, variant, gen, fuse_nb;
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
    ~Workspace() { drop_graphs(); }
};

struct qcdw_op {
    qcdw_ctx* ctx = nullptr;
    Geom g{};
    double kappa = 0, csw = 0;
    int inner = F64;
    int recon = 12;
    PoolBuf gauge64, gauge_lo;
    PoolBuf Ainv64[2], Ainv_lo[2], A64[2];
    int hop_nt[4] = {1, 1, 1, 1};  // single-RHS hop, per precision (tuned): sites per thread along t,
    int hop_cg[4] = {0, 0, 0, 0};  //   c-tiles per group swept along t (0: none)
    int hop_fma[4] = {0, 0, 0, 0};  //   and the arithmetic form (1: multiply-add form)
    Workspace ws;                  // single- and multi-RHS solves
};

// a set of operators solved together (different lattices and kappas)
struct qcdw_batch {
    qcdw_ctx* ctx = nullptr;
    std::vector<qcdw_op*> ops;
    int inner = F64;
    std::vector<long> off, len;  // element offsets / lengths of each problem in concatenated vectors
    long total = 0, nmax = 0;
    int total_tiles = 0, nbmax = 0;
    PoolBuf map, nbs, tab64, tablo;  // device: (off, len) pairs, hop tiles per problem, BatchEntry tables
    Workspace ws;
};

namespace qcdw_host {

constexpr long MAX_PARTIALS = 4096;

// fixed workspace of qcdw_dslash_noalloc (noalloc.hip): device address lookup per device, and bytes needed
hipError_t noalloc_scratch_init(int device);
size_t noalloc_dslash_bytes(long Vh, bool build_clover);  // >= blas_blocks(); hop partials are sized per lattice

struct PrecView {
    int prec;
    int recon;
    const void* gauge;
    const void* Ainv[2];
};

inline PrecView view(const qcdw_op* op, int prec)
{
    if (prec == F64) return {F64, op->recon, op->gauge64.p, {op->Ainv64[0].p, op->Ainv64[1].p}};
    return {op->inner, op->inner == F64 ? op->recon : (op->inner == F32 ? op->recon : 12), op->gauge_lo.p,
            {op->Ainv_lo[0].p, op->Ainv_lo[1].p}};
}

inline HopArgs hop_args(const Geom& g, int parity)
{
    HopArgs a{};
    a.g = g;
    a.parity = parity;
    a.nrhs = 1;
    a.nt = 1;
    return a;
}

// out_e = M_hat in_e = in_e - kappa^2 A_ee^-1 H_eo A_oo^-1 H_oe in_e, with an optional fused reduction
// (hop_blocks_nt(op->g, op->hop_nt[v.prec], op->hop_cg[v.prec]) partials); the operator's tuned form
inline hipError_t matpc(hipStream_t s, const qcdw_op* op, const PrecView& v, const void* in, void* out, void* tmp_o, int red,
                 const void* w, double* partials, const int* stop)
{
    HopArgs a = hop_args(op->g, 1);
    a.nt = op->hop_nt[v.prec];
    a.cgroup = op->hop_cg[v.prec];
    a.fma = op->hop_fma[v.prec];
    a.psi = in;
    a.out = tmp_o;
    a.gauge = v.gauge;
    a.clov = v.Ainv[1];
    a.stop = stop;
    hipError_t e = launch_hop(s, v.prec, v.recon, EPI_CLOV, RED_NONE, a);
    if (e != hipSuccess) return e;
    HopArgs b = hop_args(op->g, 0);
    b.nt = op->hop_nt[v.prec];
    b.cgroup = op->hop_cg[v.prec];
    b.fma = op->hop_fma[v.prec];
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

// right preconditioner of FGMRES: z = K(v) on FP64 even-site internal fields
using Precond = std::function<qcdw_status(const void* v, void* z)>;
qcdw_status fgmres_run(qcdw_op* op, const Precond* precond, const void* b, void* x, const qcdw_solver_params* params,
                       qcdw_solve_info* info);

inline qcdw_status read_double(qcdw_ctx* ctx, const double* dev, double& out)
{
    HIPCHK(ctx, hipMemcpyAsync(ctx->host_d, dev, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    out = ctx->host_d[0];
    return QCDW_OK;
}

}  // namespace qcdw_host

using namespace qcdw_host;
