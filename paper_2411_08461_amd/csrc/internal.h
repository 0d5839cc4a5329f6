// Host-side internal interfaces of libqcdw: launch descriptors and launcher
// declarations shared between the kernel files and the C-ABI layer.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dev.h"

namespace qcdw {

struct Scal;  // BiCGStab scalars, below

enum Prec { F64 = 0, F32 = 1, BF16 = 2, F16 = 3 };

inline int cplx_bytes(int prec) { return prec == F64 ? 16 : prec == F32 ? 8 : 4; }
inline int real_bytes(int prec) { return prec == F64 ? 8 : prec == F32 ? 4 : 2; }

// hop epilogues
enum Epi {
    EPI_NONE = 0,       // out = H psi
    EPI_CLOV = 1,       // out = B (H psi)
    EPI_CLOV_XPAY = 2,  // out = y - a B (H psi)
    EPI_XPAY_CLOVY = 3  // out = B y - a (H psi)
};
// hop fused reductions (per-block partials)
enum Red {
    RED_NONE = 0,
    RED_WDOT = 1,  // (w, out)              -> 2 doubles
    RED_TS = 2     // (out, y), ||out||^2   -> 3 doubles
};

struct HopArgs {
    const void* psi;    // input spinor, parity 1 - parity
    void* out;          // output spinor, parity `parity`
    const void* gauge;  // R entries per link at link_base / link_stride (dev.h)
    const void* clov;   // clover-type matrix of the output parity, [Vh][2][36] reordered
    const void* y;      // xpay / dot operand on the output parity
    const void* w;      // dot operand on the output parity
    double a;           // xpay coefficient
    double* partials;   // [nblocks][3]
    Geom g;
    int parity;
    int nrhs;           // right-hand sides interleaved per site (1 or more)
    const int* active;  // multi-RHS: per-RHS active flag (nullptr: all active)
    const int* stop;    // if non-null and *stop != 0 the launch does nothing
    int nt;             // single-RHS hop: output sites per thread along t (1, 2, 4 or 8; 0 means 1)
    int cgroup;         // single-RHS hop: c-tiles per group swept along t (0: no grouping)
    int fma;            // single-RHS hop: bit 0 the multiply-add form of the hop arithmetic, bit 1 the
                        // t-neighbours staged in LDS (slice groups with one site per thread group only)
};

// one problem of a batched solve (device table entry); reconstruct-12 operators
struct BatchEntry {
    Geom g;
    double kappa2;        // kappa^2 of this problem
    const void* gauge;    // links in the batch's Krylov precision
    const void* clov[2];  // A^-1 per parity, same precision
    long off;             // element offset (complex) of this problem in the concatenated vectors
    long n;               // 12 Vh
    int tile0;            // first global hop tile of this problem
    int ntiles;           // hop tiles of this problem
};

struct BatchHopArgs {
    const BatchEntry* tab;
    int nprob;
    int total_tiles;
    int parity;
    int nbmax;           // partials stride per problem (tiles)
    int use_kappa2;      // 1: xpay coefficient = kappa^2 of each problem, else `a`
    double a;
    const void* psi;     // concatenated vectors, problem k at element offset tab[k].off
    void* out;
    const void* y;
    const void* w;
    double* partials;    // [problem][nbmax][3]
    const Scal* S;       // per-problem solver scalars (flags) or nullptr
};

constexpr int HOP_SITES_PER_BLOCK = 64;  // 4 lanes per site, 256 threads
__host__ __device__ inline int hop_blocks(int Vh) { return (Vh + HOP_SITES_PER_BLOCK - 1) / HOP_SITES_PER_BLOCK; }
// the t-stepping hop (nt sites per thread along t) needs Lt % (2 nt) == 0
__host__ __device__ inline bool hop_nt_fits(const Geom& g, int nt)
{
    return nt <= 1 || ((nt == 2 || nt == 4 || nt == 8) && g.Lt % (2 * nt) == 0);
}
// tiles of 64 consecutive sites within one t-slice (eo index c in [0, Lxh Ly Lz))
__host__ __device__ inline int hop_ctiles(const Geom& g) { return (g.Lxh * g.Ly * g.Lz + 63) / 64; }
// a c-tile group size is valid if it divides the c-tiles of a slice
__host__ __device__ inline bool hop_cgroup_fits(const Geom& g, int cg)
{
    return cg == 0 || (cg > 0 && hop_ctiles(g) % cg == 0);
}
// blocks (and reduction partials) of one single-RHS hop launch
__host__ __device__ inline int hop_blocks_nt(const Geom& g, int nt, int cg)
{
    if (nt <= 1) return cg > 0 ? hop_ctiles(g) * g.Lt : hop_blocks(g.Vh);
    return hop_ctiles(g) * (g.Lt / nt);
}

// e0/e1: optional events recorded by the kernel dispatch itself (timing)
hipError_t launch_hop(hipStream_t s, int prec, int recon, int epi, int red, const HopArgs& a,
                      hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);

// BiCGStab scalars kept on the device (complex values as re, im pairs)
hipError_t launch_hop_batch(hipStream_t s, int prec, int epi, int red, const BatchHopArgs& b, int grid,
                            hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);

struct Scal {
    double rho[2];    // (r0, r)
    double rho_prev[2];  // rho of the iteration in progress (the beta step's denominator)
    double alpha[2];
    double omega[2];
    double beta[2];
    double rr;        // ||r||^2 of the iterated residual
    double r0n2;      // ||r0||^2 (breakdown thresholds)
    double stop_rr;   // convergence when rr <= stop_rr
    double hist_norm; // history entry = sqrt(rr) * hist_norm
    int iter;         // iterations completed
    int flags;        // FLAG_* below
    int fault_iter;   // > 0: force a breakdown when iter reaches this value; < 0: flag an overflow at -value
    int hist_len;     // capacity of the device history
};
enum { FLAG_CONV = 1, FLAG_BREAK = 2, FLAG_NAN = 4, FLAG_STOP = 8 /* cycle ended by the host */ };

constexpr int BLAS_THREADS = 256;
// number of blocks used by the BLAS reductions on n complex elements
inline int blas_blocks(long n)
{
    long b = (n + BLAS_THREADS * 4 - 1) / (BLAS_THREADS * 4);
    if (b < 1) b = 1;
    if (b > 2048) b = 2048;
    return (int)b;
}

// Vector kernels act on nrhs stacked fields of n complex elements each; RHS y uses
// elements [y n, (y+1) n), scalars S[y] and partials [y][blocks][..].  With a map
// (device array of (offset, length) per vector, problems of different sizes) the
// ranges come from the map and nmax is the longest length.
hipError_t launch_norm2(hipStream_t s, int prec, const void* x, long n, double* partials, double* out, int nrhs = 1,
                        const long2* map = nullptr, long nmax = 0);
hipError_t launch_xmy_norm2(hipStream_t s, int prec_b, int prec_y, const void* b, const void* y, void* r, long n,
                            double* partials, double* out, int nrhs = 1, const long2* map = nullptr,
                            long nmax = 0);  // r = b - y (FP64 r), out = ||r||^2
hipError_t launch_convert(hipStream_t s, int prec_in, int prec_out, const void* in, void* out, long n, double scale,
                          const double* scales = nullptr, int nrhs = 1, const long2* map = nullptr, long nmax = 0);
hipError_t launch_axpy_hi(hipStream_t s, int prec_x, double a, const double* coefs, const void* x, void* y, long n,
                          int nrhs = 1, const long2* map = nullptr, long nmax = 0);  // y(f64) += a x
hipError_t launch_clov_apply_internal(hipStream_t s, int prec, const Geom& g, const void* clov, const void* in,
                                      void* out);

// BiCGStab iteration pieces
// start of a Krylov cycle from the FP64 residuals rhi: r = scales[y] rhi in precision prec; unless
// resume, r0 = p = r and the scalars S are initialised from ||r||^2 (rho = ||r||^2, flags from
// stop_rr); xlo (FP32 complex, may be nullptr) is cleared.  partials: nrhs x blas_blocks doubles.
hipError_t launch_cycle_start(hipStream_t s, int prec, const void* rhi, void* r, void* r0, void* p, void* xlo, long n,
                              const double* scales, Scal* S, double* partials, int nrhs, const long2* map, long nmax,
                              bool resume);
// rho' = (r0, r), beta from the previous step's scalars, for a cycle that continues the recurrence
hipError_t launch_bicg_resume(hipStream_t s, int prec, const void* r0, const void* r, long n, Scal* S,
                              double* partials, int nrhs, const long2* map, long nmax);
// The BiCGStab vector updates.  Each takes its scalar (beta, alpha, omega) from S, recorded there by
// the matching launch_fin_* kernel, or, with fin != nullptr, forms it itself from the reduction
// partials fin [RHS][fin_nb][3] (fin_nbs: per-RHS counts, or nullptr) and records it in S: one
// launch fewer per scalar.  hist: the residual history of the beta step (fused form only).
hipError_t launch_bicg_p(hipStream_t s, int prec, void* p, const void* r, const void* v, long n, Scal* S,
                         int nrhs = 1, const long2* map = nullptr, long nmax = 0, const double* fin = nullptr,
                         int fin_nb = 0, double* hist = nullptr);
hipError_t launch_bicg_s(hipStream_t s, int prec, void* sv, const void* r, const void* v, long n, Scal* S,
                         int nrhs = 1, const long2* map = nullptr, long nmax = 0, const double* fin = nullptr,
                         int fin_nb = 0, const int* fin_nbs = nullptr);
// partials (its own output) must not overlap fin
hipError_t launch_bicg_xr(hipStream_t s, int prec, int prec_x, void* x, const void* p, const void* sv, void* r,
                          const void* t, const void* r0, long n, Scal* S, double* partials, int nrhs = 1,
                          const long2* map = nullptr, long nmax = 0, const double* fin = nullptr, int fin_nb = 0,
                          const int* fin_nbs = nullptr);
// nb: partials stride per RHS; nbs (optional, per RHS) the count actually written
hipError_t launch_fin_alpha(hipStream_t s, Scal* S, const double* partials, int nb, int nrhs = 1,
                            const int* nbs = nullptr);
hipError_t launch_fin_omega(hipStream_t s, Scal* S, const double* partials, int nb, int nrhs = 1,
                            const int* nbs = nullptr);
hipError_t launch_fin_beta(hipStream_t s, Scal* S, const double* partials, int nb, double* hist, int nrhs = 1);

// multi-RHS hop (reconstruct-12): a.nrhs stacked fields; RHS y skipped when S[y].flags != 0;
// partials [y][hop_blocks][3]
hipError_t launch_hop_mrhs(hipStream_t s, int prec, int epi, int red, const HopArgs& a, const Scal* S,
                           hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// the same with the link products on the matrix cores (BF16 / FP16 storage only; hipErrorInvalidValue
// otherwise); same grid and partials as launch_hop_mrhs
hipError_t launch_hop_mrhs_mfma(hipStream_t s, int prec, int epi, int red, const HopArgs& a, const Scal* S,
                                hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// the same operation with one block per (tile, rhs), rhs fastest (links and clover re-read from L2)
hipError_t launch_hop_rhs(hipStream_t s, int prec, int epi, int red, const HopArgs& a, const Scal* S,
                          hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);

// learned preconditioner layers (activations [parity][channel][Vh][3], FP32/BF16 storage)
// mfma: layers with a BF16 end mix channels on the BF16 matrix cores (k_net_layer_mfma)
hipError_t launch_net_layer(hipStream_t s, int pin, int pout, int cin, int cout, const void* in, void* out,
                            const void* gauge32, const void* W, const Geom& g,
                            int mfma = 0);
// out[2 cin cout] (+)= weight gradient of hop a: sum_x g_{c'} conj(T_a phi_c); partials: [blocks][2 cin cout]
hipError_t launch_net_wgrad(hipStream_t s, int cin, int cout, const void* phi, const void* gz, const void* gauge32,
                            const Geom& g, int a, double* partials, double* out, int accumulate);
hipError_t launch_net_adjoint_w(hipStream_t s, const void* W, void* Wt, int cout, int cin);
hipError_t launch_net_make_gz(hipStream_t s, const void* diff, void* gz, long n_half, double coef);
hipError_t launch_gaussian(hipStream_t s, void* out, long n, uint64_t seed, uint64_t stream);  // FP64 complex
hipError_t launch_adam(hipStream_t s, void* W, const double* G, double* m, double* v, int n, double lr, double b1,
                       double b2, double eps, int step, double gscale);

// FGMRES block Gram-Schmidt on FP64 vectors V_i = V + i stride (complex elements)
hipError_t launch_scale_inv_norm(hipStream_t s, const void* w, void* out, long n, const double* nrm2);
hipError_t launch_multidot(hipStream_t s, const void* V, long stride, int nvec, const void* w, long n,
                           double* partials, double* out);  // out[2i..] = (V_i, w); partials: 16 ceil(nvec/8) blocks
hipError_t launch_multiaxpy(hipStream_t s, const void* V, long stride, int nvec, const double* c, void* w, long n,
                            double sign);  // w += sign sum_i c_i V_i

// pack / unpack between the paper layouts and the internal ones
hipError_t launch_pack_spinor(hipStream_t s, int prec, const Geom& g, const void* paper, int parity, void* internal,
                              double scale);
hipError_t launch_unpack_spinor(hipStream_t s, int prec, const Geom& g, const void* internal, int parity, void* paper,
                                double scale);
hipError_t launch_pack_gauge(hipStream_t s, int prec, int recon, const Geom& g, const void* paper, void* internal);
hipError_t launch_pack_clover(hipStream_t s, int prec, const Geom& g, const void* paper, int parity, void* internal);

// clover kernels on the paper layouts (FP64)
// the 12 wall sources on slice t0 with spatial momentum mom (12 paper-layout fields into out)
hipError_t launch_wall_sources(hipStream_t s, const Geom& g, int t0, const int mom[3], void* out);
// meson contraction of the 12-field propagators S and T (T = S: the two-point function) into out[Lt]
// (complex FP64); site_scratch: V complex
hipError_t launch_meson_2pt(hipStream_t s, const Geom& g, const void* S, const void* T, int g_snk, int g_src,
                            const int mom[3], void* site_scratch, void* out);
// sequential sources through the sink slice t_f from the propagator S (12 fields into out)
hipError_t launch_seq_sources(hipStream_t s, const Geom& g, const void* S, int t_f, int g_f, const int mom[3],
                              void* out);
// C = wt sum_i sigma_i4 F_i4 + ws sum_{i<j} sigma_ij F_ij (wt = ws = 1: the isotropic clover field)
hipError_t launch_clover_build(hipStream_t s, const Geom& g, const void* U, void* clover, double wt = 1.0,
                               double ws = 1.0);
hipError_t launch_clover_apply(hipStream_t s, const Geom& g, const void* clover, const void* psi, void* out,
                               double kappa, double csw);
hipError_t launch_clover_invert(hipStream_t s, const Geom& g, const void* clover, double kappa, double csw,
                                void* inv, int* notpd_count);
// packed A = 1 - kappa csw C (paper clover layout) for the full-operator epilogue
// clover fermion force of the bilinear 2 Re(Y^+ M X) (force.hip); Gam: scratch of 6 x 144 V bytes
hipError_t launch_clover_force(hipStream_t s, const Geom& g, const void* U, const void* X, const void* Y,
                               double kappa, double csw, void* Gam, void* H);
hipError_t launch_clover_to_A(hipStream_t s, const Geom& g, const void* clover, double kappa, double csw, void* A);

}  // namespace qcdw
