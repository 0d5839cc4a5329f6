// Conversion between the paper's field layouts (Sec. II.A, FP64) and the
// library's internal site-major layouts, with optional down-conversion to
// FP32 / BF16 / FP16 storage (round to nearest even) and a scale factor.
#include "internal.h"

namespace qcdw {

// spinor: paper [2][Vh][4][3] complex f64  <->  internal spinor (sp_idx order) complex P
template <class P>
__global__ void k_pack_spinor(const double2* __restrict__ paper, void* out, int Vh, int parity, double scale)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;  // internal element
    if (e >= 12L * Vh) return;
    long s, site;
    int c;
    sp_coords(e, Vh, s, site, c);
    const double2 v = paper[((long)parity * Vh + site) * 12 + s * 3 + c];
    using T = typename P::real;
    P::st(out, e, cx<T>{(T)(scale * v.x), (T)(scale * v.y)});
}

template <class P>
__global__ void k_unpack_spinor(const void* in, double2* __restrict__ paper, int Vh, int parity, double scale)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 12L * Vh) return;
    long s, site;
    int c;
    sp_coords(e, Vh, s, site, c);
    const auto v = P::ld(in, e);
    paper[((long)parity * Vh + site) * 12 + s * 3 + c] = make_double2(scale * (double)v.re, scale * (double)v.im);
}

// gauge: paper [4][2][Vh][3][3]  ->  internal links of R entries (rows 0..R/3-1) at link_base
template <class P, int R>
__global__ void k_pack_gauge(const double2* __restrict__ paper, void* out, int Vh)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 8L * Vh * R) return;
    const int j = (int)(e % R);
    const long link = e / R;  // (mu*2 + parity)*Vh + site
    const int site = (int)(link % Vh), mp = (int)(link / Vh);
    const double2 v = paper[link * 9 + j];
    using T = typename P::real;
    constexpr bool soa = link_soa_for(P::cbytes);
    P::st(out, link_base(mp >> 1, mp & 1, site, Vh, R, soa) + j * link_stride(Vh, soa), cx<T>{(T)v.x, (T)v.y});
}

// clover: paper [2][Vh][2][36] -> internal (one parity) [Vh][2][36] in the reordered packing
//   [d0 d1 d2 | L10 L20 L21 | L30 L31 L32 L40 L41 L42 L50 L51 L52 | d3 d4 d5 | L43 L53 L54]
// The paper packing is [d0..d5 | L10 L20 L21 L30 L31 L32 L40 L41 L42 L43 L50 .. L54].
__device__ __forceinline__ int clover_src_pos(int m)
{
    // lower slot s of (j,k) in the paper packing is j(j-1)/2 + k at reals 6+2s, 7+2s
    if (m < 3) return m;                      // d0..d2
    if (m < 9) return 6 + (m - 3);            // L10 L20 L21  (slots 0..2)
    if (m < 27) {                             // L3x (slots 3..5), L4x (6..8), L5x (10..12)
        const int q = (m - 9) >> 1, ri = (m - 9) & 1;
        const int row = q / 3, col = q % 3;   // row 0..2 -> j = 3..5
        const int j = 3 + row;
        const int slot = j * (j - 1) / 2 + col;
        return 6 + 2 * slot + ri;
    }
    if (m < 30) return 3 + (m - 27);          // d3..d5
    const int q = (m - 30) >> 1, ri = (m - 30) & 1;  // L43 (9), L53 (13), L54 (14)
    const int slot = q == 0 ? 9 : (q == 1 ? 13 : 14);
    return 6 + 2 * slot + ri;
}

template <class P>
__global__ void k_pack_clover(const double* __restrict__ paper, void* out, int Vh, int parity)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;  // = clov_index(site, chi, m)
    if (e >= clov_reals(Vh)) return;
    const int m = (int)(e % 36);
    const long blk = e / 36;  // site * 2 + chirality
    using T = typename P::real;
    P::str(out, e, (T)paper[((long)parity * Vh * 2 + blk) * 36 + clover_src_pos(m)]);
}

static inline dim3 grid_for(long n) { return dim3((unsigned)((n + 255) / 256)); }

hipError_t launch_pack_spinor(hipStream_t s, int prec, const Geom& g, const void* paper, int parity, void* internal,
                              double scale)
{
    const long n = 12L * g.Vh;
    if (n == 0) return hipSuccess;
    const double2* pp = (const double2*)paper;
    switch (prec) {
    case F64: hipLaunchKernelGGL(k_pack_spinor<P64>, grid_for(n), dim3(256), 0, s, pp, internal, g.Vh, parity, scale); break;
    case F32: hipLaunchKernelGGL(k_pack_spinor<P32>, grid_for(n), dim3(256), 0, s, pp, internal, g.Vh, parity, scale); break;
    case BF16: hipLaunchKernelGGL(k_pack_spinor<PBF16>, grid_for(n), dim3(256), 0, s, pp, internal, g.Vh, parity, scale); break;
    case F16: hipLaunchKernelGGL(k_pack_spinor<PF16>, grid_for(n), dim3(256), 0, s, pp, internal, g.Vh, parity, scale); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_unpack_spinor(hipStream_t s, int prec, const Geom& g, const void* internal, int parity, void* paper,
                                double scale)
{
    const long n = 12L * g.Vh;
    if (n == 0) return hipSuccess;
    double2* pp = (double2*)paper;
    switch (prec) {
    case F64: hipLaunchKernelGGL(k_unpack_spinor<P64>, grid_for(n), dim3(256), 0, s, internal, pp, g.Vh, parity, scale); break;
    case F32: hipLaunchKernelGGL(k_unpack_spinor<P32>, grid_for(n), dim3(256), 0, s, internal, pp, g.Vh, parity, scale); break;
    case BF16: hipLaunchKernelGGL(k_unpack_spinor<PBF16>, grid_for(n), dim3(256), 0, s, internal, pp, g.Vh, parity, scale); break;
    case F16: hipLaunchKernelGGL(k_unpack_spinor<PF16>, grid_for(n), dim3(256), 0, s, internal, pp, g.Vh, parity, scale); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_pack_gauge(hipStream_t s, int prec, int recon, const Geom& g, const void* paper, void* internal)
{
    const double2* pp = (const double2*)paper;
    const int R = recon == 18 ? 9 : 6;
    const long n = 8L * g.Vh * R;
    if (n == 0) return hipSuccess;
    if (R == 9) {
        if (prec == F64) hipLaunchKernelGGL((k_pack_gauge<P64, 9>), grid_for(n), dim3(256), 0, s, pp, internal, g.Vh);
        else if (prec == F32) hipLaunchKernelGGL((k_pack_gauge<P32, 9>), grid_for(n), dim3(256), 0, s, pp, internal, g.Vh);
        else return hipErrorInvalidValue;
    } else {
        switch (prec) {
        case F64: hipLaunchKernelGGL((k_pack_gauge<P64, 6>), grid_for(n), dim3(256), 0, s, pp, internal, g.Vh); break;
        case F32: hipLaunchKernelGGL((k_pack_gauge<P32, 6>), grid_for(n), dim3(256), 0, s, pp, internal, g.Vh); break;
        case BF16: hipLaunchKernelGGL((k_pack_gauge<PBF16, 6>), grid_for(n), dim3(256), 0, s, pp, internal, g.Vh); break;
        case F16: hipLaunchKernelGGL((k_pack_gauge<PF16, 6>), grid_for(n), dim3(256), 0, s, pp, internal, g.Vh); break;
        default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

hipError_t launch_pack_clover(hipStream_t s, int prec, const Geom& g, const void* paper, int parity, void* internal)
{
    const long n = clov_reals(g.Vh);
    if (n == 0) return hipSuccess;
    const double* pp = (const double*)paper;
    switch (prec) {
    case F64: hipLaunchKernelGGL(k_pack_clover<P64>, grid_for(n), dim3(256), 0, s, pp, internal, g.Vh, parity); break;
    case F32: hipLaunchKernelGGL(k_pack_clover<P32>, grid_for(n), dim3(256), 0, s, pp, internal, g.Vh, parity); break;
    case BF16: hipLaunchKernelGGL(k_pack_clover<PBF16>, grid_for(n), dim3(256), 0, s, pp, internal, g.Vh, parity); break;
    case F16: hipLaunchKernelGGL(k_pack_clover<PF16>, grid_for(n), dim3(256), 0, s, pp, internal, g.Vh, parity); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace qcdw
