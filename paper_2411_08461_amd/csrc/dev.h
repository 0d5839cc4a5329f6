// Device-side building blocks shared by the qcdw HIP kernels: complex
// arithmetic, storage-precision traits for the internal layouts, lattice
// geometry and deterministic block reductions.
//
// Internal (library-owned) layouts, one parity of Vh sites each:
//   spinor  [4 spin][Vh site][3 colour] complex        (spin-major, colour inner)
//   gauge   [4 mu][2 parity][R][Vh site] complex in FP64, [4 mu][2 parity][Vh site][R] in FP32 and
//           16-bit storage; R = 6 (rows 0,1: reconstruct-12) or 9 (full link), row-major colour order
//   clover  [Vh site][2 chirality][36 entry] reals, entries in the reordered packing of
//           hop.hip, so a lane's 27-entry window is contiguous (wide per-lane loads; layouts
//           with sites fastest were measured slower on gfx950)
// Each lane of a hop kernel reads one spin (3 contiguous complex) of a
// neighbour, so consecutive sites give contiguous, fully coalesced accesses.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qcdw {

// ---------------------------------------------------------------------------
// complex
// ---------------------------------------------------------------------------
template <typename T>
struct cx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> mk(T r, T i) { return cx<T>{r, i}; }
template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }
template <typename T>
__device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.re, -a.im}; }
// conj(a) * b
template <typename T>
__device__ __forceinline__ cx<T> cmul_conj(cx<T> a, cx<T> b)
{
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// w += a b and w += conj(a) b, one multiply-add per real term (w + a * b would round the product
// first and add it separately)
template <typename T>
__device__ __forceinline__ void cmac(cx<T>& w, cx<T> a, cx<T> b)
{
    w.re += a.re * b.re;
    w.re -= a.im * b.im;
    w.im += a.re * b.im;
    w.im += a.im * b.re;
}
template <typename T>
__device__ __forceinline__ void cmac_conj(cx<T>& w, cx<T> a, cx<T> b)
{
    w.re += a.re * b.re;
    w.re += a.im * b.im;
    w.im += a.re * b.im;
    w.im -= a.im * b.re;
}
template <typename T>
__device__ __forceinline__ T norm2(cx<T> a) { return a.re * a.re + a.im * a.im; }

// ---------------------------------------------------------------------------
// storage precisions: FP64, FP32, BF16, FP16.  `real` is the arithmetic type.
// ---------------------------------------------------------------------------
// BF16 bits (low half of b) to float: exact
__device__ __forceinline__ float bf_bits2f(uint32_t b) { return __uint_as_float(b << 16); }
// float to BF16 bits, round to nearest even, in integer arithmetic (NaN kept quiet): the scalar store
// uses it so that an FP64 value is rounded to FP32 first and then to BF16, whatever the compiler folds
// (it turns a double -> float -> bfloat conversion chain into one direct rounding)
__device__ __forceinline__ uint32_t f2bf_bits(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}
// float to BF16 by the conversion instruction (v_cvt_pk_bf16_f32: round to nearest even, NaN stays
// NaN), two values packed low, high; written as a conversion, not as bit arithmetic, so that the
// compiler folds a rounded value that is rounded again into one instruction
typedef float bf_f2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf_b2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ bf_b2 f2bf2(float lo, float hi) { return __builtin_convertvector(bf_f2{lo, hi}, bf_b2); }

struct P64 {
    using real = double;
    static constexpr int cbytes = 16;  // bytes per complex
    __device__ static cx<double> ld(const void* base, long k)
    {
        double2 v = reinterpret_cast<const double2*>(base)[k];
        return {v.x, v.y};
    }
    __device__ static void st(void* base, long k, cx<double> z)
    {
        reinterpret_cast<double2*>(base)[k] = make_double2(z.re, z.im);
    }
    __device__ static cx<double> rt(cx<double> z) { return z; }
    __device__ static double ldr(const void* base, long k) { return reinterpret_cast<const double*>(base)[k]; }
    __device__ static void str(void* base, long k, double v) { reinterpret_cast<double*>(base)[k] = v; }
};

struct P32 {
    using real = float;
    static constexpr int cbytes = 8;
    __device__ static cx<float> ld(const void* base, long k)
    {
        float2 v = reinterpret_cast<const float2*>(base)[k];
        return {v.x, v.y};
    }
    __device__ static void st(void* base, long k, cx<float> z)
    {
        reinterpret_cast<float2*>(base)[k] = make_float2(z.re, z.im);
    }
    __device__ static cx<float> rt(cx<float> z) { return z; }
    __device__ static float ldr(const void* base, long k) { return reinterpret_cast<const float*>(base)[k]; }
    __device__ static void str(void* base, long k, float v) { reinterpret_cast<float*>(base)[k] = v; }
};

struct PBF16 {
    using real = float;
    static constexpr int cbytes = 4;
    __device__ static cx<float> ld(const void* base, long k)
    {
        uint32_t v = reinterpret_cast<const uint32_t*>(base)[k];
        return {bf_bits2f(v & 0xffffu), bf_bits2f(v >> 16)};
    }
    __device__ static void st(void* base, long k, cx<float> z) { reinterpret_cast<bf_b2*>(base)[k] = f2bf2(z.re, z.im); }
    __device__ static cx<float> rt(cx<float> z)
    {
        const bf_f2 f = __builtin_convertvector(f2bf2(z.re, z.im), bf_f2);
        return {f.x, f.y};
    }
    __device__ static float ldr(const void* base, long k)
    {
        return bf_bits2f(reinterpret_cast<const uint16_t*>(base)[k]);
    }
    __device__ static void str(void* base, long k, float v) { reinterpret_cast<uint16_t*>(base)[k] = (uint16_t)f2bf_bits(v); }
};

struct PF16 {
    using real = float;
    static constexpr int cbytes = 4;
    __device__ static cx<float> ld(const void* base, long k)
    {
        const _Float16* p = reinterpret_cast<const _Float16*>(base) + 2 * k;
        return {(float)p[0], (float)p[1]};
    }
    __device__ static void st(void* base, long k, cx<float> z)
    {
        _Float16* p = reinterpret_cast<_Float16*>(base) + 2 * k;
        p[0] = (_Float16)z.re;
        p[1] = (_Float16)z.im;
    }
    __device__ static cx<float> rt(cx<float> z) { return {(float)(_Float16)z.re, (float)(_Float16)z.im}; }
    __device__ static float ldr(const void* base, long k) { return (float)reinterpret_cast<const _Float16*>(base)[k]; }
    __device__ static void str(void* base, long k, float v) { reinterpret_cast<_Float16*>(base)[k] = (_Float16)v; }
};

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
struct Geom {
    int Lx, Ly, Lz, Lt;
    int Lxh;   // Lx / 2
    int Vh;    // sites per parity
    int t_bc;  // +1 / -1
    double xs = 1.0;  // weight of the spatial hops (nu / xi_0 for the anisotropic action, Sec. III.B)
};

// real index of entry m (reordered packing) of chirality block chi at `site` in an internal
// clover-type array of one parity, and the array's length in reals
constexpr int CLOV_STRIDE = 1;  // distance between consecutive entries of one matrix
__host__ __device__ inline long clov_index(int site, int chi, int m) { return ((long)site * 2 + chi) * 36 + m; }
__host__ __device__ inline long clov_reals(long Vh) { return 72L * Vh; }

// Complex index of (spin s, site, colour c) in an internal spinor of one parity of Vh sites.  Fields
// of several planes (stacks of parities, learned-net channels) use the same order with s the plane
// index.  Spin-major with colour innermost ([4][Vh][3]: a lane's spin of one site is 3 contiguous
// complex), or with QCDW_SPINOR_SOA=1 one plane per (spin, colour) ([4][3][Vh]: the sites of a wave
// read one contiguous run per load instruction).
#ifndef QCDW_SPINOR_SOA
#define QCDW_SPINOR_SOA 0
#endif
__host__ __device__ inline long sp_idx(long s, long site, int c, long Vh)
{
    return QCDW_SPINOR_SOA ? (s * 3 + c) * Vh + site : (s * Vh + site) * 3 + c;
}
// inverse of sp_idx: (s, site, c) of complex element e
__host__ __device__ inline void sp_coords(long e, long Vh, long& s, long& site, int& c)
{
    if (QCDW_SPINOR_SOA) {
        site = e % Vh;
        const long r = e / Vh;
        c = (int)(r % 3);
        s = r / 3;
    } else {
        c = (int)(e % 3);
        const long r = e / 3;
        site = r % Vh;
        s = r / Vh;
    }
}

// Internal gauge field of R complex entries per link (R = 6: the first two rows, R = 9: all), by
// direction mu and parity p.  Entry j of link (mu, p, site) sits at link_base(mu, p, site) +
// j * link_stride: link-major ([mu][p][Vh][R]), or site-fastest ([mu][p][R][Vh]), where the 16 sites
// of a wave read one contiguous run per entry instead of 16 records 6 entries apart.  The layout
// follows the storage precision: site-fastest in FP64 (the hop measured 5-7 % faster at 24^3 x 64),
// link-major in FP32 and 16-bit storage (a link's entries are fetched by wide per-lane loads there;
// site-fastest measured 10-20 % slower in BF16).  QCDW_LINK_SOA = 0 / 1 forces one layout for all.
#ifndef QCDW_LINK_SOA
#define QCDW_LINK_SOA -1
#endif
__host__ __device__ constexpr bool link_soa_for(int cbytes)
{
    return QCDW_LINK_SOA < 0 ? cbytes == 16 : QCDW_LINK_SOA != 0;
}
__host__ __device__ inline long link_base(int mu, int p, long site, long Vh, int R, bool soa)
{
    return soa ? (long)(mu * 2 + p) * R * Vh + site : ((long)(mu * 2 + p) * Vh + site) * R;
}
__host__ __device__ inline long link_stride(long Vh, bool soa) { return soa ? Vh : 1; }

// coordinates of checkerboard index i on parity p
__device__ __forceinline__ void site_coords(const Geom& g, int i, int p, int& x, int& y, int& z, int& t)
{
    int xh = i % g.Lxh;
    int r = i / g.Lxh;
    y = r % g.Ly;
    r /= g.Ly;
    z = r % g.Lz;
    t = r / g.Lz;
    x = 2 * xh + ((p + y + z + t) & 1);
}

// ---------------------------------------------------------------------------
// block mapping: consecutive logical tiles on one XCD (workgroups are
// dispatched round-robin over the 8 XCDs, each with its own L2)
// ---------------------------------------------------------------------------
#ifndef QCDW_XCD_REMAP
#define QCDW_XCD_REMAP 1
#endif
__device__ __forceinline__ int xcd_tile(int b, int nblk)
{
#if !QCDW_XCD_REMAP
    return b;
#endif
    const int nx = 8;
    int per = nblk / nx, rem = nblk % nx;
    int xcd = b % nx, k = b / nx;
    return xcd * per + (xcd < rem ? xcd : rem) + k;
}

// ---------------------------------------------------------------------------
// deterministic reductions (fixed lane/wave order)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum K values over a 256-thread block; thread 0 writes them to out[0..K).
template <int K>
__device__ __forceinline__ void block_sum_store(double (&v)[K], double* out)
{
    __shared__ double red[4][K];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; k++) v[k] = wave_sum(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; k++) red[wv][k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; k++) out[k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
    }
}

}  // namespace qcdw
