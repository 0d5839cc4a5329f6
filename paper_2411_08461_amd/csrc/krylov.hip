// Block Gram-Schmidt kernels for flexible GMRES (Saad 1993): several dot
// products against one vector in a single pass, and a combined update
// w += sign * sum_i c_i V_i.  Vectors are FP64 complex; V_i = V + i * stride.
// Reductions use a fixed order, so results are bitwise reproducible.
#include "internal.h"

namespace qcdw {

constexpr int MDOT_GROUP = 8;  // vectors per pass

// partials[(group * nb + block) * 16 + 2 j + {0,1}] = partial sum of conj(V_{8 group + j}) w
__global__ __launch_bounds__(256) void k_multidot(const double2* V, long stride, int nvec, const double2* w, long n,
                                                  double* partials)
{
    const int i0 = blockIdx.y * MDOT_GROUP;
    const int cnt = min(MDOT_GROUP, nvec - i0);
    double acc[2 * MDOT_GROUP];
#pragma unroll
    for (int j = 0; j < 2 * MDOT_GROUP; j++) acc[j] = 0.0;
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long)gridDim.x * 256) {
        const double2 we = w[e];
#pragma unroll
        for (int j = 0; j < MDOT_GROUP; j++) {
            if (j < cnt) {
                const double2 v = V[(long)(i0 + j) * stride + e];
                acc[2 * j] += v.x * we.x + v.y * we.y;
                acc[2 * j + 1] += v.x * we.y - v.y * we.x;
            }
        }
    }
    block_sum_store<2 * MDOT_GROUP>(acc, partials + ((long)blockIdx.y * gridDim.x + blockIdx.x) * 2 * MDOT_GROUP);
}

// out[2 i + {0,1}] = sum over blocks, i < nvec
__global__ __launch_bounds__(256) void k_multidot_sum(const double* partials, int nb, int nvec, double* out)
{
    const int e = blockIdx.x;  // 0 .. 2*8-1 within the group
    const int group = blockIdx.y;
    const int i = group * MDOT_GROUP + e / 2;
    double v[1] = {0.0};
    for (int b = threadIdx.x; b < nb; b += 256) v[0] += partials[((long)group * nb + b) * 2 * MDOT_GROUP + e];
    __shared__ double res[1];
    block_sum_store<1>(v, res);
    __syncthreads();
    if (threadIdx.x == 0 && i < nvec) out[2 * i + (e & 1)] = res[0];
}

// w += sign * sum_i c_i V_i
__global__ __launch_bounds__(256) void k_multiaxpy(const double2* V, long stride, int nvec, const double* c,
                                                   double2* w, long n, double sign)
{
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long)gridDim.x * 256) {
        double2 acc = w[e];
        for (int i = 0; i < nvec; i++) {
            const double2 v = V[(long)i * stride + e];
            const double cr = sign * c[2 * i], ci = sign * c[2 * i + 1];
            acc.x += cr * v.x - ci * v.y;
            acc.y += cr * v.y + ci * v.x;
        }
        w[e] = acc;
    }
}

// out = w / sqrt(*nrm2) (out = 0 if the norm is zero)
__global__ __launch_bounds__(256) void k_scale_inv_norm(const double2* w, double2* out, long n, const double* nrm2)
{
    const double q = *nrm2;
    const double sc = q > 0.0 ? 1.0 / sqrt(q) : 0.0;
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long)gridDim.x * 256) {
        const double2 v = w[e];
        out[e] = make_double2(sc * v.x, sc * v.y);
    }
}

hipError_t launch_scale_inv_norm(hipStream_t s, const void* w, void* out, long n, const double* nrm2)
{
    hipLaunchKernelGGL(k_scale_inv_norm, dim3(blas_blocks(n)), dim3(256), 0, s, (const double2*)w, (double2*)out, n,
                       nrm2);
    return hipGetLastError();
}

hipError_t launch_multidot(hipStream_t s, const void* V, long stride, int nvec, const void* w, long n,
                           double* partials, double* out)
{
    if (nvec <= 0) return hipSuccess;
    const int ng = (nvec + MDOT_GROUP - 1) / MDOT_GROUP;
    const int nb = blas_blocks(n);
    hipLaunchKernelGGL(k_multidot, dim3(nb, ng), dim3(256), 0, s, (const double2*)V, stride, nvec, (const double2*)w,
                       n, partials);
    hipLaunchKernelGGL(k_multidot_sum, dim3(2 * MDOT_GROUP, ng), dim3(256), 0, s, partials, nb, nvec, out);
    return hipGetLastError();
}

hipError_t launch_multiaxpy(hipStream_t s, const void* V, long stride, int nvec, const double* c, void* w, long n,
                            double sign)
{
    if (nvec <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_multiaxpy, dim3(blas_blocks(n)), dim3(256), 0, s, (const double2*)V, stride, nvec, c,
                       (double2*)w, n, sign);
    return hipGetLastError();
}

}  // namespace qcdw
