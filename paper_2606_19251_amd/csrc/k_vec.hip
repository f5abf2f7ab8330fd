// Streaming vector kernels, deterministic reductions and the scalar steps of the outer
// FP64 loops. Reductions always use kReduceBlocks workgroups with a grid-stride loop and
// a fixed combination tree, so every sum is bitwise reproducible from run to run.
#include <cmath>

#include "kernels.hpp"

namespace amgg {

namespace {

inline dim3 grid_for(int64_t n) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    return dim3(static_cast<unsigned>(g));
}

__device__ __forceinline__ void block_partial(double v, double* partial) {
    __shared__ double red[kBlock / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x / 64] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = red[0];
        for (int k = 1; k < kBlock / 64; ++k) s += red[k];
        partial[blockIdx.x] = s;
    }
}

// Sum of `count` partials by one workgroup, in a fixed order.
// Sum of count partials by one workgroup of kFinish threads: each thread keeps eight
// independent accumulators (eight loads in flight) over a fixed strided subset, then a
// fixed-order tree; the result does not depend on timing.
constexpr int kFinish = 1024;

__device__ __forceinline__ double sum_partials(const double* partial, int count = kReduceBlocks) {
    __shared__ double red[kFinish];
    double v[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int k = threadIdx.x;
    for (; k + 7 * kFinish < count; k += 8 * kFinish) {
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] += partial[k + q * kFinish];
    }
#pragma unroll
    for (int q = 0; q < 7; ++q)
        if (k + q * kFinish < count) v[q] += partial[k + q * kFinish];
    red[threadIdx.x] = ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
    __syncthreads();
    for (int w = kFinish / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    return red[0];
}

template <typename T>
__global__ void mul_kernel(int32_t n, const T* __restrict__ a, const T* __restrict__ b, T* __restrict__ y) {
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) y[i] = a[i] * b[i];
}

template <typename T>
__global__ void copy_kernel(int32_t n, const T* __restrict__ a, T* __restrict__ y) {
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) y[i] = a[i];
}

__global__ void zero_kernel(uint32_t* __restrict__ p, int64_t words) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i < words) p[i] = 0u;
}

template <bool DIAG>
__global__ void cast_scaled_kernel(int32_t n, const double* __restrict__ x, const double* __restrict__ scale,
                                   float* __restrict__ y, const float* __restrict__ d, float* __restrict__ u) {
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const float yi = static_cast<float>(x[i] * scale[0]);
    y[i] = yi;
    if constexpr (DIAG) u[i] = d[i] * yi;
}

__global__ void cast_scale_kernel(int64_t n, const double* __restrict__ x, double scale, float* __restrict__ y) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i < n) y[i] = static_cast<float>(x[i] * scale);
}

// out[r][k] = (float)(in[r][k] * gscale[group[r]]) (group NULL: group 0 for every row)
__global__ void cast_scale_rows_kernel(int32_t nrows, int32_t ncols, const double* __restrict__ in,
                                       const int32_t* __restrict__ group, const double* __restrict__ gscale,
                                       float* __restrict__ out) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= static_cast<int64_t>(nrows) * ncols) return;
    const int32_t r = static_cast<int32_t>(i / ncols);
    out[i] = static_cast<float>(in[i] * gscale[group ? group[r] : 0]);
}

// out[0] = (sum_i (a[i] - b[i])) / n, summed in index order by one thread (n is a handful of
// problems: the validation meshes of a training run).
__global__ void mean_difference_kernel(int32_t n, const double* __restrict__ a, const double* __restrict__ b,
                                       double* __restrict__ out) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double s = 0.0;
    for (int32_t i = 0; i < n; ++i) s += a[i] - b[i];
    out[0] = s / n;
}

__global__ void cast_d2f_kernel(int32_t n, const double* __restrict__ x, float* __restrict__ y) {
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) y[i] = static_cast<float>(x[i]);
}

__global__ void cast_f2d_kernel(int32_t n, const float* __restrict__ x, double* __restrict__ y) {
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) y[i] = static_cast<double>(x[i]);
}

__global__ void sub_mean_kernel(int32_t n, const double* __restrict__ x, const double* __restrict__ sum,
                                double* __restrict__ y) {
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) y[i] = x[i] - sum[0] / static_cast<double>(n);
}

__global__ __launch_bounds__(kBlock) void partial_dot_kernel(int32_t n, const double* __restrict__ a,
                                                            const double* __restrict__ b,
                                                            double* __restrict__ partial) {
    double v = 0.0;
    for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += kReduceBlocks * kBlock) v += a[i] * b[i];
    block_partial(v, partial);
}

__global__ __launch_bounds__(kBlock) void partial_sum_kernel(int32_t n, const double* __restrict__ a,
                                                            double* __restrict__ partial) {
    double v = 0.0;
    for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += kReduceBlocks * kBlock) v += a[i];
    block_partial(v, partial);
}

__global__ __launch_bounds__(kFinish) void finish_sum_kernel(const double* __restrict__ partial,
                                                           double* __restrict__ out) {
    const double s = sum_partials(partial);
    if (threadIdx.x == 0) out[0] = s;
}

__global__ __launch_bounds__(kFinish) void fcg_finish_pq_kernel(const double* __restrict__ partial, int count,
                                                              double* __restrict__ s) {
    const double pq = sum_partials(partial, count);
    if (threadIdx.x == 0) {
        s[kPQ] = pq;
        if (!(pq > 0.0)) s[kFlag] = 1.0;
        s[kAlpha] = s[kGamma] / pq;
    }
}

__global__ __launch_bounds__(kBlock) void fcg_update_xr_kernel(int32_t n, double* __restrict__ x,
                                                              const double* __restrict__ p,
                                                              const double* __restrict__ r,
                                                              const double* __restrict__ q,
                                                              double* __restrict__ rnew,
                                                              const double* __restrict__ s,
                                                              double* __restrict__ partial, Cast32 cs) {
    if (s[kHalt] != 0.0 || s[kFlag] != 0.0) return;  // uniform over the grid
    const double a = s[kAlpha];
    const double sc = cs.f ? s[kScaleNext] : 0.0;
    double v = 0.0;
    for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += kReduceBlocks * kBlock) {
        x[i] += a * p[i];
        const double ri = r[i] - a * q[i];
        rnew[i] = ri;
        v += ri * ri;
        if (cs.f) {  // the next cycle's FP32 right-hand side (uniform branch)
            const float fy = static_cast<float>(ri * sc);
            cs.f[i] = fy;
            if (cs.qd) cs.u[i] = cs.qd[i] * fy;
        }
    }
    block_partial(v, partial);
}

__global__ __launch_bounds__(kFinish) void fcg_finish_rr_kernel(const double* __restrict__ partial, int count,
                                                              double* __restrict__ s) {
    const double rr = sum_partials(partial, count);
    if (threadIdx.x == 0) {
        s[kRR] = rr;
        const double nrm = sqrt(rr);
        s[kNorm] = nrm;
        s[kInvNorm] = nrm > 0.0 ? 1.0 / nrm : 0.0;
    }
}

__global__ __launch_bounds__(kBlock) void fcg_castback_dots_kernel(int32_t n, const float* __restrict__ u32,
                                                                  const double* __restrict__ s,
                                                                  const double* __restrict__ rnew,
                                                                  const double* __restrict__ rold,
                                                                  double* __restrict__ z,
                                                                  double* __restrict__ partial2) {
    const double nrm = s[kUnscale];
    double a = 0.0, b = 0.0;
    for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += kReduceBlocks * kBlock) {
        const double zi = static_cast<double>(u32[i]) * nrm;
        if (z) z[i] = zi;
        a += zi * rnew[i];
        if (rold) b += zi * rold[i];
    }
    block_partial(a, partial2);
    __syncthreads();
    block_partial(b, partial2 + kReduceBlocks);
}

__global__ __launch_bounds__(kBlock) void fcg_dots64_kernel(int32_t n, const double* __restrict__ z,
                                                           const double* __restrict__ rnew,
                                                           const double* __restrict__ rold,
                                                           double* __restrict__ partial2) {
    double a = 0.0, b = 0.0;
    for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += kReduceBlocks * kBlock) {
        a += z[i] * rnew[i];
        if (rold) b += z[i] * rold[i];
    }
    block_partial(a, partial2);
    __syncthreads();
    block_partial(b, partial2 + kReduceBlocks);
}

__global__ __launch_bounds__(kFinish) void fcg_finish_beta_kernel(const double* __restrict__ partial2,
                                                                double* __restrict__ s, int first) {
    const double zr = sum_partials(partial2);
    __syncthreads();
    const double zro = sum_partials(partial2 + kReduceBlocks);
    if (threadIdx.x == 0) {
        s[kZR] = zr;
        s[kZRold] = zro;
        if (!(zr > 0.0)) s[kFlag] = 1.0;
        s[kBeta] = first ? 0.0 : (zr - zro) / s[kGamma];
        s[kGamma] = zr;
    }
}

__global__ void fcg_update_p_kernel(int32_t n, const double* __restrict__ z, double* __restrict__ p,
                                    const double* __restrict__ s, int first) {
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = first ? z[i] : z[i] + s[kBeta] * p[i];
}

// The same with z formed from the FP32 cycle output as fcg_castback_dots forms it (not stored).
__global__ void fcg_update_p32_kernel(int32_t n, const float* __restrict__ u32, double* __restrict__ p,
                                      const double* __restrict__ s, int first) {
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) {
        const double zi = static_cast<double>(u32[i]) * s[kUnscale];
        p[i] = first ? zi : zi + s[kBeta] * p[i];
    }
}

__global__ void ir_update_f32_kernel(int32_t n, double* __restrict__ x, const float* __restrict__ u32,
                                     const double* __restrict__ s) {
    if (s[kHalt] != 0.0) return;
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) x[i] += static_cast<double>(u32[i]) * s[kUnscale];
}

// 2^-e with e the binary exponent of v (v in [2^e, 2^(e+1))); 1 for v = 0 or non-finite v
__device__ __forceinline__ double pow2_scale(double v) {
    return v > 0.0 && v <= 1.7976931348623157e308 ? ldexp(1.0, -ilogb(v)) : 1.0;
}

__device__ __forceinline__ void set_scales(double* s, double next, double cast) {
    s[kScaleNext] = next;
    s[kScaleCast] = cast;
    s[kUnscale] = 1.0 / cast;  // exact: cast is a power of two
}

__global__ void ir_set_scales_kernel(double* __restrict__ s) {
    if (threadIdx.x == 0) {
        const double sc = pow2_scale(s[kNorm]);
        set_scales(s, sc, sc);
    }
}

__global__ void ir_update_f64_kernel(int32_t n, double* __restrict__ x, const double* __restrict__ e,
                                     const double* __restrict__ s) {
    if (s[kHalt] != 0.0) return;
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) x[i] += e[i];
}

__global__ void fcg_set_limits_kernel(double* __restrict__ s, double tol2, double div2) {
    if (threadIdx.x == 0) {
        s[kTolRR] = tol2 * s[kRR];
        s[kDivRR] = div2 * s[kRR];
        s[kHalt] = 0.0;
        s[kFlag] = 0.0;
        const double sc = pow2_scale(sqrt(s[kRR]));
        set_scales(s, sc, sc);
    }
}

__global__ void fcg_clear_halt_kernel(double* __restrict__ s) {
    if (threadIdx.x == 0) {
        s[kHalt] = 0.0;
        s[kFlag] = 0.0;
    }
}

__global__ __launch_bounds__(kFinish) void fcg_finish_rr_guarded_kernel(const double* __restrict__ partial, int count,
                                                                      double* __restrict__ s) {
    if (s[kHalt] != 0.0 || s[kFlag] != 0.0) return;
    const double rr = sum_partials(partial, count);
    if (threadIdx.x == 0) {
        s[kRR] = rr;
        const double nrm = sqrt(rr);
        s[kNorm] = nrm;
        s[kInvNorm] = nrm > 0.0 ? 1.0 / nrm : 0.0;
        if (rr <= s[kTolRR] || !(rr <= s[kDivRR])) s[kHalt] = 1.0;
        set_scales(s, pow2_scale(nrm), s[kScaleNext]);
    }
}

}  // namespace

template <typename T>
hipError_t vec_mul(int32_t n, const T* a, const T* b, T* y, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    mul_kernel<T><<<grid_for(n), kBlock, 0, stream>>>(n, a, b, y);
    return hipGetLastError();
}
template hipError_t vec_mul<float>(int32_t, const float*, const float*, float*, hipStream_t);
template hipError_t vec_mul<double>(int32_t, const double*, const double*, double*, hipStream_t);

template <typename T>
hipError_t vec_copy(int32_t n, const T* a, T* y, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    copy_kernel<T><<<grid_for(n), kBlock, 0, stream>>>(n, a, y);
    return hipGetLastError();
}
template hipError_t vec_copy<float>(int32_t, const float*, float*, hipStream_t);
template hipError_t vec_copy<double>(int32_t, const double*, double*, hipStream_t);
template hipError_t vec_copy<int32_t>(int32_t, const int32_t*, int32_t*, hipStream_t);

hipError_t vec_zero_bytes(void* p, size_t bytes, hipStream_t stream) {
    // a fill kernel rather than a memset node keeps the cycle capturable in a graph
    const int64_t words = static_cast<int64_t>((bytes + 3) / 4);
    if (words <= 0) return hipSuccess;
    zero_kernel<<<grid_for(words), kBlock, 0, stream>>>(static_cast<uint32_t*>(p), words);
    return hipGetLastError();
}

hipError_t cast_scaled_f64_f32(int32_t n, const double* x, const double* scale, float* y, hipStream_t stream,
                               const float* d, float* u) {
    if (n <= 0) return hipSuccess;
    if ((d == nullptr) != (u == nullptr)) return hipErrorInvalidValue;
    if (d)
        cast_scaled_kernel<true><<<grid_for(n), kBlock, 0, stream>>>(n, x, scale, y, d, u);
    else
        cast_scaled_kernel<false><<<grid_for(n), kBlock, 0, stream>>>(n, x, scale, y, nullptr, nullptr);
    return hipGetLastError();
}

hipError_t cast_scale_f64_f32(int64_t n, const double* x, double scale, float* y, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    cast_scale_kernel<<<grid_for(n), kBlock, 0, stream>>>(n, x, scale, y);
    return hipGetLastError();
}

hipError_t cast_scale_rows_f64_f32(int32_t nrows, int32_t ncols, const double* in, const int32_t* group,
                                   const double* gscale, float* out, hipStream_t stream) {
    const int64_t total = static_cast<int64_t>(nrows) * ncols;
    if (total <= 0) return hipSuccess;
    cast_scale_rows_kernel<<<grid_for(total), kBlock, 0, stream>>>(nrows, ncols, in, group, gscale, out);
    return hipGetLastError();
}

hipError_t mean_difference(int32_t n, const double* a, const double* b, double* out, hipStream_t stream) {
    mean_difference_kernel<<<1, 64, 0, stream>>>(n, a, b, out);
    return hipGetLastError();
}

hipError_t cast_f64_f32(int32_t n, const double* x, float* y, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    cast_d2f_kernel<<<grid_for(n), kBlock, 0, stream>>>(n, x, y);
    return hipGetLastError();
}

hipError_t cast_f32_f64(int32_t n, const float* x, double* y, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    cast_f2d_kernel<<<grid_for(n), kBlock, 0, stream>>>(n, x, y);
    return hipGetLastError();
}

hipError_t sub_mean(int32_t n, const double* x, const double* sum, double* y, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    sub_mean_kernel<<<grid_for(n), kBlock, 0, stream>>>(n, x, sum, y);
    return hipGetLastError();
}

hipError_t partial_dot(int32_t n, const double* a, const double* b, double* partial, hipStream_t stream) {
    partial_dot_kernel<<<kReduceBlocks, kBlock, 0, stream>>>(n, a, b, partial);
    return hipGetLastError();
}

hipError_t partial_sum(int32_t n, const double* a, double* partial, hipStream_t stream) {
    partial_sum_kernel<<<kReduceBlocks, kBlock, 0, stream>>>(n, a, partial);
    return hipGetLastError();
}

hipError_t finish_sum(const double* partial, double* out, hipStream_t stream) {
    finish_sum_kernel<<<1, kFinish, 0, stream>>>(partial, out);
    return hipGetLastError();
}

hipError_t fcg_finish_pq(const double* partial, int count, double* s, hipStream_t stream) {
    fcg_finish_pq_kernel<<<1, kFinish, 0, stream>>>(partial, count, s);
    return hipGetLastError();
}

hipError_t fcg_update_xr(int32_t n, double* x, const double* p, const double* r, const double* q, double* rnew,
                         const double* s, double* partial, hipStream_t stream, const Cast32& cast) {
    if ((cast.qd == nullptr) != (cast.u == nullptr)) return hipErrorInvalidValue;
    fcg_update_xr_kernel<<<kReduceBlocks, kBlock, 0, stream>>>(n, x, p, r, q, rnew, s, partial, cast);
    return hipGetLastError();
}

hipError_t fcg_finish_rr(const double* partial, int count, double* s, hipStream_t stream) {
    fcg_finish_rr_kernel<<<1, kFinish, 0, stream>>>(partial, count, s);
    return hipGetLastError();
}

hipError_t fcg_castback_dots(int32_t n, const float* u32, const double* s, const double* rnew, const double* rold,
                             double* z, double* partial2, hipStream_t stream) {
    fcg_castback_dots_kernel<<<kReduceBlocks, kBlock, 0, stream>>>(n, u32, s, rnew, rold, z, partial2);
    return hipGetLastError();
}

hipError_t fcg_dots64(int32_t n, const double* z, const double* rnew, const double* rold, double* partial2,
                      hipStream_t stream) {
    fcg_dots64_kernel<<<kReduceBlocks, kBlock, 0, stream>>>(n, z, rnew, rold, partial2);
    return hipGetLastError();
}

hipError_t fcg_finish_beta(const double* partial2, double* s, int first, hipStream_t stream) {
    fcg_finish_beta_kernel<<<1, kFinish, 0, stream>>>(partial2, s, first);
    return hipGetLastError();
}

hipError_t fcg_update_p(int32_t n, const double* z, double* p, const double* s, int first, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    fcg_update_p_kernel<<<grid_for(n), kBlock, 0, stream>>>(n, z, p, s, first);
    return hipGetLastError();
}

hipError_t fcg_update_p32(int32_t n, const float* u32, double* p, const double* s, int first, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    fcg_update_p32_kernel<<<grid_for(n), kBlock, 0, stream>>>(n, u32, p, s, first);
    return hipGetLastError();
}

hipError_t ir_update_f32(int32_t n, double* x, const float* u32, const double* s, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    ir_update_f32_kernel<<<grid_for(n), kBlock, 0, stream>>>(n, x, u32, s);
    return hipGetLastError();
}

hipError_t fcg_set_limits(double* s, double tol, double div, hipStream_t stream) {
    fcg_set_limits_kernel<<<1, 64, 0, stream>>>(s, tol * tol, div * div);
    return hipGetLastError();
}

hipError_t fcg_clear_halt(double* s, hipStream_t stream) {
    fcg_clear_halt_kernel<<<1, 64, 0, stream>>>(s);
    return hipGetLastError();
}

hipError_t ir_set_scales(double* s, hipStream_t stream) {
    ir_set_scales_kernel<<<1, 64, 0, stream>>>(s);
    return hipGetLastError();
}

hipError_t fcg_finish_rr_guarded(const double* partial, int count, double* s, hipStream_t stream) {
    fcg_finish_rr_guarded_kernel<<<1, kFinish, 0, stream>>>(partial, count, s);
    return hipGetLastError();
}

hipError_t ir_update_f64(int32_t n, double* x, const double* e, const double* s, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    ir_update_f64_kernel<<<grid_for(n), kBlock, 0, stream>>>(n, x, e, s);
    return hipGetLastError();
}

}  // namespace amgg
