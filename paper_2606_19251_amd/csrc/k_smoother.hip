// Sparse pseudo-inverse smoother assembly (paper Sec. 3.1, Eq. 5):
//   q_ii = f_d(a_ii/s) / a_ii,   q_ij = f_o(a_ij/s) / (a_ii + a_jj),   s = max |offdiag(A)|,
//   f_d(x) = d0 + x(d1 + x(d2 + ...)),   f_o(x) = x(o1 + x(o2 + ...)).
// Evaluated in FP64 with Horner's rule, each operation rounded on its own (this file is
// built with -ffp-contract=off and the pragma below) and IEEE division, so the values
// are reproducible bit for bit by any implementation that follows the same order.
// One thread per row: the entries of a row are contiguous, and the diagonal of the
// neighbour j is a gather from the level's diagonal array.
#include "kernels.hpp"

namespace amgg {

namespace {

__device__ __forceinline__ double horner_diag(double x, const double* c, int deg) {
#pragma clang fp contract(off)
    double t = c[deg];
    for (int k = deg - 1; k >= 0; --k) t = c[k] + x * t;
    return t;
}

__device__ __forceinline__ double horner_off(double x, const double* o, int deg) {
#pragma clang fp contract(off)
    // o[0] = o1 ... o[deg-1] = o_deg
    double t = o[deg - 1];
    for (int k = deg - 2; k >= 0; --k) t = o[k] + x * t;
    return x * t;
}

// Row i of Q and of its diagonal with coefficients c[0..2deg] and scale s.
__device__ __forceinline__ void assemble_row(int32_t i, const int32_t* __restrict__ ptr,
                                             const int32_t* __restrict__ col, const double* __restrict__ val,
                                             const double* __restrict__ diag, const double* c, int deg, double s,
                                             double* __restrict__ q64, float* __restrict__ q32,
                                             double* __restrict__ qd64, float* __restrict__ qd32) {
#pragma clang fp contract(off)
    const double aii = diag[i];
    const int32_t pb = ptr[i], pe = ptr[i + 1];
    // eight entries at a time: their columns and values, then the neighbours' diagonals, are
    // loaded together (a past-the-end slot re-reads the row's last entry and is not stored)
    constexpr int kE = 8;
    for (int32_t base = pb; base < pe; base += kE) {
        int32_t j[kE];
        double a[kE], dj[kE];
#pragma unroll
        for (int q = 0; q < kE; ++q) {
            const int32_t p = min(base + q, pe - 1);
            j[q] = col[p];
            a[q] = val[p];
        }
#pragma unroll
        for (int q = 0; q < kE; ++q) dj[q] = diag[j[q]];
#pragma unroll
        for (int q = 0; q < kE; ++q) {
            const int32_t p = base + q;
            if (p < pe) {
                const double x = a[q] / s;
                double v;
                if (j[q] == i) {
                    v = horner_diag(x, c, deg) / a[q];
                    qd64[i] = v;
                    qd32[i] = static_cast<float>(v);
                } else {
                    v = horner_off(x, c + deg + 1, deg) / (aii + dj[q]);
                }
                q64[p] = v;
                q32[p] = static_cast<float>(v);
            }
        }
    }
}

__global__ __launch_bounds__(kBlock) void assemble_kernel(int32_t n, const int32_t* __restrict__ ptr,
                                                         const int32_t* __restrict__ col,
                                                         const double* __restrict__ val,
                                                         const double* __restrict__ diag,
                                                         const double* __restrict__ scale, PolyCoeffs pc,
                                                         const float* __restrict__ coeffs_dev,
                                                         double* __restrict__ q64, float* __restrict__ q32,
                                                         double* __restrict__ qd64, float* __restrict__ qd32) {
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int deg = pc.degree;
    double c[2 * 4 + 1];
    for (int k = 0; k < 2 * deg + 1; ++k) c[k] = coeffs_dev ? static_cast<double>(coeffs_dev[k]) : pc.c[k];
    assemble_row(i, ptr, col, val, diag, c, deg, scale[0], q64, q32, qd64, qd32);
}

__global__ __launch_bounds__(kBlock) void assemble_blocks_kernel(
    int32_t n, const int32_t* __restrict__ ptr, const int32_t* __restrict__ col, const double* __restrict__ val,
    const double* __restrict__ diag, int32_t nblk, const int32_t* __restrict__ off, const double* __restrict__ scale,
    const int32_t* __restrict__ crow, PolyCoeffs pc, const float* __restrict__ coeffs_dev, int32_t stride,
    double* __restrict__ q64, float* __restrict__ q32, double* __restrict__ qd64, float* __restrict__ qd32) {
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int32_t lo = 0, hi = nblk - 1;  // block of row i
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) / 2;
        if (off[mid] <= i)
            lo = mid;
        else
            hi = mid - 1;
    }
    const int deg = pc.degree;
    const int32_t r = crow[lo];
    double c[2 * 4 + 1];
    for (int k = 0; k < 2 * deg + 1; ++k)
        c[k] = r < 0 ? 0.0 : coeffs_dev ? static_cast<double>(coeffs_dev[static_cast<int64_t>(r) * stride + k]) : pc.c[k];
    assemble_row(i, ptr, col, val, diag, c, deg, scale[lo], q64, q32, qd64, qd32);
}

}  // namespace

hipError_t assemble_smoother(int32_t n, const int32_t* ptr, const int32_t* col, const double* val,
                             const double* diag, const double* scale, const PolyCoeffs& pc,
                             const float* coeffs_dev, double* q64, float* q32, double* qd64, float* qd32,
                             hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    if (pc.degree < 1 || pc.degree > 4) return hipErrorInvalidValue;
    const dim3 grid(static_cast<unsigned>((n + kBlock - 1) / kBlock));
    assemble_kernel<<<grid, kBlock, 0, stream>>>(n, ptr, col, val, diag, scale, pc, coeffs_dev, q64, q32, qd64,
                                                  qd32);
    return hipGetLastError();
}

hipError_t assemble_smoother_blocks(int32_t n, const int32_t* ptr, const int32_t* col, const double* val,
                                    const double* diag, int32_t nblk, const int32_t* off, const double* scale,
                                    const int32_t* crow, const PolyCoeffs& pc, const float* coeffs_dev,
                                    int32_t stride, double* q64, float* q32, double* qd64, float* qd32,
                                    hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    if (pc.degree < 1 || pc.degree > 4 || nblk < 1) return hipErrorInvalidValue;
    const dim3 grid(static_cast<unsigned>((n + kBlock - 1) / kBlock));
    assemble_blocks_kernel<<<grid, kBlock, 0, stream>>>(n, ptr, col, val, diag, nblk, off, scale, crow, pc, coeffs_dev,
                                                         stride, q64, q32, qd64, qd32);
    return hipGetLastError();
}

}  // namespace amgg
