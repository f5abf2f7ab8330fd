// Sparse pseudo-inverse smoother assembly (paper Sec. 3.1, Eq. 5):
//   q_ii = f_d(a_ii/s) / a_ii,   q_ij = f_o(a_ij/s) / (a_ii + a_jj),   s = max |offdiag(A)|,
//   f_d(x) = d0 + x(d1 + x(d2 + ...)),   f_o(x) = x(o1 + x(o2 + ...)).
// Evaluated in FP64 with Horner's rule, each operation rounded on its own (this file is
// built with -ffp-contract=off and the pragma below) and IEEE division, so the values
// are reproducible bit for bit by any implementation that follows the same order.
// The entries are streamed per block of rows with the row data (coefficients, scale, a_ii) in
// LDS; the diagonal of the neighbour j is a gather from the level's diagonal array.
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

constexpr int kAsmCap = 4096;  // entries of a workgroup's rows staged through LDS
constexpr int kAsmChunk = 4;   // entries per thread per round

// A workgroup owns kBlock consecutive rows. Each thread first forms its row's coefficients,
// scale and diagonal (the per-row data of Eq. 5) in LDS and marks the row's entries with its
// local row index; the block's entries are then streamed with unit stride (coalesced column,
// value and output streams), each entry taking its row's data from LDS. The arithmetic per
// entry is the per-row form's (assemble_row), so the values are the same bit for bit; a block
// whose entries overflow the LDS map falls back to one thread per row.
// BLOCKS: block-diagonal level (coefficient row and scale of the row's block, a coefficient
// row < 0 gives zero coefficients); else one coefficient set and scale[0].
template <bool BLOCKS>
__global__ __launch_bounds__(kBlock) void assemble_stream_kernel(
    int32_t n, const int32_t* __restrict__ ptr, const int32_t* __restrict__ col, const double* __restrict__ val,
    const double* __restrict__ diag, int32_t nblk, const int32_t* __restrict__ off, const double* __restrict__ scale,
    const int32_t* __restrict__ crow, PolyCoeffs pc, const float* __restrict__ coeffs_dev, int32_t stride,
    double* __restrict__ q64, float* __restrict__ q32, double* __restrict__ qd64, float* __restrict__ qd32) {
#pragma clang fp contract(off)
    static_assert(kBlock <= 256, "local row indices are stored in 8 bits");
    __shared__ uint8_t rowof[kAsmCap];
    __shared__ double cs[kBlock][2 * 4 + 1];
    __shared__ double srow[kBlock], arow[kBlock];
    const int deg = pc.degree;
    const int t = static_cast<int>(threadIdx.x);
    const int32_t r0 = static_cast<int32_t>(blockIdx.x) * kBlock;
    const int32_t r1 = min(r0 + kBlock, n);
    const int32_t e0 = ptr[r0];
    const int32_t ne = ptr[r1] - e0;
    const bool fits = ne <= kAsmCap;
    const int32_t i = r0 + t;
    if (i < r1) {
        int32_t b = 0, r = 0;
        if constexpr (BLOCKS) {
            int32_t lo = 0, hi = nblk - 1;  // block of row i
            while (lo < hi) {
                const int32_t mid = (lo + hi + 1) / 2;
                if (off[mid] <= i)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            b = lo;
            r = crow[b];
        }
        for (int k = 0; k < 2 * deg + 1; ++k) {
            if (pc.diag_only && k > deg) {
                cs[t][k] = 0.0;
                continue;
            }
            if constexpr (BLOCKS)
                cs[t][k] = r < 0 ? 0.0
                           : coeffs_dev ? static_cast<double>(coeffs_dev[static_cast<int64_t>(r) * stride + k])
                                        : pc.c[k];
            else
                cs[t][k] = coeffs_dev ? static_cast<double>(coeffs_dev[k]) : pc.c[k];
        }
        srow[t] = scale[b];
        arow[t] = diag[i];
        if (fits)
            for (int32_t k = ptr[i] - e0; k < ptr[i + 1] - e0; ++k) rowof[k] = static_cast<uint8_t>(t);
    }
    __syncthreads();
    if (!fits) {
        if (i < r1) assemble_row(i, ptr, col, val, diag, cs[t], deg, srow[t], q64, q32, qd64, qd32);
        return;
    }
    for (int32_t base = 0; base < ne; base += kAsmChunk * kBlock) {
        int32_t j[kAsmChunk];
        double a[kAsmChunk], dj[kAsmChunk];
#pragma unroll
        for (int q = 0; q < kAsmChunk; ++q) {
            const int32_t k = min(base + t + q * kBlock, ne - 1);
            j[q] = col[e0 + k];
            a[q] = val[e0 + k];
        }
#pragma unroll
        for (int q = 0; q < kAsmChunk; ++q) dj[q] = diag[j[q]];
#pragma unroll
        for (int q = 0; q < kAsmChunk; ++q) {
            const int32_t k = base + t + q * kBlock;
            if (k < ne) {
                const int lr = rowof[k];
                const int32_t row = r0 + lr;
                const double x = a[q] / srow[lr];
                double v;
                if (j[q] == row) {
                    v = horner_diag(x, cs[lr], deg) / a[q];
                    qd64[row] = v;
                    qd32[row] = static_cast<float>(v);
                } else {
                    v = horner_off(x, cs[lr] + deg + 1, deg) / (arow[lr] + dj[q]);
                }
                q64[e0 + k] = v;
                q32[e0 + k] = static_cast<float>(v);
            }
        }
    }
}

}  // namespace

hipError_t assemble_smoother(int32_t n, const int32_t* ptr, const int32_t* col, const double* val,
                             const double* diag, const double* scale, const PolyCoeffs& pc,
                             const float* coeffs_dev, double* q64, float* q32, double* qd64, float* qd32,
                             hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    if (pc.degree < 1 || pc.degree > 4) return hipErrorInvalidValue;
    const dim3 grid(static_cast<unsigned>((n + kBlock - 1) / kBlock));
    assemble_stream_kernel<false><<<grid, kBlock, 0, stream>>>(n, ptr, col, val, diag, 1, nullptr, scale, nullptr, pc,
                                                               coeffs_dev, 0, q64, q32, qd64, qd32);
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
    assemble_stream_kernel<true><<<grid, kBlock, 0, stream>>>(n, ptr, col, val, diag, nblk, off, scale, crow, pc,
                                                              coeffs_dev, stride, q64, q32, qd64, qd32);
    return hipGetLastError();
}

}  // namespace amgg
