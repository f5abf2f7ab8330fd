// Row-wise CSR products on gfx950.
//
// Rows of up to ~32 nonzeros (every level of the P1 and finite-volume hierarchies) use the
// CSR-stream kernel: a workgroup owns a block of consecutive rows, its 256 threads walk the
// block's contiguous nonzeros with unit stride (fully coalesced value and column streams),
// multiply by the gathered x and leave the products in LDS; one thread per row then sums
// its row's products in order and applies the epilogue (residual, smoothing update,
// restriction, prolongation). The rows per block are chosen from the mean row length so
// that a block's nonzeros fit the LDS buffer; a block that still overflows (a long row)
// falls back to a per-thread loop from global memory.
//
// Longer rows use the lane kernel: `LANES` consecutive threads of a 64-wide wavefront own one
// row, stride over its entries and combine their sums with cross-lane shuffles.
//
// The FP64 outer loop's products (q = A p with p^T q, r = b - A x with r^T r) are the same
// stream kernel writing one partial sum per workgroup, reduced afterwards in a fixed order.
#include "kernels.hpp"

namespace amgg {

int lanes_for(int32_t nrows, int32_t nnz) {
    if (nrows <= 0) return 1;
    const double avg = static_cast<double>(nnz) / nrows;
    int l = 1;
    while (l < 64 && l < avg) l <<= 1;
    return l;
}

namespace {

constexpr int kStreamCap = 4096;  // products held in LDS per workgroup

// Rows per stream workgroup for a mean row length, or 0 for the lane kernel.
int stream_rows(int32_t nrows, int32_t nnz) {
    const double avg = nrows > 0 ? static_cast<double>(nnz) / nrows : 0.0;
    for (int r : {256, 128, 64, 32})
        if (r * avg * 1.25 <= kStreamCap) return r;
    return 0;
}

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b runs on XCD b mod 8), each
// with its own L2. Renumber them so that every XCD processes one contiguous range of row
// blocks: neighbouring rows gather neighbouring x entries, which then stay in one L2.
__device__ __forceinline__ int32_t xcd_block() {
    constexpr int32_t kXcd = 8;
    const int32_t b = blockIdx.x, g = gridDim.x;
    const int32_t q = g / kXcd, r = g % kXcd;
    const int32_t x = b % kXcd, k = b / kXcd;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}

template <typename T, int LANES>
__device__ __forceinline__ T group_sum(T s) {
#pragma unroll
    for (int off = LANES / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, LANES);
    return s;
}

template <typename T, Epi E>
__device__ __forceinline__ void epilogue(int32_t row, T s, T* __restrict__ y, const T* __restrict__ f,
                                         const T* __restrict__ qd, const T* __restrict__ u) {
    if constexpr (E == Epi::Store) {
        y[row] = s;
    } else if constexpr (E == Epi::Resid) {
        y[row] = f[row] - s;
    } else if constexpr (E == Epi::Add) {
        y[row] += s;
    } else if constexpr (E == Epi::Sub) {
        y[row] -= s;
    } else {
        y[row] = u[row] + qd[row] * (f[row] - s);
    }
}

// Sum of one double per thread over the workgroup into partial[blockIdx.x] (fixed tree).
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

// DOT: 0 none; 1 partial of x_i y_i (q = A p, p^T q); 2 partial of y_i^2 (r = b - A x, r^T r).
template <typename T, Epi E, int ROWS, int DOT>
__global__ __launch_bounds__(kBlock) void csr_stream_kernel(int32_t nrows, const int32_t* __restrict__ ptr,
                                                           const int32_t* __restrict__ col,
                                                           const T* __restrict__ val, const T* __restrict__ x,
                                                           T* __restrict__ y, const T* __restrict__ f,
                                                           const T* __restrict__ qd, const T* __restrict__ u,
                                                           double* __restrict__ partial) {
    __shared__ T prod[kStreamCap];
    const int32_t r0 = xcd_block() * ROWS;
    const int32_t r1 = min(r0 + ROWS, nrows);
    const int32_t e0 = ptr[r0];
    const int32_t ne = ptr[r1] - e0;
    const int32_t row = r0 + static_cast<int32_t>(threadIdx.x);
    const bool mine = threadIdx.x < ROWS && row < r1;
    T s = T(0);
    if (ne <= kStreamCap) {
        // all column/value loads of this thread first, then the gathers: more loads in flight
        constexpr int kPer = kStreamCap / kBlock;
        T v[kPer];
        int32_t c[kPer];
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int32_t k = threadIdx.x + q * kBlock;
            if (k < ne) {
                v[q] = val[e0 + k];
                c[q] = col[e0 + k];
            }
        }
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int32_t k = threadIdx.x + q * kBlock;
            if (k < ne) prod[k] = v[q] * x[c[q]];
        }
        __syncthreads();
        if (mine) {
            const int32_t end = ptr[row + 1] - e0;
            for (int32_t k = ptr[row] - e0; k < end; ++k) s += prod[k];
        }
    } else if (mine) {
        const int32_t end = ptr[row + 1];
        for (int32_t k = ptr[row]; k < end; ++k) s += val[k] * x[col[k]];
    }
    double d = 0.0;
    if (mine) {
        epilogue<T, E>(row, s, y, f, qd, u);
        if constexpr (DOT == 1) d = static_cast<double>(x[row]) * static_cast<double>(s);
        if constexpr (DOT == 2) {
            const double v = static_cast<double>(y[row]);
            d = v * v;
        }
    }
    if constexpr (DOT != 0) block_partial(d, partial);
}

template <typename T, int LANES, Epi E>
__global__ __launch_bounds__(kBlock) void csr_rows_kernel(int32_t nrows, const int32_t* __restrict__ ptr,
                                                         const int32_t* __restrict__ col,
                                                         const T* __restrict__ val, const T* __restrict__ x,
                                                         T* __restrict__ y, const T* __restrict__ f,
                                                         const T* __restrict__ qd, const T* __restrict__ u) {
    const int32_t t = blockIdx.x * kBlock + threadIdx.x;
    const int32_t row = t / LANES;
    const int lane = t % LANES;
    T s = T(0);
    if (row < nrows) {
        const int32_t end = ptr[row + 1];
        for (int32_t p = ptr[row] + lane; p < end; p += LANES) s += val[p] * x[col[p]];
    }
    s = group_sum<T, LANES>(s);
    if (row < nrows && lane == 0) epilogue<T, E>(row, s, y, f, qd, u);
}

// Lane kernel with a fixed grid and per-workgroup partial sums (long rows in the outer loop).
template <int LANES, int DOT>
__global__ __launch_bounds__(kBlock) void rows_dot_kernel(int32_t nrows, const int32_t* __restrict__ ptr,
                                                         const int32_t* __restrict__ col,
                                                         const double* __restrict__ val,
                                                         const double* __restrict__ x, const double* __restrict__ b,
                                                         double* __restrict__ y, double* __restrict__ partial) {
    constexpr int kRowsPerBlock = kBlock / LANES;
    const int lane = threadIdx.x % LANES;
    double acc = 0.0;
    for (int32_t base = blockIdx.x * kRowsPerBlock; base < nrows; base += gridDim.x * kRowsPerBlock) {
        const int32_t row = base + threadIdx.x / LANES;
        double s = 0.0;
        if (row < nrows) {
            const int32_t end = ptr[row + 1];
            for (int32_t k = ptr[row] + lane; k < end; k += LANES) s += val[k] * x[col[k]];
        }
        s = group_sum<double, LANES>(s);
        if (row < nrows && lane == 0) {
            if constexpr (DOT == 1) {
                y[row] = s;
                acc += x[row] * s;
            } else {
                const double ri = b[row] - s;
                y[row] = ri;
                acc += ri * ri;
            }
        }
    }
    block_partial(acc, partial);
}

template <typename T, Epi E, int DOT>
hipError_t launch_stream(int rows, const CsrView& m, const T* val, const T* x, T* y, const T* f, const T* qd,
                         const T* u, double* partial, hipStream_t stream) {
    const dim3 grid(static_cast<unsigned>((m.nrows + rows - 1) / rows));
    switch (rows) {
        case 256:
            csr_stream_kernel<T, E, 256, DOT><<<grid, kBlock, 0, stream>>>(m.nrows, m.ptr, m.col, val, x, y, f, qd, u, partial);
            break;
        case 128:
            csr_stream_kernel<T, E, 128, DOT><<<grid, kBlock, 0, stream>>>(m.nrows, m.ptr, m.col, val, x, y, f, qd, u, partial);
            break;
        case 64:
            csr_stream_kernel<T, E, 64, DOT><<<grid, kBlock, 0, stream>>>(m.nrows, m.ptr, m.col, val, x, y, f, qd, u, partial);
            break;
        case 32:
            csr_stream_kernel<T, E, 32, DOT><<<grid, kBlock, 0, stream>>>(m.nrows, m.ptr, m.col, val, x, y, f, qd, u, partial);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, Epi E>
hipError_t launch_rows(const CsrView& m, const T* val, const T* x, T* y, const T* f, const T* qd, const T* u,
                       hipStream_t stream) {
    if (m.nrows <= 0) return hipSuccess;
    const int rows = stream_rows(m.nrows, m.nnz);
    if (rows > 0) return launch_stream<T, E, 0>(rows, m, val, x, y, f, qd, u, nullptr, stream);
    const int64_t threads = static_cast<int64_t>(m.nrows) * m.lanes;
    const dim3 grid(static_cast<unsigned>((threads + kBlock - 1) / kBlock));
    switch (m.lanes) {
#define AMGG_CASE(L)                                                                                        \
    case L:                                                                                                 \
        csr_rows_kernel<T, L, E><<<grid, kBlock, 0, stream>>>(m.nrows, m.ptr, m.col, val, x, y, f, qd, u); \
        break;
        AMGG_CASE(1)
        AMGG_CASE(2)
        AMGG_CASE(4)
        AMGG_CASE(8)
        AMGG_CASE(16)
        AMGG_CASE(32)
        AMGG_CASE(64)
#undef AMGG_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int DOT>
int launch_outer(const CsrView& m, const double* val, const double* x, const double* b, double* y, double* partial,
                 hipStream_t stream, hipError_t* err) {
    const int rows = stream_rows(m.nrows, m.nnz);
    if (rows > 0) {
        if constexpr (DOT == 1)
            *err = launch_stream<double, Epi::Store, 1>(rows, m, val, x, y, nullptr, nullptr, nullptr, partial, stream);
        else
            *err = launch_stream<double, Epi::Resid, 2>(rows, m, val, x, y, b, nullptr, nullptr, partial, stream);
        return (m.nrows + rows - 1) / rows;
    }
    switch (m.lanes) {
#define AMGG_CASE(L)                                                                                              \
    case L:                                                                                                       \
        rows_dot_kernel<L, DOT><<<kReduceBlocks, kBlock, 0, stream>>>(m.nrows, m.ptr, m.col, val, x, b, y, partial); \
        break;
        AMGG_CASE(1)
        AMGG_CASE(2)
        AMGG_CASE(4)
        AMGG_CASE(8)
        AMGG_CASE(16)
        AMGG_CASE(32)
        AMGG_CASE(64)
#undef AMGG_CASE
        default:
            *err = hipErrorInvalidValue;
            return 0;
    }
    *err = hipGetLastError();
    return kReduceBlocks;
}

}  // namespace

int outer_partials(int32_t nrows, int32_t nnz) {
    const int rows = stream_rows(nrows, nnz);
    return rows > 0 ? (nrows + rows - 1) / rows : kReduceBlocks;
}

template <typename T>
hipError_t csr_apply(const CsrView& m, const T* val, const T* x, T* y, const T* f, const T* qd, const T* u,
                     Epi epi, hipStream_t stream) {
    switch (epi) {
        case Epi::Store:
            return launch_rows<T, Epi::Store>(m, val, x, y, f, qd, u, stream);
        case Epi::Resid:
            return launch_rows<T, Epi::Resid>(m, val, x, y, f, qd, u, stream);
        case Epi::Add:
            return launch_rows<T, Epi::Add>(m, val, x, y, f, qd, u, stream);
        case Epi::Jacobi:
            return launch_rows<T, Epi::Jacobi>(m, val, x, y, f, qd, u, stream);
        case Epi::Sub:
            return launch_rows<T, Epi::Sub>(m, val, x, y, f, qd, u, stream);
    }
    return hipErrorInvalidValue;
}

template hipError_t csr_apply<float>(const CsrView&, const float*, const float*, float*, const float*,
                                     const float*, const float*, Epi, hipStream_t);
template hipError_t csr_apply<double>(const CsrView&, const double*, const double*, double*, const double*,
                                      const double*, const double*, Epi, hipStream_t);

hipError_t csr_spmv_dot(const CsrView& m, const double* val, const double* p, double* q, double* partial, int* count,
                        hipStream_t stream) {
    hipError_t e = hipSuccess;
    *count = launch_outer<1>(m, val, p, nullptr, q, partial, stream, &e);
    return e;
}

hipError_t csr_resid_norm(const CsrView& m, const double* val, const double* x, const double* b, double* r,
                          double* partial, int* count, hipStream_t stream) {
    hipError_t e = hipSuccess;
    *count = launch_outer<2>(m, val, x, b, r, partial, stream, &e);
    return e;
}

}  // namespace amgg
