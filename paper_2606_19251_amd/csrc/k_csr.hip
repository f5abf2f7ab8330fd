// Row-wise CSR products on gfx950: a group of `LANES` consecutive threads of a 64-wide
// wavefront owns one row and strides over its entries, so that the column and value
// streams of neighbouring rows are read by neighbouring lanes (coalesced), and the
// group's partial sums are combined with cross-lane shuffles. LANES is chosen per
// matrix from its mean row length (about 7 for the fine P1 matrices, 2-3 for P, longer
// on coarse levels), which keeps most lanes busy without one wavefront per short row.
#include "kernels.hpp"

namespace amgg {

// Rows with at most this many lanes' worth of entries on average use the CSR-stream kernel.
int kStreamMaxLanes = 8;

int lanes_for(int32_t nrows, int32_t nnz) {
    if (nrows <= 0) return 1;
    const double avg = static_cast<double>(nnz) / nrows;
    int l = 1;
    while (l < 64 && l < avg) l <<= 1;
    return l;
}

namespace {

template <typename T, int LANES>
__device__ __forceinline__ T group_sum(T s) {
#pragma unroll
    for (int off = LANES / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, LANES);
    return s;
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
    if (row < nrows && lane == 0) {
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
}

// CSR-stream variant for short rows: a workgroup owns kStreamRows consecutive rows; its
// threads walk the rows' contiguous nonzeros with unit stride (fully coalesced value and
// column streams), leave the products a_ij x_j in LDS, and each thread then sums its own
// row's products in order. Blocks whose nonzeros exceed the LDS capacity fall back to a
// per-thread row loop from global memory.
constexpr int kStreamRows = kBlock;
constexpr int kStreamCap = 2048;

template <typename T, Epi E>
__global__ __launch_bounds__(kBlock) void csr_stream_kernel(int32_t nrows, const int32_t* __restrict__ ptr,
                                                           const int32_t* __restrict__ col,
                                                           const T* __restrict__ val, const T* __restrict__ x,
                                                           T* __restrict__ y, const T* __restrict__ f,
                                                           const T* __restrict__ qd, const T* __restrict__ u) {
    __shared__ T prod[kStreamCap];
    const int32_t r0 = blockIdx.x * kStreamRows;
    const int32_t r1 = min(r0 + kStreamRows, nrows);
    const int32_t e0 = ptr[r0];
    const int32_t ne = ptr[r1] - e0;
    const int32_t row = r0 + threadIdx.x;
    T s = T(0);
    if (ne <= kStreamCap) {
        for (int32_t k = threadIdx.x; k < ne; k += kBlock) prod[k] = val[e0 + k] * x[col[e0 + k]];
        __syncthreads();
        if (row < r1) {
            const int32_t end = ptr[row + 1] - e0;
            for (int32_t k = ptr[row] - e0; k < end; ++k) s += prod[k];
        }
    } else if (row < r1) {
        const int32_t end = ptr[row + 1];
        for (int32_t k = ptr[row]; k < end; ++k) s += val[k] * x[col[k]];
    }
    if (row < r1) {
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
}

template <typename T, Epi E>
hipError_t launch_rows(const CsrView& m, const T* val, const T* x, T* y, const T* f, const T* qd, const T* u,
                       hipStream_t stream) {
    if (m.nrows <= 0) return hipSuccess;
    if (m.lanes <= kStreamMaxLanes) {
        const dim3 grid(static_cast<unsigned>((m.nrows + kStreamRows - 1) / kStreamRows));
        csr_stream_kernel<T, E><<<grid, kBlock, 0, stream>>>(m.nrows, m.ptr, m.col, val, x, y, f, qd, u);
        return hipGetLastError();
    }
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

// Block-level sum of one double per thread into partial[blockIdx.x] (fixed tree order).
__device__ __forceinline__ void block_partial(double v, double* partial) {
    __shared__ double red[kBlock / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = red[0];
        for (int k = 1; k < kBlock / 64; ++k) s += red[k];
        partial[blockIdx.x] = s;
    }
}

// q = A p with the row loop strided over a fixed grid of kReduceBlocks workgroups, so the
// per-block partial sums of p_i q_i are reproducible.
template <int LANES>
__global__ __launch_bounds__(kBlock) void spmv_dot_kernel(int32_t nrows, const int32_t* __restrict__ ptr,
                                                         const int32_t* __restrict__ col,
                                                         const double* __restrict__ val,
                                                         const double* __restrict__ p, double* __restrict__ q,
                                                         double* __restrict__ partial) {
    constexpr int kRowsPerBlock = kBlock / LANES;
    const int lane = threadIdx.x % LANES;
    double acc = 0.0;
    for (int32_t base = blockIdx.x * kRowsPerBlock; base < nrows; base += gridDim.x * kRowsPerBlock) {
        const int32_t row = base + threadIdx.x / LANES;
        double s = 0.0;
        if (row < nrows) {
            const int32_t end = ptr[row + 1];
            for (int32_t k = ptr[row] + lane; k < end; k += LANES) s += val[k] * p[col[k]];
        }
        s = group_sum<double, LANES>(s);
        if (row < nrows && lane == 0) {
            q[row] = s;
            acc += p[row] * s;
        }
    }
    block_partial(acc, partial);
}

template <int LANES>
__global__ __launch_bounds__(kBlock) void resid_norm_kernel(int32_t nrows, const int32_t* __restrict__ ptr,
                                                           const int32_t* __restrict__ col,
                                                           const double* __restrict__ val,
                                                           const double* __restrict__ x,
                                                           const double* __restrict__ b, double* __restrict__ r,
                                                           double* __restrict__ partial) {
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
            const double ri = b[row] - s;
            r[row] = ri;
            acc += ri * ri;
        }
    }
    block_partial(acc, partial);
}

}  // namespace

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

hipError_t csr_spmv_dot(const CsrView& m, const double* val, const double* p, double* q, double* partial,
                        hipStream_t stream) {
    switch (m.lanes) {
#define AMGG_CASE(L)                                                                                  \
    case L:                                                                                           \
        spmv_dot_kernel<L><<<kReduceBlocks, kBlock, 0, stream>>>(m.nrows, m.ptr, m.col, val, p, q, partial); \
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

hipError_t csr_resid_norm(const CsrView& m, const double* val, const double* x, const double* b, double* r,
                          double* partial, hipStream_t stream) {
    switch (m.lanes) {
#define AMGG_CASE(L)                                                                                       \
    case L:                                                                                                \
        resid_norm_kernel<L><<<kReduceBlocks, kBlock, 0, stream>>>(m.nrows, m.ptr, m.col, val, x, b, r, partial); \
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

}  // namespace amgg
