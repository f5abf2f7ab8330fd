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
#include "xcd.hpp"

namespace amgg {

LaunchEvents& armed_events() {
    static thread_local LaunchEvents ev;
    return ev;
}

int lanes_for(int32_t nrows, int32_t nnz) {
    if (nrows <= 0) return 1;
    const double avg = static_cast<double>(nnz) / nrows;
    int l = 1;
    while (l < 64 && l < avg) l <<= 1;
    return l;
}

namespace {


// Rows per stream workgroup for a mean row length, or 0 for the lane kernel: the most rows whose
// entries fill most of one product round (then every block streams its entries in one round of
// dependent loads; 8M tet mesh, level 1 at 10.9 entries per row: 128 instead of 256 rows, solves
// 0.7-1 % faster), else the most rows whose entries fit the product buffer.
int stream_rows(int32_t nrows, int32_t nnz) {
    const double avg = nrows > 0 ? static_cast<double>(nnz) / nrows : 0.0;
    for (int r : {256, 128, 64})
        if (r * avg <= 0.9 * kStreamRound) return r;
    for (int r : {256, 128, 64, 32})
        if (r * avg * 1.25 <= kStreamCap) return r;
    return 0;
}

template <typename T, int LANES>
__device__ __forceinline__ T group_sum(T s) {
#pragma unroll
    for (int off = LANES / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, LANES);
    return s;
}

template <typename T, Epi E>
__device__ __forceinline__ void epilogue(int32_t row, T s, T* __restrict__ y, const T* __restrict__ f,
                                         const T* __restrict__ qd, const T* __restrict__ u, T* __restrict__ y2) {
    if constexpr (E == Epi::Store) {
        y[row] = s;
    } else if constexpr (E == Epi::StoreScaled) {
        y[row] = s;
        y2[row] = qd[row] * s;
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

constexpr int kChunk = 8;  // entries per thread per round of a product stream

// out[k] = m[k] * g(col[k]) for k < ne, where m and col are already offset to the block's first
// entry and g(j) = x[j] (or d[j] * x[j] with SCALED, rounded as a separate product). Every round
// gives each thread kChunk entries; a thread past the end re-reads the last entry (same cache
// line) and stores its unused product past ne instead of branching, so that all value/column
// loads of a round are issued together and then all of its gathers: each wave keeps many loads
// in flight. out must hold ne rounded up to a multiple of kChunk * kBlock.
template <typename T, class Gather>
__device__ __forceinline__ void stream_products_g(int32_t ne, const T* __restrict__ m,
                                                  const int32_t* __restrict__ col, Gather gather, T* __restrict__ out) {
    for (int32_t base = 0; base < ne; base += kChunk * kBlock) {
        T v[kChunk];
        int32_t c[kChunk];
#pragma unroll
        for (int q = 0; q < kChunk; ++q) {
            const int32_t k = min(base + static_cast<int32_t>(threadIdx.x) + q * kBlock, ne - 1);
            v[q] = m[k];
            c[q] = col[k];
        }
        T p[kChunk];
#pragma unroll
        for (int q = 0; q < kChunk; ++q) p[q] = v[q] * gather(c[q]);
#pragma unroll
        for (int q = 0; q < kChunk; ++q) out[base + static_cast<int32_t>(threadIdx.x) + q * kBlock] = p[q];
    }
}

// The same products from packed columns (ColPack): a round loads 2-byte offsets instead of
// 4-byte columns. A far entry (offset kFarCol) gathers the block's base column instead (in
// range, and branch-free, so that all gathers of a round stay in flight together); after a
// barrier far_products overwrites its slot from the block's far list, so every slot ends up
// holding exactly the product of the plain walk.
template <typename T, class Gather>
__device__ __forceinline__ void stream_products_packed(int32_t ne, const T* __restrict__ m,
                                                       const uint16_t* __restrict__ off, int32_t cbase, Gather gather,
                                                       T* __restrict__ out) {
    for (int32_t base = 0; base < ne; base += kChunk * kBlock) {
        T v[kChunk];
        int32_t c[kChunk];
#pragma unroll
        for (int q = 0; q < kChunk; ++q) {
            const int32_t k = min(base + static_cast<int32_t>(threadIdx.x) + q * kBlock, ne - 1);
            v[q] = m[k];
            const uint32_t o = off[k];
            c[q] = cbase + static_cast<int32_t>(o == kFarCol ? 0u : o);
        }
        T p[kChunk];
#pragma unroll
        for (int q = 0; q < kChunk; ++q) p[q] = v[q] * gather(c[q]);
#pragma unroll
        for (int q = 0; q < kChunk; ++q) out[base + static_cast<int32_t>(threadIdx.x) + q * kBlock] = p[q];
    }
}

template <typename T, class Gather>
__device__ __forceinline__ void far_products(int32_t f0, int32_t f1, const T* __restrict__ m,
                                             const uint16_t* __restrict__ fslot, const int32_t* __restrict__ fcol,
                                             Gather gather, T* __restrict__ out) {
    for (int32_t j = f0 + static_cast<int32_t>(threadIdx.x); j < f1; j += kBlock) {
        const int32_t s = fslot[j];
        out[s] = m[s] * gather(fcol[j]);
    }
}

// Products of block b's entries (ne <= kStreamCap) into out, from packed or plain columns.
template <typename T, bool PACKED, class Gather>
__device__ __forceinline__ void block_products(int32_t b, int32_t e0, int32_t ne, const T* __restrict__ val,
                                               const int32_t* __restrict__ col, const ColPack& cp, Gather gather,
                                               T* __restrict__ out) {
    if constexpr (PACKED) {
        const int32_t f0 = cp.foff[b], f1 = cp.foff[b + 1];
        stream_products_packed<T>(ne, val + e0, cp.off + e0, cp.base[b], gather, out);
        if (f1 > f0) {  // uniform over the workgroup
            __syncthreads();  // the stand-in products of the far slots are stored
            far_products<T>(f0, f1, val + e0, cp.fslot, cp.fcol, gather, out);
        }
    } else {
        stream_products_g<T>(ne, val + e0, col + e0, gather, out);
    }
}

template <typename T, bool SCALED = false>
__device__ __forceinline__ void stream_products(int32_t ne, const T* __restrict__ m, const int32_t* __restrict__ col,
                                                const T* __restrict__ x, const T* __restrict__ d,
                                                T* __restrict__ out) {
    if constexpr (SCALED)
        stream_products_g<T>(ne, m, col, [&](int32_t j) { return d[j] * x[j]; }, out);
    else
        stream_products_g<T>(ne, m, col, [&](int32_t j) { return x[j]; }, out);
}
static_assert(kStreamCap % (kChunk * kBlock) == 0, "product buffers hold whole rounds");
static_assert(kStreamRound == kChunk * kBlock, "a product round");

// Two product streams in the same rounds (out1[k] = m1[k] x[c1[k]], k < n1, and likewise for
// stream 2): a round issues the value/column loads of both, then the gathers of both, so the
// two dependent load chains overlap instead of running one after the other. Same products and
// storage as two stream_products calls.
template <typename T>
__device__ __forceinline__ void stream_products_pair(int32_t n1, const T* __restrict__ m1, const int32_t* __restrict__ c1,
                                                     T* __restrict__ out1, int32_t n2, const T* __restrict__ m2,
                                                     const int32_t* __restrict__ c2, T* __restrict__ out2,
                                                     const T* __restrict__ x) {
    const int32_t n = max(n1, n2);
    for (int32_t base = 0; base < n; base += kChunk * kBlock) {
        const bool a = base < n1, b = base < n2;
        T v1[kChunk], v2[kChunk];
        int32_t i1[kChunk], i2[kChunk];
        if (a) {
#pragma unroll
            for (int q = 0; q < kChunk; ++q) {
                const int32_t k = min(base + static_cast<int32_t>(threadIdx.x) + q * kBlock, n1 - 1);
                v1[q] = m1[k];
                i1[q] = c1[k];
            }
        }
        if (b) {
#pragma unroll
            for (int q = 0; q < kChunk; ++q) {
                const int32_t k = min(base + static_cast<int32_t>(threadIdx.x) + q * kBlock, n2 - 1);
                v2[q] = m2[k];
                i2[q] = c2[k];
            }
        }
        T p1[kChunk], p2[kChunk];
        if (a) {
#pragma unroll
            for (int q = 0; q < kChunk; ++q) p1[q] = v1[q] * x[i1[q]];
        }
        if (b) {
#pragma unroll
            for (int q = 0; q < kChunk; ++q) p2[q] = v2[q] * x[i2[q]];
        }
        if (a) {
#pragma unroll
            for (int q = 0; q < kChunk; ++q) out1[base + static_cast<int32_t>(threadIdx.x) + q * kBlock] = p1[q];
        }
        if (b) {
#pragma unroll
            for (int q = 0; q < kChunk; ++q) out2[base + static_cast<int32_t>(threadIdx.x) + q * kBlock] = p2[q];
        }
    }
}

// Sum of buf[pb..pe) from left to right (the order of the stored row); the LDS reads are
// issued four at a time ahead of the dependent additions.
template <typename T>
__device__ __forceinline__ T row_sum(const T* buf, int32_t pb, int32_t pe) {
    T s = T(0);
    int32_t k = pb;
    for (; k + 4 <= pe; k += 4) {
        const T a0 = buf[k], a1 = buf[k + 1], a2 = buf[k + 2], a3 = buf[k + 3];
        s += a0;
        s += a1;
        s += a2;
        s += a3;
    }
    for (; k < pe; ++k) s += buf[k];
    return s;
}

// DOT: 0 none; 1 partial of x_i y_i (q = A p, p^T q); 2 partial of y_i^2 (r = b - A x, r^T r);
// 3 as 2, with the scaled FP32 copy of y written through cs instead of y itself.
// PACKED: columns from cp (packed for blocks of ROWS rows), else from col.
template <typename T, Epi E, int ROWS, int DOT, bool PACKED>
__global__ __launch_bounds__(kBlock) void csr_stream_kernel(int32_t nrows, const int32_t* __restrict__ ptr,
                                                           const int32_t* __restrict__ col, ColPack cp,
                                                           const T* __restrict__ val, const T* __restrict__ x,
                                                           T* __restrict__ y, const T* __restrict__ f,
                                                           const T* __restrict__ qd, const T* __restrict__ u,
                                                           T* __restrict__ y2, double* __restrict__ partial,
                                                           int32_t cap, Cast32 cs) {
    static_assert(DOT != 3 || (E == Epi::Resid && sizeof(T) == 8), "the FP32 copy is of an FP64 residual");
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T* prod = reinterpret_cast<T*>(lds_raw);  // cap products (dynamic LDS)
    const int32_t blk = xcd_block();
    const int32_t r0 = blk * ROWS;
    const int32_t r1 = min(r0 + ROWS, nrows);
    const int32_t e0 = ptr[r0];
    const int32_t ne = ptr[r1] - e0;
    const int32_t row = r0 + static_cast<int32_t>(threadIdx.x);
    const bool mine = threadIdx.x < ROWS && row < r1;
    // the row's own operands, loaded while the products stream
    int32_t pb = 0, pe = 0;
    T fr = T(0), qr = T(0), ur = T(0), yr = T(0), xr = T(0);
    if (mine) {
        pb = ptr[row];
        pe = ptr[row + 1];
        if constexpr (E == Epi::Resid || E == Epi::Jacobi) fr = f[row];
        if constexpr (E == Epi::Jacobi) {
            qr = qd[row];
            ur = u[row];
        }
        if constexpr (E == Epi::StoreScaled) qr = qd[row];
        if constexpr (E == Epi::Add || E == Epi::Sub) yr = y[row];
        if constexpr (DOT == 1) xr = x[row];
    }
    T s = T(0);
    if (ne <= cap) {
        block_products<T, PACKED>(blk, e0, ne, val, col, cp, [&](int32_t j) { return x[j]; }, prod);
        __syncthreads();
        if (mine) s = row_sum(prod, pb - e0, pe - e0);
    } else if (mine) {
        for (int32_t k = pb; k < pe; ++k) s += val[k] * x[col[k]];
    }
    double d = 0.0;
    if (mine) {
        T out;
        if constexpr (E == Epi::Store || E == Epi::StoreScaled) out = s;
        if constexpr (E == Epi::StoreScaled) y2[row] = qr * s;
        if constexpr (E == Epi::Resid) out = fr - s;
        if constexpr (E == Epi::Add) out = yr + s;
        if constexpr (E == Epi::Sub) out = yr - s;
        if constexpr (E == Epi::Jacobi) out = ur + qr * (fr - s);
        if constexpr (DOT == 3) {
            const float fy = static_cast<float>(out * cs.scale[0]);
            cs.f[row] = fy;
            if (cs.qd) cs.u[row] = cs.qd[row] * fy;
        } else {
            y[row] = out;
        }
        if constexpr (DOT == 1) d = static_cast<double>(xr) * static_cast<double>(s);
        if constexpr (DOT >= 2) d = static_cast<double>(out) * static_cast<double>(out);
    }
    if constexpr (DOT != 0) block_partial(d, partial);
}

template <typename T, int LANES, Epi E>
__global__ __launch_bounds__(kBlock) void csr_rows_kernel(int32_t nrows, const int32_t* __restrict__ ptr,
                                                         const int32_t* __restrict__ col,
                                                         const T* __restrict__ val, const T* __restrict__ x,
                                                         T* __restrict__ y, const T* __restrict__ f,
                                                         const T* __restrict__ qd, const T* __restrict__ u,
                                                         T* __restrict__ y2) {
    const int32_t t = blockIdx.x * kBlock + threadIdx.x;
    const int32_t row = t / LANES;
    const int lane = t % LANES;
    T s = T(0);
    if (row < nrows) {
        const int32_t end = ptr[row + 1];
        for (int32_t p = ptr[row] + lane; p < end; p += LANES) s += val[p] * x[col[p]];
    }
    s = group_sum<T, LANES>(s);
    if (row < nrows && lane == 0) epilogue<T, E>(row, s, y, f, qd, u, y2);
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
                         const T* u, T* y2, double* partial, hipStream_t stream, const Cast32& cs = Cast32{}) {
    const dim3 grid(static_cast<unsigned>((m.nrows + rows - 1) / rows));
    const bool packed = m.cp.rows == rows && m.cp.off != nullptr;
    if (m.cap < kStreamRound || m.cap > kStreamCap || m.cap % kStreamRound) return hipErrorInvalidValue;
    const size_t lds = static_cast<size_t>(m.cap) * sizeof(T);
    switch (rows) {
#define AMGG_CASE(R)                                                                                              \
    case R:                                                                                                       \
        return packed ? launch_kernel_lds(csr_stream_kernel<T, E, R, DOT, true>, grid, dim3(kBlock), lds, stream,    \
                                          m.nrows, m.ptr, m.col, m.cp, val, x, y, f, qd, u, y2, partial, m.cap, cs)  \
                      : launch_kernel_lds(csr_stream_kernel<T, E, R, DOT, false>, grid, dim3(kBlock), lds, stream,   \
                                          m.nrows, m.ptr, m.col, ColPack{}, val, x, y, f, qd, u, y2, partial, m.cap, \
                                          cs);
        AMGG_CASE(256)
        AMGG_CASE(128)
        AMGG_CASE(64)
        AMGG_CASE(32)
#undef AMGG_CASE
        default:
            return hipErrorInvalidValue;
    }
}

template <typename T, Epi E>
hipError_t launch_rows(const CsrView& m, const T* val, const T* x, T* y, const T* f, const T* qd, const T* u,
                       T* y2, hipStream_t stream) {
    if (m.nrows <= 0) return hipSuccess;
    const int rows = stream_rows(m.nrows, m.nnz);
    if (rows > 0) return launch_stream<T, E, 0>(rows, m, val, x, y, f, qd, u, y2, nullptr, stream);
    const int64_t threads = static_cast<int64_t>(m.nrows) * m.lanes;
    const dim3 grid(static_cast<unsigned>((threads + kBlock - 1) / kBlock));
    switch (m.lanes) {
#define AMGG_CASE(L)                                                                                        \
    case L:                                                                                                 \
        return launch_kernel(csr_rows_kernel<T, L, E>, grid, dim3(kBlock), stream, m.nrows, m.ptr, m.col, val, x, y, \
                             f, qd, u, y2);
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
}

template <int DOT>
int launch_outer(const CsrView& m, const double* val, const double* x, const double* b, double* y, double* partial,
                 hipStream_t stream, hipError_t* err) {
    const int rows = stream_rows(m.nrows, m.nnz);
    if (rows > 0) {
        if constexpr (DOT == 1)
            *err = launch_stream<double, Epi::Store, 1>(rows, m, val, x, y, nullptr, nullptr, nullptr, nullptr, partial,
                                                        stream);
        else
            *err = launch_stream<double, Epi::Resid, 2>(rows, m, val, x, y, b, nullptr, nullptr, nullptr, partial,
                                                        stream);
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


// ---------------------------------------------------------------------------------------
// Fused smoothing steps (one workgroup per block of ROWS rows plus its halo).
//
// Phase 1 evaluates z = epi1(M1 x) on the block's own rows and on its halo rows and keeps z
// in LDS; phase 2 evaluates y = epi2(M2 z) on the own rows, gathering z from LDS through the
// precomputed slots. The own rows' entries and the halo rows' entries are both read as flat
// streams shared evenly by the workgroup's threads (all loads issued before the gathers);
// products go to LDS and every row is then summed by one thread in stored order, so the
// results are bitwise those of the separate passes.
//   PRE:  M1 = Q, x = f, z = Q f (also written to u); M2 = A, y = f - A z
//   POST: M1 = A, x = u, z = f - A u;                 M2 = Q, y = u + Q z
// ---------------------------------------------------------------------------------------
enum class Fused : int { Pre = 0, Post = 1 };

template <typename T, int ROWS, Fused M>
__global__ __launch_bounds__(kBlock) void csr_halo_kernel(int32_t nrows, const int32_t* __restrict__ ptr,
                                                         const int32_t* __restrict__ col, HaloView h,
                                                         const T* __restrict__ m1, const T* __restrict__ hm1,
                                                         const T* __restrict__ m2, const T* __restrict__ x,
                                                         const T* __restrict__ f, T* __restrict__ y,
                                                         T* __restrict__ uout) {
    constexpr int kHRows = kHaloCap / kBlock;
    __shared__ T prod[kStreamCap];
    __shared__ T hprod[kStreamCap];  // >= kHaloEntCap, whole rounds
    __shared__ T z[ROWS + kHaloCap];
    const int32_t b = xcd_block();
    const int32_t r0 = b * ROWS;
    const int32_t r1 = min(r0 + ROWS, nrows);
    const int32_t row = r0 + static_cast<int32_t>(threadIdx.x);
    const bool mine = threadIdx.x < ROWS && row < r1;
    const int32_t e0 = ptr[r0];
    const int32_t ne = ptr[r1] - e0;
    const int32_t h0 = h.hoff[b];
    const int32_t nh = h.hoff[b + 1] - h0;
    const int32_t he0 = h.heoff[b];
    const int32_t nhe = h.heoff[b + 1] - he0;
    // operands that do not depend on phase 1: the own row's bounds and f (and u for POST), the
    // halo rows' entry ranges (and f there for POST), phase 2's first round of values and slots
    int32_t pb = 0, pe = 0;
    T fr = T(0), xr = T(0);
    if (mine) {
        pb = ptr[row] - e0;
        pe = ptr[row + 1] - e0;
        fr = f[row];
        if constexpr (M == Fused::Post) xr = x[row];
    }
    int32_t hb[kHRows], hx[kHRows];
    T hf[kHRows];
    if (nh > 0) {  // clamped instead of branching, so the loads are in flight together
#pragma unroll
        for (int q = 0; q < kHRows; ++q) {
            const int32_t hh = min(static_cast<int32_t>(threadIdx.x) + q * kBlock, nh - 1);
            hb[q] = hh > 0 ? h.hend[h0 + hh - 1] : 0;
            hx[q] = h.hend[h0 + hh];
            hf[q] = T(0);
            if constexpr (M == Fused::Post) hf[q] = f[h.halo[h0 + hh]];
        }
    }
    const bool fits = ne <= kStreamCap;
    T v2[kChunk];
    uint16_t l2[kChunk];
    if (fits && ne > 0) {
#pragma unroll
        for (int q = 0; q < kChunk; ++q) {
            const int32_t k = min(static_cast<int32_t>(threadIdx.x) + q * kBlock, ne - 1);
            v2[q] = m2[e0 + k];
            l2[q] = h.loc[e0 + k];
        }
    }
    // phase 1: z on the own rows and the halo rows
    stream_products_pair<T>(fits ? ne : 0, m1 + e0, col + e0, prod, nhe, hm1 + he0, h.hcol + he0, hprod, x);
    __syncthreads();
    if (mine) {
        T s = T(0);
        if (fits) {
            s = row_sum(prod, pb, pe);
        } else {
            for (int32_t k = pb; k < pe; ++k) s += m1[e0 + k] * x[col[e0 + k]];
        }
        if constexpr (M == Fused::Pre) {
            z[threadIdx.x] = s;
            uout[row] = s;
        } else {
            z[threadIdx.x] = fr - s;
        }
    }
#pragma unroll
    for (int q = 0; q < kHRows; ++q) {
        const int32_t hh = static_cast<int32_t>(threadIdx.x) + q * kBlock;
        if (hh < nh) {
            const T s = row_sum(hprod, hb[q], hx[q]);
            if constexpr (M == Fused::Pre)
                z[ROWS + hh] = s;
            else
                z[ROWS + hh] = hf[q] - s;
        }
    }
    __syncthreads();
    // phase 2: M2 z on the own rows, z gathered from LDS
    if (fits) {
        for (int32_t base = 0; base < ne; base += kChunk * kBlock) {
            if (base > 0) {
#pragma unroll
                for (int q = 0; q < kChunk; ++q) {
                    const int32_t k = min(base + static_cast<int32_t>(threadIdx.x) + q * kBlock, ne - 1);
                    v2[q] = m2[e0 + k];
                    l2[q] = h.loc[e0 + k];
                }
            }
#pragma unroll
            for (int q = 0; q < kChunk; ++q) prod[base + static_cast<int32_t>(threadIdx.x) + q * kBlock] = v2[q] * z[l2[q]];
        }
    }
    __syncthreads();
    if (mine) {
        T s = T(0);
        if (fits) {
            s = row_sum(prod, pb, pe);
        } else {
            for (int32_t k = pb; k < pe; ++k) s += m2[e0 + k] * z[h.loc[e0 + k]];
        }
        if constexpr (M == Fused::Pre)
            y[row] = fr - s;
        else
            y[row] = xr + s;
    }
}

// First diagonal smoothing step from u = 0 (u = d f) fused with the pass after it: the row
// products gather d_j f_j, rounded exactly as the separate u = d f pass rounds them.
//   NEXT_RESID: u_i = d_i f_i, y_i = f_i - (A u)_i
//   otherwise:  y_i = d_i f_i + d_i (f_i - (A u)_i)
template <typename T, int ROWS, bool NEXT_RESID, bool PACKED>
__global__ __launch_bounds__(kBlock) void csr_jpre_kernel(int32_t nrows, const int32_t* __restrict__ ptr,
                                                         const int32_t* __restrict__ col, ColPack cp,
                                                         const T* __restrict__ val, const T* __restrict__ d,
                                                         const T* __restrict__ f, T* __restrict__ y,
                                                         T* __restrict__ uout, int32_t cap) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T* prod = reinterpret_cast<T*>(lds_raw);  // cap products (dynamic LDS)
    const int32_t blk = xcd_block();
    const int32_t r0 = blk * ROWS;
    const int32_t r1 = min(r0 + ROWS, nrows);
    const int32_t e0 = ptr[r0];
    const int32_t ne = ptr[r1] - e0;
    const int32_t row = r0 + static_cast<int32_t>(threadIdx.x);
    const bool mine = threadIdx.x < ROWS && row < r1;
    int32_t pb = 0, pe = 0;
    T fr = T(0), dr = T(0);
    if (mine) {
        pb = ptr[row];
        pe = ptr[row + 1];
        fr = f[row];
        dr = d[row];
    }
    T s = T(0);
    if (ne <= cap) {
        block_products<T, PACKED>(blk, e0, ne, val, col, cp, [&](int32_t j) { return d[j] * f[j]; }, prod);
        __syncthreads();
        if (mine) s = row_sum(prod, pb - e0, pe - e0);
    } else if (mine) {
        for (int32_t k = pb; k < pe; ++k) {
            const T uj = d[col[k]] * f[col[k]];
            s += val[k] * uj;
        }
    }
    if (mine) {
        const T ui = dr * fr;
        if constexpr (NEXT_RESID) {
            uout[row] = ui;
            y[row] = fr - s;
        } else {
            y[row] = ui + dr * (fr - s);
        }
    }
}

template <typename T, Fused M>
hipError_t launch_halo(const CsrView& m, const HaloView& h, const T* m1, const T* hm1, const T* m2, const T* x,
                       const T* f, T* y, T* uout, hipStream_t stream) {
    if (m.nrows <= 0) return hipSuccess;
    const dim3 grid(static_cast<unsigned>((m.nrows + h.rows - 1) / h.rows));
    switch (h.rows) {
#define AMGG_CASE(R)                                                                                              \
    case R:                                                                                                       \
        return launch_kernel(csr_halo_kernel<T, R, M>, grid, dim3(kBlock), stream, m.nrows, m.ptr, m.col, h, m1, hm1, \
                             m2, x, f, y, uout);
        AMGG_CASE(256)
        AMGG_CASE(128)
        AMGG_CASE(64)
        AMGG_CASE(32)
#undef AMGG_CASE
        default:
            return hipErrorInvalidValue;
    }
}

__global__ void gather_kernel(int32_t n, const int32_t* __restrict__ idx, const double* __restrict__ s64,
                              const float* __restrict__ s32, double* __restrict__ d64, float* __restrict__ d32) {
    const int32_t k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    const int32_t i = idx[k];
    if (d64) d64[k] = s64[i];
    if (d32) d32[k] = s32[i];
}

template <typename T, bool NEXT_RESID>
hipError_t launch_jpre(const CsrView& m, const T* a, const T* d, const T* f, T* y, T* u, hipStream_t stream) {
    if (m.nrows <= 0) return hipSuccess;
    const int rows = stream_rows(m.nrows, m.nnz);
    if (rows == 0) {  // long rows: the separate passes (u = d f, then r = f - A u)
        if constexpr (!NEXT_RESID) return hipErrorInvalidValue;  // would need a third buffer
        hipError_t e = vec_mul<T>(m.nrows, d, f, u, stream);
        if (e != hipSuccess) return e;
        return csr_apply<T>(m, a, u, y, f, nullptr, nullptr, Epi::Resid, stream);
    }
    const dim3 grid(static_cast<unsigned>((m.nrows + rows - 1) / rows));
    const bool packed = m.cp.rows == rows && m.cp.off != nullptr;
    if (m.cap < kStreamRound || m.cap > kStreamCap || m.cap % kStreamRound) return hipErrorInvalidValue;
    const size_t lds = static_cast<size_t>(m.cap) * sizeof(T);
    switch (rows) {
#define AMGG_CASE(R)                                                                                             \
    case R:                                                                                                      \
        return packed ? launch_kernel_lds(csr_jpre_kernel<T, R, NEXT_RESID, true>, grid, dim3(kBlock), lds, stream, \
                                          m.nrows, m.ptr, m.col, m.cp, a, d, f, y, u, m.cap)                     \
                      : launch_kernel_lds(csr_jpre_kernel<T, R, NEXT_RESID, false>, grid, dim3(kBlock), lds,     \
                                          stream, m.nrows, m.ptr, m.col, ColPack{}, a, d, f, y, u, m.cap);
        AMGG_CASE(256)
        AMGG_CASE(128)
        AMGG_CASE(64)
        AMGG_CASE(32)
#undef AMGG_CASE
        default:
            return hipErrorInvalidValue;
    }
}

__global__ __launch_bounds__(kBlock) void block_max_kernel(int32_t nrows, const int32_t* __restrict__ ptr, int rows,
                                                          int32_t* __restrict__ out) {
    __shared__ int32_t red[kBlock / 64];
    const int64_t b = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int64_t r0 = b * rows;
    int32_t m = 0;
    if (r0 < nrows) m = ptr[min(r0 + rows, static_cast<int64_t>(nrows))] - ptr[r0];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x / 64] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < kBlock / 64; ++k) m = max(m, red[k]);
        atomicMax(out, m);
    }
}

}  // namespace

hipError_t block_max_entries(int32_t nrows, const int32_t* ptr, int rows, int32_t* out, hipStream_t stream) {
    if (nrows <= 0 || rows <= 0) return hipSuccess;
    const int64_t nb = (static_cast<int64_t>(nrows) + rows - 1) / rows;
    block_max_kernel<<<static_cast<unsigned>((nb + kBlock - 1) / kBlock), kBlock, 0, stream>>>(nrows, ptr, rows, out);
    return hipGetLastError();
}

int stream_rows_for(int32_t nrows, int32_t nnz) { return stream_rows(nrows, nnz); }

int outer_partials(int32_t nrows, int32_t nnz) {
    const int rows = stream_rows(nrows, nnz);
    return rows > 0 ? (nrows + rows - 1) / rows : kReduceBlocks;
}

template <typename T>
hipError_t csr_apply(const CsrView& m, const T* val, const T* x, T* y, const T* f, const T* qd, const T* u,
                     Epi epi, hipStream_t stream, T* y2) {
    switch (epi) {
        case Epi::Store:
            return launch_rows<T, Epi::Store>(m, val, x, y, f, qd, u, nullptr, stream);
        case Epi::Resid:
            return launch_rows<T, Epi::Resid>(m, val, x, y, f, qd, u, nullptr, stream);
        case Epi::Add:
            return launch_rows<T, Epi::Add>(m, val, x, y, f, qd, u, nullptr, stream);
        case Epi::Jacobi:
            return launch_rows<T, Epi::Jacobi>(m, val, x, y, f, qd, u, nullptr, stream);
        case Epi::Sub:
            return launch_rows<T, Epi::Sub>(m, val, x, y, f, qd, u, nullptr, stream);
        case Epi::StoreScaled:
            if (!qd || !y2) return hipErrorInvalidValue;
            return launch_rows<T, Epi::StoreScaled>(m, val, x, y, f, qd, u, y2, stream);
    }
    return hipErrorInvalidValue;
}

template hipError_t csr_apply<float>(const CsrView&, const float*, const float*, float*, const float*,
                                     const float*, const float*, Epi, hipStream_t, float*);
template hipError_t csr_apply<double>(const CsrView&, const double*, const double*, double*, const double*,
                                      const double*, const double*, Epi, hipStream_t, double*);

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

hipError_t csr_resid_cast(const CsrView& m, const double* val, const double* x, const double* b, const Cast32& cast,
                          double* partial, int* count, hipStream_t stream) {
    const int rows = stream_rows(m.nrows, m.nnz);
    if (rows <= 0 || !cast.f || !cast.scale || (cast.qd == nullptr) != (cast.u == nullptr)) return hipErrorInvalidValue;
    *count = (m.nrows + rows - 1) / rows;
    return launch_stream<double, Epi::Resid, 3>(rows, m, val, x, nullptr, b, nullptr, nullptr, nullptr, partial, stream,
                                                cast);
}

template <typename T>
hipError_t smooth_pre_fused(const CsrView& m, const HaloView& h, const T* a, const T* q, const T* hq, const T* f,
                            T* u, T* r, hipStream_t stream) {
    return launch_halo<T, Fused::Pre>(m, h, q, hq, a, f, f, r, u, stream);
}
template <typename T>
hipError_t smooth_post_fused(const CsrView& m, const HaloView& h, const T* a, const T* ha, const T* q, const T* f,
                             const T* u, T* y, hipStream_t stream) {
    return launch_halo<T, Fused::Post>(m, h, a, ha, q, u, f, y, nullptr, stream);
}
hipError_t gather_values(int32_t n, const int32_t* idx, const double* src64, const float* src32, double* dst64,
                         float* dst32, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    gather_kernel<<<(n + kBlock - 1) / kBlock, kBlock, 0, stream>>>(n, idx, src64, src32, dst64, dst32);
    return hipGetLastError();
}
template <typename T>
hipError_t jacobi_pre_resid(const CsrView& m, const T* a, const T* d, const T* f, T* u, T* r, hipStream_t stream) {
    return launch_jpre<T, true>(m, a, d, f, r, u, stream);
}
template <typename T>
hipError_t jacobi_pre_step(const CsrView& m, const T* a, const T* d, const T* f, T* y, hipStream_t stream) {
    return launch_jpre<T, false>(m, a, d, f, y, nullptr, stream);
}
#define AMGG_INST(T)                                                                                                \
    template hipError_t smooth_pre_fused<T>(const CsrView&, const HaloView&, const T*, const T*, const T*, const T*, \
                                            T*, T*, hipStream_t);                                                  \
    template hipError_t smooth_post_fused<T>(const CsrView&, const HaloView&, const T*, const T*, const T*,         \
                                             const T*, const T*, T*, hipStream_t);                                 \
    template hipError_t jacobi_pre_resid<T>(const CsrView&, const T*, const T*, const T*, T*, T*, hipStream_t);     \
    template hipError_t jacobi_pre_step<T>(const CsrView&, const T*, const T*, const T*, T*, hipStream_t);
AMGG_INST(float)
AMGG_INST(double)
#undef AMGG_INST

}  // namespace amgg
