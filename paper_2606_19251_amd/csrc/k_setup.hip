// Setup-side kernels: diagonal and off-diagonal scale of each level, the exact transpose
// R = P^T, and the dense coarsest-level factorisation, inverse and per-cycle product.
#include <algorithm>
#include <cmath>

#include "kernels.hpp"

namespace amgg {

namespace {

inline dim3 grid_for(int64_t n) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    return dim3(static_cast<unsigned>(g));
}

__global__ void extract_diag_kernel(int32_t n, const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                    const double* __restrict__ val, double* __restrict__ diag,
                                    int32_t* __restrict__ bad) {
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double d = 0.0;
    bool found = false;
    for (int32_t p = ptr[i]; p < ptr[i + 1]; ++p)
        if (col[p] == i) {
            d = val[p];
            found = true;
        }
    diag[i] = d;
    if (!found || !(d > 0.0)) atomicOr(bad, 1);
}

__global__ __launch_bounds__(kBlock) void absmax_partial_kernel(int32_t n, const int32_t* __restrict__ ptr,
                                                               const int32_t* __restrict__ col,
                                                               const double* __restrict__ val,
                                                               double* __restrict__ partial) {
    __shared__ double red[kBlock];
    double m = -1.0;  // -1 marks "no off-diagonal seen"
    for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += kReduceBlocks * kBlock)
        for (int32_t p = ptr[i]; p < ptr[i + 1]; ++p)
            if (col[p] != i) m = fmax(m, fabs(val[p]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kBlock) void absmax_final_kernel(const double* __restrict__ partial,
                                                             double* __restrict__ scale) {
    __shared__ double red[kBlock];
    double m = -1.0;
    for (int k = threadIdx.x; k < kReduceBlocks; k += kBlock) m = fmax(m, partial[k]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) scale[0] = red[0] <= 0.0 ? 1.0 : red[0];  // no nonzero off-diagonal: s = 1
}

// --- transpose -----------------------------------------------------------------------
__global__ void count_cols_kernel(int32_t nnz, const int32_t* __restrict__ col, int32_t* __restrict__ cnt) {
    const int32_t p = blockIdx.x * kBlock + threadIdx.x;
    if (p < nnz) atomicAdd(&cnt[col[p] + 1], 1);
}

// In-place inclusive scan of a[1..m] (setup only): the range is cut into at most
// kScanParts contiguous pieces; pass 1 sums each piece, pass 2 scans the piece sums, pass 3
// scans each piece from its offset. Integer sums: the result does not depend on the order.
constexpr int kScanBlock = 1024;  // 16 wavefronts
constexpr int64_t kScanParts = 1024;  // at most ceil(m / kScanBlock) <= m pieces
static_assert(kScanParts <= kScanPartsMax, "pack_columns scratch holds the piece sums");

__device__ int32_t block_inclusive_scan(int32_t v, int32_t* lds, int32_t* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    if (lane == 63) lds[wave] = v;
    __syncthreads();
    if (wave == 0) {
        int32_t w = lane < kScanBlock / 64 ? lds[lane] : 0;
        for (int o = 1; o < kScanBlock / 64; o <<= 1) {
            const int32_t t = __shfl_up(w, o, 64);
            if (lane >= o) w += t;
        }
        if (lane < kScanBlock / 64) lds[lane] = w;
    }
    __syncthreads();
    if (wave > 0) v += lds[wave - 1];
    *total = lds[kScanBlock / 64 - 1];
    __syncthreads();
    return v;
}

__global__ __launch_bounds__(kScanBlock) void scan_reduce_kernel(int32_t m, int32_t piece,
                                                                 const int32_t* __restrict__ a,
                                                                 int32_t* __restrict__ parts) {
    __shared__ int32_t lds[kScanBlock / 64];
    const int64_t lo = 1 + static_cast<int64_t>(blockIdx.x) * piece;
    const int64_t hi = min(lo + piece, static_cast<int64_t>(m) + 1);
    int32_t s = 0;
    for (int64_t k = lo + threadIdx.x; k < hi; k += kScanBlock) s += a[k];
    int32_t total;
    block_inclusive_scan(s, lds, &total);
    if (threadIdx.x == 0) parts[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanBlock) void scan_parts_kernel(int32_t nparts, int32_t* __restrict__ parts) {
    __shared__ int32_t lds[kScanBlock / 64];
    const int32_t v = threadIdx.x < nparts ? parts[threadIdx.x] : 0;
    int32_t total;
    const int32_t incl = block_inclusive_scan(v, lds, &total);
    if (threadIdx.x < nparts) parts[threadIdx.x] = incl - v;  // exclusive
}

__global__ __launch_bounds__(kScanBlock) void scan_apply_kernel(int32_t m, int32_t piece, int32_t* __restrict__ a,
                                                                const int32_t* __restrict__ parts) {
    __shared__ int32_t lds[kScanBlock / 64];
    const int64_t lo = 1 + static_cast<int64_t>(blockIdx.x) * piece;
    const int64_t hi = min(lo + piece, static_cast<int64_t>(m) + 1);
    int32_t carry = parts[blockIdx.x];
    for (int64_t base = lo; base < hi; base += kScanBlock) {
        const int64_t k = base + threadIdx.x;
        const int32_t v = k < hi ? a[k] : 0;
        int32_t total;
        const int32_t incl = block_inclusive_scan(v, lds, &total);
        if (k < hi) a[k] = carry + incl;
        carry += total;
    }
}

__global__ void scatter_transpose_kernel(int32_t nf, const int32_t* __restrict__ p_ptr,
                                         const int32_t* __restrict__ p_col, const double* __restrict__ p_val,
                                         int32_t* __restrict__ cursor, int32_t* __restrict__ r_col,
                                         double* __restrict__ r_val) {
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= nf) return;
    for (int32_t p = p_ptr[i]; p < p_ptr[i + 1]; ++p) {
        const int32_t dst = atomicAdd(&cursor[p_col[p]], 1);
        r_col[dst] = i;
        r_val[dst] = p_val[p];
    }
}

// The scatter order within a row depends on atomics; sorting by column restores the one
// exact transpose.
__global__ void sort_rows_kernel(int32_t nc, const int32_t* __restrict__ r_ptr, int32_t* __restrict__ r_col,
                                 double* __restrict__ r_val) {
    const int32_t c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= nc) return;
    const int32_t lo = r_ptr[c], hi = r_ptr[c + 1];
    for (int32_t a = lo + 1; a < hi; ++a) {
        const int32_t key = r_col[a];
        const double v = r_val[a];
        int32_t b = a - 1;
        while (b >= lo && r_col[b] > key) {
            r_col[b + 1] = r_col[b];
            r_val[b + 1] = r_val[b];
            --b;
        }
        r_col[b + 1] = key;
        r_val[b + 1] = v;
    }
}

// --- dense coarsest level --------------------------------------------------------------
__global__ void dense_zero_kernel(int64_t total, double* __restrict__ M) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (k < total) M[k] = 0.0;
}

// Rows [0, n) of ptr (columns shifted by -col0) into the dense n x n matrix M.
__global__ void dense_scatter_kernel(int32_t n, const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                     const double* __restrict__ val, int32_t col0, double* __restrict__ M) {
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    for (int32_t p = ptr[i]; p < ptr[i + 1]; ++p) M[static_cast<int64_t>(i) * n + (col[p] - col0)] = val[p];
}

// A_L + alpha 1 1^T with alpha = mean(diag)/n (constant null space of all-Neumann problems).
__global__ __launch_bounds__(1024) void dense_rank_one_kernel(int32_t n, double* __restrict__ M) {
    __shared__ double red[1024];
    double s = 0.0;
    for (int32_t i = threadIdx.x; i < n; i += 1024) s += M[static_cast<int64_t>(i) * n + i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double alpha = red[0] / n / n;
    const int64_t total = static_cast<int64_t>(n) * n;
    for (int64_t k = threadIdx.x; k < total; k += 1024) M[k] += alpha;
}

// LU with partial pivoting (largest |pivot|, smallest row index on ties) by one workgroup.
__global__ __launch_bounds__(1024) void dense_lu_kernel(int32_t n, double* __restrict__ M, int32_t* __restrict__ piv,
                                                        int32_t* __restrict__ bad) {
    __shared__ double sval[1024];
    __shared__ int32_t sidx[1024];
    const int tid = threadIdx.x;
    for (int32_t k = tid; k < n; k += 1024) piv[k] = k;
    __syncthreads();
    for (int32_t k = 0; k < n; ++k) {
        double best = -1.0;
        int32_t bi = n;
        for (int32_t i = k + tid; i < n; i += 1024) {
            const double v = fabs(M[static_cast<int64_t>(i) * n + k]);
            if (v > best) {
                best = v;
                bi = i;
            }
        }
        sval[tid] = best;
        sidx[tid] = bi;
        __syncthreads();
        for (int w = 512; w > 0; w >>= 1) {
            if (tid < w) {
                const double ov = sval[tid + w];
                const int32_t oi = sidx[tid + w];
                if (ov > sval[tid] || (ov == sval[tid] && oi < sidx[tid])) {
                    sval[tid] = ov;
                    sidx[tid] = oi;
                }
            }
            __syncthreads();
        }
        const int32_t p = sidx[0];
        const double pv = sval[0];
        __syncthreads();
        if (!(pv > 0.0)) {
            if (tid == 0) bad[0] = 1;
            return;
        }
        if (p != k)
            for (int32_t j = tid; j < n; j += 1024) {
                const double t = M[static_cast<int64_t>(k) * n + j];
                M[static_cast<int64_t>(k) * n + j] = M[static_cast<int64_t>(p) * n + j];
                M[static_cast<int64_t>(p) * n + j] = t;
            }
        if (tid == 0) piv[k] = p;
        __syncthreads();
        const double pivot = M[static_cast<int64_t>(k) * n + k];
        for (int32_t i = k + 1 + tid; i < n; i += 1024) M[static_cast<int64_t>(i) * n + k] /= pivot;
        __syncthreads();
        const int32_t m = n - k - 1;
        const int64_t cnt = static_cast<int64_t>(m) * m;
        for (int64_t e = tid; e < cnt; e += 1024) {
            const int32_t i = k + 1 + static_cast<int32_t>(e / m);
            const int32_t j = k + 1 + static_cast<int32_t>(e % m);
            M[static_cast<int64_t>(i) * n + j] -= M[static_cast<int64_t>(i) * n + k] * M[static_cast<int64_t>(k) * n + j];
        }
        __syncthreads();
    }
}

// Column j of the inverse: solve L U x = Perm e_j, one workgroup per column, x in LDS.
__global__ __launch_bounds__(kBlock) void dense_inverse_cols_kernel(int32_t n, const double* __restrict__ LU,
                                                                   const int32_t* __restrict__ piv,
                                                                   const int32_t* __restrict__ bad,
                                                                   double* __restrict__ inv) {
    extern __shared__ double b[];
    if (bad[0]) return;  // factorisation failed: leave the inverse untouched
    const int32_t j = blockIdx.x;
    const int tid = threadIdx.x;
    for (int32_t i = tid; i < n; i += kBlock) b[i] = (i == j) ? 1.0 : 0.0;
    __syncthreads();
    if (tid == 0)
        for (int32_t k = 0; k < n; ++k) {
            const int32_t p = piv[k];
            if (p != k && p >= 0 && p < n) {
                const double t = b[k];
                b[k] = b[p];
                b[p] = t;
            }
        }
    __syncthreads();
    for (int32_t k = 0; k < n; ++k) {
        const double bk = b[k];
        for (int32_t i = k + 1 + tid; i < n; i += kBlock) b[i] -= LU[static_cast<int64_t>(i) * n + k] * bk;
        __syncthreads();
    }
    for (int32_t k = n - 1; k >= 0; --k) {
        if (tid == 0) b[k] /= LU[static_cast<int64_t>(k) * n + k];
        __syncthreads();
        const double bk = b[k];
        for (int32_t i = tid; i < k; i += kBlock) b[i] -= LU[static_cast<int64_t>(i) * n + k] * bk;
        __syncthreads();
    }
    for (int32_t i = tid; i < n; i += kBlock) inv[static_cast<int64_t>(i) * n + j] = b[i];
}

// y = inv x in FP64, one wavefront per row (coalesced row reads of the inverse).
template <typename T>
__global__ __launch_bounds__(kBlock) void dense_gemv_kernel(int32_t n, const double* __restrict__ inv,
                                                           const T* __restrict__ x, T* __restrict__ y) {
    const int32_t row = blockIdx.x * (kBlock / 64) + threadIdx.x / 64;
    const int lane = threadIdx.x & 63;
    double s = 0.0;
    if (row < n) {
        const double* a = inv + static_cast<int64_t>(row) * n;
        for (int32_t j = lane; j < n; j += 64) s += a[j] * static_cast<double>(x[j]);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (row < n && lane == 0) y[row] = static_cast<T>(s);
}


// --- block-diagonal levels ---------------------------------------------------------------
__device__ __forceinline__ int32_t block_of(int32_t i, int32_t nblk, const int32_t* __restrict__ off) {
    int32_t lo = 0, hi = nblk - 1;  // largest b with off[b] <= i
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) / 2;
        if (off[mid] <= i)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// scale[b] = max |a_ij| over the off-diagonal entries of block b's rows (1 if none), one
// workgroup per block; a maximum does not depend on the order.
__global__ __launch_bounds__(kBlock) void block_absmax_kernel(const int32_t* __restrict__ off,
                                                             const int32_t* __restrict__ ptr,
                                                             const int32_t* __restrict__ col,
                                                             const double* __restrict__ val,
                                                             double* __restrict__ scale) {
    __shared__ double red[kBlock];
    const int32_t b = blockIdx.x;
    double m = -1.0;
    for (int32_t i = off[b] + threadIdx.x; i < off[b + 1]; i += kBlock)
        for (int32_t p = ptr[i]; p < ptr[i + 1]; ++p)
            if (col[p] != i) m = fmax(m, fabs(val[p]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) scale[b] = red[0] <= 0.0 ? 1.0 : red[0];
}

// bad = 1 if an entry of P couples fine block b with another coarse block.
__global__ void prolong_blocks_kernel(int32_t n, const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                      int32_t nblk, const int32_t* __restrict__ foff,
                                      const int32_t* __restrict__ coff, int32_t* __restrict__ bad) {
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int32_t b = block_of(i, nblk, foff);
    for (int32_t p = ptr[i]; p < ptr[i + 1]; ++p)
        if (col[p] < coff[b] || col[p] >= coff[b + 1]) bad[0] = 1;
}

// y = blockdiag(inv_b) x: row i of block b is a dot product with row (i - off[b]) of inv_b,
// summed exactly as dense_gemv_kernel sums a row of a single inverse.
template <typename T>
__global__ __launch_bounds__(kBlock) void block_dense_gemv_kernel(int32_t n, int32_t nblk,
                                                                 const int32_t* __restrict__ off,
                                                                 const int64_t* __restrict__ doff,
                                                                 const double* __restrict__ inv,
                                                                 const T* __restrict__ x, T* __restrict__ y) {
    const int32_t row = blockIdx.x * (kBlock / 64) + threadIdx.x / 64;
    const int lane = threadIdx.x & 63;
    double s = 0.0;
    if (row < n) {
        const int32_t b = block_of(row, nblk, off);
        const int32_t o = off[b], nb = off[b + 1] - o;
        const double* a = inv + doff[b] + static_cast<int64_t>(row - o) * nb;
        for (int32_t j = lane; j < nb; j += 64) s += a[j] * static_cast<double>(x[o + j]);
    }
#pragma unroll
    for (int off2 = 32; off2 > 0; off2 >>= 1) s += __shfl_xor(s, off2, 64);
    if (row < n && lane == 0) y[row] = static_cast<T>(s);
}

}  // namespace

hipError_t extract_diag(int32_t n, const int32_t* ptr, const int32_t* col, const double* val, double* diag,
                        int32_t* bad, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    extract_diag_kernel<<<grid_for(n), kBlock, 0, stream>>>(n, ptr, col, val, diag, bad);
    return hipGetLastError();
}

hipError_t offdiag_absmax(int32_t n, const int32_t* ptr, const int32_t* col, const double* val, double* partial,
                          double* scale, hipStream_t stream) {
    absmax_partial_kernel<<<kReduceBlocks, kBlock, 0, stream>>>(n, ptr, col, val, partial);
    absmax_final_kernel<<<1, kBlock, 0, stream>>>(partial, scale);
    return hipGetLastError();
}

// --- packed columns --------------------------------------------------------------------
// One workgroup per row block: the base column (the middle entry of the block's middle row,
// less 32767, at least 0: with sorted columns that entry sits among the row's near neighbours,
// the diagonal for a level matrix, so the 16-bit window is centred on the block's own
// neighbourhood), every entry's offset from it, and the count of far entries into cnt[b + 1]
// (none for a block beyond the product buffer, whose rows read the plain columns).
__global__ __launch_bounds__(kBlock) void pack_count_kernel(int32_t nrows, int rows, const int32_t* __restrict__ ptr,
                                                           const int32_t* __restrict__ col, uint16_t* __restrict__ off,
                                                           int32_t* __restrict__ base, int32_t* __restrict__ cnt) {
    __shared__ int32_t nfar;
    const int32_t b = blockIdx.x;
    const int32_t r0 = b * rows, r1 = min(r0 + rows, nrows);
    const int32_t e0 = ptr[r0], ne = ptr[r1] - e0;
    const int32_t rm = r0 + (r1 - r0) / 2;
    const int32_t mb = ptr[rm], me = ptr[rm + 1];
    const int32_t anchor = me > mb ? col[mb + (me - mb) / 2] : (ne > 0 ? col[e0 + ne / 2] : 0);
    const int32_t bs = max(0, anchor - 32767);
    if (threadIdx.x == 0) nfar = 0;
    __syncthreads();
    int32_t mine = 0;
    for (int32_t k = threadIdx.x; k < ne; k += kBlock) {
        const int64_t o = static_cast<int64_t>(col[e0 + k]) - bs;
        const bool near = o >= 0 && o < kFarCol;
        off[e0 + k] = near ? static_cast<uint16_t>(o) : kFarCol;
        mine += near ? 0 : 1;
    }
    if (mine) atomicAdd(&nfar, mine);
    __syncthreads();
    if (threadIdx.x == 0) {
        base[b] = bs;
        cnt[b + 1] = ne <= kStreamCap ? nfar : 0;
    }
}

// Far entries of each block at foff[b]..: entry index within the block and full column. Their
// order within a block is immaterial (each one is written to its own product slot).
__global__ __launch_bounds__(kBlock) void pack_far_kernel(int32_t nrows, int rows, const int32_t* __restrict__ ptr,
                                                         const int32_t* __restrict__ col,
                                                         const uint16_t* __restrict__ off,
                                                         const int32_t* __restrict__ foff,
                                                         uint16_t* __restrict__ fslot, int32_t* __restrict__ fcol) {
    __shared__ int32_t pos;
    const int32_t b = blockIdx.x;
    const int32_t r0 = b * rows, r1 = min(r0 + rows, nrows);
    const int32_t e0 = ptr[r0], ne = ptr[r1] - e0;
    if (ne > kStreamCap || foff[b + 1] == foff[b]) return;  // uniform over the workgroup
    const int32_t f0 = foff[b];
    if (threadIdx.x == 0) pos = 0;
    __syncthreads();
    for (int32_t k = threadIdx.x; k < ne; k += kBlock)
        if (off[e0 + k] == kFarCol) {
            const int32_t j = f0 + atomicAdd(&pos, 1);
            fslot[j] = static_cast<uint16_t>(k);
            fcol[j] = col[e0 + k];
        }
}

hipError_t pack_columns(int32_t nrows, int32_t nnz, const int32_t* ptr, const int32_t* col, int rows, uint16_t* off,
                        int32_t* base, int32_t* foff, uint16_t* fslot, int32_t* fcol, int64_t cap, int32_t* parts,
                        int64_t* nfar, hipStream_t stream) {
    *nfar = -1;
    if (nrows <= 0 || nnz <= 0 || rows <= 0) return hipSuccess;
    const int32_t nb = (nrows + rows - 1) / rows;
    hipError_t e = vec_zero_bytes(foff, sizeof(int32_t), stream);
    if (e != hipSuccess) return e;
    pack_count_kernel<<<nb, kBlock, 0, stream>>>(nrows, rows, ptr, col, off, base, foff);
    // in-place inclusive scan of the counts foff[1..nb]: foff[b] = far entries before block b
    const int32_t nparts = static_cast<int32_t>(
        std::min<int64_t>(kScanParts, (static_cast<int64_t>(nb) + kScanBlock - 1) / kScanBlock));
    const int32_t piece = static_cast<int32_t>((static_cast<int64_t>(nb) + nparts - 1) / nparts);
    scan_reduce_kernel<<<nparts, kScanBlock, 0, stream>>>(nb, piece, foff, parts);
    scan_parts_kernel<<<1, kScanBlock, 0, stream>>>(nparts, parts);
    scan_apply_kernel<<<nparts, kScanBlock, 0, stream>>>(nb, piece, foff, parts);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    int32_t total = 0;
    if ((e = hipMemcpyAsync(&total, foff + nb, sizeof(int32_t), hipMemcpyDeviceToHost, stream)) != hipSuccess ||
        (e = hipStreamSynchronize(stream)) != hipSuccess)
        return e;
    *nfar = total;
    if (total > cap || total == 0) return hipSuccess;  // over capacity: the plain columns stay in use
    pack_far_kernel<<<nb, kBlock, 0, stream>>>(nrows, rows, ptr, col, off, foff, fslot, fcol);
    return hipGetLastError();
}

hipError_t transpose_csr(int32_t nf, int32_t nc, int32_t nnz, const int32_t* p_ptr, const int32_t* p_col,
                         const double* p_val, int32_t* r_ptr, int32_t* r_col, double* r_val, int32_t* cursor,
                         hipStream_t stream) {
    hipError_t e = vec_zero_bytes(r_ptr, sizeof(int32_t) * (nc + 1), stream);
    if (e != hipSuccess) return e;
    if (nnz > 0) count_cols_kernel<<<grid_for(nnz), kBlock, 0, stream>>>(nnz, p_col, r_ptr);
    // piece sums live in `cursor`, which is free until the scatter below
    const int32_t nparts = static_cast<int32_t>(std::min<int64_t>(kScanParts, (static_cast<int64_t>(nc) + kScanBlock - 1) / kScanBlock));
    const int32_t piece = static_cast<int32_t>((static_cast<int64_t>(nc) + nparts - 1) / nparts);
    scan_reduce_kernel<<<nparts, kScanBlock, 0, stream>>>(nc, piece, r_ptr, cursor);
    scan_parts_kernel<<<1, kScanBlock, 0, stream>>>(nparts, cursor);
    scan_apply_kernel<<<nparts, kScanBlock, 0, stream>>>(nc, piece, r_ptr, cursor);
    if ((e = vec_copy<int32_t>(nc, r_ptr, cursor, stream)) != hipSuccess) return e;
    scatter_transpose_kernel<<<grid_for(nf), kBlock, 0, stream>>>(nf, p_ptr, p_col, p_val, cursor, r_col, r_val);
    sort_rows_kernel<<<grid_for(nc), kBlock, 0, stream>>>(nc, r_ptr, r_col, r_val);
    return hipGetLastError();
}

hipError_t dense_from_csr(int32_t n, const int32_t* ptr, const int32_t* col, const double* val, double* M,
                          int singular, hipStream_t stream, int32_t col0) {
    const int64_t total = static_cast<int64_t>(n) * n;
    dense_zero_kernel<<<grid_for(total), kBlock, 0, stream>>>(total, M);
    dense_scatter_kernel<<<grid_for(n), kBlock, 0, stream>>>(n, ptr, col, val, col0, M);
    if (singular) dense_rank_one_kernel<<<1, 1024, 0, stream>>>(n, M);
    return hipGetLastError();
}

hipError_t dense_lu_inverse(int32_t n, double* M, int32_t* piv, double* inv, int32_t* bad, hipStream_t stream) {
    dense_lu_kernel<<<1, 1024, 0, stream>>>(n, M, piv, bad);
    dense_inverse_cols_kernel<<<n, kBlock, sizeof(double) * n, stream>>>(n, M, piv, bad, inv);
    return hipGetLastError();
}

template <typename T>
hipError_t dense_gemv(int32_t n, const double* inv, const T* x, T* y, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const dim3 grid(static_cast<unsigned>((n + kBlock / 64 - 1) / (kBlock / 64)));
    return launch_kernel(dense_gemv_kernel<T>, grid, dim3(kBlock), stream, n, inv, x, y);
}
template hipError_t dense_gemv<float>(int32_t, const double*, const float*, float*, hipStream_t);
template hipError_t dense_gemv<double>(int32_t, const double*, const double*, double*, hipStream_t);

hipError_t block_absmax(int32_t nblk, const int32_t* off, const int32_t* ptr, const int32_t* col, const double* val,
                        double* scale, hipStream_t stream) {
    if (nblk <= 0) return hipSuccess;
    block_absmax_kernel<<<nblk, kBlock, 0, stream>>>(off, ptr, col, val, scale);
    return hipGetLastError();
}

hipError_t prolong_blocks_check(int32_t n, const int32_t* ptr, const int32_t* col, int32_t nblk, const int32_t* foff,
                                const int32_t* coff, int32_t* bad, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    prolong_blocks_kernel<<<grid_for(n), kBlock, 0, stream>>>(n, ptr, col, nblk, foff, coff, bad);
    return hipGetLastError();
}

template <typename T>
hipError_t block_dense_gemv(int32_t n, int32_t nblk, const int32_t* off, const int64_t* doff, const double* inv,
                            const T* x, T* y, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const dim3 grid(static_cast<unsigned>((n + kBlock / 64 - 1) / (kBlock / 64)));
    return launch_kernel(block_dense_gemv_kernel<T>, grid, dim3(kBlock), stream, n, nblk, off, doff, inv, x, y);
}
template hipError_t block_dense_gemv<float>(int32_t, int32_t, const int32_t*, const int64_t*, const double*,
                                            const float*, float*, hipStream_t);
template hipError_t block_dense_gemv<double>(int32_t, int32_t, const int32_t*, const int64_t*, const double*,
                                             const double*, double*, hipStream_t);

}  // namespace amgg
