// Device setup of one level (paper Sec. 2.2; Sec. 4: classical Ruge-Stueben, strength threshold
// theta; Alg. 1, step 2), bitwise equal to the host RS setup: strength of connection, direct
// interpolation from a given C/F split (the split itself, a sequential greedy, stays on the
// host) and the Galerkin product A_c = R (A P) with R = P^T.
//
// Each sparse product C = L * M is formed in two phases:
//   symbolic  every product L_ij M_jk is expanded to a key (row i, column k); one radix sort
//             of the keys and a unique pass give C's pattern (rows in order, columns
//             ascending) without any floating point;
//   numeric   one thread per entry c_ik walks row i of L in ascending column order and adds
//             L_ij M_jk for every j whose row of M holds column k (binary search), starting
//             from 0.0, with product and sum rounded separately.
// The numeric order is exactly the row-by-row accumulation of the host product, so the
// result does not depend on how the symbolic phase orders or batches its work. The
// expansion is processed in row chunks that bound the temporary memory.
// This file is compiled with -ffp-contract=off: no product may be fused into its sum.
#include <hip/hip_runtime.h>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/device/device_select.hpp>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "amggnn.h"
#include "errors.hpp"
#include "kernels.hpp"

namespace amgg {
int hip_fail(hipError_t e, const char* where);
}

using namespace amgg;

namespace {

constexpr int kThreads = 256;

inline unsigned blocks_for(int64_t n) { return static_cast<unsigned>((n + kThreads - 1) / kThreads); }

// One thread per item; nothing is launched for zero items.
template <typename... KArgs, typename... Args>
void launch(void (*kernel)(KArgs...), int64_t items, hipStream_t st, Args... args) {
    if (items > 0)
        hipLaunchKernelGGL(kernel, dim3(blocks_for(items)), dim3(kThreads), 0, st, static_cast<KArgs>(args)...);
}

inline int bit_width(uint64_t v) {
    int b = 0;
    while (v) {
        ++b;
        v >>= 1;
    }
    return b;
}

// bad = 1 unless rows [0, n) form a CSR pattern with nnz entries and strictly ascending
// columns in [0, ncols); `bad` must be 0 on entry.
__global__ void validate_csr_kernel(int32_t n, int32_t ncols, int32_t nnz, const int32_t* __restrict__ ptr,
                                    const int32_t* __restrict__ col, int32_t* __restrict__ bad) {
    const int32_t i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const int32_t lo = ptr[i], hi = ptr[i + 1];
    bool ok = lo >= 0 && hi >= lo && hi <= nnz && (i > 0 || lo == 0) && (i < n - 1 || hi == nnz);
    for (int32_t p = lo; ok && p < hi; ++p) {
        const int32_t c = col[p];
        ok = c >= 0 && c < ncols && (p == lo || c > col[p - 1]);
    }
    if (!ok) *bad = 1;
}

// row[p] = i for every entry p of row i.
__global__ void row_index_kernel(int32_t n, const int32_t* __restrict__ ptr, int32_t* __restrict__ row) {
    const int32_t i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    for (int32_t p = ptr[i]; p < ptr[i + 1]; ++p) row[p] = i;
}

// cnt[p] = length of the row of M that L's entry p selects; cnt[nnz_l] = 0 (scan sentinel).
__global__ void product_count_kernel(int32_t nnz_l, const int32_t* __restrict__ lcol,
                                     const int32_t* __restrict__ mptr, int64_t* __restrict__ cnt) {
    const int32_t p = blockIdx.x * kThreads + threadIdx.x;
    if (p > nnz_l) return;
    int64_t c = 0;
    if (p < nnz_l) {
        const int32_t j = lcol[p];
        c = mptr[j + 1] - mptr[j];
    }
    cnt[p] = c;
}

// Row chunk boundaries: bounds[m] = the last row r with (products before r) <= m * budget;
// bounds[0] = 0, bounds[m_count] = n. boff[m] = products before bounds[m].
__global__ void chunk_bounds_kernel(int32_t n, const int32_t* __restrict__ lptr, const int64_t* __restrict__ loff,
                                    int64_t budget, int32_t m_count, int32_t* __restrict__ bounds,
                                    int64_t* __restrict__ boff) {
    const int32_t m = blockIdx.x * kThreads + threadIdx.x;
    if (m > m_count) return;
    int32_t r;
    if (m == 0) {
        r = 0;
    } else if (m == m_count) {
        r = n;
    } else {
        const int64_t target = budget * m;
        int32_t lo = 0, hi = n;  // invariant: poff(lo) <= target; answer in [lo, hi]
        while (lo < hi) {
            const int32_t mid = lo + (hi - lo + 1) / 2;
            if (loff[lptr[mid]] <= target)
                lo = mid;
            else
                hi = mid - 1;
        }
        r = lo;
    }
    bounds[m] = r;
    boff[m] = loff[lptr[r]];
}

// Keys of the products of L's entries [p0, p1): (row - r0) << kb | column of M.
__global__ void expand_kernel(int32_t p0, int32_t p1, const int32_t* __restrict__ lrow,
                              const int32_t* __restrict__ lcol, const int64_t* __restrict__ loff, int64_t base,
                              int32_t r0, int kb, const int32_t* __restrict__ mptr, const int32_t* __restrict__ mcol,
                              uint64_t* __restrict__ keys) {
    const int32_t p = p0 + blockIdx.x * kThreads + threadIdx.x;
    if (p >= p1) return;
    const int32_t j = lcol[p];
    const uint64_t hi = static_cast<uint64_t>(lrow[p] - r0) << kb;
    uint64_t* out = keys + (loff[p] - base);
    for (int32_t q = mptr[j]; q < mptr[j + 1]; ++q) *out++ = hi | static_cast<uint32_t>(mcol[q]);
}

__global__ void decode_cols_kernel(int32_t u, const uint64_t* __restrict__ uniq, uint64_t mask,
                                   int32_t* __restrict__ col) {
    const int32_t e = blockIdx.x * kThreads + threadIdx.x;
    if (e < u) col[e] = static_cast<int32_t>(uniq[e] & mask);
}

// rowptr[r] = base + (number of unique keys of rows before r), for the chunk's rows.
__global__ void decode_rowptr_kernel(int32_t rows, const uint64_t* __restrict__ uniq, int32_t u, int kb,
                                     int32_t base, int32_t* __restrict__ rowptr) {
    const int32_t r = blockIdx.x * kThreads + threadIdx.x;
    if (r >= rows) return;
    const uint64_t key = static_cast<uint64_t>(r) << kb;
    int32_t lo = 0, hi = u;
    while (lo < hi) {
        const int32_t mid = lo + (hi - lo) / 2;
        if (uniq[mid] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    rowptr[r] = base + lo;
}

__global__ void set_int_kernel(int32_t* __restrict__ dst, int32_t v) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *dst = v;
}

// c_ik = sum over L's row i, ascending j, of L_ij * M_jk where M_jk is stored.
__global__ void numeric_kernel(int32_t u, const int32_t* __restrict__ crow, const int32_t* __restrict__ ccol,
                               const int32_t* __restrict__ lptr, const int32_t* __restrict__ lcol,
                               const double* __restrict__ lval, const int32_t* __restrict__ mptr,
                               const int32_t* __restrict__ mcol, const double* __restrict__ mval,
                               double* __restrict__ cval) {
    const int32_t e = blockIdx.x * kThreads + threadIdx.x;
    if (e >= u) return;
    const int32_t i = crow[e], k = ccol[e];
    double s = 0.0;
    for (int32_t p = lptr[i]; p < lptr[i + 1]; ++p) {
        const int32_t j = lcol[p];
        const int32_t end = mptr[j + 1];
        int32_t lo = mptr[j], hi = end;
        while (lo < hi) {
            const int32_t mid = lo + (hi - lo) / 2;
            if (mcol[mid] < k)
                lo = mid + 1;
            else
                hi = mid;
        }
        if (lo < end && mcol[lo] == k) s = s + lval[p] * mval[lo];
    }
    cval[e] = s;
}

// flag[e] = 1 for entries kept in A_c (nonzero or diagonal); flag[u] = 0 (scan sentinel).
__global__ void keep_flag_kernel(int32_t u, const int32_t* __restrict__ crow, const int32_t* __restrict__ ccol,
                                 const double* __restrict__ cval, int32_t* __restrict__ flag) {
    const int32_t e = blockIdx.x * kThreads + threadIdx.x;
    if (e > u) return;
    flag[e] = e < u && (cval[e] != 0.0 || ccol[e] == crow[e]) ? 1 : 0;
}

__global__ void compact_kernel(int32_t u, const int32_t* __restrict__ flag, const int32_t* __restrict__ pos,
                               const int32_t* __restrict__ ccol, const double* __restrict__ cval,
                               int32_t* __restrict__ col2, double* __restrict__ val2) {
    const int32_t e = blockIdx.x * kThreads + threadIdx.x;
    if (e >= u || !flag[e]) return;
    col2[pos[e]] = ccol[e];
    val2[pos[e]] = cval[e];
}

__global__ void remap_rowptr_kernel(int32_t n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ pos,
                                    int32_t* __restrict__ rowptr2) {
    const int32_t i = blockIdx.x * kThreads + threadIdx.x;
    if (i <= n) rowptr2[i] = pos[rowptr[i]];
}

// ---------------------------------------------------------------------------------------
// Host orchestration
// ---------------------------------------------------------------------------------------
struct Failure {
    int code;
    std::string msg;
};

void check(hipError_t e, const char* where) {
    if (e != hipSuccess) throw Failure{AMGG_EHIP, std::string(where) + ": " + hipGetErrorString(e)};
}

// Device memory from the caller's allocator; what is not taken as a result is released
// when the pool goes out of scope.
class Pool {
  public:
    Pool(amgg_alloc_fn a, amgg_release_fn r, void* u, hipStream_t st) : alloc_(a), release_(r), user_(u), st_(st) {}
    ~Pool() {
        if (!live_.empty()) (void)hipStreamSynchronize(st_);  // queued work may still use them
        for (void* p : live_) release_(p, user_);
    }
    template <class T>
    T* get(int64_t count) {
        const size_t bytes = static_cast<size_t>(std::max<int64_t>(count, 1)) * sizeof(T);
        void* p = alloc_(bytes, user_);
        if (!p) throw Failure{AMGG_EWORKSPACE, "amgg_galerkin_device: allocation of " + std::to_string(bytes) +
                                                   " bytes failed"};
        live_.push_back(p);
        return static_cast<T*>(p);
    }
    void put(const void* p) {
        auto it = std::find(live_.begin(), live_.end(), p);
        if (it == live_.end()) return;
        check(hipStreamSynchronize(st_), "hipStreamSynchronize");
        release_(*it, user_);
        live_.erase(it);
    }
    void keep(const void* p) {  // hand to the caller
        auto it = std::find(live_.begin(), live_.end(), p);
        if (it != live_.end()) live_.erase(it);
    }

  private:
    amgg_alloc_fn alloc_;
    amgg_release_fn release_;
    void* user_;
    hipStream_t st_;
    std::vector<void*> live_;
};


struct DevCsr {
    int32_t nrows = 0, ncols = 0, nnz = 0;
    int32_t* ptr = nullptr;
    int32_t* col = nullptr;
    double* val = nullptr;
};

struct ConstCsr {
    int32_t nrows, ncols, nnz;
    const int32_t* ptr;
    const int32_t* col;
    const double* val;
};

template <class T>
T read_back(const T* dev, hipStream_t st) {
    T v{};
    check(hipMemcpyAsync(&v, dev, sizeof(T), hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    check(hipStreamSynchronize(st), "hipStreamSynchronize");
    return v;
}

// C = L * M with the pattern of every structurally generated entry (zeros kept).
DevCsr spgemm(Pool& pool, const ConstCsr& L, const ConstCsr& M, int64_t budget, hipStream_t st) {
    const int32_t n = L.nrows;
    DevCsr C;
    C.nrows = n;
    C.ncols = M.ncols;
    C.ptr = pool.get<int32_t>(static_cast<int64_t>(n) + 1);
    // products per entry of L and their offsets (row i's products start at loff[lptr[i]])
    int32_t* lrow = pool.get<int32_t>(L.nnz);
    int64_t* cnt = pool.get<int64_t>(static_cast<int64_t>(L.nnz) + 1);
    int64_t* loff = pool.get<int64_t>(static_cast<int64_t>(L.nnz) + 1);
    launch(row_index_kernel, n, st, n, L.ptr, lrow);
    launch(product_count_kernel, static_cast<int64_t>(L.nnz) + 1, st,
                       L.nnz, L.col, M.ptr, cnt);
    check(hipGetLastError(), "product count");
    size_t tb = 0;
    check(rocprim::exclusive_scan(nullptr, tb, cnt, loff, int64_t{0}, static_cast<size_t>(L.nnz) + 1,
                                  rocprim::plus<int64_t>(), st),
          "scan size");
    void* tmp = pool.get<unsigned char>(static_cast<int64_t>(tb));
    check(rocprim::exclusive_scan(tmp, tb, cnt, loff, int64_t{0}, static_cast<size_t>(L.nnz) + 1,
                                  rocprim::plus<int64_t>(), st),
          "product offsets");
    pool.put(tmp);
    pool.put(cnt);
    const int64_t total = read_back(loff + L.nnz, st);

    // row chunks of at most about `budget` products
    const int32_t m_count = static_cast<int32_t>(std::max<int64_t>(1, (total + budget - 1) / budget));
    int32_t* dbounds = pool.get<int32_t>(m_count + 1);
    int64_t* dboff = pool.get<int64_t>(m_count + 1);
    launch(chunk_bounds_kernel, m_count + 1, st, n, L.ptr, loff,
                       budget, m_count, dbounds, dboff);
    check(hipGetLastError(), "chunk bounds");
    std::vector<int32_t> bounds(m_count + 1);
    std::vector<int64_t> boff(m_count + 1);
    check(hipMemcpyAsync(bounds.data(), dbounds, sizeof(int32_t) * (m_count + 1), hipMemcpyDeviceToHost, st), "copy");
    check(hipMemcpyAsync(boff.data(), dboff, sizeof(int64_t) * (m_count + 1), hipMemcpyDeviceToHost, st), "copy");
    check(hipStreamSynchronize(st), "hipStreamSynchronize");
    pool.put(dbounds);
    pool.put(dboff);

    const int kb = std::max(1, bit_width(static_cast<uint64_t>(std::max(M.ncols, 1) - 1)));
    const uint64_t mask = (uint64_t{1} << kb) - 1;
    std::vector<int32_t*> part_col;
    std::vector<int32_t> part_u;
    int64_t u_total = 0;
    int32_t* dnum = pool.get<int32_t>(1);
    for (int32_t m = 0; m < m_count; ++m) {
        const int32_t r0 = bounds[m], r1 = bounds[m + 1];
        if (r1 <= r0) continue;
        const int64_t tc = boff[m + 1] - boff[m];
        if (tc > INT32_MAX) throw Failure{AMGG_EINVAL, "amgg_galerkin_device: a row holds more than 2^31 - 1 products"};
        int32_t u = 0;
        int32_t* col = pool.get<int32_t>(std::max<int64_t>(tc, 1));
        if (tc > 0) {
            const int rb = std::max(1, bit_width(static_cast<uint64_t>(r1 - r0 - 1)));
            uint64_t* ka = pool.get<uint64_t>(tc);
            uint64_t* kbuf = pool.get<uint64_t>(tc);
            int32_t p0 = 0, p1 = 0;
            check(hipMemcpyAsync(&p0, L.ptr + r0, sizeof(int32_t), hipMemcpyDeviceToHost, st), "copy");
            check(hipMemcpyAsync(&p1, L.ptr + r1, sizeof(int32_t), hipMemcpyDeviceToHost, st), "copy");
            check(hipStreamSynchronize(st), "hipStreamSynchronize");
            launch(expand_kernel, p1 - p0, st, p0, p1, lrow, L.col,
                               loff, boff[m], r0, kb, M.ptr, M.col, ka);
            check(hipGetLastError(), "expand");
            rocprim::double_buffer<uint64_t> db(ka, kbuf);
            size_t sb = 0, ub = 0;
            const unsigned int end_bit = static_cast<unsigned int>(kb + rb);
            check(rocprim::radix_sort_keys(nullptr, sb, db, static_cast<size_t>(tc), 0u, end_bit, st), "sort size");
            check(rocprim::unique(nullptr, ub, db.current(), db.alternate(), dnum, static_cast<size_t>(tc),
                                  rocprim::equal_to<uint64_t>(), st),
                  "unique size");
            void* t2 = pool.get<unsigned char>(static_cast<int64_t>(std::max(sb, ub)));
            check(rocprim::radix_sort_keys(t2, sb, db, static_cast<size_t>(tc), 0u, end_bit, st), "sort");
            uint64_t* sorted = db.current();
            uint64_t* uniq = db.alternate();
            check(rocprim::unique(t2, ub, sorted, uniq, dnum, static_cast<size_t>(tc), rocprim::equal_to<uint64_t>(),
                                  st),
                  "unique");
            pool.put(t2);
            u = read_back(dnum, st);
            if (u_total + u > INT32_MAX)
                throw Failure{AMGG_EINVAL, "amgg_galerkin_device: product has more than 2^31 - 1 entries"};
            launch(decode_cols_kernel, u, st, u, uniq, mask, col);
            launch(decode_rowptr_kernel, r1 - r0, st, r1 - r0, uniq,
                               u, kb, static_cast<int32_t>(u_total), C.ptr + r0);
            check(hipGetLastError(), "decode");
            check(hipStreamSynchronize(st), "hipStreamSynchronize");
            pool.put(ka);
            pool.put(kbuf);
        } else {
            launch(decode_rowptr_kernel, r1 - r0, st, r1 - r0,
                               static_cast<const uint64_t*>(nullptr), 0, kb, static_cast<int32_t>(u_total), C.ptr + r0);
            check(hipGetLastError(), "decode");
        }
        part_col.push_back(col);
        part_u.push_back(u);
        u_total += u;
    }
    pool.put(dnum);
    pool.put(lrow);
    pool.put(loff);
    hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(1), 0, st, C.ptr + n, static_cast<int32_t>(u_total));
    check(hipGetLastError(), "row pointer");
    C.nnz = static_cast<int32_t>(u_total);
    if (part_col.size() == 1) {
        C.col = part_col[0];
    } else {
        C.col = pool.get<int32_t>(u_total);
        int64_t at = 0;
        for (size_t c = 0; c < part_col.size(); ++c) {
            if (part_u[c] > 0)
                check(hipMemcpyAsync(C.col + at, part_col[c], sizeof(int32_t) * part_u[c], hipMemcpyDeviceToDevice,
                                     st),
                      "copy");
            at += part_u[c];
        }
        check(hipStreamSynchronize(st), "hipStreamSynchronize");
        for (int32_t* p : part_col) pool.put(p);
    }
    // numeric phase
    int32_t* crow = pool.get<int32_t>(C.nnz);
    C.val = pool.get<double>(C.nnz);
    launch(row_index_kernel, n, st, n, C.ptr, crow);
    launch(numeric_kernel, C.nnz, st, C.nnz, crow, C.col, L.ptr,
                       L.col, L.val, M.ptr, M.col, M.val, C.val);
    check(hipGetLastError(), "numeric");
    check(hipStreamSynchronize(st), "hipStreamSynchronize");
    pool.put(crow);
    return C;
}

// Drops exact zeros off the diagonal; the result's arrays replace C's.
DevCsr drop_zeros(Pool& pool, const DevCsr& C, hipStream_t st) {
    int32_t* crow = pool.get<int32_t>(C.nnz);
    int32_t* flag = pool.get<int32_t>(static_cast<int64_t>(C.nnz) + 1);
    int32_t* pos = pool.get<int32_t>(static_cast<int64_t>(C.nnz) + 1);
    launch(row_index_kernel, C.nrows, st, C.nrows, C.ptr, crow);
    launch(keep_flag_kernel, static_cast<int64_t>(C.nnz) + 1, st,
                       C.nnz, crow, C.col, C.val, flag);
    check(hipGetLastError(), "keep flags");
    size_t tb = 0;
    check(rocprim::exclusive_scan(nullptr, tb, flag, pos, int32_t{0}, static_cast<size_t>(C.nnz) + 1,
                                  rocprim::plus<int32_t>(), st),
          "scan size");
    void* tmp = pool.get<unsigned char>(static_cast<int64_t>(tb));
    check(rocprim::exclusive_scan(tmp, tb, flag, pos, int32_t{0}, static_cast<size_t>(C.nnz) + 1,
                                  rocprim::plus<int32_t>(), st),
          "keep positions");
    pool.put(tmp);
    const int32_t kept = read_back(pos + C.nnz, st);
    DevCsr D = C;
    if (kept != C.nnz) {
        D.nnz = kept;
        D.ptr = pool.get<int32_t>(static_cast<int64_t>(C.nrows) + 1);
        D.col = pool.get<int32_t>(kept);
        D.val = pool.get<double>(kept);
        launch(compact_kernel, C.nnz, st, C.nnz, flag, pos, C.col,
                           C.val, D.col, D.val);
        launch(remap_rowptr_kernel, static_cast<int64_t>(C.nrows) + 1, st, C.nrows, C.ptr, pos, D.ptr);
        check(hipGetLastError(), "compact");
        check(hipStreamSynchronize(st), "hipStreamSynchronize");
        pool.put(C.ptr);
        pool.put(C.col);
        pool.put(C.val);
    }
    pool.put(crow);
    pool.put(flag);
    pool.put(pos);
    return D;
}

// ---------------------------------------------------------------------------------------
// Strength and direct interpolation: one thread per row, the host setup's formulas in the
// host setup's order (entries in stored, ascending column order; every operation rounded).
// ---------------------------------------------------------------------------------------
// strong[p] = 1 when entry p (column j != i) of row i has -a_ij >= theta max_{k != i}(-a_ik)
// and that max is positive.
__global__ void strength_kernel(int32_t n, const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                const double* __restrict__ val, double theta, uint8_t* __restrict__ strong) {
    const int32_t i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const int32_t pb = ptr[i], pe = ptr[i + 1];
    double big = -INFINITY;
    bool any_off = false;
    for (int32_t p = pb; p < pe; ++p) {
        if (col[p] == i) continue;
        any_off = true;
        const double v = -val[p];
        big = big < v ? v : big;
    }
    const bool some = any_off && big > 0.0;
    const double cut = theta * big;
    for (int32_t p = pb; p < pe; ++p) strong[p] = some && col[p] != i && -val[p] >= cut ? 1 : 0;
}

// cf as int32 with a trailing 0 (its exclusive scan numbers the C points)
__global__ void cf_to_int_kernel(int32_t n, const int8_t* __restrict__ cf, int32_t* __restrict__ out) {
    const int32_t i = blockIdx.x * kThreads + threadIdx.x;
    if (i < n) out[i] = cf[i] != 0 ? 1 : 0;
    if (i == n) out[i] = 0;
}

// entries of P's row i: 1 for a C point, else the strong C neighbours (0: no interpolation)
__global__ void interp_count_kernel(int32_t n, const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                    const uint8_t* __restrict__ strong, const int8_t* __restrict__ cf,
                                    int32_t* __restrict__ cnt) {
    const int32_t i = blockIdx.x * kThreads + threadIdx.x;
    if (i == n) cnt[i] = 0;
    if (i >= n) return;
    if (cf[i] != 0) {
        cnt[i] = 1;
        return;
    }
    int32_t c = 0;
    for (int32_t p = ptr[i]; p < ptr[i + 1]; ++p) c += strong[p] && cf[col[p]] != 0 ? 1 : 0;
    cnt[i] = c;
}

// Direct interpolation with positive couplings lumped on the diagonal: an F row with strong C
// neighbours C_i gets w_ik = -(alpha_i a_ik) / (a_ii + sum of its positive off-diagonals), with
// alpha_i = (sum of its negative off-diagonals) / (sum of a_ik over C_i); a C row is the identity.
__global__ void interp_fill_kernel(int32_t n, const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                   const double* __restrict__ val, const uint8_t* __restrict__ strong,
                                   const int8_t* __restrict__ cf, const int32_t* __restrict__ cidx,
                                   const int32_t* __restrict__ prow, int32_t* __restrict__ pcol,
                                   double* __restrict__ pval) {
    const int32_t i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    int32_t q = prow[i];
    if (cf[i] != 0) {
        pcol[q] = cidx[i];
        pval[q] = 1.0;
        return;
    }
    if (prow[i + 1] == q) return;
    const int32_t pb = ptr[i], pe = ptr[i + 1];
    double a_ii = 0.0;
    for (int32_t p = pb; p < pe; ++p)
        if (col[p] == i) a_ii = val[p];
    double lumped = a_ii, neg_sum = 0.0, strong_c_sum = 0.0;
    for (int32_t p = pb; p < pe; ++p) {
        const int32_t k = col[p];
        if (k == i) continue;
        const double a = val[p];
        if (a > 0.0) lumped = lumped + a;
        if (a < 0.0) neg_sum = neg_sum + a;
        if (strong[p] && cf[k] != 0) strong_c_sum = strong_c_sum + a;
    }
    const double ratio = neg_sum / strong_c_sum;
    for (int32_t p = pb; p < pe; ++p) {
        const int32_t k = col[p];
        if (!(strong[p] && cf[k] != 0)) continue;
        pcol[q] = cidx[k];
        pval[q] = -(ratio * val[p]) / lumped;
        ++q;
    }
}

// bad[0] = 1 unless (ptr, col) is a CSR pattern of n rows, nnz entries, ascending columns < n
void validate_square(Pool& pool, int32_t n, int32_t nnz, const int32_t* ptr, const int32_t* col, const char* who,
                     hipStream_t st) {
    int32_t* bad = pool.get<int32_t>(1);
    hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(1), 0, st, bad, 0);
    launch(validate_csr_kernel, n, st, n, n, nnz, ptr, col, bad);
    check(hipGetLastError(), "validate");
    if (read_back(bad, st))
        throw Failure{AMGG_EINVAL, std::string(who) + ": not a CSR pattern of the stated size with ascending columns"};
    pool.put(bad);
}

template <typename T>
void exclusive_scan_i32(Pool& pool, const T* in, int32_t* out, int64_t count, hipStream_t st) {
    size_t tb = 0;
    check(rocprim::exclusive_scan(nullptr, tb, in, out, int32_t{0}, static_cast<size_t>(count),
                                  rocprim::plus<int32_t>(), st),
          "scan size");
    void* tmp = pool.get<unsigned char>(static_cast<int64_t>(tb));
    check(rocprim::exclusive_scan(tmp, tb, in, out, int32_t{0}, static_cast<size_t>(count), rocprim::plus<int32_t>(),
                                  st),
          "scan");
    pool.put(tmp);
}

}  // namespace

extern "C" int amgg_strength_device(int device, int32_t n, const int32_t* rowptr, const int32_t* col,
                                    const double* val, int32_t nnz, double theta, uint8_t* strong,
                                    amgg_alloc_fn alloc, amgg_release_fn release, void* user, void* stream) {
    return guarded([&]() -> int {
        if (n <= 0 || nnz < 0 || !rowptr || !alloc || !release || (nnz > 0 && (!col || !val || !strong)))
            return fail(AMGG_EINVAL, "amgg_strength_device: NULL argument or bad size");
        if (!(theta > 0.0 && theta < 1.0)) return fail(AMGG_EINVAL, "amgg_strength_device: theta outside (0, 1)");
        hipError_t e = hipSetDevice(device);
        if (e != hipSuccess) return hip_fail(e, "amgg_strength_device: hipSetDevice");
        const hipStream_t st = static_cast<hipStream_t>(stream);
        try {
            Pool pool(alloc, release, user, st);
            validate_square(pool, n, nnz, rowptr, col, "amgg_strength_device", st);
            launch(strength_kernel, n, st, n, rowptr, col, val, theta, strong);
            check(hipGetLastError(), "strength");
            return AMGG_OK;
        } catch (const Failure& f) {
            (void)hipStreamSynchronize(st);
            return fail(f.code, f.msg);
        }
    });
}

extern "C" int amgg_interp_device(int device, int32_t n, const int32_t* rowptr, const int32_t* col, const double* val,
                                  int32_t nnz, const uint8_t* strong, const int8_t* cf, amgg_alloc_fn alloc,
                                  amgg_release_fn release, void* user, int32_t* nc, int32_t** p_rowptr,
                                  int32_t** p_col, double** p_val, int32_t* p_nnz, void* stream) {
    return guarded([&]() -> int {
        if (n <= 0 || nnz < 0 || !rowptr || !cf || !alloc || !release || !nc || !p_rowptr || !p_col || !p_val ||
            !p_nnz || (nnz > 0 && (!col || !val || !strong)))
            return fail(AMGG_EINVAL, "amgg_interp_device: NULL argument or bad size");
        hipError_t e = hipSetDevice(device);
        if (e != hipSuccess) return hip_fail(e, "amgg_interp_device: hipSetDevice");
        const hipStream_t st = static_cast<hipStream_t>(stream);
        try {
            Pool pool(alloc, release, user, st);
            validate_square(pool, n, nnz, rowptr, col, "amgg_interp_device", st);
            int32_t* tmp = pool.get<int32_t>(static_cast<int64_t>(n) + 1);
            int32_t* cidx = pool.get<int32_t>(static_cast<int64_t>(n) + 1);
            launch(cf_to_int_kernel, static_cast<int64_t>(n) + 1, st, n, cf, tmp);
            exclusive_scan_i32(pool, tmp, cidx, static_cast<int64_t>(n) + 1, st);
            const int32_t ncoarse = read_back(cidx + n, st);
            if (ncoarse <= 0) throw Failure{AMGG_EINVAL, "amgg_interp_device: no C point"};
            int32_t* prow = pool.get<int32_t>(static_cast<int64_t>(n) + 1);
            launch(interp_count_kernel, static_cast<int64_t>(n) + 1, st, n, rowptr, col, strong, cf, tmp);
            exclusive_scan_i32(pool, tmp, prow, static_cast<int64_t>(n) + 1, st);
            const int32_t total = read_back(prow + n, st);
            pool.put(tmp);
            int32_t* pcol = pool.get<int32_t>(total);
            double* pval = pool.get<double>(total);
            launch(interp_fill_kernel, n, st, n, rowptr, col, val, strong, cf, cidx, prow, pcol, pval);
            check(hipGetLastError(), "interpolation");
            check(hipStreamSynchronize(st), "hipStreamSynchronize");
            pool.put(cidx);
            pool.keep(prow);
            pool.keep(pcol);
            pool.keep(pval);
            *nc = ncoarse;
            *p_rowptr = prow;
            *p_col = pcol;
            *p_val = pval;
            *p_nnz = total;
            return AMGG_OK;
        } catch (const Failure& f) {
            (void)hipStreamSynchronize(st);
            return fail(f.code, f.msg);
        }
    });
}

extern "C" int amgg_galerkin_device(int device, int32_t n, int32_t nc, const int32_t* a_rowptr, const int32_t* a_col,
                                    const double* a_val, int32_t a_nnz, const int32_t* p_rowptr, const int32_t* p_col,
                                    const double* p_val, int32_t p_nnz, amgg_alloc_fn alloc, amgg_release_fn release,
                                    void* user, int64_t chunk_products, int32_t** ac_rowptr, int32_t** ac_col,
                                    double** ac_val, int32_t* ac_nnz, void* stream) {
    return guarded([&]() -> int {
        if (n <= 0 || nc <= 0 || a_nnz < 0 || p_nnz < 0 || !a_rowptr || !p_rowptr || !alloc || !release ||
            !ac_rowptr || !ac_col || !ac_val || !ac_nnz || (a_nnz > 0 && (!a_col || !a_val)) ||
            (p_nnz > 0 && (!p_col || !p_val)) || chunk_products < 0)
            return fail(AMGG_EINVAL, "amgg_galerkin_device: NULL argument or bad size");
        const int64_t budget = chunk_products > 0 ? chunk_products : (int64_t{1} << 27);
        if (budget > INT32_MAX) return fail(AMGG_EINVAL, "amgg_galerkin_device: chunk_products above 2^31 - 1");
        hipError_t e = hipSetDevice(device);
        if (e != hipSuccess) return hip_fail(e, "amgg_galerkin_device: hipSetDevice");
        const hipStream_t st = static_cast<hipStream_t>(stream);
        try {
            Pool pool(alloc, release, user, st);
            int32_t* bad = pool.get<int32_t>(2);
            hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(1), 0, st, bad, 0);
            hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(1), 0, st, bad + 1, 0);
            launch(validate_csr_kernel, n, st, n, n, a_nnz, a_rowptr, a_col, bad);
            launch(validate_csr_kernel, n, st, n, nc, p_nnz, p_rowptr, p_col, bad + 1);
            check(hipGetLastError(), "validate");
            int32_t flags[2] = {0, 0};
            check(hipMemcpyAsync(flags, bad, sizeof(flags), hipMemcpyDeviceToHost, st), "copy");
            check(hipStreamSynchronize(st), "hipStreamSynchronize");
            if (flags[0] || flags[1])
                throw Failure{AMGG_EINVAL, std::string("amgg_galerkin_device: ") + (flags[0] ? "A" : "P") +
                                               " is not a CSR pattern of the stated size with ascending columns"};
            pool.put(bad);
            // R = P^T, the exact transpose (rows in ascending fine index)
            DevCsr R;
            R.nrows = nc;
            R.ncols = n;
            R.nnz = p_nnz;
            R.ptr = pool.get<int32_t>(static_cast<int64_t>(nc) + 1);
            R.col = pool.get<int32_t>(p_nnz);
            R.val = pool.get<double>(p_nnz);
            int32_t* cursor = pool.get<int32_t>(static_cast<int64_t>(nc) + 1);
            check(transpose_csr(n, nc, p_nnz, p_rowptr, p_col, p_val, R.ptr, R.col, R.val, cursor, st), "transpose");
            const ConstCsr A{n, n, a_nnz, a_rowptr, a_col, a_val};
            const ConstCsr P{n, nc, p_nnz, p_rowptr, p_col, p_val};
            DevCsr AP = spgemm(pool, A, P, budget, st);
            pool.put(cursor);
            const ConstCsr Rc{R.nrows, R.ncols, R.nnz, R.ptr, R.col, R.val};
            const ConstCsr APc{AP.nrows, AP.ncols, AP.nnz, AP.ptr, AP.col, AP.val};
            DevCsr G = spgemm(pool, Rc, APc, budget, st);
            pool.put(AP.ptr);
            pool.put(AP.col);
            pool.put(AP.val);
            pool.put(R.ptr);
            pool.put(R.col);
            pool.put(R.val);
            DevCsr Ac = drop_zeros(pool, G, st);
            pool.keep(Ac.ptr);
            pool.keep(Ac.col);
            pool.keep(Ac.val);
            *ac_rowptr = Ac.ptr;
            *ac_col = Ac.col;
            *ac_val = Ac.val;
            *ac_nnz = Ac.nnz;
            return AMGG_OK;
        } catch (const Failure& f) {
            (void)hipStreamSynchronize(st);  // the failure is what is reported
            return fail(f.code, f.msg);
        }
    });
}
