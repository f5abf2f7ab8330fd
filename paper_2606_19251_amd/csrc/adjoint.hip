// Residual-reduction loss of V-cycles and its gradient with respect to every level's
// smoother coefficients (paper Sec. 3.3, Eq. 11; Alg. 1, steps 9-13). The paper obtains the
// gradient by automatic differentiation; here the reverse sweep is written by hand:
//
//   smoothing step  u' = u + Q (f - A u):   ubar = ubar' - A (Q ubar'),  fbar += Q ubar',
//                                          Qbar_ij = ubar'_i r_j  (reduced at once into cbar)
//   restriction     f_c = R (f - A u):      rbar = P fbar_c,  ubar -= A rbar,  fbar += rbar
//   prolongation    u'' = u + P e_c:        ebar_c = R ubar''
//   coarsest        e = A_L^{-1} f:          fbar = A_L^{-1} ebar
//
// using A = A^T, Q = Q^T, R = P^T (symmetric up to rounding). dq_ii/dd_m = x_ii^m / a_ii and
// dq_ij/do_m = x_ij^m / (a_ii + a_jj) with x = a/s. Smoothing iterates are not stored: each
// level keeps its entry iterate and the iterate after its coarse-grid correction, and the
// backward sweep recomputes the k-th smoothing iterate from these.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "amggnn.h"
#include "ctx.hpp"
#include "errors.hpp"
#include "kernels.hpp"

using namespace amgg;

namespace {

constexpr int kMaxC = 2 * AMGG_MAX_DEGREE + 1;

inline dim3 grid_for(int64_t n) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    return dim3(static_cast<unsigned>(g));
}

__device__ __forceinline__ double block_sum(double v) {
    __shared__ double red[kBlock / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x / 64] = v;
    __syncthreads();
    double s = red[0];
    for (int k = 1; k < kBlock / 64; ++k) s += red[k];
    __syncthreads();
    return s;
}

// Row i of t = Q ubar, and its terms of the coefficient gradient:
//   g[m]       += ubar_i r_i x_ii^m / a_ii                  m = 0..deg      (diagonal part)
//   g[deg+m]   += ubar_i r_j x_ij^m / (a_ii + a_jj)   j != i, m = 1..deg      (off-diagonal part)
template <typename T>
__device__ __forceinline__ void adj_smooth_row(int32_t i, const int32_t* __restrict__ ptr,
                                               const int32_t* __restrict__ col, const double* __restrict__ val,
                                               const double* __restrict__ diag, double s, const T* __restrict__ q,
                                               const T* __restrict__ ubar, const T* __restrict__ r,
                                               T* __restrict__ t, int deg, double* g) {
    const double ui = static_cast<double>(ubar[i]);
    const double aii = diag[i];
    const int32_t pb = ptr[i], pe = ptr[i + 1];
    T acc = T(0);
    // eight entries at a time: their columns and values, then the gathers at the neighbours, are
    // loaded together; the sums still run over the entries in stored order (a past-the-end slot
    // re-reads the row's last entry and is not used)
    constexpr int kE = 8;
    for (int32_t base = pb; base < pe; base += kE) {
        int32_t jv[kE];
        T qv[kE], uj[kE], rj[kE];
        double av[kE], dj[kE];
#pragma unroll
        for (int e = 0; e < kE; ++e) {
            const int32_t p = min(base + e, pe - 1);
            jv[e] = col[p];
            qv[e] = q[p];
            av[e] = val[p];
        }
#pragma unroll
        for (int e = 0; e < kE; ++e) {
            uj[e] = ubar[jv[e]];
            rj[e] = r[jv[e]];
            dj[e] = diag[jv[e]];
        }
#pragma unroll
        for (int e = 0; e < kE; ++e) {
            if (base + e >= pe) break;
            const int32_t j = jv[e];
            acc += qv[e] * uj[e];
            const double x = av[e] / s;
            if (j == i) {
                double w = ui * static_cast<double>(rj[e]) / aii;
                for (int m = 0; m <= deg; ++m) {
                    g[m] += w;
                    w *= x;
                }
            } else {
                double w = ui * static_cast<double>(rj[e]) / (aii + dj[e]) * x;
                for (int m = 1; m <= deg; ++m) {
                    g[deg + m] += w;
                    w *= x;
                }
            }
        }
    }
    t[i] = acc;
}

// t = Q ubar and per-workgroup partial sums of the coefficient gradient (grid-stride rows).
template <typename T>
__global__ __launch_bounds__(kBlock) void adj_smooth_kernel(int32_t n, const int32_t* __restrict__ ptr,
                                                           const int32_t* __restrict__ col,
                                                           const double* __restrict__ val,
                                                           const double* __restrict__ diag,
                                                           const double* __restrict__ scale,
                                                           const T* __restrict__ q, const T* __restrict__ ubar,
                                                           const T* __restrict__ r, T* __restrict__ t, int deg,
                                                           double* __restrict__ partial) {
    double g[kMaxC];
    for (int m = 0; m < kMaxC; ++m) g[m] = 0.0;
    const double s = scale[0];
    for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += kReduceBlocks * kBlock)
        adj_smooth_row<T>(i, ptr, col, val, diag, s, q, ubar, r, t, deg, g);
    for (int m = 0; m <= 2 * deg; ++m) {
        const double v = block_sum(g[m]);
        if (threadIdx.x == 0) partial[m * kReduceBlocks + blockIdx.x] = v;
    }
}

__device__ __forceinline__ int32_t block_of_row(int32_t i, int32_t nblk, const int32_t* __restrict__ off) {
    int32_t lo = 0, hi = nblk - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) / 2;
        if (off[mid] <= i)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Block-diagonal level: workgroup c takes the rows of chunk c (all in one block, whose scale
// it uses) and writes its partial sums to partial[m * nchunk + c].
template <typename T>
__global__ __launch_bounds__(kBlock) void adj_smooth_blocks_kernel(
    int32_t nchunk, const int32_t* __restrict__ chunk_row, int32_t nblk, const int32_t* __restrict__ off,
    const double* __restrict__ scale, const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
    const double* __restrict__ val, const double* __restrict__ diag, const T* __restrict__ q,
    const T* __restrict__ ubar, const T* __restrict__ r, T* __restrict__ t, int deg, double* __restrict__ partial) {
    double g[kMaxC];
    for (int m = 0; m < kMaxC; ++m) g[m] = 0.0;
    const int32_t c = blockIdx.x;
    const int32_t r0 = chunk_row[c], r1 = chunk_row[c + 1];
    const double s = scale[block_of_row(r0, nblk, off)];
    for (int32_t i = r0 + threadIdx.x; i < r1; i += kBlock) adj_smooth_row<T>(i, ptr, col, val, diag, s, q, ubar, r, t, deg, g);
    for (int m = 0; m <= 2 * deg; ++m) {
        const double v = block_sum(g[m]);
        if (threadIdx.x == 0) partial[m * nchunk + c] = v;
    }
}

// cbar[crow[b]][m] += sum of block b's chunk partials (in chunk order), one workgroup per block.
// The first nkeep of each row's ncoef gradients are accumulated (the diagonal form of Eq. 5 keeps
// d0..d_deg only: its off-diagonal coefficients are no parameters and keep a zero gradient).
__global__ __launch_bounds__(kBlock) void adj_coeff_reduce_blocks_kernel(const double* __restrict__ partial,
                                                                        int32_t nchunk, int ncoef, int nkeep,
                                                                        const int32_t* __restrict__ blk_chunk,
                                                                        const int32_t* __restrict__ crow,
                                                                        double* __restrict__ cbar) {
    const int32_t b = blockIdx.x;
    const int32_t row = crow[b];
    if (row < 0) return;  // uniform over the workgroup
    const int32_t c0 = blk_chunk[b], c1 = blk_chunk[b + 1];
    for (int m = 0; m < nkeep; ++m) {
        double v = 0.0;
        for (int32_t k = c0 + threadIdx.x; k < c1; k += kBlock) v += partial[m * nchunk + k];
        v = block_sum(v);
        if (threadIdx.x == 0) cbar[static_cast<int64_t>(row) * ncoef + m] += v;
    }
}

// Per-block dot products of a level's vectors: chunk partials, then one sum per block.
template <typename T>
__global__ __launch_bounds__(kBlock) void dot_chunks_kernel(const int32_t* __restrict__ chunk_row,
                                                           const T* __restrict__ a, const T* __restrict__ b,
                                                           double* __restrict__ partial) {
    const int32_t c = blockIdx.x;
    double v = 0.0;
    for (int32_t i = chunk_row[c] + threadIdx.x; i < chunk_row[c + 1]; i += kBlock)
        v += static_cast<double>(a[i]) * static_cast<double>(b[i]);
    v = block_sum(v);
    if (threadIdx.x == 0) partial[c] = v;
}

__global__ __launch_bounds__(kBlock) void dot_blocks_final_kernel(const double* __restrict__ partial,
                                                                 const int32_t* __restrict__ blk_chunk,
                                                                 double* __restrict__ out) {
    const int32_t b = blockIdx.x;
    double v = 0.0;
    for (int32_t k = blk_chunk[b] + threadIdx.x; k < blk_chunk[b + 1]; k += kBlock) v += partial[k];
    v = block_sum(v);
    if (threadIdx.x == 0) out[b] = v;
}

// per block: loss_b = log10(||r_N|| / ||r_0||), s2_b = -1 / (ln 10 ||r_N||^2)
__global__ void loss_blocks_kernel(int32_t nblk, const double* __restrict__ s0, const double* __restrict__ s1,
                                   double* __restrict__ s2, double* __restrict__ loss) {
    const int32_t b = blockIdx.x * kBlock + threadIdx.x;
    if (b >= nblk) return;
    loss[b] = 0.5 * log10(s1[b] / s0[b]);
    s2[b] = -1.0 / (log(10.0) * s1[b]);
}

template <typename T>
__global__ void scale_blocks_kernel(int32_t n, T* __restrict__ y, int32_t nblk, const int32_t* __restrict__ off,
                                    const double* __restrict__ s) {
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) y[i] = static_cast<T>(static_cast<double>(y[i]) * s[block_of_row(i, nblk, off)]);
}

__global__ __launch_bounds__(kBlock) void adj_coeff_reduce_kernel(const double* __restrict__ partial, int nkeep,
                                                                 double* __restrict__ cbar) {
    __shared__ double red[kBlock];
    for (int m = 0; m < nkeep; ++m) {
        double v = 0.0;
        for (int k = threadIdx.x; k < kReduceBlocks; k += kBlock) v += partial[m * kReduceBlocks + k];
        red[threadIdx.x] = v;
        __syncthreads();
        for (int w = kBlock / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) cbar[m] += red[0];
        __syncthreads();
    }
}

template <typename T>
__global__ void axpy_kernel(int32_t n, const T* __restrict__ x, T* __restrict__ y) {
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) y[i] += x[i];
}

template <typename T>
__global__ void scale_dev_kernel(int32_t n, T* __restrict__ y, const double* __restrict__ s) {
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) y[i] = static_cast<T>(static_cast<double>(y[i]) * s[0]);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void dot_partial_kernel(int32_t n, const T* __restrict__ a,
                                                            const T* __restrict__ b, double* __restrict__ partial) {
    double v = 0.0;
    for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += kReduceBlocks * kBlock)
        v += static_cast<double>(a[i]) * static_cast<double>(b[i]);
    v = block_sum(v);
    if (threadIdx.x == 0) partial[blockIdx.x] = v;
}

// s[0] = ||r_0||^2, s[1] = ||r_N||^2  ->  loss = log10(||r_N|| / ||r_0||),  s[2] = -1 / (ln 10 ||r_N||^2)
__global__ void loss_kernel(double* __restrict__ s, double* __restrict__ loss) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        loss[0] = 0.5 * log10(s[1] / s[0]);
        s[2] = -1.0 / (log(10.0) * s[1]);
    }
}

struct Adj {
    amgg_ctx* c;
    hipStream_t st;
    int nu1, nu2, deg;
    double* cbar;
    bool blocked = false;  // per-block losses; gradients to the blocks' coefficient rows
    hipError_t e = hipSuccess;
    void ok(hipError_t r) {
        if (r != hipSuccess && e == hipSuccess) e = r;
    }

    template <typename T>
    void axpy(int32_t n, const T* x, T* y) {
        if (n > 0) axpy_kernel<T><<<grid_for(n), kBlock, 0, st>>>(n, x, y);
        ok(hipGetLastError());
    }

    // a . b, or per block (out[b]) on a block-diagonal hierarchy
    template <typename T>
    double* dot(int32_t n, const T* a, const T* b, double* out) {
        if (blocked) {
            const Level& L0 = c->lv[0];
            dot_chunks_kernel<T><<<L0.nchunk(), kBlock, 0, st>>>(L0.chunk_row, a, b, c->blk_partial);
            ok(hipGetLastError());
            dot_blocks_final_kernel<<<L0.nblk, kBlock, 0, st>>>(c->blk_partial, L0.blk_chunk, out);
            ok(hipGetLastError());
            return out;
        }
        dot_partial_kernel<T><<<kReduceBlocks, kBlock, 0, st>>>(n, a, b, c->adj_partial);
        ok(hipGetLastError());
        ok(finish_sum(c->adj_partial, out, st));
        return out;
    }

    // Iterate before smoothing step k (1-based) of a sequence starting at `entry` (nullptr = 0);
    // returns nullptr when that iterate is the zero vector.
    template <typename T>
    const T* recompute(Level& L, const T* f, const T* entry, int k) {
        if (k == 1) return entry;
        T* cur = L.adj<T>(kAdjW);
        T* oth = L.adj<T>(kAdjT);
        if (entry) ok(vec_copy<T>(L.n, entry, cur, st));
        for (int j = 1; j < k; ++j) ok(smooth_step<T>(L, f, cur, oth, L.r<T>(), entry == nullptr && j == 1, st));
        return cur;
    }

    // Reverse one smoothing step u' = u + Q (f - A u) whose input iterate is w (nullptr = 0).
    template <typename T>
    void step_back(int l, const T* f, const T* w) {
        Level& L = c->lv[l];
        const T* r = f;
        if (w) {
            ok(csr_apply<T>(L.A(), L.aval<T>(), w, L.adj<T>(kAdjR), f, nullptr, nullptr, Epi::Resid, st));
            r = L.adj<T>(kAdjR);
        }
        T* ub = L.adj<T>(kAdjUbar);
        T* tq = L.t<T>();
        if (blocked) {
            const int32_t nch = L.nchunk();
            adj_smooth_blocks_kernel<T><<<nch, kBlock, 0, st>>>(nch, L.chunk_row, L.nblk, L.blk_off, L.blk_scale, L.ptr,
                                                                L.col, L.val, L.diag, L.qval<T>(), ub, r, tq, deg,
                                                                c->blk_partial);
            ok(hipGetLastError());
            adj_coeff_reduce_blocks_kernel<<<L.nblk, kBlock, 0, st>>>(c->blk_partial, nch, 2 * deg + 1,
                                                                      L.diag_form ? deg + 1 : 2 * deg + 1,
                                                                      L.blk_chunk, L.blk_crow, cbar);
        } else {
            adj_smooth_kernel<T><<<kReduceBlocks, kBlock, 0, st>>>(L.n, L.ptr, L.col, L.val, L.diag, L.scale,
                                                                    L.qval<T>(), ub, r, tq, deg, c->adj_partial);
            ok(hipGetLastError());
            adj_coeff_reduce_kernel<<<1, kBlock, 0, st>>>(c->adj_partial, L.diag_form ? deg + 1 : 2 * deg + 1,
                                                          cbar + l * (2 * deg + 1));
        }
        ok(hipGetLastError());
        axpy<T>(L.n, tq, L.adj<T>(kAdjFbar));
        ok(csr_apply<T>(L.A(), L.aval<T>(), tq, ub, nullptr, nullptr, nullptr, Epi::Sub, st));
    }

    // Given ubar of level l's output (in adj(kAdjUbar)), leave ubar of its input there and the
    // adjoint of its right-hand side in adj(kAdjFbar).
    template <typename T>
    void level_back(int l, const T* f, const T* entry) {
        Level& L = c->lv[l];
        T* ub = L.adj<T>(kAdjUbar);
        T* fb = L.adj<T>(kAdjFbar);
        if (l == c->nlevels - 1) {
            ok(coarse_solve<T>(L, ub, fb, st));
            return;
        }
        ok(vec_zero_bytes(fb, sizeof(T) * L.n, st));
        for (int k = nu2; k >= 1; --k) step_back<T>(l, f, recompute<T>(L, f, L.adj<T>(kAdjUmid), k));
        Level& C = c->lv[l + 1];
        ok(csr_apply<T>(L.R(), L.rv<T>(), ub, C.adj<T>(kAdjUbar), nullptr, nullptr, nullptr, Epi::Store, st));
        level_back<T>(l + 1, C.f<T>(), nullptr);
        ok(csr_apply<T>(L.P(), L.pv<T>(), C.adj<T>(kAdjFbar), L.adj<T>(kAdjR), nullptr, nullptr, nullptr, Epi::Store,
                        st));
        ok(csr_apply<T>(L.A(), L.aval<T>(), L.adj<T>(kAdjR), ub, nullptr, nullptr, nullptr, Epi::Sub, st));
        axpy<T>(L.n, L.adj<T>(kAdjR), fb);
        for (int k = nu1; k >= 1; --k) step_back<T>(l, f, recompute<T>(L, f, entry, k));
    }

    // u_m from u_0 by m cycles; the level vectors of the m-th cycle are kept for the sweep.
    // On return adj(kAdjUin) of level 0 holds u_{m-1}.
    template <typename T>
    T* forward_to(int m, const T* f0, const T* u0) {
        Level& L0 = c->lv[0];
        T* uin = L0.adj<T>(kAdjUin);
        if (u0)
            ok(vec_copy<T>(L0.n, u0, uin, st));
        else
            ok(vec_zero_bytes(uin, sizeof(T) * L0.n, st));
        T* res = nullptr;
        for (int i = 1; i <= m; ++i) {
            if (i > 1) ok(vec_copy<T>(L0.n, res, uin, st));
            ok(vec_copy<T>(L0.n, uin, L0.u<T>(), st));
            ok(vcycle_level<T>(c, 0, f0, L0.u<T>(), L0.t<T>(), false, nu1, nu2, st, &res, i == m));
        }
        return res;
    }

    template <typename T>
    void run(int nvc, const T* f0, const T* u0, double* loss) {
        Level& L0 = c->lv[0];
        const int32_t n = L0.n;
        // scalars: ||r_0||^2, ||r_N||^2 and the seed scale (one each, or one per block)
        const int32_t k = blocked ? c->nblk : 1;
        double* s = blocked ? c->blk_scal : c->adj_scal;
        T* r0 = L0.adj<T>(kAdjR);
        if (u0) {
            ok(csr_apply<T>(L0.A(), L0.aval<T>(), u0, r0, f0, nullptr, nullptr, Epi::Resid, st));
            dot<T>(n, r0, r0, s + 0);
        } else {
            dot<T>(n, f0, f0, s + 0);
        }
        // forward, r_N, loss and the seed ubar_N = -(1/ln10) A r_N / ||r_N||^2
        T* uN = forward_to<T>(nvc, f0, u0);
        T* rN = L0.adj<T>(kAdjR);
        ok(csr_apply<T>(L0.A(), L0.aval<T>(), uN, rN, f0, nullptr, nullptr, Epi::Resid, st));
        dot<T>(n, rN, rN, s + k);
        T* ub = L0.adj<T>(kAdjUbar);
        if (blocked) {
            loss_blocks_kernel<<<grid_for(k), kBlock, 0, st>>>(k, s, s + k, s + 2 * k, loss);
            ok(hipGetLastError());
            ok(csr_apply<T>(L0.A(), L0.aval<T>(), rN, ub, nullptr, nullptr, nullptr, Epi::Store, st));
            scale_blocks_kernel<T><<<grid_for(n), kBlock, 0, st>>>(n, ub, L0.nblk, L0.blk_off, s + 2 * k);
        } else {
            loss_kernel<<<1, 1, 0, st>>>(s, loss);
            ok(hipGetLastError());
            ok(csr_apply<T>(L0.A(), L0.aval<T>(), rN, ub, nullptr, nullptr, nullptr, Epi::Store, st));
            scale_dev_kernel<T><<<grid_for(n), kBlock, 0, st>>>(n, ub, s + 2);
        }
        ok(hipGetLastError());
        for (int m = nvc; m >= 1; --m) {
            // recompute cycle m (a later cycle overwrote its level vectors); the forward pass
            // does not touch ubar
            if (m < nvc) forward_to<T>(m, f0, u0);
            level_back<T>(0, f0, L0.adj<T>(kAdjUin));
        }
    }
};

}  // namespace

static int loss_adjoint(const char* who, amgg_ctx* c, int nu1, int nu2, int precision, int nvc, const double* f,
                        const double* u0, double* loss_dev, double* dcoeffs_dev, int32_t dcoeff_rows, bool blocked,
                        void* stream) {
    const std::string w(who);
    int rc = check_ready(c, who);
    if (rc) return rc;
    if (!f || !loss_dev || !dcoeffs_dev) return fail(AMGG_EINVAL, w + ": null argument");
    if (nu1 < 0 || nu1 > 8 || nu2 < 0 || nu2 > 8 || nvc < 1 || nvc > 16)
        return fail(AMGG_EINVAL, w + ": nu or nvc out of range");
    if (precision != 32 && precision != 64) return fail(AMGG_EINVAL, w + ": precision must be 32 or 64");
    if (blocked != (c->nblk > 0))
        return fail(AMGG_ESTATE, w + (blocked ? ": the hierarchy has no blocks" : ": the hierarchy is block-diagonal; "
                                                                                  "use amgg_vcycle_loss_adjoint_blocks"));
    const int deg = c->lv[0].degree;
    for (int l = 0; l + 1 < c->nlevels; ++l)
        if (c->lv[l].degree != deg)
            return fail(AMGG_EINVAL, w + ": every level needs the same polynomial degree");
    if (c->nlevels > 1 && deg < 1) return fail(AMGG_ESTATE, w + ": smoothers not set");
    const int d = c->nlevels > 1 ? deg : 1;
    int64_t zero_rows = c->nlevels;
    if (blocked) {
        for (int l = 0; l < c->nlevels; ++l)
            for (int32_t r : c->lv[l].blk_crow_h)
                if (r >= dcoeff_rows) return fail(AMGG_EINVAL, w + ": a block's coefficient row is beyond dcoeff_rows");
        zero_rows = dcoeff_rows;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    Adj A{c, st, nu1, nu2, d, dcoeffs_dev, blocked};
    A.ok(hipSetDevice(c->device));
    A.ok(vec_zero_bytes(dcoeffs_dev, sizeof(double) * zero_rows * (2 * d + 1), st));
    Level& L0 = c->lv[0];
    if (precision == 64) {
        A.run<double>(nvc, f, u0, loss_dev);
    } else {
        A.ok(cast_f64_f32(L0.n, f, c->adj_f32, st));
        float* u32 = nullptr;
        if (u0) {
            // the fine level's own right-hand-side buffer is not used by the sweep (f comes
            // from adj_f32), so it holds the FP32 copy of u0
            u32 = L0.f<float>();
            A.ok(cast_f64_f32(L0.n, u0, u32, st));
        }
        A.run<float>(nvc, c->adj_f32, u32, loss_dev);
    }
    if (A.e != hipSuccess) return hip_fail(A.e, who);
    return AMGG_OK;
}

extern "C" int amgg_vcycle_loss_adjoint(amgg_ctx* c, int nu1, int nu2, int precision, int nvc, const double* f,
                                        const double* u0, double* loss_dev, double* dcoeffs_dev, void* stream) {
    return guarded([&]() -> int {
        return loss_adjoint("amgg_vcycle_loss_adjoint", c, nu1, nu2, precision, nvc, f, u0, loss_dev, dcoeffs_dev, 0,
                            false, stream);
    });
}

extern "C" int amgg_vcycle_loss_adjoint_blocks(amgg_ctx* c, int nu1, int nu2, int precision, int nvc,
                                               const double* f, const double* u0, double* loss_dev,
                                               double* dcoeffs_dev, int32_t dcoeff_rows, void* stream) {
    return guarded([&]() -> int {
        if (dcoeff_rows < 1) return fail(AMGG_EINVAL, "amgg_vcycle_loss_adjoint_blocks: dcoeff_rows < 1");
        return loss_adjoint("amgg_vcycle_loss_adjoint_blocks", c, nu1, nu2, precision, nvc, f, u0, loss_dev,
                            dcoeffs_dev, dcoeff_rows, true, stream);
    });
}
