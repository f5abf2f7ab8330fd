// Launchers of the gfx950 kernels used by the solver. Every launcher enqueues work on
// `stream` and returns hipSuccess or the launch error; none synchronises.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>

namespace amgg {

// ---------------------------------------------------------------------------------------
// Launch helper. When a pair of events is armed on the calling thread, the next kernel
// launched through launch_kernel records them at its own start and end (hipExtLaunchKernel)
// and disarms them; otherwise it is a plain launch.
// ---------------------------------------------------------------------------------------
struct LaunchEvents {
    hipEvent_t start = nullptr;
    hipEvent_t stop = nullptr;
};
LaunchEvents& armed_events();  // per host thread

template <typename... KArgs, typename... Args>
inline hipError_t launch_kernel(void (*kernel)(KArgs...), dim3 grid, dim3 block, hipStream_t stream,
                                Args... args) {
    LaunchEvents& ev = armed_events();
    if (ev.start != nullptr) {
        const hipEvent_t s = ev.start, e = ev.stop;
        ev = LaunchEvents{};
        hipExtLaunchKernelGGL(kernel, grid, block, 0, stream, s, e, 0, static_cast<KArgs>(args)...);
    } else {
        hipLaunchKernelGGL(kernel, grid, block, 0, stream, static_cast<KArgs>(args)...);
    }
    return hipGetLastError();
}

// The same with `lds` bytes of dynamic LDS.
template <typename... KArgs, typename... Args>
inline hipError_t launch_kernel_lds(void (*kernel)(KArgs...), dim3 grid, dim3 block, size_t lds, hipStream_t stream,
                                    Args... args) {
    LaunchEvents& ev = armed_events();
    if (ev.start != nullptr) {
        const hipEvent_t s = ev.start, e = ev.stop;
        ev = LaunchEvents{};
        hipExtLaunchKernelGGL(kernel, grid, block, lds, stream, s, e, 0, static_cast<KArgs>(args)...);
    } else {
        hipLaunchKernelGGL(kernel, grid, block, lds, stream, static_cast<KArgs>(args)...);
    }
    return hipGetLastError();
}

constexpr int kBlock = 256;         // threads per workgroup (4 wavefronts of 64)
constexpr int kStreamCap = 4096;    // products a CSR-stream workgroup holds in LDS
constexpr int kReduceBlocks = 1024; // fixed partial count: reductions are deterministic

// ---------------------------------------------------------------------------------------
// Row-wise CSR products y = epilogue(sum_j a_ij x_j); `lanes` threads cooperate on a row.
// ---------------------------------------------------------------------------------------
enum class Epi : int {
    Store = 0,   // y_i = s
    Resid = 1,   // y_i = f_i - s
    Add = 2,     // y_i += s
    Jacobi = 3,  // y_i = u_i + qd_i (f_i - s)      (one-pass diagonal smoothing step)
    Sub = 4,     // y_i -= s
    StoreScaled = 5,  // y_i = s and y2_i = qd_i s (a restriction that also forms the coarse
                      // level's first diagonal smoothing step from zero, u = qd f)
};

// Column indices of a CSR matrix packed for the CSR-stream kernels: rows are grouped in blocks
// of `rows` consecutive rows (the kernels' row blocks), every entry stores its column as a 16-bit
// offset from its block's base column, and the few entries whose column lies outside
// [base, base + 65534] ("far" entries, offset kFarCol) are listed per block with their entry
// index within the block and their full column. The kernels form exactly the products of the
// plain CSR walk (only the loads of the columns change), so results are bitwise the same.
constexpr uint16_t kFarCol = 0xFFFF;
struct ColPack {
    const uint16_t* off = nullptr;    // [nnz]
    const int32_t* base = nullptr;    // [blocks]
    const int32_t* foff = nullptr;    // [blocks + 1] far entries of each block
    const uint16_t* fslot = nullptr;  // entry index within the block of each far entry
    const int32_t* fcol = nullptr;    // column of each far entry
    int rows = 0;                     // rows per block of the encoding (0: none, plain columns)
};

// The FP32 right-hand side of the next cycle, written by the outer loop's residual kernel instead
// of the FP64 residual: f[i] = (float)(r_i * scale[0]) and, with qd, u[i] = qd[i] * f[i] (the first
// diagonal smoothing step from zero of the cycle that receives f).
struct Cast32 {
    float* f = nullptr;
    const float* qd = nullptr;
    float* u = nullptr;
    const double* scale = nullptr;
};

struct CsrView {
    int32_t nrows;
    int32_t nnz;
    const int32_t* ptr;
    const int32_t* col;
    int lanes;        // 1, 2, 4, ..., 64
    ColPack cp = {};  // packed columns (cp.rows == the stream kernel's rows per block), if any
    // products the CSR-stream kernel keeps in LDS per workgroup: a whole number of product
    // rounds covering the matrix's largest row block, at most kStreamCap (blocks beyond it sum
    // their rows from global memory). Smaller buffers let more workgroups share a compute unit.
    int32_t cap = kStreamCap;
};

// LDS product capacity for a matrix whose largest row block (of the stream kernel's rows) holds
// `maxblk` entries.
constexpr int32_t kStreamRound = 2048;  // entries of one product round (8 per thread)
inline int32_t stream_cap_for(int32_t maxblk) {
    const int32_t c = (maxblk + kStreamRound - 1) / kStreamRound * kStreamRound;
    return c < kStreamRound ? kStreamRound : (c > kStreamCap ? kStreamCap : c);
}
// out[0] = max over row blocks of `rows` rows of the block's entries (out[0] must start at 0).
hipError_t block_max_entries(int32_t nrows, const int32_t* ptr, int rows, int32_t* out, hipStream_t stream);

// Pack the columns of an nrows-row CSR matrix for row blocks of `rows` rows (a value of
// stream_rows_for): off [nnz], base [blocks], foff [blocks + 1], and at most `cap` far entries
// in fslot / fcol. `parts` is scratch of at least kScanParts + 1 ints. Synchronises the stream;
// *nfar receives the number of far entries (the packing is unusable when it exceeds cap).
// Blocks whose entries exceed the stream kernels' product buffer record no far entries (their
// rows are summed from the plain columns).
hipError_t pack_columns(int32_t nrows, int32_t nnz, const int32_t* ptr, const int32_t* col, int rows, uint16_t* off,
                        int32_t* base, int32_t* foff, uint16_t* fslot, int32_t* fcol, int64_t cap, int32_t* parts,
                        int64_t* nfar, hipStream_t stream);
constexpr int64_t kScanPartsMax = 1024;  // scratch of pack_columns: kScanPartsMax + 1 ints
// Matrices with fewer entries keep their plain columns: measured on one MI355X, packing pays only
// where a pass streams its matrix from HBM (8M-cell mesh: fine-level residual 91 -> 84 us,
// solves 1-3 % faster); a matrix that stays in the 256 MB last-level cache is latency-bound,
// and there the far-entry pass costs more than the saved bytes (1M P1 mesh: solves 2-5 %
// slower with every matrix packed). 2^24 entries = 128 MB of FP32 values and plain columns.
constexpr int32_t kPackMinEntries = 1 << 24;

int lanes_for(int32_t nrows, int32_t nnz);

template <typename T>
hipError_t csr_apply(const CsrView& m, const T* val, const T* x, T* y, const T* f, const T* qd, const T* u,
                     Epi epi, hipStream_t stream, T* y2 = nullptr);

// Rows per workgroup of the CSR-stream kernels for a matrix of this shape (0: lane kernel).
int stream_rows_for(int32_t nrows, int32_t nnz);

// Fused smoothing steps on a level (Q values on A's pattern). Rows are grouped in blocks of
// h.rows consecutive rows (= stream_rows_for(A)); each block has at most kHaloCap halo rows
// with at most kHaloEntCap stored entries between them (lists built on the host, halo.hpp).
// Levels with more rows than this stay with separate passes: there the halo rows' extra
// traffic (about 0.4-0.9 of the block's own entries) costs more than the saved launch.
constexpr int32_t kFuseMaxRows = 65536;
constexpr int kHaloCap = 1024;
constexpr int kHaloEntCap = 3072;  // <= the kernels' LDS product buffer (4096)
struct HaloView {
    int rows;
    const int32_t* hoff;   // [blocks + 1] into halo / hend
    const int32_t* halo;   // halo row ids
    const uint16_t* hend;  // end of each halo row's entries within its block's flat list
    const int32_t* heoff;  // [blocks + 1] into the flat halo-entry arrays
    const int32_t* hcol;   // column of each halo entry
    const uint16_t* loc;   // [nnz] block-local slot of each stored entry's column
};
// first pre-smoothing step from u = 0 and the residual after it: u = Q f, r = f - A u
// (hq: Q's values at the halo entries, in flat halo-entry order)
template <typename T>
hipError_t smooth_pre_fused(const CsrView& m, const HaloView& h, const T* a, const T* q, const T* hq, const T* f,
                            T* u, T* r, hipStream_t stream);
// one smoothing step into another buffer: y = u + Q (f - A u)   (y must not alias u;
// ha: A's values at the halo entries)
template <typename T>
hipError_t smooth_post_fused(const CsrView& m, const HaloView& h, const T* a, const T* ha, const T* q, const T* f,
                             const T* u, T* y, hipStream_t stream);
// dst[k] = src[idx[k]] for k < n, in both precisions (either pair may be null)
hipError_t gather_values(int32_t n, const int32_t* idx, const double* src64, const float* src32, double* dst64,
                         float* dst32, hipStream_t stream);
// Diagonal smoother d: first step from u = 0 fused with what follows it.
//   jacobi_pre_resid: u = d f and r = f - A u
//   jacobi_pre_step:  y = d f + d (f - A (d f))   (two steps)
template <typename T>
hipError_t jacobi_pre_resid(const CsrView& m, const T* a, const T* d, const T* f, T* u, T* r, hipStream_t stream);
template <typename T>
hipError_t jacobi_pre_step(const CsrView& m, const T* a, const T* d, const T* f, T* y, hipStream_t stream);

// q = A p and per-workgroup partial sums of p_i q_i (FP64 outer loop); *count = partials written.
hipError_t csr_spmv_dot(const CsrView& m, const double* val, const double* p, double* q, double* partial, int* count,
                        hipStream_t stream);
// r = b - A x and per-workgroup partial sums of r_i^2; *count = partials written.
hipError_t csr_resid_norm(const CsrView& m, const double* val, const double* x, const double* b, double* r,
                          double* partial, int* count, hipStream_t stream);
// r = b - A x with the partials of r_i^2 as csr_resid_norm, but r itself is not stored: the kernel
// writes its scaled FP32 copy (Cast32). Only for matrices the CSR-stream kernels serve
// (stream_rows_for > 0); hipErrorInvalidValue otherwise.
hipError_t csr_resid_cast(const CsrView& m, const double* val, const double* x, const double* b, const Cast32& cast,
                          double* partial, int* count, hipStream_t stream);
// Number of partial sums the calls above write for a matrix of this shape.
int outer_partials(int32_t nrows, int32_t nnz);

// ---------------------------------------------------------------------------------------
// Vector kernels
// ---------------------------------------------------------------------------------------
template <typename T>
hipError_t vec_mul(int32_t n, const T* a, const T* b, T* y, hipStream_t stream);  // y = a * b
template <typename T>
hipError_t vec_copy(int32_t n, const T* a, T* y, hipStream_t stream);
hipError_t vec_zero_bytes(void* p, size_t bytes, hipStream_t stream);
// y32 = (float)(x * scale[0]) ; scale on device. With d and u: also u = d y32 (FP32 product),
// the first diagonal smoothing step from zero of the cycle that receives y32.
hipError_t cast_scaled_f64_f32(int32_t n, const double* x, const double* scale, float* y, hipStream_t stream,
                               const float* d = nullptr, float* u = nullptr);
hipError_t cast_f64_f32(int32_t n, const double* x, float* y, hipStream_t stream);
hipError_t cast_scale_f64_f32(int64_t n, const double* x, double scale, float* y, hipStream_t stream);
hipError_t cast_scale_rows_f64_f32(int32_t nrows, int32_t ncols, const double* in, const int32_t* group,
                                   const double* gscale, float* out, hipStream_t stream);
hipError_t mean_difference(int32_t n, const double* a, const double* b, double* out, hipStream_t stream);
hipError_t cast_f32_f64(int32_t n, const float* x, double* y, hipStream_t stream);
// y = x - mean, mean = sum/n from a device scalar sum
hipError_t sub_mean(int32_t n, const double* x, const double* sum, double* y, hipStream_t stream);

// Deterministic two-stage reductions into partial[kReduceBlocks]
hipError_t partial_dot(int32_t n, const double* a, const double* b, double* partial, hipStream_t stream);
hipError_t partial_sum(int32_t n, const double* a, double* partial, hipStream_t stream);
// final: scalars[out] = sum(partial[0..kReduceBlocks))
hipError_t finish_sum(const double* partial, double* out, hipStream_t stream);  // kReduceBlocks partials

// FCG pieces; s = device scalars (see fcg_slot)
enum FcgSlot : int {
    kGamma = 0,   // z^T r
    kAlpha = 1,
    kBeta = 2,
    kRR = 3,      // ||r||^2
    kPQ = 4,      // p^T A p
    kNorm = 5,    // ||r||
    kInvNorm = 6, // 1/||r||
    kZR = 7,
    kZRold = 8,
    kBB = 9,      // ||b||^2
    kSum = 10,    // scratch sum (mean projection)
    kFlag = 11,   // breakdown flag (1.0 = breakdown)
    kTolRR = 12,  // tol^2 ||b||^2: the guarded steps halt below it
    kDivRR = 13,  // div^2 ||b||^2: ... and above it (or on a non-finite norm)
    kHalt = 14,   // 1.0 once a guarded step has halted the iteration
    // The outer loops with FP32 cycles scale each residual by a power of two (exact in both
    // directions) fixed before the residual is formed, so that the kernel forming it can write
    // the cycle's FP32 right-hand side itself: r_k is scaled by 2^-e, e the exponent of
    // ||r_{k-1}|| (r_k is at most about ||r_{k-1}||, so the FP32 values stay near 1).
    kScaleNext = 15,  // scale for the residual about to be formed
    kScaleCast = 16,  // scale of the residual held in FP32 (or to be cast next)
    kUnscale = 17,    // 1 / kScaleCast, applied to the cycle's output
    kSlots = 18
};
// Halting. An outer iteration may be enqueued before the host has read the previous one's
// residual; the guarded steps below then leave x and the residual norm unchanged once the
// iteration has converged, diverged or broken down (kHalt or kFlag set).
// s[kTolRR] = tol^2 s[kRR], s[kDivRR] = div^2 s[kRR], s[kHalt] = s[kFlag] = 0 (from the initial residual)
hipError_t fcg_set_limits(double* s, double tol, double div, hipStream_t stream);
// the three scale slots from s[kNorm] (at the start of a solve and after a restart)
hipError_t ir_set_scales(double* s, hipStream_t stream);
hipError_t fcg_clear_halt(double* s, hipStream_t stream);  // s[kHalt] = s[kFlag] = 0
// guarded fcg_finish_rr: skipped when halted; sets kHalt when rr <= s[kTolRR] or !(rr <= s[kDivRR]);
// moves kScaleNext to kScaleCast (and its inverse to kUnscale) and sets kScaleNext from the new norm
hipError_t fcg_finish_rr_guarded(const double* partial, int count, double* s, hipStream_t stream);
hipError_t fcg_finish_pq(const double* partial, int count, double* s, hipStream_t stream);  // pq, alpha = gamma/pq
// x += a p ; rnew = r - a q (skipped, partials included, when halted); with cast.f also the next
// cycle's FP32 right-hand side from rnew scaled by s[kScaleNext] (Cast32; cast.scale unused)
hipError_t fcg_update_xr(int32_t n, double* x, const double* p, const double* r, const double* q, double* rnew,
                         const double* s, double* partial, hipStream_t stream, const Cast32& cast = Cast32{});
hipError_t fcg_finish_rr(const double* partial, int count, double* s, hipStream_t stream);  // rr, norm, invnorm
// z = (double)u32 * s[kUnscale] (stored unless z is null) and partials of z.rnew, z.rold (2 * kReduceBlocks)
hipError_t fcg_castback_dots(int32_t n, const float* u32, const double* s, const double* rnew, const double* rold,
                             double* z, double* partial2, hipStream_t stream);
hipError_t fcg_dots64(int32_t n, const double* z, const double* rnew, const double* rold, double* partial2,
                      hipStream_t stream);
hipError_t fcg_finish_beta(const double* partial2, double* s, int first, hipStream_t stream);
hipError_t fcg_update_p(int32_t n, const double* z, double* p, const double* s, int first, hipStream_t stream);
// p = z (+ beta p) with z = (double)u32 * s[kUnscale] formed in place, as fcg_castback_dots forms it
hipError_t fcg_update_p32(int32_t n, const float* u32, double* p, const double* s, int first, hipStream_t stream);
// IR: x += (double)u32 * norm  (or x += e64); skipped when halted
hipError_t ir_update_f32(int32_t n, double* x, const float* u32, const double* s, hipStream_t stream);
hipError_t ir_update_f64(int32_t n, double* x, const double* e, const double* s, hipStream_t stream);

// ---------------------------------------------------------------------------------------
// Setup kernels
// ---------------------------------------------------------------------------------------
// diag[i] = a_ii; bad[0] set to 1 when a row has no positive stored diagonal
hipError_t extract_diag(int32_t n, const int32_t* ptr, const int32_t* col, const double* val, double* diag,
                        int32_t* bad, hipStream_t stream);
// scale[0] = max |a_ij| over off-diagonal entries, or 1 when there are none
hipError_t offdiag_absmax(int32_t n, const int32_t* ptr, const int32_t* col, const double* val, double* partial,
                          double* scale, hipStream_t stream);
// R = P^T (rows in ascending fine index): counts, scan, scatter, per-row sort; r_ptr has
// n_c + 1 entries, cursor n_c + 1 entries of scratch
hipError_t transpose_csr(int32_t nf, int32_t nc, int32_t nnz, const int32_t* p_ptr, const int32_t* p_col,
                         const double* p_val, int32_t* r_ptr, int32_t* r_col, double* r_val, int32_t* cursor,
                         hipStream_t stream);

struct PolyCoeffs {
    double c[2 * 4 + 1];
    int degree;
    int diag_only = 0;  // the diagonal form of Eq. 5: f_o taken as 0 whatever the coefficients say
};
// Eq. (5) smoother values on A's pattern; also the diagonal of Q^{-1} in both precisions.
hipError_t assemble_smoother(int32_t n, const int32_t* ptr, const int32_t* col, const double* val,
                             const double* diag, const double* scale, const PolyCoeffs& pc,
                             const float* coeffs_dev, double* q64, float* q32, double* qd64, float* qd32,
                             hipStream_t stream);
// The same values on a block-diagonal level: block b (rows off[b]..off[b+1]) uses scale[b]
// and the coefficients coeffs_dev + crow[b] * stride (or pc when coeffs_dev is null);
// crow[b] < 0 gives Q = 0 on that block.
hipError_t assemble_smoother_blocks(int32_t n, const int32_t* ptr, const int32_t* col, const double* val,
                                    const double* diag, int32_t nblk, const int32_t* off, const double* scale,
                                    const int32_t* crow, const PolyCoeffs& pc, const float* coeffs_dev,
                                    int32_t stride, double* q64, float* q32, double* qd64, float* qd32,
                                    hipStream_t stream);

// Dense coarse solve (rows [0, n) of ptr; columns shifted by -col0 for a diagonal block)
hipError_t dense_from_csr(int32_t n, const int32_t* ptr, const int32_t* col, const double* val, double* M,
                          int singular, hipStream_t stream, int32_t col0 = 0);
hipError_t dense_lu_inverse(int32_t n, double* M, int32_t* piv, double* inv, int32_t* bad, hipStream_t stream);
template <typename T>
hipError_t dense_gemv(int32_t n, const double* inv, const T* x, T* y, hipStream_t stream);
// Block-diagonal levels: off[nblk+1] row offsets; inverse of block b at inv + doff[b].
hipError_t block_absmax(int32_t nblk, const int32_t* off, const int32_t* ptr, const int32_t* col, const double* val,
                        double* scale, hipStream_t stream);
hipError_t prolong_blocks_check(int32_t n, const int32_t* ptr, const int32_t* col, int32_t nblk, const int32_t* foff,
                                const int32_t* coff, int32_t* bad, hipStream_t stream);
template <typename T>
hipError_t block_dense_gemv(int32_t n, int32_t nblk, const int32_t* off, const int64_t* doff, const double* inv,
                            const T* x, T* y, hipStream_t stream);

}  // namespace amgg
