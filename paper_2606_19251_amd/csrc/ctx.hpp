// Internal state of a solver context: per-level views of the caller's hierarchy arrays
// and the arrays carved from the caller's workspace.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <type_traits>
#include <vector>

#include "amggnn.h"
#include "kernels.hpp"

namespace amgg {

enum : int { kSmootherNone = 0, kSmootherDiagonal = 1, kSmootherSparse = 2 };
constexpr int kChunkRows = 256;  // rows per workgroup of the segmented (per-block) sums
constexpr int kMaxCoef = 2 * AMGG_MAX_DEGREE + 1;
// Outer iterations of a solve enqueued at once (the one the host inspects and those behind it), so
// that a host thread late by up to kPipeline - 1 iterations leaves no gap on the stream.
constexpr int kPipeline = 3;

struct Level {
    bool loaded = false, p_loaded = false;
    // A_l (caller-owned, device)
    int32_t n = 0, nnz = 0;
    const int32_t* ptr = nullptr;
    const int32_t* col = nullptr;
    const double* val = nullptr;
    // P_l (caller-owned, device), n x nc
    int32_t pn_f = 0, nc = 0, pnnz = 0;
    const int32_t* pptr = nullptr;
    const int32_t* pcol = nullptr;
    const double* pval = nullptr;
    // workspace
    float* val32 = nullptr;
    float* pval32 = nullptr;
    int32_t* rptr = nullptr;
    int32_t* rcol = nullptr;
    double* rval = nullptr;
    float* rval32 = nullptr;
    double* diag = nullptr;
    double* scale = nullptr;
    double* q64 = nullptr;
    float* q32 = nullptr;
    double* qd64 = nullptr;
    float* qd32 = nullptr;
    double *u64 = nullptr, *f64 = nullptr, *r64 = nullptr, *t64 = nullptr;
    float *u32 = nullptr, *f32 = nullptr, *r32 = nullptr, *t32 = nullptr;
    double* dense = nullptr;
    double* inv = nullptr;
    int32_t* piv = nullptr;
    // halo lists of the fused smoothing kernels (hrows = rows per block, 0 = not available)
    int hrows = 0;
    int32_t nhent = 0;  // halo entries over all blocks
    int32_t* hoff = nullptr;
    int32_t* halo = nullptr;
    uint16_t* hend = nullptr;
    int32_t* heoff = nullptr;
    int32_t* hent = nullptr;  // global entry index of each halo entry
    int32_t* hcol = nullptr;
    double* ha64 = nullptr;  // A and Q values at the halo entries
    float* ha32 = nullptr;
    double* hq64 = nullptr;
    float* hq32 = nullptr;
    uint16_t* hloc = nullptr;
    bool fuse = true;  // use the fused kernels where available
    // packed columns (ColPack) of A_l (which Q_l shares), P_l and R_l for the CSR-stream kernels
    struct Pack {
        uint16_t* off = nullptr;
        int32_t* base = nullptr;
        int32_t* foff = nullptr;
        uint16_t* fslot = nullptr;
        int32_t* fcol = nullptr;
        int rows = 0;       // rows per block the packing is for (0: none)
        int64_t cap = 0;    // far-entry capacity
        int64_t nfar = -1;  // far entries found at finalize (-1: not built)
        bool usable() const { return rows > 0 && nfar >= 0 && nfar <= cap; }
        // mode 0: plain columns; 1: packed for matrices of at least kPackMinEntries entries;
        // 2: packed wherever the packing fits
        ColPack view(int mode, int32_t nz) const {
            if (mode == 0 || !usable() || (mode == 1 && nz < kPackMinEntries)) return ColPack{};
            return ColPack{off, base, foff, fslot, fcol, rows};
        }
    };
    Pack pa, pp, pr;
    int pack = 1;  // packing mode of the CSR-stream kernels (see Pack::view)
    // adjoint scratch, kAdjVecs vectors of n per precision (see AdjVec)
    double* adj64[8] = {};
    float* adj32[8] = {};
    // block-diagonal (batched) level: nblk independent problems, rows of block b are
    // [blk_off[b], blk_off[b+1]); host copies are kept for the device tables and the chunks
    // of at most kChunkRows rows (never spanning two blocks) that segmented sums use
    int32_t nblk = 0;
    std::vector<int32_t> blk_off_h, blk_crow_h, chunk_row_h, blk_chunk_h;
    std::vector<int32_t> blk_sing_h;
    std::vector<int64_t> dense_off_h;
    int32_t* blk_off = nullptr;
    int32_t* blk_crow = nullptr;  // coefficient row of each block (-1: no smoother)
    double* blk_scale = nullptr;
    int32_t* chunk_row = nullptr;  // nchunk + 1 row starts
    int32_t* blk_chunk = nullptr;  // nblk + 1 chunk offsets
    int64_t* dense_off = nullptr;  // coarsest level: offset of each block's dense inverse
    int32_t nchunk() const { return static_cast<int32_t>(chunk_row_h.empty() ? 0 : chunk_row_h.size() - 1); }
    // smoother state
    int smoother = kSmootherNone;
    int degree = 0;
    bool baseline = false;  // exactly the omega = 2/3 Jacobi smoother (the fallback target)
    bool diag_form = false; // diagonal form of Eq. 5 (f_o = 0): the off-diagonal coefficients are no
                            // parameters of the level, their gradient is zero

    // LDS product capacity of the CSR-stream kernels for A (and Q), P and R (set at finalize)
    int32_t acap = kStreamCap, pcap = kStreamCap, rcap = kStreamCap;

    CsrView A() const { return {n, nnz, ptr, col, lanes_for(n, nnz), pa.view(pack, nnz), acap}; }
    CsrView P() const { return {n, pnnz, pptr, pcol, lanes_for(n, pnnz), pp.view(pack, pnnz), pcap}; }
    CsrView R() const { return {nc, pnnz, rptr, rcol, lanes_for(nc, pnnz), pr.view(pack, pnnz), rcap}; }
    HaloView H() const { return {hrows, hoff, halo, hend, heoff, hcol, hloc}; }
    template <typename T> const T* hav() const { if constexpr (std::is_same_v<T, double>) return ha64; else return ha32; }
    template <typename T> const T* hqv() const { if constexpr (std::is_same_v<T, double>) return hq64; else return hq32; }

    template <typename T> const T* aval() const { if constexpr (std::is_same_v<T, double>) return val; else return val32; }
    template <typename T> const T* qval() const { if constexpr (std::is_same_v<T, double>) return q64; else return q32; }
    template <typename T> const T* qd() const { if constexpr (std::is_same_v<T, double>) return qd64; else return qd32; }
    template <typename T> const T* pv() const { if constexpr (std::is_same_v<T, double>) return pval; else return pval32; }
    template <typename T> const T* rv() const { if constexpr (std::is_same_v<T, double>) return rval; else return rval32; }
    template <typename T> T* u() const { if constexpr (std::is_same_v<T, double>) return u64; else return u32; }
    template <typename T> T* f() const { if constexpr (std::is_same_v<T, double>) return f64; else return f32; }
    template <typename T> T* r() const { if constexpr (std::is_same_v<T, double>) return r64; else return r32; }
    template <typename T> T* t() const { if constexpr (std::is_same_v<T, double>) return t64; else return t32; }
    template <typename T> T* adj(int k) const { if constexpr (std::is_same_v<T, double>) return adj64[k]; else return adj32[k]; }
};

// Adjoint work vectors of a level
enum AdjVec : int {
    kAdjUin = 0,   // entry iterate of the level (fine level only; coarser levels start from 0)
    kAdjUmid = 1,  // iterate after the coarse-grid correction (entry of post-smoothing)
    kAdjUbar = 2,  // adjoint of the level's iterate
    kAdjFbar = 3,  // adjoint of the level's right-hand side
    kAdjR = 4,     // recomputed residual / restricted adjoint
    kAdjW = 5,     // recomputed smoothing iterate
    kAdjT = 6,     // second buffer of the recomputation (diagonal step ping-pong) / Q ubar
    kAdjVecs = 7
};

}  // namespace amgg

struct amgg_ctx {
    int device = 0;
    int nlevels = 0;
    amgg::Level lv[AMGG_MAX_LEVELS];
    bool finalized = false;
    int singular = 0;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    double* host_scal = nullptr;  // pinned host copies of the device scalars: 1 + kPipeline slots of kSlots
    hipStream_t cap_stream = nullptr;  // private stream for graph capture
    hipEvent_t ev[amgg::kPipeline] = {};  // completion of the pipelined scalar copies
    struct Graph {
        std::string key;
        hipGraphExec_t exec;
    };
    std::vector<Graph> graphs;  // captured outer-iteration bodies
    // workspace
    double* scal = nullptr;
    double* partial = nullptr;
    double* partial2 = nullptr;
    int32_t* flags = nullptr;
    int32_t* cursor = nullptr;
    int32_t* pack_parts = nullptr;  // scan scratch of the column packing
    int32_t* blkmax = nullptr;      // largest row block of A, P and R per level (3 x AMGG_MAX_LEVELS)
    double *ra = nullptr, *rb = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *bproj = nullptr;
    double* adj_partial = nullptr;
    double* adj_scal = nullptr;
    float* adj_f32 = nullptr;
    // block-diagonal contexts (every level split into nblk blocks)
    int32_t nblk = 0;
    double* blk_scal = nullptr;     // per-block loss scalars, 4 x nblk
    double* blk_partial = nullptr;  // per-chunk partial sums, kMaxCoef x (most chunks of a level)
};

namespace amgg {

size_t layout(amgg_ctx* c, uintptr_t base);
int hip_fail(hipError_t e, const char* where);
int check_ready(const amgg_ctx* c, const char* where);
template <typename T>
hipError_t vcycle_level(amgg_ctx* c, int l, const T* f, T* u, T* t, bool zero, int nu1, int nu2, hipStream_t st,
                        T** result, bool store = false, bool u_ready = false);
// True when a cycle from u = 0 on level l starts with a diagonal smoothing step u = qd f that
// the producer of f may form in the same pass (vcycle_level's u_ready).
bool takes_ready_u(const amgg_ctx* c, int l, int nu1);
template <typename T>
hipError_t smooth_step(Level& L, const T* f, T*& cur, T*& oth, T* r, bool from_zero, hipStream_t st);
// Coarsest-level solve: the dense inverse, or the block inverses of a block-diagonal level.
template <typename T>
hipError_t coarse_solve(const Level& L, const T* f, T* u, hipStream_t st);

}  // namespace amgg
