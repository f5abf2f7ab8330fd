// GCIN smoother-coefficient predictor on gfx950 (paper Sec. 3.2, Eqs. 6-10; App. A.1,
// Tab. 5): forward, hand-written backward and Adam.
//
// Layout. All graphs of a batch (every level of every problem, Alg. 1 steps 3-6) are
// concatenated; each graph starts on a 64-row tile boundary (pad rows carry no edges and
// are masked), so a tile belongs to exactly one graph and per-graph statistics are fixed
// order sums of per-tile partials (no atomics, bitwise reproducible). Activations are
// FP32 [N x 64] row-major; a tile is processed by one 256-thread workgroup (4 wavefronts x
// 16 rows, lane = channel), so every row access is one coalesced 256-byte transaction.
//
// Each GCIN layer is one pass: the neighbour features are normalised and rectified on
// load (InstanceNorm + ReLU of the previous layer applied by the consumer), aggregated
// with the edge weights (A_hat = (A - D) + I), multiplied by Theta_l (64 x 64) and the
// per-tile sums of y and y^2 are emitted for the next InstanceNorm. In BF16 mode the
// 64 x 64 products run on v_mfma_f32_16x16x32_bf16 with FP32 accumulation.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "amggnn.h"
#include "errors.hpp"
#include "gcin.h"

namespace {

// The hidden width HD (64, or 32 for the smaller variant) is a template parameter of every
// kernel below; a workgroup has 4 HD threads (4 groups of HD lanes, lane = channel).
constexpr int NL = 4;      // GCIN layers
constexpr int RO = 32;     // readout width per layer
constexpr int JK = RO * NL;
constexpr int M1 = 128, M2 = 64;
constexpr int TILE = 64;
constexpr int kAdamThreads = 256;
constexpr int kWBlocks = 512; // fixed grid of the weight-gradient reductions
constexpr int kMaxOut = 9;    // 2 d + 1 for d <= 4
constexpr float kEps = 1e-5f;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------------------------------
// parameter offsets (order documented in gcin.h)
// ------------------------------------------------------------------------------------------
struct Offs {
    int64_t convW[NL], convb[NL], gam[NL], bet[NL], roW[NL], rob[NL];
    int64_t lng, lnb, m0W, m0b, m1W, m1b, m2W, m2b, head0, total;
    int nout;
};

Offs offsets(int d, int HD) {
    Offs o{};
    int64_t k = 0;
    for (int l = 0; l < NL; ++l) {
        const int in = l == 0 ? 2 : HD;
        o.convW[l] = k; k += in * HD;
        o.convb[l] = k; k += HD;
        o.gam[l] = k; k += HD;
        o.bet[l] = k; k += HD;
    }
    o.head0 = k;
    for (int l = 0; l < NL; ++l) {
        o.roW[l] = k; k += 2 * HD * RO;
        o.rob[l] = k; k += RO;
    }
    o.nout = 2 * d + 1;
    o.lng = k; k += JK;
    o.lnb = k; k += JK;
    o.m0W = k; k += JK * M1;
    o.m0b = k; k += M1;
    o.m1W = k; k += M1 * M2;
    o.m1b = k; k += M2;
    o.m2W = k; k += M2 * o.nout;
    o.m2b = k; k += o.nout;
    o.total = k;
    return o;
}

__device__ __forceinline__ unsigned short f2bf(float f) {
    // round to nearest even (inputs are finite)
    unsigned int u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return static_cast<unsigned short>(u >> 16);
}

__device__ __forceinline__ float normrelu(float y, float mu, float rs, float ga, float be) {
    return fmaxf((y - mu) * rs * ga + be, 0.0f);
}

// Aggregation over the stored entries of a lane group's rows [r0, r1) of the batched graph (W
// lanes, one per channel, share the row index; r1 - r0 < W). The group's row bounds are loaded
// once, one per lane, and read across lanes at each row change, so that the walk over the rows
// has no dependent global load. Entries are visited in stored order, a batch at a time: the
// batch's column indices and weights are spread over the group's lanes (lane l holds entry l),
// its gathers load(j) are issued together while the next batch's indices load, and use(w, v)
// is then applied in entry order, each entry's index and weight read across lanes; done(row) is
// called once per row after its last entry (rows without entries included). A 64-lane group
// owns its wavefront, so the indices it reads are uniform (scalar registers) and it takes 32
// entries per batch; a 32-lane group (two per wavefront, on different rows) takes kAggBatch.
constexpr int kAggBatch = 16;

template <int W, typename V, class Load, class Use, class Done>
__device__ __forceinline__ void visit_rows(const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                           const float* __restrict__ w, int32_t r0, int32_t r1, Load load, Use use,
                                           Done done) {
    static_assert(W == 64 || W == 32, "lane groups of 64 or 32");
    const int32_t rp = ptr[r0 + min(static_cast<int32_t>(threadIdx.x % W), r1 - r0)];
    auto bound = [&](int32_t i) {  // ptr[r0 + i], i <= r1 - r0
        const int32_t v = __shfl(rp, i, W);
        if constexpr (W == 64) return __builtin_amdgcn_readfirstlane(v);
        return v;
    };
    const int32_t kend = bound(r1 - r0);
    int32_t r = r0;
    int32_t rnext = bound(1);
    const int32_t kbeg = bound(0);
    auto walk = [&](int32_t k, int q, float wq, const V& v) {
        if (k + q < kend) {
            while (k + q >= rnext) {
                done(r);
                ++r;
                rnext = bound(r + 1 - r0);
            }
            use(wq, v);
        }
    };
    if constexpr (W == 64) {
        constexpr int B = 2 * kAggBatch;  // 32 gathers in flight per wavefront
        const int32_t l = static_cast<int32_t>(threadIdx.x % 64) % B;
        int32_t cl = 0;
        float wl = 0.0f;
        if (kbeg < kend) {
            const int32_t kk = min(kbeg + l, kend - 1);
            cl = col[kk];
            wl = w[kk];
        }
        for (int32_t k = kbeg; k < kend; k += B) {
            V vj[B];
#pragma unroll
            for (int q = 0; q < B; ++q) vj[q] = load(__builtin_amdgcn_readlane(cl, q));
            const float wcur = wl;
            if (k + B < kend) {
                const int32_t kk = min(k + B + l, kend - 1);
                cl = col[kk];
                wl = w[kk];
            }
#pragma unroll
            for (int q = 0; q < B; ++q)
                walk(k, q, __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, wcur), q)), vj[q]);
        }
    } else {
        const int32_t l = static_cast<int32_t>(threadIdx.x % W) % kAggBatch;
        int32_t cl = 0;
        float wl = 0.0f;
        if (kbeg < kend) {
            const int32_t kk = min(kbeg + l, kend - 1);
            cl = col[kk];
            wl = w[kk];
        }
        for (int32_t k = kbeg; k < kend; k += kAggBatch) {
            V vj[kAggBatch];
#pragma unroll
            for (int q = 0; q < kAggBatch; ++q) vj[q] = load(__shfl(cl, q, W));
            const float wcur = wl;
            if (k + kAggBatch < kend) {
                const int32_t kk = min(k + kAggBatch + l, kend - 1);
                cl = col[kk];
                wl = w[kk];
            }
#pragma unroll
            for (int q = 0; q < kAggBatch; ++q) walk(k, q, __shfl(wcur, q, W), vj[q]);
        }
    }
    for (; r < r1; ++r) done(r);
}

// The same walk with 16-byte gathers: the HD / 4 = G lanes of group q (of the 4 HD lanes that own
// rows [r0, r0 + 16)) own the rows [r0 + 4 q, r0 + 4 q + 4) and lane p of the group holds channels
// 4 p .. 4 p + 3, so that one load instruction brings 64 / G neighbour rows (the load units
// process a wavefront's addresses a few lanes per cycle, which bounds a gather of one 4-byte
// channel per lane). Each row's entries are still visited in stored order, so every channel's sum
// is the one visit_rows forms. A group takes its entries kBatchX4 at a time, their indices and
// weights held by its first lanes; use(w, v, s) gets the four channels as a float4 and s = the
// row when the entry is the row's own (column = row), else -1; done(row) is called once per row
// of the group.
constexpr int kBatchX4 = 8;

template <int G, class Load, class Use, class Done>
__device__ __forceinline__ void visit_rows_x4(const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                              const float* __restrict__ w, int32_t r0, Load load, Use use,
                                              Done done) {
    static_assert(G == 16 || G == 8, "groups of 16 (64 channels) or 8 (32 channels) lanes");
    constexpr int B = kBatchX4;
    const int p = static_cast<int>(threadIdx.x % G);
    const int32_t g0 = r0 + 4 * static_cast<int32_t>((threadIdx.x % (4 * G)) / G);  // the group's first row
    const int32_t rp = ptr[g0 + min(p, 4)];
    auto bound = [&](int32_t i) { return __shfl(rp, i, G); };  // ptr[g0 + i], i <= 4
    const int32_t kbeg = bound(0), kend = bound(4);
    int32_t r = g0;
    int32_t rnext = bound(1);
    const int32_t l = p % B;
    int32_t cl = 0;
    float wl = 0.0f;
    if (kbeg < kend) {
        const int32_t kk = min(kbeg + l, kend - 1);
        cl = col[kk];
        wl = w[kk];
    }
    for (int32_t k = kbeg; k < kend; k += B) {
        float4 vj[B];
#pragma unroll
        for (int q = 0; q < B; ++q) vj[q] = load(__shfl(cl, q, G));
        const float wcur = wl;
        const int32_t ccur = cl;
        if (k + B < kend) {
            const int32_t kk = min(k + B + l, kend - 1);
            cl = col[kk];
            wl = w[kk];
        }
#pragma unroll
        for (int q = 0; q < B; ++q) {
            const float wq = __shfl(wcur, q, G);
            const int32_t jq = __shfl(ccur, q, G);
            if (k + q < kend) {
                while (k + q >= rnext) {
                    done(r);
                    ++r;
                    rnext = bound(r + 1 - g0);
                }
                use(wq, vj[q], jq == r ? r : -1);
            }
        }
    }
    for (; r < g0 + 4; ++r) done(r);
}

// Sum over the 4 wavefronts of a workgroup, per channel (lane), into out[c] (thread wave 0).
template <int HD>
__device__ __forceinline__ double wave4_sum(double v, double (*sh)[HD]) {
    const int wv = threadIdx.x / HD, c = threadIdx.x % HD;
    sh[wv][c] = v;
    __syncthreads();
    const double s = sh[0][c] + sh[1][c] + sh[2][c] + sh[3][c];
    __syncthreads();
    return s;
}

// ------------------------------------------------------------------------------------------
// batch construction
// ------------------------------------------------------------------------------------------
// A workgroup owns 256 consecutive rows of the level graph. Each thread writes its row's
// pointer and degree feature and marks the row's entries in an LDS map; the entries are then
// copied with unit stride (columns shifted to the graph's first batch row, weights a_ij, 1 for
// the self-loop of A_hat, whose entry also writes the a_ii feature). The map holds 64 entries per
// row on average (the coarse levels of the 3D hierarchies have 25-60); a block whose entries do
// not fit it is copied row by row.
constexpr int kFillCap = 16384;

__global__ __launch_bounds__(256) void fill_graph_kernel(int32_t n, const int32_t* __restrict__ rp,
                                                        const int32_t* __restrict__ cl,
                                                        const double* __restrict__ va, int32_t row0, int32_t e0,
                                                        int32_t* __restrict__ ptr, int32_t* __restrict__ col,
                                                        float* __restrict__ w, float* __restrict__ x0) {
    __shared__ uint8_t rowof[kFillCap];
    const int t = static_cast<int>(threadIdx.x);
    const int32_t r0 = static_cast<int32_t>(blockIdx.x) * 256;
    const int32_t r1 = min(r0 + 256, n);
    const int32_t b0 = rp[r0];
    const int32_t ne = rp[r1] - b0;
    const bool fits = ne <= kFillCap;
    const int32_t i = r0 + t;
    int32_t b = 0, e = 0;
    if (i < r1) {
        b = rp[i];
        e = rp[i + 1];
        ptr[row0 + i] = e0 + b;
        x0[2 * (row0 + i)] = 0.0f;  // a_ii; the diagonal entry writes it below
        x0[2 * (row0 + i) + 1] = static_cast<float>(e - b - 1);
        if (fits)
            for (int32_t k = b - b0; k < e - b0; ++k) rowof[k] = static_cast<uint8_t>(t);
    }
    __syncthreads();
    if (!fits) {
        if (i < r1)
            for (int32_t p = b; p < e; ++p) {
                const int32_t j = cl[p];
                col[e0 + p] = row0 + j;
                w[e0 + p] = j == i ? 1.0f : static_cast<float>(va[p]);
                if (j == i) x0[2 * (row0 + i)] = static_cast<float>(va[p]);
            }
        return;
    }
    for (int32_t k = t; k < ne; k += 256) {
        const int32_t p = b0 + k;
        const int32_t j = cl[p];
        const int32_t row = r0 + rowof[k];
        col[e0 + p] = row0 + j;
        if (j == row) {
            w[e0 + p] = 1.0f;  // self-loop of A_hat
            x0[2 * (row0 + row)] = static_cast<float>(va[p]);
        } else {
            w[e0 + p] = static_cast<float>(va[p]);
        }
    }
}

__global__ void set_int_kernel(int32_t* __restrict__ p, int32_t v) { p[0] = v; }

__global__ void pad_rows_kernel(int32_t from, int32_t to, int32_t eptr, int32_t* __restrict__ ptr,
                                float* __restrict__ x0) {
    const int32_t i = from + blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= to) return;
    ptr[i] = eptr;
    x0[2 * i] = 0.0f;
    x0[2 * i + 1] = 0.0f;
}

// ------------------------------------------------------------------------------------------
// forward
// ------------------------------------------------------------------------------------------
// Output of layer 0 at a node from its two aggregated input features h = (A_hat x0)_i:
// y_c = b0_c + h0 W0[0][c] + h1 W0[1][c]. The input features span two dimensions, so y is never
// stored: every consumer (the layer's statistics and pooling, layer 1's aggregation, the
// backward) forms it from h with this one expression, 8 bytes per node instead of 4 HD.
__device__ __forceinline__ float y0_of(float2 h, float w0, float w1, float bb) {
    return __builtin_fmaf(h.y, w1, __builtin_fmaf(h.x, w0, bb));
}

// Layer 0 of a tile: H0 = A_hat x0 (two features per node; 4 HD / 64 lanes per row, each summing
// every such entry of the row, combined in a fixed butterfly) and the per-tile sums of y and
// y^2 for the InstanceNorm statistics.
template <int HD>
__global__ __launch_bounds__(4 * HD) void layer0_kernel(const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                                    const float* __restrict__ w, const float* __restrict__ x0,
                                                    const int32_t* __restrict__ tile_graph,
                                                    const int32_t* __restrict__ gend, const float* __restrict__ W0,
                                                    const float* __restrict__ b0, float* __restrict__ H0,
                                                    double* __restrict__ tstat) {
    constexpr int LPR = 4 * HD / TILE;
    __shared__ double sh[4][HD];
    __shared__ float2 hs[TILE];
    const int tile = blockIdx.x, wv = threadIdx.x / HD, c = threadIdx.x % HD;
    const int32_t end = gend[tile_graph[tile]];
    {
        const int lr = threadIdx.x / LPR, q = threadIdx.x % LPR;
        const int32_t row = tile * TILE + lr;
        float h0 = 0.0f, h1 = 0.0f;
        if (row < end) {
            const int32_t pe = ptr[row + 1];
            for (int32_t k = ptr[row] + q; k < pe; k += LPR) {
                const float wk = w[k];
                const float2 xv = *reinterpret_cast<const float2*>(x0 + 2 * static_cast<int64_t>(col[k]));
                h0 = __builtin_fmaf(wk, xv.x, h0);
                h1 = __builtin_fmaf(wk, xv.y, h1);
            }
        }
#pragma unroll
        for (int off = 1; off < LPR; off <<= 1) {
            h0 += __shfl_xor(h0, off, LPR);
            h1 += __shfl_xor(h1, off, LPR);
        }
        if (q == 0) {
            const float2 hv = make_float2(h0, h1);
            hs[lr] = hv;
            reinterpret_cast<float2*>(H0)[row] = hv;
        }
    }
    __syncthreads();
    const float w0 = W0[c], w1 = W0[HD + c], bb = b0[c];
    double s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int lr = wv * 16 + r;
        if (tile * TILE + lr < end) {
            const float y = y0_of(hs[lr], w0, w1, bb);
            s1 += y;
            s2 += static_cast<double>(y) * y;
        }
    }
    s1 = wave4_sum(s1, sh);
    s2 = wave4_sum(s2, sh);
    if (wv == 0) {
        tstat[tile * 2 * HD + c] = s1;
        tstat[tile * 2 * HD + HD + c] = s2;
    }
}

// y (64 values of `rows` in LDS tile A[64][65]) times B (64 x 64) -> D tile [64][65] in LDS.
// FP32: lane c computes column c. BF16: v_mfma_f32_16x16x32_bf16 on the wavefront's 16 rows;
// Bt is the bf16 copy of B stored [col][k] (k contiguous) in LDS.
//
// SPLIT: A is passed as a_hi + a_lo, two bf16 numbers (16 significant bits), with one MFMA
// each. The aggregated features of a GCIN layer have a per-graph mean that is large next to
// their spread across nodes (the raw features a_ii, deg(i) are not centred), and the
// InstanceNorm that follows subtracts that mean: rounding each node's A row to a single bf16
// would be amplified by |A| / std(A) in the normalised output. Rounding of the weights is
// not amplified (it moves the mean and the rows alike), so B stays single bf16.
__device__ __forceinline__ void split_bf16(float x, unsigned short& hi, unsigned short& lo) {
    hi = f2bf(x);
    lo = f2bf(x - __uint_as_float(static_cast<unsigned int>(hi) << 16));
}

// SPLITB: B is passed as b_hi + b_lo as well and the product a_hi b_lo is added (the
// a_lo b_lo term is below FP32 resolution): an FP32-accurate product on the BF16 MFMA
// units, used where the result feeds non-smooth operations (ReLU masks, arg-max pooling)
// whose gradients must match an FP32/FP64 evaluation.
// GB: the bf16 copies of B (and of its low parts) are read from global memory, row-major [col][k]
// with row stride HD (Bg, Bglo; formed once per forward by weights_bf16_kernel), not from LDS:
// the weights are shared by every tile and stay in cache, and a workgroup's LDS holds no copy of
// them.
template <int HD, bool MFMA, bool SPLIT = false, bool SPLITB = false, bool GB = false>
__device__ __forceinline__ void tile_gemm(const float (*A)[HD + 1], const float* __restrict__ Bf,
                                          const unsigned short (*Bt)[HD + 8], float (*D)[HD + 1],
                                          const unsigned short (*Btlo)[HD + 8] = nullptr,
                                          const unsigned short* __restrict__ Bg = nullptr,
                                          const unsigned short* __restrict__ Bglo = nullptr) {
    static_assert(!MFMA || HD == 64, "the MFMA tiling is written for 64 channels");
    const int wv = threadIdx.x / HD, lane = threadIdx.x % HD;
    if constexpr (!MFMA) {
        for (int r = 0; r < 16; ++r) {
            const int lr = wv * 16 + r;
            float acc = 0.0f;
#pragma unroll 8
            for (int k = 0; k < HD; ++k) acc += A[lr][k] * Bf[k * HD + lane];
            D[lr][lane] = acc;
        }
    } else {
        const int i = lane % 16, kq = (lane / 16) * 8;
        f32x4 acc[4];
        for (int nb = 0; nb < 4; ++nb) acc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
        for (int ks = 0; ks < HD; ks += 32) {
            u16x8 av, alv;
            for (int e = 0; e < 8; ++e) {
                if constexpr (SPLIT) {
                    unsigned short h, l;
                    split_bf16(A[wv * 16 + i][ks + kq + e], h, l);
                    av[e] = h;
                    alv[e] = l;
                } else {
                    av[e] = f2bf(A[wv * 16 + i][ks + kq + e]);
                }
            }
            const bf16x8 a = __builtin_bit_cast(bf16x8, av);
            const bf16x8 al = __builtin_bit_cast(bf16x8, alv);
            for (int nb = 0; nb < 4; ++nb) {
                u16x8 bv;
                if constexpr (GB)
                    bv = *reinterpret_cast<const u16x8*>(Bg + (nb * 16 + i) * HD + ks + kq);
                else
                    for (int e = 0; e < 8; ++e) bv[e] = Bt[nb * 16 + i][ks + kq + e];
                const bf16x8 b = __builtin_bit_cast(bf16x8, bv);
                acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[nb], 0, 0, 0);
                if constexpr (SPLIT) acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, b, acc[nb], 0, 0, 0);
                if constexpr (SPLITB) {
                    u16x8 blv;
                    if constexpr (GB)
                        blv = *reinterpret_cast<const u16x8*>(Bglo + (nb * 16 + i) * HD + ks + kq);
                    else
                        for (int e = 0; e < 8; ++e) blv[e] = Btlo[nb * 16 + i][ks + kq + e];
                    const bf16x8 bl = __builtin_bit_cast(bf16x8, blv);
                    acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bl, acc[nb], 0, 0, 0);
                }
            }
        }
        for (int nb = 0; nb < 4; ++nb)
            for (int e = 0; e < 4; ++e) D[wv * 16 + (lane / 16) * 4 + e][nb * 16 + i] = acc[nb][e];
    }
}

// Stage a 64 x 64 FP32 matrix M (row-major [k][c]) for tile_gemm: bf16 copy as Bt[c][k] when
// `transpose`, else as Bt[k'][c'] = M[k'][c'] (used for products with M^T).
template <int HD>
__device__ __forceinline__ void stage_bf16(const float* __restrict__ M, bool transpose, unsigned short (*Bt)[HD + 8]) {
    for (int e = threadIdx.x; e < HD * HD; e += 4 * HD) {
        const int k = e / HD, c = e % HD;
        if (transpose)
            Bt[c][k] = f2bf(M[e]);
        else
            Bt[k][c] = f2bf(M[e]);
    }
}

// hi/lo bf16 pair of M^T (Bt[c][k] = hi, Btlo[c][k] = lo of M[k][c]).
template <int HD>
__device__ __forceinline__ void stage_bf16_split_t(const float* __restrict__ M, unsigned short (*Bt)[HD + 8],
                                                   unsigned short (*Btlo)[HD + 8]) {
    for (int e = threadIdx.x; e < HD * HD; e += 4 * HD) {
        const int k = e / HD, c = e % HD;
        unsigned short h, l;
        split_bf16(M[e], h, l);
        Bt[c][k] = h;
        Btlo[c][k] = l;
    }
}

// Y0: the layer below is layer 0, whose output is formed from H0 (y0_of) instead of read from Yp.
// bf16 hi / lo parts of the 64 x 64 weights of layers 1 .. NL-1, transposed ([col][k]) for
// tile_gemm's global-memory operand: block l - 1 forms layer l into wbf + (l - 1) 2 HD^2 (hi) and
// the HD^2 entries after it (lo).
template <int HD>
__global__ __launch_bounds__(256) void weights_bf16_kernel(const float* __restrict__ P, Offs o,
                                                         unsigned short* __restrict__ wbf) {
    const int l = blockIdx.x + 1;
    const float* W = P + o.convW[l];
    unsigned short* hi = wbf + static_cast<int64_t>(blockIdx.x) * 2 * HD * HD;
    for (int e = threadIdx.x; e < HD * HD; e += blockDim.x) {
        const int k = e / HD, c = e % HD;
        unsigned short h, lo;
        split_bf16(W[e], h, lo);
        hi[c * HD + k] = h;
        hi[HD * HD + c * HD + k] = lo;
    }
}

template <int HD, bool MFMA, bool X3, bool Y0>
__global__ __launch_bounds__(4 * HD) void layer_kernel(const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                                   const float* __restrict__ w, const int32_t* __restrict__ tile_graph,
                                                   const int32_t* __restrict__ gend, const float* __restrict__ Yp,
                                                   const float* __restrict__ H0, const float* __restrict__ W0,
                                                   const float* __restrict__ b0,
                                                   const float* __restrict__ mup, const float* __restrict__ rsp,
                                                   const float* __restrict__ gam, const float* __restrict__ bet,
                                                   const float* __restrict__ W, const float* __restrict__ b,
                                                   const unsigned short* __restrict__ wbf,
                                                   float* __restrict__ Hout, float* __restrict__ Y,
                                                   double* __restrict__ tstat, double* __restrict__ psum,
                                                   float* __restrict__ pmax, int32_t* __restrict__ parg) {
    // The kernel also forms the per-tile readout partials of the layer below (psum / pmax / parg
    // as pool_tile_kernel writes them): every row's own entry of A_hat brings that row's
    // normalised, rectified input x, which is kept in Xs and pooled in the output loop in
    // pool_tile_kernel's order, so the layer below needs no pooling pass.
    // The product overwrites the aggregates in place: every wavefront reads only its own 16
    // rows of Hs and writes the same rows, each output after all of its row's reads (the
    // stores depend on them), so one tile buffer serves both, and after the output loop it holds
    // the per-tile reductions; with the weights' bf16 parts read from global memory (wbf: hi,
    // then lo) the tile and the rows' own inputs Xs are all the LDS a workgroup holds (33 KB with
    // 64 channels: 4 workgroups per CU, as many as the registers admit).
    __shared__ __align__(16) float Hs[TILE][HD + 1];  // aggregates, products, then the reductions
    float (*Ds)[HD + 1] = Hs;
    __shared__ float Xs[TILE][HD + 1];
    const int tile = blockIdx.x, wv = threadIdx.x / HD, c = threadIdx.x % HD;
    const int g = tile_graph[tile];
    const int32_t end = gend[g];
    const int32_t r0 = tile * TILE + wv * 16;
    {
        // channels 4 p .. 4 p + 3 of the lane's group (see visit_rows_x4)
        constexpr int G = HD / 4;
        const int c4 = 4 * static_cast<int>(threadIdx.x % G);
        const float4 mu4 = *reinterpret_cast<const float4*>(mup + g * HD + c4);
        const float4 rs4 = *reinterpret_cast<const float4*>(rsp + g * HD + c4);
        const float4 ga4 = *reinterpret_cast<const float4*>(gam + c4);
        const float4 be4 = *reinterpret_cast<const float4*>(bet + c4);
        float4 w04 = make_float4(0.f, 0.f, 0.f, 0.f), w14 = w04, bb4 = w04;
        if constexpr (Y0) {
            w04 = *reinterpret_cast<const float4*>(W0 + c4);
            w14 = *reinterpret_cast<const float4*>(W0 + HD + c4);
            bb4 = *reinterpret_cast<const float4*>(b0 + c4);
        }
        float4 h4 = make_float4(0.f, 0.f, 0.f, 0.f);
        visit_rows_x4<G>(
            ptr, col, w, r0,
            [&](int32_t j) {
                if constexpr (Y0) {
                    const float2 hv = reinterpret_cast<const float2*>(H0)[j];
                    return make_float4(y0_of(hv, w04.x, w14.x, bb4.x), y0_of(hv, w04.y, w14.y, bb4.y),
                                       y0_of(hv, w04.z, w14.z, bb4.z), y0_of(hv, w04.w, w14.w, bb4.w));
                } else {
                    return *reinterpret_cast<const float4*>(Yp + static_cast<int64_t>(j) * HD + c4);
                }
            },
            [&](float wp, const float4& v, int32_t self) {
                const float4 x = make_float4(normrelu(v.x, mu4.x, rs4.x, ga4.x, be4.x),
                                             normrelu(v.y, mu4.y, rs4.y, ga4.y, be4.y),
                                             normrelu(v.z, mu4.z, rs4.z, ga4.z, be4.z),
                                             normrelu(v.w, mu4.w, rs4.w, ga4.w, be4.w));
                h4.x += wp * x.x;
                h4.y += wp * x.y;
                h4.z += wp * x.z;
                h4.w += wp * x.w;
                if (self >= 0) {
                    float* xs = &Xs[self - tile * TILE][c4];
                    xs[0] = x.x;
                    xs[1] = x.y;
                    xs[2] = x.z;
                    xs[3] = x.w;
                }
            },
            [&](int32_t row) {
                const float4 hv = row < end ? h4 : make_float4(0.f, 0.f, 0.f, 0.f);
                float* hs = &Hs[row - tile * TILE][c4];
                hs[0] = hv.x;
                hs[1] = hv.y;
                hs[2] = hv.z;
                hs[3] = hv.w;
                if (Hout) *reinterpret_cast<float4*>(Hout + static_cast<int64_t>(row) * HD + c4) = hv;
                h4 = make_float4(0.f, 0.f, 0.f, 0.f);
            });
    }
    __syncthreads();
    tile_gemm<HD, MFMA, true, X3, true>(Hs, W, nullptr, Ds, nullptr, wbf, wbf + HD * HD);
    __syncthreads();
    // y of the wave's rows with the per-tile sums of y and y^2 and the readout partials of the
    // layer below (sum, max and first arg-max of x per channel; each row's x came with its own
    // entry, rows past the graph have none), each summed over the rows in order
    const float bc = b[c];
    double s1 = 0.0, s2 = 0.0, ps = 0.0;
    float mx = -INFINITY;
    int32_t am = INT32_MAX;
    for (int r = 0; r < 16; ++r) {
        const int lr = wv * 16 + r;
        const int32_t row = tile * TILE + lr;
        float y = 0.0f;
        if (row < end) {
            y = Ds[lr][c] + bc;
            s1 += y;
            s2 += static_cast<double>(y) * y;
            const float x = Xs[lr][c];
            ps += x;
            if (x > mx) {
                mx = x;
                am = row;
            }
        }
        Y[static_cast<int64_t>(row) * HD + c] = y;
    }
    // every wave has read its rows of the tile, whose space now holds the four waves' partials;
    // wave 0 combines them in wave order
    __syncthreads();
    double (*r1)[HD] = reinterpret_cast<double (*)[HD]>(&Hs[0][0]);
    double (*r2)[HD] = r1 + 4;
    double (*rp)[HD] = r1 + 8;
    float (*rmax)[HD] = reinterpret_cast<float (*)[HD]>(r1 + 12);
    int32_t (*rarg)[HD] = reinterpret_cast<int32_t (*)[HD]>(rmax + 4);
    r1[wv][c] = s1;
    r2[wv][c] = s2;
    rp[wv][c] = ps;
    rmax[wv][c] = mx;
    rarg[wv][c] = am;
    __syncthreads();
    if (wv == 0) {
        tstat[tile * 2 * HD + c] = r1[0][c] + r1[1][c] + r1[2][c] + r1[3][c];
        tstat[tile * 2 * HD + HD + c] = r2[0][c] + r2[1][c] + r2[2][c] + r2[3][c];
        for (int k = 1; k < 4; ++k)
            if (rmax[k][c] > mx) {
                mx = rmax[k][c];
                am = rarg[k][c];
            }
        psum[tile * HD + c] = rp[0][c] + rp[1][c] + rp[2][c] + rp[3][c];
        pmax[tile * HD + c] = mx;
        parg[tile * HD + c] = am;
    }
}

// Per-graph reductions over tiles run in two fixed-order stages so that large graphs (the fine
// level has n/64 tiles) are spread over many workgroups: stage 1 sums the tiles of each chunk
// (at most kChunkTiles consecutive tiles of one graph, chunks counted from the graph's first
// tile), stage 2 the chunks of each graph. In both, wave w of the workgroup sums items w, w+4,
// w+8, ... in order and the four wave sums are added in wave order: deterministic, and a
// graph's result does not depend on the other graphs of the batch.
constexpr int kChunkTiles = 256;

// out[k][j][c] = sum over items i in [bounds[k], bounds[k+1]) of in[i][j][c], j < K, c < HD
template <int HD, int K>
__global__ __launch_bounds__(4 * HD) void chunk_sum_kernel(const double* __restrict__ in, const int32_t* __restrict__ bounds,
                                                       double* __restrict__ out) {
    __shared__ double sh[4][K][HD];
    const int k = blockIdx.x, wv = threadIdx.x / HD, c = threadIdx.x % HD;
    double s[K];
#pragma unroll
    for (int j = 0; j < K; ++j) s[j] = 0.0;
    // items wv, wv + 4, ... in order; four items' loads are issued ahead of their additions
    const int32_t i1 = bounds[k + 1];
    int32_t i = bounds[k] + wv;
    for (; i + 12 < i1; i += 16) {
        double v[4][K];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int j = 0; j < K; ++j) v[u][j] = in[(static_cast<int64_t>(i + 4 * u) * K + j) * HD + c];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int j = 0; j < K; ++j) s[j] += v[u][j];
    }
    for (; i < i1; i += 4)
#pragma unroll
        for (int j = 0; j < K; ++j) s[j] += in[(static_cast<int64_t>(i) * K + j) * HD + c];
#pragma unroll
    for (int j = 0; j < K; ++j) sh[wv][j][c] = s[j];
    __syncthreads();
    if (wv == 0)
#pragma unroll
        for (int j = 0; j < K; ++j)
            out[(static_cast<int64_t>(k) * K + j) * HD + c] = ((sh[0][j][c] + sh[1][j][c]) + sh[2][j][c]) + sh[3][j][c];
}

// Per graph and channel: mean and 1/sqrt(biased variance + eps) from the chunk sums.
template <int HD>
__global__ __launch_bounds__(4 * HD) void stats_final_kernel(const double* __restrict__ cstat,
                                                         const int32_t* __restrict__ gchunk,
                                                         const float* __restrict__ gcnt, float* __restrict__ mu,
                                                         float* __restrict__ rstd) {
    __shared__ double sh[4][2][HD];
    const int g = blockIdx.x, wv = threadIdx.x / HD, c = threadIdx.x % HD;
    double s1 = 0.0, s2 = 0.0;
    for (int32_t k = gchunk[g] + wv; k < gchunk[g + 1]; k += 4) {
        s1 += cstat[static_cast<int64_t>(k) * 2 * HD + c];
        s2 += cstat[static_cast<int64_t>(k) * 2 * HD + HD + c];
    }
    sh[wv][0][c] = s1;
    sh[wv][1][c] = s2;
    __syncthreads();
    if (wv != 0) return;
    s1 = ((sh[0][0][c] + sh[1][0][c]) + sh[2][0][c]) + sh[3][0][c];
    s2 = ((sh[0][1][c] + sh[1][1][c]) + sh[2][1][c]) + sh[3][1][c];
    const double n = gcnt[g];
    const double m = s1 / n;
    double var = s2 / n - m * m;
    if (var < 0.0) var = 0.0;
    mu[g * HD + c] = static_cast<float>(m);
    rstd[g * HD + c] = static_cast<float>(1.0 / sqrt(var + static_cast<double>(kEps)));
}

// y of rows r0 .. r0 + 15 in channel c (0 past the graph's end): read from Y, or formed from H0
// for layer 0; the 16 loads are issued together.
template <int HD, bool Y0>
__device__ __forceinline__ void load_rows(float (&yv)[16], int32_t r0, int32_t end, int c, const float* __restrict__ Y,
                                          const float* __restrict__ H0, const float* __restrict__ W0,
                                          const float* __restrict__ b0) {
    if constexpr (Y0) {
        const float w0 = W0[c], w1 = W0[HD + c], bb = b0[c];
        float2 hv[16];
#pragma unroll
        for (int r = 0; r < 16; ++r)
            hv[r] = r0 + r < end ? reinterpret_cast<const float2*>(H0)[r0 + r] : make_float2(0.0f, 0.0f);
#pragma unroll
        for (int r = 0; r < 16; ++r) yv[r] = r0 + r < end ? y0_of(hv[r], w0, w1, bb) : 0.0f;
    } else {
#pragma unroll
        for (int r = 0; r < 16; ++r) yv[r] = r0 + r < end ? Y[static_cast<int64_t>(r0 + r) * HD + c] : 0.0f;
    }
}

// Per tile: sum, max and first arg-max of x = ReLU(IN(y)) per channel.
template <int HD, bool Y0>
__global__ __launch_bounds__(4 * HD) void pool_tile_kernel(const int32_t* __restrict__ tile_graph,
                                                       const int32_t* __restrict__ gend, const float* __restrict__ Y,
                                                       const float* __restrict__ H0, const float* __restrict__ W0,
                                                       const float* __restrict__ b0,
                                                       const float* __restrict__ mu, const float* __restrict__ rstd,
                                                       const float* __restrict__ gam, const float* __restrict__ bet,
                                                       double* __restrict__ tsum, float* __restrict__ tmax,
                                                       int32_t* __restrict__ targ) {
    __shared__ double sh[4][HD];
    __shared__ float smax[4][HD];
    __shared__ int32_t sarg[4][HD];
    const int tile = blockIdx.x, wv = threadIdx.x / HD, c = threadIdx.x % HD;
    const int g = tile_graph[tile];
    const int32_t end = gend[g];
    const float m = mu[g * HD + c], rs = rstd[g * HD + c], ga = gam[c], be = bet[c];
    double s = 0.0;
    float mx = -INFINITY;
    int32_t am = INT32_MAX;
    float yv[16];  // the 16 rows' loads are issued together
    load_rows<HD, Y0>(yv, tile * TILE + wv * 16, end, c, Y, H0, W0, b0);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int32_t row = tile * TILE + wv * 16 + r;
        if (row < end) {
            const float x = normrelu(yv[r], m, rs, ga, be);
            s += x;
            if (x > mx) {
                mx = x;
                am = row;
            }
        }
    }
    smax[wv][c] = mx;
    sarg[wv][c] = am;
    s = wave4_sum(s, sh);
    if (wv == 0) {
        for (int k = 1; k < 4; ++k)
            if (smax[k][c] > mx) {
                mx = smax[k][c];
                am = sarg[k][c];
            }
        tsum[tile * HD + c] = s;
        tmax[tile * HD + c] = mx;
        targ[tile * HD + c] = am;
    }
}

// Max with its arg-max, ties to the lowest node index (any combination order gives the same).
__device__ __forceinline__ void max_merge(float& mx, int32_t& am, float m2, int32_t a2) {
    if (m2 > mx || (m2 == mx && a2 < am)) {
        mx = m2;
        am = a2;
    }
}

// Stage 1 of the pooling reduction (see chunk_sum_kernel): per chunk, sum, max and arg-max.
template <int HD>
__global__ __launch_bounds__(4 * HD) void pool_chunk_kernel(const double* __restrict__ tsum, const float* __restrict__ tmax,
                                                        const int32_t* __restrict__ targ,
                                                        const int32_t* __restrict__ bounds, double* __restrict__ csum,
                                                        float* __restrict__ cmax, int32_t* __restrict__ carg) {
    __shared__ double ss[4][HD];
    __shared__ float sm[4][HD];
    __shared__ int32_t sa[4][HD];
    const int k = blockIdx.x, wv = threadIdx.x / HD, c = threadIdx.x % HD;
    double s = 0.0;
    float mx = -INFINITY;
    int32_t am = INT32_MAX;
    // tiles wv, wv + 4, ... in order; four tiles' loads are issued ahead of their use
    const int32_t t1 = bounds[k + 1];
    int32_t t = bounds[k] + wv;
    for (; t + 12 < t1; t += 16) {
        double vs[4];
        float vm[4];
        int32_t va[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t e = static_cast<int64_t>(t + 4 * u) * HD + c;
            vs[u] = tsum[e];
            vm[u] = tmax[e];
            va[u] = targ[e];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            s += vs[u];
            max_merge(mx, am, vm[u], va[u]);
        }
    }
    for (; t < t1; t += 4) {
        s += tsum[static_cast<int64_t>(t) * HD + c];
        max_merge(mx, am, tmax[static_cast<int64_t>(t) * HD + c], targ[static_cast<int64_t>(t) * HD + c]);
    }
    ss[wv][c] = s;
    sm[wv][c] = mx;
    sa[wv][c] = am;
    __syncthreads();
    if (wv != 0) return;
    for (int w = 1; w < 4; ++w) max_merge(mx, am, sm[w][c], sa[w][c]);
    csum[static_cast<int64_t>(k) * HD + c] = ((ss[0][c] + ss[1][c]) + ss[2][c]) + ss[3][c];
    cmax[static_cast<int64_t>(k) * HD + c] = mx;
    carg[static_cast<int64_t>(k) * HD + c] = am;
}

template <int HD>
__global__ __launch_bounds__(4 * HD) void pool_final_kernel(const double* __restrict__ csum, const float* __restrict__ cmax,
                                                        const int32_t* __restrict__ carg,
                                                        const int32_t* __restrict__ gchunk,
                                                        const float* __restrict__ gcnt, int layer,
                                                        float* __restrict__ pooled, int32_t* __restrict__ argmax) {
    __shared__ double ss[4][HD];
    __shared__ float sm[4][HD];
    __shared__ int32_t sa[4][HD];
    const int g = blockIdx.x, wv = threadIdx.x / HD, c = threadIdx.x % HD;
    double s = 0.0;
    float mx = -INFINITY;
    int32_t am = INT32_MAX;
    for (int32_t k = gchunk[g] + wv; k < gchunk[g + 1]; k += 4) {
        s += csum[static_cast<int64_t>(k) * HD + c];
        max_merge(mx, am, cmax[static_cast<int64_t>(k) * HD + c], carg[static_cast<int64_t>(k) * HD + c]);
    }
    ss[wv][c] = s;
    sm[wv][c] = mx;
    sa[wv][c] = am;
    __syncthreads();
    if (wv != 0) return;
    for (int w = 1; w < 4; ++w) max_merge(mx, am, sm[w][c], sa[w][c]);
    s = ((ss[0][c] + ss[1][c]) + ss[2][c]) + ss[3][c];
    pooled[(g * NL + layer) * 2 * HD + c] = static_cast<float>(s / gcnt[g]);
    pooled[(g * NL + layer) * 2 * HD + HD + c] = mx;
    argmax[(g * NL + layer) * HD + c] = am;
}

__device__ __forceinline__ float block128_sum(float v, float* red) {
    // 128 threads
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = 64; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    const float r = red[0];
    __syncthreads();
    return r;
}

struct HeadSave {
    float* z;    // [G][128] readout concatenation
    float* ln;   // [G][2]   mean, rstd
    float* s;    // [G][128] sigmoid output
    float* a1;   // [G][128]
    float* a2;   // [G][64]
};

// Readout, LayerNorm, sigmoid and predictive MLP of one graph per workgroup (128 threads).
template <int HD>
__global__ __launch_bounds__(128) void head_fwd_kernel(const float* __restrict__ P, Offs o,
                                                       const float* __restrict__ pooled, HeadSave hs,
                                                       float* __restrict__ out) {
    __shared__ float p[NL * 2 * HD], z[JK], s[JK], a1[M1], a2[M2], red[128];
    const int g = blockIdx.x, t = threadIdx.x;
    for (int k = t; k < NL * 2 * HD; k += 128) p[k] = pooled[g * NL * 2 * HD + k];
    __syncthreads();
    {
        const int l = t / RO, oo = t % RO;
        float acc = P[o.rob[l] + oo];
        for (int k = 0; k < 2 * HD; ++k) acc += p[l * 2 * HD + k] * P[o.roW[l] + k * RO + oo];
        z[t] = acc;
    }
    __syncthreads();
    const float m = block128_sum(z[t], red) / JK;
    const float dz = z[t] - m;
    const float v = block128_sum(dz * dz, red) / JK;
    const float rs = 1.0f / sqrtf(v + kEps);
    const float zn = dz * rs * P[o.lng + t] + P[o.lnb + t];
    s[t] = 1.0f / (1.0f + expf(-zn));
    __syncthreads();
    {
        float acc = P[o.m0b + t];
        for (int k = 0; k < JK; ++k) acc += s[k] * P[o.m0W + k * M1 + t];
        a1[t] = fmaxf(acc, 0.0f);
    }
    __syncthreads();
    if (t < M2) {
        float acc = P[o.m1b + t];
        for (int k = 0; k < M1; ++k) acc += a1[k] * P[o.m1W + k * M2 + t];
        a2[t] = fmaxf(acc, 0.0f);
    }
    __syncthreads();
    if (t < o.nout) {
        float acc = P[o.m2b + t];
        for (int k = 0; k < M2; ++k) acc += a2[k] * P[o.m2W + k * o.nout + t];
        out[g * o.nout + t] = acc;
    }
    hs.z[g * JK + t] = z[t];
    hs.s[g * JK + t] = s[t];
    hs.a1[g * M1 + t] = a1[t];
    if (t < M2) hs.a2[g * M2 + t] = a2[t];
    if (t == 0) {
        hs.ln[2 * g] = m;
        hs.ln[2 * g + 1] = rs;
    }
}

// ------------------------------------------------------------------------------------------
// backward
// ------------------------------------------------------------------------------------------
// Head backward of one graph; writes this graph's head-parameter gradients (relative to
// o.head0) into gh[g][*] and the pooled-feature gradients into dpooled[g].
template <int HD>
__global__ __launch_bounds__(128) void head_bwd_kernel(const float* __restrict__ P, Offs o,
                                                       const float* __restrict__ pooled, HeadSave hs,
                                                       const float* __restrict__ dout, float* __restrict__ gh,
                                                       int64_t ghstride, float* __restrict__ dpooled) {
    __shared__ float p[NL * 2 * HD], s[JK], a1[M1], a2[M2], d2[M2], d1[M1], dzv[JK], red[128], dov[kMaxOut];
    const int g = blockIdx.x, t = threadIdx.x;
    float* const gbase = gh + g * ghstride;
    auto G = [&](int64_t off) -> float& { return gbase[off - o.head0]; };  // absolute parameter offsets
    for (int k = t; k < NL * 2 * HD; k += 128) p[k] = pooled[g * NL * 2 * HD + k];
    s[t] = hs.s[g * JK + t];
    a1[t] = hs.a1[g * M1 + t];
    if (t < M2) a2[t] = hs.a2[g * M2 + t];
    if (t < o.nout) dov[t] = dout[g * o.nout + t];
    __syncthreads();
    // out = a2 W3 + b3
    if (t < o.nout) G(o.m2b + t) = dov[t];
    for (int e = t; e < M2 * o.nout; e += 128) G(o.m2W + e) = a2[e / o.nout] * dov[e % o.nout];
    if (t < M2) {
        float acc = 0.0f;
        for (int q = 0; q < o.nout; ++q) acc += dov[q] * P[o.m2W + t * o.nout + q];
        d2[t] = a2[t] > 0.0f ? acc : 0.0f;
    }
    __syncthreads();
    // a2 = relu(a1 W2 + b2)
    if (t < M2) G(o.m1b + t) = d2[t];
    for (int e = t; e < M1 * M2; e += 128) G(o.m1W + e) = a1[e / M2] * d2[e % M2];
    {
        float acc = 0.0f;
        for (int q = 0; q < M2; ++q) acc += d2[q] * P[o.m1W + t * M2 + q];
        d1[t] = a1[t] > 0.0f ? acc : 0.0f;
    }
    __syncthreads();
    // a1 = relu(s W1 + b1)
    G(o.m0b + t) = d1[t];
    for (int e = t; e < JK * M1; e += 128) G(o.m0W + e) = s[e / M1] * d1[e % M1];
    float ds = 0.0f;
    for (int q = 0; q < M1; ++q) ds += d1[q] * P[o.m0W + t * M1 + q];
    // s = sigmoid(zn), zn = zhat gamma + beta, zhat = (z - m) rstd
    const float dzn = ds * s[t] * (1.0f - s[t]);
    const float m = hs.ln[2 * g], rs = hs.ln[2 * g + 1];
    const float zh = (hs.z[g * JK + t] - m) * rs;
    G(o.lng + t) = dzn * zh;
    G(o.lnb + t) = dzn;
    const float dzh = dzn * P[o.lng + t];
    const float mean_a = block128_sum(dzh, red) / JK;
    const float mean_b = block128_sum(dzh * zh, red) / JK;
    dzv[t] = rs * (dzh - mean_a - zh * mean_b);
    __syncthreads();
    // z[l*32+o] = rob_l[o] + sum_k p_l[k] roW_l[k][o]
    for (int l = 0; l < NL; ++l) {
        if (t < RO) G(o.rob[l] + t) = dzv[l * RO + t];
        for (int e = t; e < 2 * HD * RO; e += 128) G(o.roW[l] + e) = p[l * 2 * HD + e / RO] * dzv[l * RO + e % RO];
        for (int k = t; k < 2 * HD; k += 128) {
            float acc = 0.0f;
            for (int q = 0; q < RO; ++q) acc += dzv[l * RO + q] * P[o.roW[l] + k * RO + q];
            dpooled[(g * NL + l) * 2 * HD + k] = acc;
        }
    }
}

// Layer backward, first half, per tile: dX from pooling (mean and arg-max) and, below the last
// layer, from the next layer's aggregation (A_hat^T dH = A_hat dH, A symmetric); ReLU and the
// affine part of InstanceNorm; per-tile sums for the normalisation backward and gamma/beta.
template <int HD, bool Y0>
__global__ __launch_bounds__(4 * HD) void bwd_a_kernel(const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                                   const float* __restrict__ w, const int32_t* __restrict__ tile_graph,
                                                   const int32_t* __restrict__ gend, const float* __restrict__ gcnt,
                                                   const float* __restrict__ Y, const float* __restrict__ H0,
                                                   const float* __restrict__ W0, const float* __restrict__ b0,
                                                   const float* __restrict__ mu,
                                                   const float* __restrict__ rstd, const float* __restrict__ gam,
                                                   const float* __restrict__ bet, const float* __restrict__ dpooled,
                                                   const int32_t* __restrict__ argmax, int layer,
                                                   const float* __restrict__ dHn, float* __restrict__ dxh,
                                                   double* __restrict__ tb) {
    __shared__ double sh[4][HD];
    const int tile = blockIdx.x, wv = threadIdx.x / HD, c = threadIdx.x % HD;
    const int g = tile_graph[tile];
    const int32_t end = gend[g];
    const float m = mu[g * HD + c], rs = rstd[g * HD + c], ga = gam[c], be = bet[c];
    const float dmean = dpooled[(g * NL + layer) * 2 * HD + c] / gcnt[g];
    const float dmax = dpooled[(g * NL + layer) * 2 * HD + HD + c];
    const int32_t am = argmax[(g * NL + layer) * HD + c];
    __shared__ float aggs[TILE][HD];  // per row: sum of w * dH of the layer above (A_hat^T = A_hat)
    double sa = 0.0, sb = 0.0, sg = 0.0, sbe = 0.0;
    const int32_t r0 = tile * TILE + wv * 16;
    float yv[16];  // this wavefront's rows of Y, loaded together while the aggregation runs
    load_rows<HD, Y0>(yv, r0, end, c, Y, H0, W0, b0);
    float acc = 0.0f;
    if (dHn) {
        visit_rows<HD, float>(
            ptr, col, w, r0, r0 + 16, [&](int32_t j) { return dHn[static_cast<int64_t>(j) * HD + c]; },
            [&](float wp, float v) { acc += wp * v; },
            [&](int32_t row) {
                aggs[row - tile * TILE][c] = acc;
                acc = 0.0f;
            });
    } else {
#pragma unroll
        for (int r = 0; r < 16; ++r) aggs[wv * 16 + r][c] = 0.0f;
    }
    // each lane reads back only what it wrote (same wavefront, same channel): no barrier needed
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int32_t row = r0 + r;
        float d = 0.0f;
        if (row < end) {
            const float dx = dmean + (row == am ? dmax : 0.0f) + aggs[wv * 16 + r][c];
            const float xh = (yv[r] - m) * rs;
            const float xn = xh * ga + be;
            const float dxn = xn > 0.0f ? dx : 0.0f;
            d = dxn * ga;
            sa += d;
            sb += static_cast<double>(d) * xh;
            sg += static_cast<double>(dxn) * xh;
            sbe += dxn;
        }
        dxh[static_cast<int64_t>(row) * HD + c] = d;
    }
    sa = wave4_sum(sa, sh);
    sb = wave4_sum(sb, sh);
    sg = wave4_sum(sg, sh);
    sbe = wave4_sum(sbe, sh);
    if (wv == 0) {
        tb[tile * 4 * HD + c] = sa;
        tb[tile * 4 * HD + HD + c] = sb;
        tb[tile * 4 * HD + 2 * HD + c] = sg;
        tb[tile * 4 * HD + 3 * HD + c] = sbe;
    }
}

// Per graph: means of dxhat and dxhat*xhat; gamma/beta gradients of the graph (from the chunk
// sums of the four per-tile quantities, as in stats_final_kernel).
template <int HD>
__global__ __launch_bounds__(4 * HD) void bwd_final_kernel(const double* __restrict__ ctb, const int32_t* __restrict__ gchunk,
                                                       const float* __restrict__ gcnt, float* __restrict__ gmean,
                                                       double* __restrict__ ggb) {
    __shared__ double sh[4][4][HD];
    const int g = blockIdx.x, wv = threadIdx.x / HD, c = threadIdx.x % HD;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int32_t k = gchunk[g] + wv; k < gchunk[g + 1]; k += 4)
#pragma unroll
        for (int j = 0; j < 4; ++j) s[j] += ctb[(static_cast<int64_t>(k) * 4 + j) * HD + c];
#pragma unroll
    for (int j = 0; j < 4; ++j) sh[wv][j][c] = s[j];
    __syncthreads();
    if (wv != 0) return;
#pragma unroll
    for (int j = 0; j < 4; ++j) s[j] = ((sh[0][j][c] + sh[1][j][c]) + sh[2][j][c]) + sh[3][j][c];
    gmean[g * 2 * HD + c] = static_cast<float>(s[0] / gcnt[g]);
    gmean[g * 2 * HD + HD + c] = static_cast<float>(s[1] / gcnt[g]);
    ggb[g * 2 * HD + c] = s[2];
    ggb[g * 2 * HD + HD + c] = s[3];
}

// Layer backward, second half. dY = rstd (dxhat - mean(dxhat) - xhat mean(dxhat xhat));
// dH = dY W^T (stored for the layer below unless first); partial dW = H^T dY and db = sum dY
// accumulated over the tiles a workgroup visits (fixed grid of kWBlocks, fixed order).
template <int HD, bool MFMA, bool Y0>
__global__ __launch_bounds__(4 * HD) void bwd_b_kernel(int ntiles, const int32_t* __restrict__ tile_graph,
                                                   const int32_t* __restrict__ gend, const float* __restrict__ Y,
                                                   const float* __restrict__ H0, const float* __restrict__ W0,
                                                   const float* __restrict__ b0,
                                                   const float* __restrict__ mu, const float* __restrict__ rstd,
                                                   const float* __restrict__ gmean, const float* __restrict__ dxh,
                                                   const float* __restrict__ H, int in_dim,
                                                   const float* __restrict__ W, float* __restrict__ dH,
                                                   float* __restrict__ wpart, double* __restrict__ bpart) {
    __shared__ float dYs[TILE][HD + 1];
    __shared__ float Hs[TILE][HD + 1];
    float (*Ds)[HD + 1] = Hs;  // the dH product is formed after dW no longer needs Hs
    __shared__ unsigned short Bt[HD][HD + 8];
    __shared__ double sh[4][HD];
    const int wv = threadIdx.x / HD, c = threadIdx.x % HD;
    static_assert(!MFMA || HD == 64, "the MFMA tiling is written for 64 channels");
    constexpr int NT = 4 * HD, NW = HD / 4;  // threads; dW entries per thread (in_dim <= HD)
    if constexpr (MFMA) {
        if (dH) stage_bf16<HD>(W, false, Bt);  // dH = dY W^T: B[c'][k] = W[k][c'] read as rows of W
    }
    // dW accumulator: thread owns W entries e = threadIdx.x + q*NT (in_dim*HD entries)
    float accw[NW];
    for (int q = 0; q < NW; ++q) accw[q] = 0.0f;
    double accb = 0.0;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int g = tile_graph[tile];
        const int32_t end = gend[g];
        const float m = mu[g * HD + c], rs = rstd[g * HD + c];
        const float ma = gmean[g * 2 * HD + c], mb = gmean[g * 2 * HD + HD + c];
        // eight rows at a time, their loads issued together
        for (int r8 = 0; r8 < 16; r8 += 8) {
            float yv[8], dv[8], hv[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const int32_t row = tile * TILE + wv * 16 + r8 + r;
                const int64_t k = static_cast<int64_t>(row) * HD + c;
                const bool ok = row < end;
                if constexpr (Y0)
                    yv[r] = ok ? y0_of(reinterpret_cast<const float2*>(H0)[row], W0[c], W0[HD + c], b0[c]) : 0.0f;
                else
                    yv[r] = ok ? Y[k] : 0.0f;
                dv[r] = ok ? dxh[k] : 0.0f;
                hv[r] = ok && c < in_dim ? H[static_cast<int64_t>(row) * in_dim + c] : 0.0f;
            }
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const int lr = wv * 16 + r8 + r;
                const int32_t row = tile * TILE + lr;
                float dy = 0.0f;
                if (row < end) {
                    const float xh = (yv[r] - m) * rs;
                    dy = rs * (dv[r] - ma - xh * mb);
                }
                dYs[lr][c] = dy;
                Hs[lr][c] = hv[r];
                accb += dy;
            }
        }
        __syncthreads();
        // dW[k][c'] += sum_rows H[row][k] dY[row][c']
        if constexpr (!MFMA) {
            for (int q = 0; q < NW; ++q) {
                const int e = threadIdx.x + q * NT;
                if (e < in_dim * HD) {
                    const int k = e / HD, cc = e % HD;
                    float acc = 0.0f;
                    for (int r = 0; r < TILE; ++r) acc += Hs[r][k] * dYs[r][cc];
                    accw[q] += acc;
                }
            }
        } else {
            if (in_dim == HD) {
                // 64 x 64 = (H^T)(64 x 64 rows) (dY): wavefront wv owns output rows k in [16 wv, 16 wv + 16)
                const int lane = c, i = lane % 16, kq = (lane / 16) * 8;
                f32x4 acc[4];
                for (int nb = 0; nb < 4; ++nb) acc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
                for (int ks = 0; ks < TILE; ks += 32) {
                    // H^T is the uncentred operand here as in the forward product: split it
                    u16x8 av, alv;
                    for (int e = 0; e < 8; ++e) {
                        unsigned short h, l;
                        split_bf16(Hs[ks + kq + e][wv * 16 + i], h, l);
                        av[e] = h;
                        alv[e] = l;
                    }
                    const bf16x8 a = __builtin_bit_cast(bf16x8, av);
                    const bf16x8 al = __builtin_bit_cast(bf16x8, alv);
                    for (int nb = 0; nb < 4; ++nb) {
                        u16x8 bv;
                        for (int e = 0; e < 8; ++e) bv[e] = f2bf(dYs[ks + kq + e][nb * 16 + i]);
                        const bf16x8 b = __builtin_bit_cast(bf16x8, bv);
                        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[nb], 0, 0, 0);
                        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, b, acc[nb], 0, 0, 0);
                    }
                }
                // lane holds rows k = 16 wv + 4 (lane/16) + e, column 16 nb + i; map to accw slots
                for (int nb = 0; nb < 4; ++nb)
                    for (int e = 0; e < 4; ++e) accw[nb * 4 + e] += acc[nb][e];
            } else {
                for (int q = 0; q < NW; ++q) {
                    const int e = threadIdx.x + q * NT;
                    if (e < in_dim * HD) {
                        const int k = e / HD, cc = e % HD;
                        float acc = 0.0f;
                        for (int r = 0; r < TILE; ++r) acc += Hs[r][k] * dYs[r][cc];
                        accw[q] += acc;
                    }
                }
            }
        }
        if (dH) {  // dH = dY W^T into the rows of Hs
            __syncthreads();
            if constexpr (!MFMA) {
                for (int r = 0; r < 16; ++r) {
                    const int lr = wv * 16 + r;
                    float acc = 0.0f;
#pragma unroll 8
                    for (int q = 0; q < HD; ++q) acc += dYs[lr][q] * W[c * HD + q];
                    Ds[lr][c] = acc;
                }
            } else {
                tile_gemm<HD, true>(dYs, W, Bt, Ds);
            }
            __syncthreads();
            for (int r = 0; r < 16; ++r) {
                const int lr = wv * 16 + r;
                const int32_t row = tile * TILE + lr;
                dH[static_cast<int64_t>(row) * HD + c] = row < end ? Ds[lr][c] : 0.0f;
            }
        }
        __syncthreads();
    }
    // write this workgroup's partials in plain [k][c] order
    if (MFMA && in_dim == HD) {
        const int lane = c, i = lane % 16;
        for (int nb = 0; nb < 4; ++nb)
            for (int e = 0; e < 4; ++e) {
                const int k = wv * 16 + (lane / 16) * 4 + e, cc = nb * 16 + i;
                wpart[static_cast<int64_t>(blockIdx.x) * HD * HD + k * HD + cc] = accw[nb * 4 + e];
            }
    } else {
        for (int q = 0; q < NW; ++q) {
            const int e = threadIdx.x + q * NT;
            if (e < in_dim * HD) wpart[static_cast<int64_t>(blockIdx.x) * HD * HD + e] = accw[q];
        }
    }
    accb = wave4_sum(accb, sh);
    if (wv == 0) bpart[blockIdx.x * HD + c] = accb;
}

// One workgroup: D1 = A B by the FP32 path and D2 = A B by the BF16 MFMA path of tile_gemm.
__global__ __launch_bounds__(256) void tile_gemm_check_kernel(const float* __restrict__ A, const float* __restrict__ B,
                                                              float* __restrict__ D1, float* __restrict__ D2) {
    constexpr int HD = 64, NT = 256;
    __shared__ float As[TILE][HD + 1];
    __shared__ float Ds[TILE][HD + 1];
    __shared__ unsigned short Bt[HD][HD + 8];
    for (int e = threadIdx.x; e < TILE * HD; e += NT) As[e / HD][e % HD] = A[e];
    stage_bf16<HD>(B, true, Bt);
    __syncthreads();
    tile_gemm<HD, false>(As, B, Bt, Ds);
    __syncthreads();
    for (int e = threadIdx.x; e < TILE * HD; e += NT) D1[e] = Ds[e / HD][e % HD];
    __syncthreads();
    tile_gemm<HD, true, true>(As, B, Bt, Ds);
    __syncthreads();
    for (int e = threadIdx.x; e < TILE * HD; e += NT) D2[e] = Ds[e / HD][e % HD];
}

// out[e] = sum over the `parts` partial arrays (stride `stride`) of part[k][e], one wavefront
// per output: lane l sums parts l, l + 64, ... in order, then a fixed shuffle tree (the same
// order in every run).
template <typename T>
__global__ __launch_bounds__(64) void reduce_parts_kernel(const T* __restrict__ part, int parts, int64_t stride,
                                                          float* __restrict__ out) {
    const int64_t e = blockIdx.x;
    double s = 0.0;
    for (int k = threadIdx.x; k < parts; k += 64) s += static_cast<double>(part[k * stride + e]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (threadIdx.x == 0) out[e] = static_cast<float>(s);
}

template <typename T>
void reduce_parts(const T* part, int parts, int64_t stride, int64_t count, float* out, hipStream_t st) {
    if (count > 0) reduce_parts_kernel<T><<<static_cast<unsigned>(count), 64, 0, st>>>(part, parts, stride, out);
}

// ------------------------------------------------------------------------------------------
// Adam
// ------------------------------------------------------------------------------------------
constexpr int kAdamBlocks = 256;

__global__ __launch_bounds__(kAdamThreads) void sumsq_kernel(const float* __restrict__ g, int64_t n,
                                                             double* __restrict__ part) {
    constexpr int NT = kAdamThreads;
    __shared__ double red[NT];
    double s = 0.0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x; i < n; i += static_cast<int64_t>(gridDim.x) * NT)
        s += static_cast<double>(g[i]) * g[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void clipcoef_kernel(const double* __restrict__ part, float clip, double* __restrict__ scal,
                                float* __restrict__ gnorm_out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int k = 0; k < kAdamBlocks; ++k) s += part[k];
    const double nrm = sqrt(s);
    double coef = 1.0;
    if (clip > 0.0f) {
        coef = static_cast<double>(clip) / (nrm + 1e-6);
        if (coef > 1.0) coef = 1.0;
    }
    scal[0] = coef;
    scal[1] = nrm;
    if (gnorm_out) gnorm_out[0] = static_cast<float>(nrm);
}

__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float bc1,
                            float bc2, const double* __restrict__ scal) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = static_cast<float>(g[i] * scal[0]);
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

inline dim3 grid_of(int64_t n, int block) { return dim3(static_cast<unsigned>((n + block - 1) / block)); }

}  // namespace

// ------------------------------------------------------------------------------------------
// batch object
// ------------------------------------------------------------------------------------------
struct gcin_batch {
    int G = 0;
    int64_t N = 0, E = 0;
    int ntiles = 0;
    std::vector<int32_t> goff, gend, gtile, gn;
    std::vector<int32_t> cbound, gchunk;  // chunk tile bounds [nchunks + 1], graph chunk bounds [G + 1]
    int nchunks = 0;
    // device
    int32_t *d_gend = nullptr, *d_gtile = nullptr, *d_tile_graph = nullptr;
    int32_t *d_cbound = nullptr, *d_gchunk = nullptr;
    double* cbuf = nullptr;  // chunk partial sums (up to 4 HD doubles per chunk)
    float* cmax = nullptr;
    int32_t* carg = nullptr;
    float* d_gcnt = nullptr;
    int32_t *ptr = nullptr, *col = nullptr;
    float *w = nullptr, *x0 = nullptr, *H0 = nullptr;
    unsigned short* wbf = nullptr;  // bf16 hi / lo parts of the weights of layers 1 .. NL-1
    float* Y[NL] = {};
    float* H[NL] = {};
    double* tstat = nullptr;
    float* mu[NL] = {};
    float* rstd[NL] = {};
    double* tpsum = nullptr;
    float* tpmax = nullptr;
    int32_t* tparg = nullptr;
    float* pooled = nullptr;
    int32_t* argmax = nullptr;
    HeadSave hs{};
    float *dpooled = nullptr, *ghead = nullptr, *dxh = nullptr, *dHa = nullptr, *dHb = nullptr;
    double* tb = nullptr;
    float* gmean = nullptr;
    double* ggb = nullptr;
    float* wpart = nullptr;
    double* bpart = nullptr;
    int64_t ghstride = 0;
    int last_degree = -1;
    int hd = 64;         // hidden width
    bool infer = false;  // forward only: no activations kept for a backward (GCIN_INFERENCE)
};

namespace {

struct Carve {
    uintptr_t base;
    size_t off = 0;
    template <class T>
    T* take(size_t count) {
        off = (off + 255) & ~static_cast<size_t>(255);
        T* p = reinterpret_cast<T*>(base + off);
        off += (count ? count : 1) * sizeof(T);
        return p;
    }
};

size_t layout_batch(gcin_batch* b, uintptr_t base) {
    Carve cv{base};
    const size_t G = b->G, N = b->N, E = b->E, T = b->ntiles, HD = b->hd;
    b->d_gend = cv.take<int32_t>(G);
    b->d_gtile = cv.take<int32_t>(G + 1);
    b->d_tile_graph = cv.take<int32_t>(T);
    b->d_gcnt = cv.take<float>(G);
    b->d_cbound = cv.take<int32_t>(static_cast<size_t>(b->nchunks) + 1);
    b->d_gchunk = cv.take<int32_t>(G + 1);
    b->cbuf = cv.take<double>(static_cast<size_t>(b->nchunks) * 4 * HD);
    b->cmax = cv.take<float>(static_cast<size_t>(b->nchunks) * HD);
    b->carg = cv.take<int32_t>(static_cast<size_t>(b->nchunks) * HD);
    b->ptr = cv.take<int32_t>(N + 1);
    b->col = cv.take<int32_t>(E);
    b->w = cv.take<float>(E);
    b->x0 = cv.take<float>(2 * N);
    b->H0 = cv.take<float>(2 * N);
    for (int l = 0; l < NL; ++l) {
        // forward only: a layer reads the layer below and its pooling reads the layer itself, so
        // two activation buffers in turn suffice (layers 1, 2, then 3 in layer 1's) and the
        // aggregates are not kept
        // layer 0's output is formed from H0 where needed and never stored
        b->Y[l] = l == 0 ? nullptr : b->infer && l >= 3 ? b->Y[l - 2] : cv.take<float>(N * HD);
        b->H[l] = l == 0 || b->infer ? nullptr : cv.take<float>(N * HD);
        b->mu[l] = cv.take<float>(G * HD);
        b->rstd[l] = cv.take<float>(G * HD);
    }
    b->tstat = cv.take<double>(T * 2 * HD);
    b->tpsum = cv.take<double>(T * HD);
    b->tpmax = cv.take<float>(T * HD);
    b->tparg = cv.take<int32_t>(T * HD);
    b->pooled = cv.take<float>(G * NL * 2 * HD);
    b->argmax = cv.take<int32_t>(G * NL * HD);
    b->hs.z = cv.take<float>(G * JK);
    b->hs.ln = cv.take<float>(G * 2);
    b->hs.s = cv.take<float>(G * JK);
    b->hs.a1 = cv.take<float>(G * M1);
    b->hs.a2 = cv.take<float>(G * M2);
    b->wbf = cv.take<unsigned short>(static_cast<size_t>(NL - 1) * 2 * HD * HD);
    if (b->infer) return (cv.off + 255) & ~static_cast<size_t>(255);  // no backward buffers
    b->dpooled = cv.take<float>(G * NL * 2 * HD);
    const Offs o4 = offsets(AMGG_MAX_DEGREE, b->hd);
    b->ghstride = ((o4.total - o4.head0) + 63) / 64 * 64;
    b->ghead = cv.take<float>(G * b->ghstride);
    b->dxh = cv.take<float>(N * HD);
    b->dHa = cv.take<float>(N * HD);
    b->dHb = cv.take<float>(N * HD);
    b->tb = cv.take<double>(T * 4 * HD);
    b->gmean = cv.take<float>(G * 2 * HD);
    b->ggb = cv.take<double>(G * 2 * HD);
    b->wpart = cv.take<float>(static_cast<size_t>(kWBlocks) * HD * HD);
    b->bpart = cv.take<double>(static_cast<size_t>(kWBlocks) * HD);
    return (cv.off + 255) & ~static_cast<size_t>(255);
}

int plan_batch(gcin_batch* b, int ngraphs, const int32_t* n, const int32_t* nnz) {
    if (ngraphs < 1 || ngraphs > GCIN_MAX_GRAPHS) return amgg::fail(AMGG_EINVAL, "gcin: ngraphs out of range");
    b->G = ngraphs;
    b->goff.assign(ngraphs + 1, 0);
    b->gend.assign(ngraphs, 0);
    b->gtile.assign(ngraphs + 1, 0);
    b->gn.assign(ngraphs, 0);
    int64_t rows = 0, edges = 0;
    for (int g = 0; g < ngraphs; ++g) {
        if (n[g] < 1 || nnz[g] < n[g]) return amgg::fail(AMGG_EINVAL, "gcin: a graph has n < 1 or nnz < n");
        b->goff[g] = static_cast<int32_t>(rows);
        b->gend[g] = static_cast<int32_t>(rows + n[g]);
        b->gtile[g] = static_cast<int32_t>(rows / TILE);
        b->gn[g] = n[g];
        rows += (static_cast<int64_t>(n[g]) + TILE - 1) / TILE * TILE;
        edges += nnz[g];
        if (rows > INT32_MAX / 2 || edges > INT32_MAX / 2) return amgg::fail(AMGG_EINVAL, "gcin: batch too large");
    }
    b->goff[ngraphs] = static_cast<int32_t>(rows);
    b->gtile[ngraphs] = static_cast<int32_t>(rows / TILE);
    b->cbound.clear();
    b->gchunk.assign(ngraphs + 1, 0);
    for (int g = 0; g < ngraphs; ++g) {
        b->gchunk[g] = static_cast<int32_t>(b->cbound.size());
        for (int32_t t = b->gtile[g]; t < b->gtile[g + 1]; t += kChunkTiles) b->cbound.push_back(t);
    }
    b->gchunk[ngraphs] = static_cast<int32_t>(b->cbound.size());
    b->nchunks = static_cast<int>(b->cbound.size());
    b->cbound.push_back(b->gtile[ngraphs]);
    b->N = rows;
    b->E = edges;
    b->ntiles = static_cast<int>(rows / TILE);
    return AMGG_OK;
}

int hip_err(hipError_t e, const char* where) {
    return amgg::fail(AMGG_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

}  // namespace

static bool hidden_ok(int hidden) { return hidden == 64 || hidden == 32; }

extern "C" int64_t gcin_param_count_hidden(int degree, int hidden) {
    if (degree < 1 || degree > AMGG_MAX_DEGREE || !hidden_ok(hidden)) return -1;
    return offsets(degree, hidden).total;
}

extern "C" int64_t gcin_param_count(int degree) { return gcin_param_count_hidden(degree, 64); }

extern "C" int gcin_batch_workspace_bytes_ex(int hidden, int flags, int ngraphs, const int32_t* n, const int32_t* nnz,
                                             size_t* bytes) {
    return amgg::guarded([&]() -> int {
        if (!n || !nnz || !bytes) return amgg::fail(AMGG_EINVAL, "gcin_batch_workspace_bytes: null argument");
        if (!hidden_ok(hidden)) return amgg::fail(AMGG_EINVAL, "gcin_batch_workspace_bytes: hidden must be 64 or 32");
        if (flags & ~GCIN_INFERENCE) return amgg::fail(AMGG_EINVAL, "gcin_batch_workspace_bytes: unknown flag");
        gcin_batch b;
        b.hd = hidden;
        b.infer = (flags & GCIN_INFERENCE) != 0;
        int rc = plan_batch(&b, ngraphs, n, nnz);
        if (rc) return rc;
        *bytes = layout_batch(&b, 0);
        return AMGG_OK;
    });
}

extern "C" int gcin_batch_workspace_bytes_hidden(int hidden, int ngraphs, const int32_t* n, const int32_t* nnz,
                                                 size_t* bytes) {
    return gcin_batch_workspace_bytes_ex(hidden, 0, ngraphs, n, nnz, bytes);
}

extern "C" int gcin_batch_workspace_bytes(int ngraphs, const int32_t* n, const int32_t* nnz, size_t* bytes) {
    return gcin_batch_workspace_bytes_hidden(64, ngraphs, n, nnz, bytes);
}

extern "C" int gcin_batch_create_ex(int hidden, int flags, int ngraphs, const gcin_graph* graphs, void* workspace,
                                    size_t ws_bytes, void* stream, gcin_batch** out) {
    return amgg::guarded([&]() -> int {
        if (!hidden_ok(hidden)) return amgg::fail(AMGG_EINVAL, "gcin_batch_create: hidden must be 64 or 32");
        if (flags & ~GCIN_INFERENCE) return amgg::fail(AMGG_EINVAL, "gcin_batch_create: unknown flag");
        if (!graphs || !out || !workspace) return amgg::fail(AMGG_EINVAL, "gcin_batch_create: null argument");
        if (reinterpret_cast<uintptr_t>(workspace) & 255u)
            return amgg::fail(AMGG_EWORKSPACE, "gcin_batch_create: workspace not 256-byte aligned");
        if (ngraphs < 1 || ngraphs > GCIN_MAX_GRAPHS) return amgg::fail(AMGG_EINVAL, "gcin_batch_create: ngraphs out of range");
        std::vector<int32_t> n(ngraphs), z(ngraphs);
        for (int g = 0; g < ngraphs; ++g) {
            n[g] = graphs[g].n;
            z[g] = graphs[g].nnz;
            if (!graphs[g].rowptr || !graphs[g].col || !graphs[g].val)
                return amgg::fail(AMGG_EINVAL, "gcin_batch_create: null graph array");
        }
        auto* b = new gcin_batch();
        b->hd = hidden;
        b->infer = (flags & GCIN_INFERENCE) != 0;
        int rc = plan_batch(b, ngraphs, n.data(), z.data());
        if (rc) {
            delete b;
            return rc;
        }
        const size_t need = layout_batch(b, 0);
        if (ws_bytes < need) {
            delete b;
            return amgg::fail(AMGG_EWORKSPACE, "gcin_batch_create: workspace too small");
        }
        layout_batch(b, reinterpret_cast<uintptr_t>(workspace));
        hipStream_t st = static_cast<hipStream_t>(stream);
        // tables
        std::vector<int32_t> tile_graph(b->ntiles);
        std::vector<float> cnt(ngraphs);
        for (int g = 0; g < ngraphs; ++g) {
            for (int t = b->gtile[g]; t < b->gtile[g + 1]; ++t) tile_graph[t] = g;
            cnt[g] = static_cast<float>(b->gn[g]);
        }
        hipError_t e = hipMemcpyAsync(b->d_gend, b->gend.data(), sizeof(int32_t) * ngraphs, hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(b->d_gtile, b->gtile.data(), sizeof(int32_t) * (ngraphs + 1), hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(b->d_tile_graph, tile_graph.data(), sizeof(int32_t) * b->ntiles, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(b->d_gcnt, cnt.data(), sizeof(float) * ngraphs, hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(b->d_cbound, b->cbound.data(), sizeof(int32_t) * b->cbound.size(), hipMemcpyHostToDevice,
                               st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(b->d_gchunk, b->gchunk.data(), sizeof(int32_t) * b->gchunk.size(), hipMemcpyHostToDevice,
                               st);
        int64_t e0 = 0;
        for (int g = 0; g < ngraphs && e == hipSuccess; ++g) {
            fill_graph_kernel<<<grid_of(n[g], 256), 256, 0, st>>>(n[g], graphs[g].rowptr, graphs[g].col, graphs[g].val,
                                                                 b->goff[g], static_cast<int32_t>(e0), b->ptr, b->col,
                                                                 b->w, b->x0);
            const int32_t from = b->gend[g], to = b->goff[g + 1];
            e0 += z[g];
            if (to > from)
                pad_rows_kernel<<<grid_of(to - from, 256), 256, 0, st>>>(from, to, static_cast<int32_t>(e0), b->ptr, b->x0);
            e = hipGetLastError();
        }
        if (e == hipSuccess) {
            set_int_kernel<<<1, 1, 0, st>>>(b->ptr + b->N, static_cast<int32_t>(b->E));
            e = hipGetLastError();
        }
        // the host tables above must stay alive until the copies complete
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            delete b;
            return hip_err(e, "gcin_batch_create");
        }
        *out = b;
        return AMGG_OK;
    });
}

extern "C" int gcin_batch_create_hidden(int hidden, int ngraphs, const gcin_graph* graphs, void* workspace,
                                        size_t ws_bytes, void* stream, gcin_batch** out) {
    return gcin_batch_create_ex(hidden, 0, ngraphs, graphs, workspace, ws_bytes, stream, out);
}

extern "C" int gcin_batch_create(int ngraphs, const gcin_graph* graphs, void* workspace, size_t ws_bytes, void* stream,
                                 gcin_batch** out) {
    return gcin_batch_create_hidden(64, ngraphs, graphs, workspace, ws_bytes, stream, out);
}

extern "C" int gcin_batch_destroy(gcin_batch* b) {
    delete b;
    return AMGG_OK;
}

namespace {

// The tile products run on MFMA for 64 channels; the 32-channel variant keeps them in FP32.
template <int HD>
void forward_impl(gcin_batch* b, int degree, int precision, const float* P, float* coeffs_out, hipStream_t st) {
    constexpr int NT = 4 * HD;
    const Offs o = offsets(degree, HD);
    const int T = b->ntiles, G = b->G;
    const float *W0 = P + o.convW[0], *b0 = P + o.convb[0];
    layer0_kernel<HD><<<T, NT, 0, st>>>(b->ptr, b->col, b->w, b->x0, b->d_tile_graph, b->d_gend, W0, b0, b->H0,
                                        b->tstat);
    const int C = b->nchunks;
    // Statistics of layer l, then its readout, which feeds no later layer: pooling each layer as
    // soon as its statistics exist leaves every result as it is and lets an inference-only batch
    // reuse the buffer of layer l - 1 for layer l + 1. The readout partials of layer l are formed
    // by the kernel of layer l + 1 (from the rows' own entries of A_hat), the last layer's by a
    // pooling pass; the per-graph reductions follow.
    auto stats = [&](int l) {
        chunk_sum_kernel<HD, 2><<<C, NT, 0, st>>>(b->tstat, b->d_cbound, b->cbuf);
        stats_final_kernel<HD><<<G, NT, 0, st>>>(b->cbuf, b->d_gchunk, b->d_gcnt, b->mu[l], b->rstd[l]);
    };
    auto pool_tiles = [&](int l) {
        (l == 0 ? pool_tile_kernel<HD, true> : pool_tile_kernel<HD, false>)<<<T, NT, 0, st>>>(
            b->d_tile_graph, b->d_gend, b->Y[l], b->H0, W0, b0, b->mu[l], b->rstd[l], P + o.gam[l], P + o.bet[l],
            b->tpsum, b->tpmax, b->tparg);
    };
    auto pool_graphs = [&](int l) {
        pool_chunk_kernel<HD><<<C, NT, 0, st>>>(b->tpsum, b->tpmax, b->tparg, b->d_cbound, b->cbuf, b->cmax, b->carg);
        pool_final_kernel<HD><<<G, NT, 0, st>>>(b->cbuf, b->cmax, b->carg, b->d_gchunk, b->d_gcnt, l, b->pooled,
                                                b->argmax);
    };
    stats(0);
    const bool mfma = HD == 64 && precision != GCIN_FP32;
    if (mfma) weights_bf16_kernel<HD><<<NL - 1, 256, 0, st>>>(P, o, b->wbf);
    for (int l = 1; l < NL; ++l) {
        const bool y0 = l == 1;
        auto kern = y0 ? layer_kernel<HD, false, false, true> : layer_kernel<HD, false, false, false>;
        if constexpr (HD == 64) {
            if (precision == GCIN_BF16X3)
                kern = y0 ? layer_kernel<HD, true, true, true> : layer_kernel<HD, true, true, false>;
            else if (precision == GCIN_BF16)
                kern = y0 ? layer_kernel<HD, true, false, true> : layer_kernel<HD, true, false, false>;
        }
        kern<<<T, NT, 0, st>>>(b->ptr, b->col, b->w, b->d_tile_graph, b->d_gend, b->Y[l - 1], b->H0, W0, b0,
                               b->mu[l - 1], b->rstd[l - 1], P + o.gam[l - 1], P + o.bet[l - 1], P + o.convW[l],
                               P + o.convb[l], b->wbf + static_cast<int64_t>(l - 1) * 2 * HD * HD, b->H[l], b->Y[l],
                               b->tstat, b->tpsum, b->tpmax, b->tparg);
        pool_graphs(l - 1);
        stats(l);
    }
    pool_tiles(NL - 1);
    pool_graphs(NL - 1);
    head_fwd_kernel<HD><<<G, 128, 0, st>>>(P, o, b->pooled, b->hs, coeffs_out);
}

template <int HD>
void backward_impl(gcin_batch* b, int degree, int precision, const float* P, const float* dcoeffs, float* grads,
                   hipStream_t st) {
    constexpr int NT = 4 * HD;
    const Offs o = offsets(degree, HD);
    const int T = b->ntiles, G = b->G;
    head_bwd_kernel<HD><<<G, 128, 0, st>>>(P, o, b->pooled, b->hs, dcoeffs, b->ghead, b->ghstride, b->dpooled);
    // head parameters: sum over graphs
    const int64_t nhead = o.total - o.head0;
    reduce_parts<float>(b->ghead, G, b->ghstride, nhead, grads + o.head0, st);
    float* dHn = nullptr;  // dH of the layer above (for the aggregation backward)
    float* bufs[2] = {b->dHa, b->dHb};
    for (int l = NL - 1; l >= 0; --l) {
        const float *W0 = P + o.convW[0], *b0 = P + o.convb[0];
        (l == 0 ? bwd_a_kernel<HD, true> : bwd_a_kernel<HD, false>)<<<T, NT, 0, st>>>(
            b->ptr, b->col, b->w, b->d_tile_graph, b->d_gend, b->d_gcnt, b->Y[l], b->H0, W0, b0, b->mu[l], b->rstd[l],
            P + o.gam[l], P + o.bet[l], b->dpooled, b->argmax, l, dHn, b->dxh, b->tb);
        chunk_sum_kernel<HD, 4><<<b->nchunks, NT, 0, st>>>(b->tb, b->d_cbound, b->cbuf);
        bwd_final_kernel<HD><<<G, NT, 0, st>>>(b->cbuf, b->d_gchunk, b->d_gcnt, b->gmean, b->ggb);
        // gamma / beta of this layer
        reduce_parts<double>(b->ggb, G, 2 * HD, HD, grads + o.gam[l], st);
        reduce_parts<double>(b->ggb + HD, G, 2 * HD, HD, grads + o.bet[l], st);
        float* dHout = l > 0 ? bufs[l & 1] : nullptr;
        const int in_dim = l == 0 ? 2 : HD;
        const float* Hin = l == 0 ? b->H0 : b->H[l];
        const int grid = T < kWBlocks ? T : kWBlocks;
        auto kern = l == 0 ? bwd_b_kernel<HD, false, true> : bwd_b_kernel<HD, false, false>;
        if constexpr (HD == 64)
            if (precision != GCIN_FP32) kern = l == 0 ? bwd_b_kernel<HD, true, true> : bwd_b_kernel<HD, true, false>;
        kern<<<grid, NT, 0, st>>>(T, b->d_tile_graph, b->d_gend, b->Y[l], b->H0, W0, b0, b->mu[l], b->rstd[l],
                                  b->gmean, b->dxh, Hin, in_dim, P + o.convW[l], dHout, b->wpart, b->bpart);
        reduce_parts<float>(b->wpart, grid, HD * HD, in_dim * HD, grads + o.convW[l], st);
        reduce_parts<double>(b->bpart, grid, HD, HD, grads + o.convb[l], st);
        dHn = dHout;
    }
}

}  // namespace

extern "C" int gcin_forward(gcin_batch* b, int degree, int precision, const float* P, float* coeffs_out, void* stream) {
    return amgg::guarded([&]() -> int {
        if (!b || !P || !coeffs_out) return amgg::fail(AMGG_EINVAL, "gcin_forward: null argument");
        if (degree < 1 || degree > AMGG_MAX_DEGREE) return amgg::fail(AMGG_EINVAL, "gcin_forward: degree out of range");
        if (precision < GCIN_FP32 || precision > GCIN_BF16X3) return amgg::fail(AMGG_EINVAL, "gcin_forward: bad precision");
        hipStream_t st = static_cast<hipStream_t>(stream);
        if (b->hd == 32)
            forward_impl<32>(b, degree, precision, P, coeffs_out, st);
        else
            forward_impl<64>(b, degree, precision, P, coeffs_out, st);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_err(e, "gcin_forward");
        b->last_degree = degree;
        return AMGG_OK;
    });
}

extern "C" int gcin_backward(gcin_batch* b, int degree, int precision, const float* P, const float* dcoeffs,
                             float* grads, void* stream) {
    return amgg::guarded([&]() -> int {
        if (!b || !P || !dcoeffs || !grads) return amgg::fail(AMGG_EINVAL, "gcin_backward: null argument");
        if (b->infer) return amgg::fail(AMGG_ESTATE, "gcin_backward: the batch was created for inference only");
        if (degree != b->last_degree) return amgg::fail(AMGG_ESTATE, "gcin_backward: no forward pass of this degree");
        if (precision < GCIN_FP32 || precision > GCIN_BF16X3) return amgg::fail(AMGG_EINVAL, "gcin_backward: bad precision");
        hipStream_t st = static_cast<hipStream_t>(stream);
        if (b->hd == 32)
            backward_impl<32>(b, degree, precision, P, dcoeffs, grads, st);
        else
            backward_impl<64>(b, degree, precision, P, dcoeffs, grads, st);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_err(e, "gcin_backward");
        return AMGG_OK;
    });
}

extern "C" int gcin_tile_gemm_check(const float* A, const float* B, float* D_fp32, float* D_bf16, void* stream) {
    if (!A || !B || !D_fp32 || !D_bf16) return amgg::fail(AMGG_EINVAL, "gcin_tile_gemm_check: null argument");
    tile_gemm_check_kernel<<<1, 256, 0, static_cast<hipStream_t>(stream)>>>(A, B, D_fp32, D_bf16);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_err(e, "gcin_tile_gemm_check");
    return AMGG_OK;
}

constexpr size_t kAdamScratchDoubles = kAdamBlocks + 8;  // partial sums of ||g||^2, then the clip scalars

extern "C" size_t adam_scratch_bytes(void) { return sizeof(double) * kAdamScratchDoubles; }

namespace {
// The three launches of one Adam step; `work` holds kAdamScratchDoubles doubles of device memory.
// Every entry of `work` that is read was written earlier in the same step (each partial by its
// workgroup, the scalars by the one-thread kernel), so it needs no clearing between calls.
hipError_t adam_launch(float* params, const float* grads, float* m, float* v, int64_t n, float lr, float b1,
                       float b2, float eps, int step, float clip, float* gnorm_out, double* work, hipStream_t st) {
    double* part = work;
    double* scal = part + kAdamBlocks;
    sumsq_kernel<<<kAdamBlocks, kAdamThreads, 0, st>>>(grads, n, part);
    clipcoef_kernel<<<1, 1, 0, st>>>(part, clip, scal, gnorm_out);
    const float bc1 = 1.0f - std::pow(b1, static_cast<float>(step));
    const float bc2 = 1.0f - std::pow(b2, static_cast<float>(step));
    adam_kernel<<<grid_of(n, 256), 256, 0, st>>>(params, grads, m, v, n, lr, b1, b2, eps, bc1, bc2, scal);
    return hipGetLastError();
}

bool adam_args_ok(const float* params, const float* grads, const float* m, const float* v, int64_t n, int step) {
    return params && grads && m && v && n > 0 && step >= 1;
}
}  // namespace

extern "C" int adam_step(float* params, const float* grads, float* m, float* v, int64_t n, float lr, float b1, float b2,
                         float eps, int step, float clip, float* gnorm_out, void* workspace, void* stream) {
    return amgg::guarded([&]() -> int {
        if (!adam_args_ok(params, grads, m, v, n, step) || !workspace)
            return amgg::fail(AMGG_EINVAL, "adam_step: bad argument");
        const hipError_t e = adam_launch(params, grads, m, v, n, lr, b1, b2, eps, step, clip, gnorm_out,
                                         static_cast<double*>(workspace), static_cast<hipStream_t>(stream));
        if (e != hipSuccess) return hip_err(e, "adam_step");
        return AMGG_OK;
    });
}

// ------------------------------------------------------------------------------------------
// Adam step without any allocation: the step's scratch (kAdamScratchDoubles doubles) is this
// file-scope device array, one copy per GPU, held until the process ends. Host code never
// passes `scratch` itself to a kernel (on the host it names a stand-in, not device memory):
// it uses the address hipGetSymbolAddress returns on each device, looked up once per device.
// ------------------------------------------------------------------------------------------
static __device__ __align__(256) double scratch[kAdamScratchDoubles];
static_assert(sizeof(scratch) == sizeof(double) * kAdamScratchDoubles, "one Adam step's scratch, whatever n");

namespace {
std::mutex g_scratch_mu;
double* g_scratch_ptr[64] = {};  // per device ordinal: the address of `scratch` on that device

// Address of `scratch` on `device`, looked up on the first call for that device with the device
// current (the caller's current device is restored afterwards).
hipError_t scratch_on(int device, double** out) {
    if (device < 0 || device >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int prev = -1;
        hipError_t e = hipGetDevice(&prev);
        if (e == hipSuccess && prev != device) e = hipSetDevice(device);
        void* p = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (prev >= 0 && prev != device) {
            const hipError_t e2 = hipSetDevice(prev);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}
}  // namespace

extern "C" int adam_step_noalloc(float* params, const float* grads, float* m, float* v, int64_t n, float lr,
                                 float b1, float b2, float eps, int step, float clip, float* gnorm_out,
                                 void* stream) {
    return amgg::guarded([&]() -> int {
        if (!adam_args_ok(params, grads, m, v, n, step)) return amgg::fail(AMGG_EINVAL, "adam_step_noalloc: bad argument");
        const hipStream_t st = static_cast<hipStream_t>(stream);
        int device = -1;
        hipError_t e = st ? hipStreamGetDevice(st, &device) : hipGetDevice(&device);
        double* work = nullptr;
        if (e == hipSuccess) e = scratch_on(device, &work);
        if (e == hipSuccess) e = adam_launch(params, grads, m, v, n, lr, b1, b2, eps, step, clip, gnorm_out, work, st);
        if (e != hipSuccess) return hip_err(e, "adam_step_noalloc");
        return AMGG_OK;
    });
}
