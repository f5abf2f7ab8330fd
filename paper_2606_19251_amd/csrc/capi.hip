// C interface of the solver: context and workspace management, hierarchy load, smoother
// assembly, the V-cycle (paper Sec. 2.2; Alg. 1, step 9) and the outer FP64 loops.
// Host code here only sequences kernels on the caller's stream; every arithmetic step of
// the solve runs in the kernels of k_*.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "amggnn.h"
#include "ctx.hpp"
#include "errors.hpp"
#include "halo.hpp"
#include "kernels.hpp"

using namespace amgg;

namespace amgg {

int hip_fail(hipError_t e, const char* where) {
    return fail(AMGG_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

namespace {

struct Bump {
    uintptr_t base;
    size_t off = 0;
    template <class T>
    T* take(size_t count) {
        off = (off + 255) & ~static_cast<size_t>(255);
        T* p = reinterpret_cast<T*>(base + off);
        off += std::max<size_t>(count, 1) * sizeof(T);
        return p;
    }
};

}  // namespace

// Carve the workspace; with base == 0 only the size is computed.
size_t layout(amgg_ctx* c, uintptr_t base) {
    Bump b{base};
    c->nblk = c->lv[0].nblk;
    int32_t max_nc = 1;
    int32_t max_chunks = 1;
    for (int l = 0; l < c->nlevels; ++l) {
        Level& L = c->lv[l];
        const size_t n = L.n, z = L.nnz;
        L.val32 = b.take<float>(z);
        L.q64 = b.take<double>(z);
        L.q32 = b.take<float>(z);
        L.diag = b.take<double>(n);
        L.qd64 = b.take<double>(n);
        L.qd32 = b.take<float>(n);
        L.scale = b.take<double>(1);
        L.u64 = b.take<double>(n);
        L.f64 = b.take<double>(n);
        L.r64 = b.take<double>(n);
        L.t64 = b.take<double>(n);
        L.u32 = b.take<float>(n);
        L.f32 = b.take<float>(n);
        L.r32 = b.take<float>(n);
        L.t32 = b.take<float>(n);
        // packed columns of A (Q shares them), and of P and R below
        auto take_pack = [&](Level::Pack& pk, int32_t rows_m, int32_t nz) {
            pk.rows = stream_rows_for(rows_m, nz);
            pk.nfar = -1;
            if (pk.rows <= 0 || nz <= 0) {
                pk.rows = 0;
                return;
            }
            const size_t nb = (static_cast<size_t>(rows_m) + pk.rows - 1) / pk.rows;
            pk.cap = static_cast<int64_t>(nz) / 8 + 64;  // beyond 1/8 of the entries far, plain columns
            pk.off = b.take<uint16_t>(nz);
            pk.base = b.take<int32_t>(nb);
            pk.foff = b.take<int32_t>(nb + 1);
            pk.fslot = b.take<uint16_t>(pk.cap);
            pk.fcol = b.take<int32_t>(pk.cap);
        };
        take_pack(L.pa, L.n, L.nnz);
        if (l + 1 < c->nlevels) {
            const size_t pz = L.pnnz;
            take_pack(L.pp, L.n, L.pnnz);
            take_pack(L.pr, L.nc, L.pnnz);
            L.pval32 = b.take<float>(pz);
            L.rptr = b.take<int32_t>(L.nc + 1);
            L.rcol = b.take<int32_t>(pz);
            L.rval = b.take<double>(pz);
            L.rval32 = b.take<float>(pz);
            max_nc = std::max(max_nc, L.nc);
            L.dense = L.inv = nullptr;
            L.piv = nullptr;
            const int rows = L.n <= kFuseMaxRows ? stream_rows_for(L.n, L.nnz) : 0;
            if (rows > 0) {
                const size_t nb = (n + rows - 1) / rows;
                L.hoff = b.take<int32_t>(nb + 1);
                L.halo = b.take<int32_t>(z);  // at most one halo row per stored entry
                L.hend = b.take<uint16_t>(z);
                L.heoff = b.take<int32_t>(nb + 1);
                // flat halo-entry arrays; levels whose halos hold more entries are not fused
                L.hent = b.take<int32_t>(z);
                L.hcol = b.take<int32_t>(z);
                L.ha64 = b.take<double>(z);
                L.ha32 = b.take<float>(z);
                L.hq64 = b.take<double>(z);
                L.hq32 = b.take<float>(z);
                L.hloc = b.take<uint16_t>(z);
            }
        } else if (L.nblk > 0) {
            const size_t dz = static_cast<size_t>(L.dense_off_h.back());
            L.dense = b.take<double>(dz);
            L.inv = b.take<double>(dz);
            L.piv = b.take<int32_t>(n);
            L.dense_off = b.take<int64_t>(L.nblk + 1);
        } else {
            L.dense = b.take<double>(n * n);
            L.inv = b.take<double>(n * n);
            L.piv = b.take<int32_t>(n);
        }
        if (L.nblk > 0) {
            L.blk_off = b.take<int32_t>(L.nblk + 1);
            L.blk_crow = b.take<int32_t>(L.nblk);
            L.blk_scale = b.take<double>(L.nblk);
            L.chunk_row = b.take<int32_t>(L.nchunk() + 1);
            L.blk_chunk = b.take<int32_t>(L.nblk + 1);
            max_chunks = std::max(max_chunks, L.nchunk());
        }
        for (int k = 0; k < kAdjVecs; ++k) {
            L.adj64[k] = b.take<double>(n);
            L.adj32[k] = b.take<float>(n);
        }
    }
    const size_t n0 = c->lv[0].n;
    c->scal = b.take<double>(kSlots);
    c->partial = b.take<double>(std::max(kReduceBlocks, outer_partials(c->lv[0].n, c->lv[0].nnz)));
    c->partial2 = b.take<double>(2 * kReduceBlocks);
    c->flags = b.take<int32_t>(8);
    c->cursor = b.take<int32_t>(max_nc + 1);
    c->pack_parts = b.take<int32_t>(kScanPartsMax + 1);
    c->blkmax = b.take<int32_t>(3 * AMGG_MAX_LEVELS);
    c->ra = b.take<double>(n0);
    c->rb = b.take<double>(n0);
    c->z = b.take<double>(n0);
    c->p = b.take<double>(n0);
    c->q = b.take<double>(n0);
    c->bproj = b.take<double>(n0);
    c->adj_partial = b.take<double>(static_cast<size_t>(2 * AMGG_MAX_DEGREE + 1) * kReduceBlocks);
    c->adj_scal = b.take<double>(64);
    c->adj_f32 = b.take<float>(n0);
    if (c->nblk > 0) {
        c->blk_scal = b.take<double>(4 * static_cast<size_t>(c->nblk));
        c->blk_partial = b.take<double>(static_cast<size_t>(kMaxCoef) * max_chunks);
    }
    return (b.off + 255) & ~static_cast<size_t>(255);
}

// ------------------------------------------------------------------------------------
// V-cycle
// ------------------------------------------------------------------------------------
template <typename T>
hipError_t coarse_solve(const Level& L, const T* f, T* u, hipStream_t st) {
    if (L.nblk > 0) return block_dense_gemv<T>(L.n, L.nblk, L.blk_off, L.dense_off, L.inv, f, u, st);
    return dense_gemv<T>(L.n, L.inv, f, u, st);
}
template hipError_t coarse_solve<float>(const Level&, const float*, float*, hipStream_t);
template hipError_t coarse_solve<double>(const Level&, const double*, double*, hipStream_t);

template <typename T>
hipError_t smooth_step(Level& L, const T* f, T*& cur, T*& oth, T* r, bool from_zero, hipStream_t st) {
    const CsrView A = L.A();
    hipError_t e;
    if (L.smoother == kSmootherDiagonal) {
        if (from_zero) return vec_mul<T>(L.n, L.qd<T>(), f, cur, st);
        e = csr_apply<T>(A, L.aval<T>(), cur, oth, f, L.qd<T>(), cur, Epi::Jacobi, st);
        std::swap(cur, oth);
        return e;
    }
    if (from_zero) return csr_apply<T>(A, L.qval<T>(), f, cur, nullptr, nullptr, nullptr, Epi::Store, st);
    if (L.fuse && L.hrows > 0) {
        e = smooth_post_fused<T>(A, L.H(), L.aval<T>(), L.hav<T>(), L.qval<T>(), f, cur, oth, st);
        std::swap(cur, oth);
        return e;
    }
    if ((e = csr_apply<T>(A, L.aval<T>(), cur, r, f, nullptr, nullptr, Epi::Resid, st)) != hipSuccess) return e;
    return csr_apply<T>(A, L.qval<T>(), r, cur, nullptr, nullptr, nullptr, Epi::Add, st);
}
template hipError_t smooth_step<float>(Level&, const float*, float*&, float*&, float*, bool, hipStream_t);
template hipError_t smooth_step<double>(Level&, const double*, double*&, double*&, double*, bool, hipStream_t);

bool takes_ready_u(const amgg_ctx* c, int l, int nu1) {
    if (l >= c->nlevels - 1 || nu1 < 1) return false;
    const Level& L = c->lv[l];
    return L.fuse && L.smoother == kSmootherDiagonal;
}

// u_ready (only with zero): u already holds qd f, the first diagonal smoothing step from zero,
// formed by the pass that produced f (the restriction or the outer loop's cast). The step after
// it then reads u like any other iterate: the same products and roundings as the fused kernel
// that forms d_j f_j per gathered entry, with one gathered vector instead of two.
template <typename T>
hipError_t vcycle_level(amgg_ctx* c, int l, const T* f, T* u, T* t, bool zero, int nu1, int nu2, hipStream_t st,
                        T** result, bool store, bool u_ready) {
    Level& L = c->lv[l];
    hipError_t e;
    if (l == c->nlevels - 1) {
        *result = u;
        return coarse_solve<T>(L, f, u, st);
    }
    if (u_ready && !(zero && takes_ready_u(c, l, nu1))) return hipErrorInvalidValue;
    T* cur = u;
    T* oth = t;
    T* r = L.r<T>();
    // The first pre-smoothing step from u = 0 is fused with the pass after it where the level
    // allows (same values, one kernel fewer): diagonal smoother u = d f with the residual (or
    // with the second step), sparse smoother u = Q f with the residual.
    int k0 = 0;
    bool have_r = false;
    if (u_ready) {
        if (nu1 == 1) {
            if ((e = csr_apply<T>(L.A(), L.aval<T>(), cur, r, f, nullptr, nullptr, Epi::Resid, st)) != hipSuccess)
                return e;
            have_r = true;
        } else {
            if ((e = csr_apply<T>(L.A(), L.aval<T>(), cur, oth, f, L.qd<T>(), cur, Epi::Jacobi, st)) != hipSuccess)
                return e;
            std::swap(cur, oth);
        }
        k0 = nu1 == 1 ? 1 : 2;
    } else if (zero && nu1 >= 1 && L.fuse) {
        if (L.smoother == kSmootherDiagonal) {
            if (nu1 == 1) {
                if ((e = jacobi_pre_resid<T>(L.A(), L.aval<T>(), L.qd<T>(), f, cur, r, st)) != hipSuccess) return e;
                have_r = true;
                k0 = 1;
            } else if (stream_rows_for(L.n, L.nnz) > 0) {
                if ((e = jacobi_pre_step<T>(L.A(), L.aval<T>(), L.qd<T>(), f, oth, st)) != hipSuccess) return e;
                std::swap(cur, oth);
                k0 = 2;
            }
        } else if (L.hrows > 0) {
            if ((e = smooth_pre_fused<T>(L.A(), L.H(), L.aval<T>(), L.qval<T>(), L.hqv<T>(), f, cur, r, st)) != hipSuccess)
                return e;
            have_r = nu1 == 1;
            k0 = 1;
        }
    }
    for (int k = k0; k < nu1; ++k)
        if ((e = smooth_step<T>(L, f, cur, oth, r, zero && k == 0, st)) != hipSuccess) return e;
    const bool still_zero = zero && nu1 == 0;
    const T* res = f;
    if (!still_zero && have_r) {
        res = r;
    } else if (!still_zero) {
        if ((e = csr_apply<T>(L.A(), L.aval<T>(), cur, r, f, nullptr, nullptr, Epi::Resid, st)) != hipSuccess)
            return e;
        res = r;
    }
    Level& C = c->lv[l + 1];
    // the restriction also forms the coarse level's first smoothing step where that is diagonal
    const bool ready = takes_ready_u(c, l + 1, nu1);
    if ((e = csr_apply<T>(L.R(), L.rv<T>(), res, C.f<T>(), nullptr, ready ? C.qd<T>() : nullptr, nullptr,
                          ready ? Epi::StoreScaled : Epi::Store, st, ready ? C.u<T>() : nullptr)) != hipSuccess)
        return e;
    T* ec = nullptr;
    if ((e = vcycle_level<T>(c, l + 1, C.f<T>(), C.u<T>(), C.t<T>(), true, nu1, nu2, st, &ec, store, ready)) !=
        hipSuccess)
        return e;
    if ((e = csr_apply<T>(L.P(), L.pv<T>(), ec, cur, nullptr, nullptr, nullptr, still_zero ? Epi::Store : Epi::Add,
                          st)) != hipSuccess)
        return e;
    // the adjoint recomputes post-smoothing from this iterate
    if (store && (e = vec_copy<T>(L.n, cur, L.adj<T>(kAdjUmid), st)) != hipSuccess) return e;
    for (int k = 0; k < nu2; ++k)
        if ((e = smooth_step<T>(L, f, cur, oth, r, false, st)) != hipSuccess) return e;
    *result = cur;
    return hipSuccess;
}

template hipError_t vcycle_level<float>(amgg_ctx*, int, const float*, float*, float*, bool, int, int, hipStream_t,
                                        float**, bool, bool);
template hipError_t vcycle_level<double>(amgg_ctx*, int, const double*, double*, double*, bool, int, int,
                                         hipStream_t, double**, bool, bool);

int check_ready(const amgg_ctx* c, const char* where) {
    if (!c) return fail(AMGG_EINVAL, std::string(where) + ": null context");
    if (!c->finalized) return fail(AMGG_ESTATE, std::string(where) + ": hierarchy not finalized");
    for (int l = 0; l + 1 < c->nlevels; ++l)
        if (c->lv[l].smoother == kSmootherNone)
            return fail(AMGG_ESTATE, std::string(where) + ": smoother of level " + std::to_string(l) + " not set");
    return AMGG_OK;
}

}  // namespace amgg

// ------------------------------------------------------------------------------------
// Context and hierarchy
// ------------------------------------------------------------------------------------
extern "C" int amgg_create(amgg_ctx** out, int device, int nlevels) {
    return guarded([&]() -> int {
        if (!out) return fail(AMGG_EINVAL, "amgg_create: null output");
        if (nlevels < 1 || nlevels > AMGG_MAX_LEVELS) return fail(AMGG_EINVAL, "amgg_create: nlevels out of range");
        int count = 0;
        hipError_t e = hipGetDeviceCount(&count);
        if (e != hipSuccess) return hip_fail(e, "amgg_create");
        if (device < 0 || device >= count) return fail(AMGG_EINVAL, "amgg_create: no such device");
        auto* c = new amgg_ctx();
        c->device = device;
        c->nlevels = nlevels;
        if ((e = hipSetDevice(device)) == hipSuccess &&
            (e = hipHostMalloc(&c->host_scal, sizeof(double) * kSlots * (1 + kPipeline))) == hipSuccess &&
            (e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking)) == hipSuccess)
            for (hipEvent_t& ev : c->ev)
                if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) break;
        if (e != hipSuccess) {
            for (hipEvent_t ev : c->ev)
                if (ev) (void)hipEventDestroy(ev);
            if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
            if (c->host_scal) (void)hipHostFree(c->host_scal);
            delete c;
            return hip_fail(e, "amgg_create");
        }
        *out = c;
        return AMGG_OK;
    });
}

static void drop_graphs(amgg_ctx* c) {
    for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.exec);
    c->graphs.clear();
}

extern "C" int amgg_destroy(amgg_ctx* c) {
    if (!c) return AMGG_OK;
    drop_graphs(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (hipEvent_t ev : c->ev)
        if (ev) (void)hipEventDestroy(ev);
    if (c->host_scal) (void)hipHostFree(c->host_scal);
    delete c;
    return AMGG_OK;
}

extern "C" int amgg_load_level(amgg_ctx* c, int lvl, int32_t n, int32_t nnz, const int32_t* rowptr,
                               const int32_t* col, const double* val) {
    if (!c || lvl < 0 || lvl >= c->nlevels) return fail(AMGG_EINVAL, "amgg_load_level: bad context or level");
    if (n <= 0 || nnz < n || !rowptr || !col || !val) return fail(AMGG_EINVAL, "amgg_load_level: bad sizes or null array");
    Level& L = c->lv[lvl];
    L.n = n;
    L.nnz = nnz;
    L.ptr = rowptr;
    L.col = col;
    L.val = val;
    L.loaded = true;
    c->finalized = false;
    return AMGG_OK;
}

extern "C" int amgg_load_prolong(amgg_ctx* c, int lvl, int32_t n_f, int32_t n_c, int32_t nnz,
                                 const int32_t* rowptr, const int32_t* col, const double* val) {
    if (!c || lvl < 0 || lvl + 1 >= c->nlevels) return fail(AMGG_EINVAL, "amgg_load_prolong: bad context or level");
    if (n_f <= 0 || n_c <= 0 || nnz < 0 || !rowptr || (nnz > 0 && (!col || !val)))
        return fail(AMGG_EINVAL, "amgg_load_prolong: bad sizes or null array");
    Level& L = c->lv[lvl];
    L.pn_f = n_f;
    L.nc = n_c;
    L.pnnz = nnz;
    L.pptr = rowptr;
    L.pcol = col;
    L.pval = val;
    L.p_loaded = true;
    c->finalized = false;
    return AMGG_OK;
}

static int check_loaded(const amgg_ctx* c, const char* where) {
    for (int l = 0; l < c->nlevels; ++l) {
        const Level& L = c->lv[l];
        if (!L.loaded) return fail(AMGG_ESTATE, std::string(where) + ": level " + std::to_string(l) + " not loaded");
        if (l + 1 < c->nlevels) {
            if (!L.p_loaded)
                return fail(AMGG_ESTATE, std::string(where) + ": prolongation " + std::to_string(l) + " not loaded");
            if (L.pn_f != L.n || L.nc != c->lv[l + 1].n)
                return fail(AMGG_EINVAL, std::string(where) + ": prolongation " + std::to_string(l) +
                                             " does not match the level sizes");
        }
    }
    const Level& Lc = c->lv[c->nlevels - 1];
    int32_t nL = Lc.n;
    if (Lc.nblk > 0) {
        nL = 0;
        for (int32_t b = 0; b < Lc.nblk; ++b) nL = std::max(nL, Lc.blk_off_h[b + 1] - Lc.blk_off_h[b]);
    }
    int32_t nblk = -1;
    for (int l = 0; l < c->nlevels; ++l) {
        const int32_t k = c->lv[l].nblk;
        if (nblk < 0) nblk = k;
        if (k != nblk)
            return fail(AMGG_EINVAL, std::string(where) + ": every level needs the same block count (level " +
                                         std::to_string(l) + " has " + std::to_string(k) + ")");
    }
    if (nL > AMGG_MAX_COARSE_DENSE)
        return fail(AMGG_EINVAL, std::string(where) + ": coarsest level has " + std::to_string(nL) +
                                     " rows, more than the dense limit " + std::to_string(AMGG_MAX_COARSE_DENSE));
    return AMGG_OK;
}

extern "C" int amgg_workspace_bytes(const amgg_ctx* c, size_t* bytes) {
    return guarded([&]() -> int {
        if (!c || !bytes) return fail(AMGG_EINVAL, "amgg_workspace_bytes: null argument");
        int rc = check_loaded(c, "amgg_workspace_bytes");
        if (rc) return rc;
        amgg_ctx tmp = *c;
        *bytes = layout(&tmp, 0);
        return AMGG_OK;
    });
}

// Halo lists of every smoothing level for the fused kernels, built on the host from a copy of
// the level's pattern (setup only).
static hipError_t build_halos(amgg_ctx* c, hipStream_t st) {
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    std::vector<int32_t> ptr, col;
    HaloLists h;
    auto up = [&](void* dst, const void* src, size_t bytes) {
        if (e == hipSuccess && bytes > 0) e = hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
    };
    for (int l = 0; l + 1 < c->nlevels; ++l) {
        Level& L = c->lv[l];
        L.hrows = 0;
        const int rows = L.n <= kFuseMaxRows ? stream_rows_for(L.n, L.nnz) : 0;
        if (rows == 0 || L.hoff == nullptr) continue;
        ptr.resize(static_cast<size_t>(L.n) + 1);
        col.resize(static_cast<size_t>(L.nnz));
        if ((e = hipMemcpy(ptr.data(), L.ptr, sizeof(int32_t) * ptr.size(), hipMemcpyDeviceToHost)) != hipSuccess ||
            (e = hipMemcpy(col.data(), L.col, sizeof(int32_t) * col.size(), hipMemcpyDeviceToHost)) != hipSuccess)
            return e;
        if (!build_halo(L.n, ptr.data(), col.data(), rows, kHaloCap, kHaloEntCap, static_cast<size_t>(L.nnz), h))
            continue;
        up(L.hoff, h.hoff.data(), sizeof(int32_t) * h.hoff.size());
        up(L.halo, h.halo.data(), sizeof(int32_t) * h.halo.size());
        up(L.hend, h.hend.data(), sizeof(uint16_t) * h.hend.size());
        up(L.heoff, h.heoff.data(), sizeof(int32_t) * h.heoff.size());
        up(L.hent, h.hent.data(), sizeof(int32_t) * h.hent.size());
        std::vector<int32_t> hc(h.hent.size());
        for (size_t k = 0; k < hc.size(); ++k) hc[k] = col[h.hent[k]];
        up(L.hcol, hc.data(), sizeof(int32_t) * hc.size());
        up(L.hloc, h.loc.data(), sizeof(uint16_t) * h.loc.size());
        if (e != hipSuccess) return e;
        L.nhent = static_cast<int32_t>(h.hent.size());
        if ((e = gather_values(L.nhent, L.hent, L.val, L.val32, L.ha64, L.ha32, st)) != hipSuccess) return e;
        L.hrows = rows;
    }
    return hipSuccess;
}

extern "C" int amgg_finalize(amgg_ctx* c, int singular, void* workspace, size_t ws_bytes, void* stream) {
    return guarded([&]() -> int {
        if (!c) return fail(AMGG_EINVAL, "amgg_finalize: null context");
        int rc = check_loaded(c, "amgg_finalize");
        if (rc) return rc;
        if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255u))
            return fail(AMGG_EWORKSPACE, "amgg_finalize: workspace null or not 256-byte aligned");
        amgg_ctx tmp = *c;
        const size_t need = layout(&tmp, 0);
        if (ws_bytes < need)
            return fail(AMGG_EWORKSPACE, "amgg_finalize: workspace has " + std::to_string(ws_bytes) + " bytes, needs " +
                                             std::to_string(need));
        hipError_t e = hipSetDevice(c->device);
        if (e != hipSuccess) return hip_fail(e, "amgg_finalize");
        drop_graphs(c);
        c->nblk = c->lv[0].nblk;
        layout(c, reinterpret_cast<uintptr_t>(workspace));
        c->ws = workspace;
        c->ws_bytes = ws_bytes;
        c->singular = singular ? 1 : 0;
        hipStream_t st = static_cast<hipStream_t>(stream);
        auto ok = [&](hipError_t r) { if (r != hipSuccess && e == hipSuccess) e = r; };
        ok(vec_zero_bytes(c->flags, sizeof(int32_t) * 8, st));
        ok(vec_zero_bytes(c->scal, sizeof(double) * kSlots, st));
        for (int l = 0; l < c->nlevels; ++l) {
            Level& L = c->lv[l];
            L.smoother = kSmootherNone;
            ok(extract_diag(L.n, L.ptr, L.col, L.val, L.diag, c->flags + 0, st));
            ok(offdiag_absmax(L.n, L.ptr, L.col, L.val, c->partial, L.scale, st));
            ok(cast_f64_f32(L.nnz, L.val, L.val32, st));
            if (l + 1 < c->nlevels) {
                ok(cast_f64_f32(L.pnnz, L.pval, L.pval32, st));
                ok(transpose_csr(L.n, L.nc, L.pnnz, L.pptr, L.pcol, L.pval, L.rptr, L.rcol, L.rval, c->cursor, st));
                ok(cast_f64_f32(L.pnnz, L.rval, L.rval32, st));
            }
        }
        Level& Lc = c->lv[c->nlevels - 1];
        if (c->nblk > 0) {
            auto up = [&](void* dst, const void* src, size_t bytes) {
                ok(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
            };
            for (int l = 0; l < c->nlevels; ++l) {
                Level& L = c->lv[l];
                up(L.blk_off, L.blk_off_h.data(), sizeof(int32_t) * L.blk_off_h.size());
                up(L.blk_crow, L.blk_crow_h.data(), sizeof(int32_t) * L.blk_crow_h.size());
                up(L.chunk_row, L.chunk_row_h.data(), sizeof(int32_t) * L.chunk_row_h.size());
                up(L.blk_chunk, L.blk_chunk_h.data(), sizeof(int32_t) * L.blk_chunk_h.size());
            }
            for (int l = 0; l < c->nlevels; ++l) {  // after every level's tables are on the device
                Level& L = c->lv[l];
                ok(block_absmax(L.nblk, L.blk_off, L.ptr, L.col, L.val, L.blk_scale, st));
                if (l + 1 < c->nlevels)
                    ok(prolong_blocks_check(L.n, L.pptr, L.pcol, L.nblk, L.blk_off, c->lv[l + 1].blk_off,
                                            c->flags + 2, st));
            }
            up(Lc.dense_off, Lc.dense_off_h.data(), sizeof(int64_t) * Lc.dense_off_h.size());
            for (int32_t b = 0; b < Lc.nblk; ++b) {
                const int32_t o = Lc.blk_off_h[b], nb = Lc.blk_off_h[b + 1] - o;
                double* M = Lc.dense + Lc.dense_off_h[b];
                ok(dense_from_csr(nb, Lc.ptr + o, Lc.col, Lc.val, M, Lc.blk_sing_h[b], st, o));
                ok(dense_lu_inverse(nb, M, Lc.piv + o, Lc.inv + Lc.dense_off_h[b], c->flags + 1, st));
            }
        } else {
            ok(dense_from_csr(Lc.n, Lc.ptr, Lc.col, Lc.val, Lc.dense, c->singular, st));
            ok(dense_lu_inverse(Lc.n, Lc.dense, Lc.piv, Lc.inv, c->flags + 1, st));
        }
        if (e != hipSuccess) return hip_fail(e, "amgg_finalize (launch)");
        // packed columns of every CSR-stream matrix (each call synchronises to read its far count)
        for (int l = 0; l < c->nlevels && e == hipSuccess; ++l) {
            Level& L = c->lv[l];
            auto pack = [&](Level::Pack& pk, int32_t rows_m, int32_t nz, const int32_t* ptr, const int32_t* col) {
                if (pk.rows > 0 && e == hipSuccess)
                    ok(pack_columns(rows_m, nz, ptr, col, pk.rows, pk.off, pk.base, pk.foff, pk.fslot, pk.fcol, pk.cap,
                                    c->pack_parts, &pk.nfar, st));
            };
            pack(L.pa, L.n, L.nnz, L.ptr, L.col);
            if (l + 1 < c->nlevels) {
                pack(L.pp, L.n, L.pnnz, L.pptr, L.pcol);
                pack(L.pr, L.nc, L.pnnz, L.rptr, L.rcol);
            }
        }
        if (e != hipSuccess) return hip_fail(e, "amgg_finalize (column packing)");
        // largest row block of every CSR-stream matrix: sizes the kernels' LDS product buffers
        ok(vec_zero_bytes(c->blkmax, sizeof(int32_t) * 3 * AMGG_MAX_LEVELS, st));
        for (int l = 0; l < c->nlevels && e == hipSuccess; ++l) {
            Level& L = c->lv[l];
            int32_t* m = c->blkmax + 3 * l;
            ok(block_max_entries(L.n, L.ptr, stream_rows_for(L.n, L.nnz), m, st));
            if (l + 1 < c->nlevels) {
                ok(block_max_entries(L.n, L.pptr, stream_rows_for(L.n, L.pnnz), m + 1, st));
                ok(block_max_entries(L.nc, L.rptr, stream_rows_for(L.nc, L.pnnz), m + 2, st));
            }
        }
        if (e != hipSuccess) return hip_fail(e, "amgg_finalize (row blocks)");
        if ((e = build_halos(c, st)) != hipSuccess) return hip_fail(e, "amgg_finalize (halo lists)");
        int32_t flags[3] = {0, 0, 0};
        std::vector<int32_t> bmax(3 * AMGG_MAX_LEVELS, 0);
        if ((e = hipMemcpyAsync(flags, c->flags, sizeof(flags), hipMemcpyDeviceToHost, st)) != hipSuccess ||
            (e = hipMemcpyAsync(bmax.data(), c->blkmax, sizeof(int32_t) * bmax.size(), hipMemcpyDeviceToHost, st)) !=
                hipSuccess ||
            (e = hipStreamSynchronize(st)) != hipSuccess)
            return hip_fail(e, "amgg_finalize (sync)");
        for (int l = 0; l < c->nlevels; ++l) {
            c->lv[l].acap = stream_cap_for(bmax[3 * l]);
            c->lv[l].pcap = stream_cap_for(bmax[3 * l + 1]);
            c->lv[l].rcap = stream_cap_for(bmax[3 * l + 2]);
        }
        if (flags[0]) return fail(AMGG_EINVAL, "amgg_finalize: a level matrix has a missing or non-positive diagonal");
        if (flags[1]) return fail(AMGG_EINVAL, "amgg_finalize: coarsest matrix is singular (zero pivot)");
        if (flags[2]) return fail(AMGG_EINVAL, "amgg_finalize: a prolongation couples different blocks");
        c->finalized = true;
        return AMGG_OK;
    });
}

extern "C" int amgg_set_fusion(amgg_ctx* c, int enable) {
    if (!c) return fail(AMGG_EINVAL, "amgg_set_fusion: null context");
    for (int l = 0; l < c->nlevels; ++l) c->lv[l].fuse = enable != 0;
    drop_graphs(c);
    return AMGG_OK;
}

extern "C" int amgg_set_packed_columns(amgg_ctx* c, int mode) {
    if (!c || mode < 0 || mode > 2) return fail(AMGG_EINVAL, "amgg_set_packed_columns: null context or bad mode");
    for (int l = 0; l < c->nlevels; ++l) c->lv[l].pack = mode;
    drop_graphs(c);
    return AMGG_OK;
}

extern "C" int amgg_level_view_get(const amgg_ctx* c, int lvl, amgg_level_view* v) {
    if (!c || !v || lvl < 0 || lvl >= c->nlevels) return fail(AMGG_EINVAL, "amgg_level_view_get: bad argument");
    if (!c->finalized) return fail(AMGG_ESTATE, "amgg_level_view_get: hierarchy not finalized");
    const Level& L = c->lv[lvl];
    const bool coarse = lvl == c->nlevels - 1;
    std::memset(v, 0, sizeof(*v));
    v->n = L.n;
    v->nnz = L.nnz;
    v->n_coarse = coarse ? 0 : L.nc;
    v->p_nnz = coarse ? 0 : L.pnnz;
    v->r_rowptr = coarse ? nullptr : L.rptr;
    v->r_col = coarse ? nullptr : L.rcol;
    v->r_val = coarse ? nullptr : L.rval;
    v->a_val32 = L.val32;
    v->p_val32 = coarse ? nullptr : L.pval32;
    v->r_val32 = coarse ? nullptr : L.rval32;
    v->q_val = L.q64;
    v->q_val32 = L.q32;
    v->diag = L.diag;
    v->scale = L.scale;
    v->coarse_inv = coarse ? L.inv : nullptr;
    v->fused_rows = L.hrows;
    const Level::Pack* packs[3] = {&L.pa, &L.pp, &L.pr};
    for (int k = 0; k < 3; ++k) {
        const bool use = packs[k]->view(L.pack, k == 0 ? L.nnz : L.pnnz).off != nullptr && (k == 0 || !coarse);
        v->pack_rows[k] = use ? packs[k]->rows : 0;
        v->pack_far[k] = use ? packs[k]->nfar : 0;
    }
    v->stream_cap[0] = L.acap;
    v->stream_cap[1] = coarse ? 0 : L.pcap;
    v->stream_cap[2] = coarse ? 0 : L.rcap;
    return AMGG_OK;
}

// ------------------------------------------------------------------------------------
// Smoother
// ------------------------------------------------------------------------------------
static int set_coeffs_impl(amgg_ctx* c, int lvl, int degree, const double* coeffs, const float* dev, void* stream,
                           int diag_only = 0) {
    if (!c || lvl < 0 || lvl >= c->nlevels) return fail(AMGG_EINVAL, "amgg_set_smoother: bad context or level");
    if (!c->finalized) return fail(AMGG_ESTATE, "amgg_set_smoother: hierarchy not finalized");
    if (degree < 1 || degree > AMGG_MAX_DEGREE) return fail(AMGG_EINVAL, "amgg_set_smoother: degree out of range");
    if (!coeffs && !dev) return fail(AMGG_EINVAL, "amgg_set_smoother: null coefficients");
    PolyCoeffs pc{};
    pc.degree = degree;
    pc.diag_only = diag_only ? 1 : 0;
    bool diagonal = diag_only != 0, baseline = false;
    if (coeffs) {
        diagonal = true;
        baseline = coeffs[0] == 2.0 / 3.0;
        for (int k = 0; k < 2 * degree + 1; ++k) {
            if (!std::isfinite(coeffs[k])) return fail(AMGG_ENONFINITE, "amgg_set_smoother: non-finite coefficient");
            pc.c[k] = coeffs[k];
            if (k > degree && coeffs[k] != 0.0) diagonal = false;
            if (k > 0 && coeffs[k] != 0.0) baseline = false;
        }
    }
    Level& L = c->lv[lvl];
    hipError_t e = hipSetDevice(c->device);
    if (e == hipSuccess && L.nblk > 0)  // the same coefficients on every block, each with its own scale
        e = assemble_smoother_blocks(L.n, L.ptr, L.col, L.val, L.diag, L.nblk, L.blk_off, L.blk_scale, L.blk_crow, pc,
                                     coeffs ? nullptr : dev, 0, L.q64, L.q32, L.qd64, L.qd32,
                                     static_cast<hipStream_t>(stream));
    else if (e == hipSuccess)
        e = assemble_smoother(L.n, L.ptr, L.col, L.val, L.diag, L.scale, pc, coeffs ? nullptr : dev, L.q64, L.q32,
                              L.qd64, L.qd32, static_cast<hipStream_t>(stream));
    if (e == hipSuccess && L.hrows > 0)
        e = gather_values(L.nhent, L.hent, L.q64, L.q32, L.hq64, L.hq32, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "amgg_set_smoother");
    L.smoother = diagonal ? kSmootherDiagonal : kSmootherSparse;
    L.degree = degree;
    L.baseline = baseline;
    L.diag_form = diag_only != 0;
    return AMGG_OK;
}

extern "C" int amgg_get_smoother_values(const amgg_ctx* c, int lvl, double* q_out, void* stream) {
    return guarded([&]() -> int {
        if (!c || !q_out || lvl < 0 || lvl >= c->nlevels)
            return fail(AMGG_EINVAL, "amgg_get_smoother_values: null argument or bad level");
        if (!c->finalized) return fail(AMGG_ESTATE, "amgg_get_smoother_values: hierarchy not finalized");
        const Level& L = c->lv[lvl];
        if (L.smoother == kSmootherNone) return fail(AMGG_ESTATE, "amgg_get_smoother_values: no smoother set");
        hipError_t e = hipSetDevice(c->device);
        if (e == hipSuccess && L.nnz > 0)
            e = hipMemcpyAsync(q_out, L.q64, sizeof(double) * L.nnz, hipMemcpyDeviceToDevice,
                               static_cast<hipStream_t>(stream));
        if (e != hipSuccess) return hip_fail(e, "amgg_get_smoother_values");
        return AMGG_OK;
    });
}

extern "C" int amgg_set_smoother_coeffs(amgg_ctx* c, int lvl, int degree, const double* coeffs, void* stream) {
    return guarded([&] { return set_coeffs_impl(c, lvl, degree, coeffs, nullptr, stream); });
}

extern "C" int amgg_set_smoother_coeffs_device(amgg_ctx* c, int lvl, int degree, const float* coeffs_dev,
                                               void* stream) {
    return guarded([&] { return set_coeffs_impl(c, lvl, degree, nullptr, coeffs_dev, stream); });
}

extern "C" int amgg_set_smoother_coeffs_device_form(amgg_ctx* c, int lvl, int degree, const float* coeffs_dev,
                                                    int diagonal, void* stream) {
    return guarded([&] { return set_coeffs_impl(c, lvl, degree, nullptr, coeffs_dev, stream, diagonal ? 1 : 0); });
}

extern "C" int amgg_set_smoother_jacobi(amgg_ctx* c, int lvl, double omega, void* stream) {
    double cf[3] = {omega, 0.0, 0.0};
    return guarded([&] { return set_coeffs_impl(c, lvl, 1, cf, nullptr, stream); });
}

static int set_coeffs_blocks_impl(amgg_ctx* c, int lvl, int degree, const float* coeffs_dev, int32_t stride,
                                  int diag_only, void* stream) {
    return guarded([&]() -> int {
        if (!c || lvl < 0 || lvl >= c->nlevels) return fail(AMGG_EINVAL, "amgg_set_smoother_coeffs_blocks: bad level");
        if (!c->finalized) return fail(AMGG_ESTATE, "amgg_set_smoother_coeffs_blocks: hierarchy not finalized");
        Level& L = c->lv[lvl];
        if (L.nblk == 0) return fail(AMGG_ESTATE, "amgg_set_smoother_coeffs_blocks: level has no blocks");
        if (degree < 1 || degree > AMGG_MAX_DEGREE || !coeffs_dev || stride < 2 * degree + 1)
            return fail(AMGG_EINVAL, "amgg_set_smoother_coeffs_blocks: bad degree, stride or null coefficients");
        PolyCoeffs pc{};
        pc.degree = degree;
        pc.diag_only = diag_only ? 1 : 0;
        const hipStream_t st = static_cast<hipStream_t>(stream);
        hipError_t e = hipSetDevice(c->device);
        if (e == hipSuccess)
            e = assemble_smoother_blocks(L.n, L.ptr, L.col, L.val, L.diag, L.nblk, L.blk_off, L.blk_scale, L.blk_crow,
                                         pc, coeffs_dev, stride, L.q64, L.q32, L.qd64, L.qd32, st);
        if (e == hipSuccess && L.hrows > 0) e = gather_values(L.nhent, L.hent, L.q64, L.q32, L.hq64, L.hq32, st);
        if (e != hipSuccess) return hip_fail(e, "amgg_set_smoother_coeffs_blocks");
        L.smoother = diag_only ? kSmootherDiagonal : kSmootherSparse;
        L.degree = degree;
        L.baseline = false;
        L.diag_form = diag_only != 0;
        return AMGG_OK;
    });
}

extern "C" int amgg_set_smoother_coeffs_blocks(amgg_ctx* c, int lvl, int degree, const float* coeffs_dev,
                                               int32_t stride, void* stream) {
    return set_coeffs_blocks_impl(c, lvl, degree, coeffs_dev, stride, 0, stream);
}

extern "C" int amgg_set_smoother_coeffs_blocks_form(amgg_ctx* c, int lvl, int degree, const float* coeffs_dev,
                                                    int32_t stride, int diagonal, void* stream) {
    return set_coeffs_blocks_impl(c, lvl, degree, coeffs_dev, stride, diagonal ? 1 : 0, stream);
}

extern "C" int amgg_set_level_blocks(amgg_ctx* c, int lvl, int32_t nblk, const int32_t* offsets,
                                     const int32_t* coeff_rows, const int32_t* singular) {
    return guarded([&]() -> int {
        if (!c || lvl < 0 || lvl >= c->nlevels) return fail(AMGG_EINVAL, "amgg_set_level_blocks: bad context or level");
        Level& L = c->lv[lvl];
        if (!L.loaded) return fail(AMGG_ESTATE, "amgg_set_level_blocks: load the level first");
        if (nblk < 1 || !offsets) return fail(AMGG_EINVAL, "amgg_set_level_blocks: nblk < 1 or null offsets");
        if (offsets[0] != 0 || offsets[nblk] != L.n)
            return fail(AMGG_EINVAL, "amgg_set_level_blocks: offsets must run from 0 to the level's row count");
        for (int32_t b = 0; b < nblk; ++b)
            if (offsets[b + 1] <= offsets[b]) return fail(AMGG_EINVAL, "amgg_set_level_blocks: empty or unordered block");
        std::vector<int32_t> rows(nblk);
        for (int32_t b = 0; b < nblk; ++b) rows[b] = coeff_rows ? coeff_rows[b] : b;
        std::vector<int32_t> used;
        for (int32_t r : rows)
            if (r >= 0) used.push_back(r);
        std::sort(used.begin(), used.end());
        if (std::adjacent_find(used.begin(), used.end()) != used.end())
            return fail(AMGG_EINVAL, "amgg_set_level_blocks: two blocks share a coefficient row");
        L.nblk = nblk;
        L.blk_off_h.assign(offsets, offsets + nblk + 1);
        L.blk_crow_h = rows;
        L.blk_sing_h.assign(nblk, 0);
        if (singular)
            for (int32_t b = 0; b < nblk; ++b) L.blk_sing_h[b] = singular[b] ? 1 : 0;
        L.chunk_row_h.clear();
        L.blk_chunk_h.assign(nblk + 1, 0);
        for (int32_t b = 0; b < nblk; ++b) {
            L.blk_chunk_h[b] = static_cast<int32_t>(L.chunk_row_h.size());
            for (int32_t r = offsets[b]; r < offsets[b + 1]; r += kChunkRows) L.chunk_row_h.push_back(r);
        }
        L.blk_chunk_h[nblk] = static_cast<int32_t>(L.chunk_row_h.size());
        L.chunk_row_h.push_back(L.n);
        L.dense_off_h.assign(nblk + 1, 0);
        for (int32_t b = 0; b < nblk; ++b) {
            const int64_t nb = offsets[b + 1] - offsets[b];
            L.dense_off_h[b + 1] = L.dense_off_h[b] + nb * nb;
        }
        c->finalized = false;
        return AMGG_OK;
    });
}

// ------------------------------------------------------------------------------------
// V-cycle entry point
// ------------------------------------------------------------------------------------
extern "C" int amgg_vcycle(amgg_ctx* c, int nu1, int nu2, int precision, const double* f, double* u, void* stream) {
    return guarded([&]() -> int {
        int rc = check_ready(c, "amgg_vcycle");
        if (rc) return rc;
        if (!f || !u) return fail(AMGG_EINVAL, "amgg_vcycle: null vector");
        if (nu1 < 0 || nu1 > 8 || nu2 < 0 || nu2 > 8) return fail(AMGG_EINVAL, "amgg_vcycle: nu out of range");
        if (precision != 64 && precision != 32) return fail(AMGG_EINVAL, "amgg_vcycle: precision must be 64 or 32");
        hipStream_t st = static_cast<hipStream_t>(stream);
        hipError_t e = hipSetDevice(c->device);
        Level& L0 = c->lv[0];
        if (e == hipSuccess && precision == 64) {
            double* res = nullptr;
            e = vec_copy<double>(L0.n, u, L0.u64, st);
            if (e == hipSuccess) e = vcycle_level<double>(c, 0, f, L0.u64, L0.t64, false, nu1, nu2, st, &res);
            if (e == hipSuccess) e = vec_copy<double>(L0.n, res, u, st);
        } else if (e == hipSuccess) {
            float* res = nullptr;
            e = cast_f64_f32(L0.n, f, L0.f32, st);
            if (e == hipSuccess) e = cast_f64_f32(L0.n, u, L0.u32, st);
            if (e == hipSuccess) e = vcycle_level<float>(c, 0, L0.f32, L0.u32, L0.t32, false, nu1, nu2, st, &res);
            if (e == hipSuccess) e = cast_f32_f64(L0.n, res, u, st);
        }
        if (e != hipSuccess) return hip_fail(e, "amgg_vcycle");
        return AMGG_OK;
    });
}

// ------------------------------------------------------------------------------------
// Single level operators
// ------------------------------------------------------------------------------------
namespace {

template <typename T>
hipError_t level_apply_t(amgg_ctx* c, int lvl, int op, const T* x, T* y, const T* f, hipStream_t st) {
    Level& L = c->lv[lvl];
    switch (op) {
        case AMGG_OP_SPMV:
            return csr_apply<T>(L.A(), L.aval<T>(), x, y, nullptr, nullptr, nullptr, Epi::Store, st);
        case AMGG_OP_RESIDUAL:
            return csr_apply<T>(L.A(), L.aval<T>(), x, y, f, nullptr, nullptr, Epi::Resid, st);
        case AMGG_OP_SMOOTH:
            return csr_apply<T>(L.A(), L.qval<T>(), x, y, nullptr, nullptr, nullptr, Epi::Add, st);
        case AMGG_OP_JACOBI:
            return csr_apply<T>(L.A(), L.aval<T>(), x, y, f, L.qd<T>(), x, Epi::Jacobi, st);
        case AMGG_OP_RESTRICT:
            return csr_apply<T>(L.R(), L.rv<T>(), x, y, nullptr, nullptr, nullptr, Epi::Store, st);
        case AMGG_OP_PROLONG:
            return csr_apply<T>(L.P(), L.pv<T>(), x, y, nullptr, nullptr, nullptr, Epi::Add, st);
        case AMGG_OP_COARSE:
            return coarse_solve<T>(L, x, y, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace

namespace {

int level_apply_checked(amgg_ctx* c, int lvl, int op, int precision, const void* x, void* y, const void* f,
                        void* stream, void* start_event, void* stop_event, const char* name) {
    return guarded([&]() -> int {
        if (!c || lvl < 0 || lvl >= c->nlevels) return fail(AMGG_EINVAL, std::string(name) + ": bad context or level");
        if (!c->finalized) return fail(AMGG_ESTATE, std::string(name) + ": hierarchy not finalized");
        if (op < AMGG_OP_SPMV || op > AMGG_OP_COARSE) return fail(AMGG_EINVAL, std::string(name) + ": unknown op");
        if (precision != 32 && precision != 64) return fail(AMGG_EINVAL, std::string(name) + ": precision must be 32 or 64");
        const bool coarsest = lvl == c->nlevels - 1;
        if ((op == AMGG_OP_RESTRICT || op == AMGG_OP_PROLONG) && coarsest)
            return fail(AMGG_EINVAL, std::string(name) + ": no transfer below the coarsest level");
        if (op == AMGG_OP_COARSE && !coarsest) return fail(AMGG_EINVAL, std::string(name) + ": COARSE needs the coarsest level");
        if ((op == AMGG_OP_SMOOTH || op == AMGG_OP_JACOBI) && c->lv[lvl].smoother == kSmootherNone)
            return fail(AMGG_ESTATE, std::string(name) + ": smoother not set");
        if (!x || !y || ((op == AMGG_OP_RESIDUAL || op == AMGG_OP_JACOBI) && !f))
            return fail(AMGG_EINVAL, std::string(name) + ": null vector");
        if ((start_event == nullptr) != (stop_event == nullptr))
            return fail(AMGG_EINVAL, std::string(name) + ": give both events or neither");
        hipStream_t st = static_cast<hipStream_t>(stream);
        hipError_t e = hipSetDevice(c->device);
        if (e == hipSuccess) {
            armed_events() = LaunchEvents{static_cast<hipEvent_t>(start_event), static_cast<hipEvent_t>(stop_event)};
            if (precision == 64)
                e = level_apply_t<double>(c, lvl, op, static_cast<const double*>(x), static_cast<double*>(y),
                                          static_cast<const double*>(f), st);
            else
                e = level_apply_t<float>(c, lvl, op, static_cast<const float*>(x), static_cast<float*>(y),
                                         static_cast<const float*>(f), st);
            armed_events() = LaunchEvents{};
        }
        if (e != hipSuccess) return hip_fail(e, name);
        return AMGG_OK;
    });
}

}  // namespace

extern "C" int amgg_level_apply(amgg_ctx* c, int lvl, int op, int precision, const void* x, void* y, const void* f,
                                void* stream) {
    return level_apply_checked(c, lvl, op, precision, x, y, f, stream, nullptr, nullptr, "amgg_level_apply");
}

extern "C" int amgg_level_apply_timed(amgg_ctx* c, int lvl, int op, int precision, const void* x, void* y,
                                      const void* f, void* start_event, void* stop_event, void* stream) {
    if (!start_event || !stop_event) return fail(AMGG_EINVAL, "amgg_level_apply_timed: null event");
    return level_apply_checked(c, lvl, op, precision, x, y, f, stream, start_event, stop_event,
                               "amgg_level_apply_timed");
}

extern "C" int amgg_chain_loss_grad(int32_t nrows, int32_t ncols, const double* dcoeffs, const int32_t* row_problem,
                                    const double* dloss, float* out, void* stream) {
    if (!dcoeffs || !dloss || !out || nrows < 0 || ncols < 1)
        return fail(AMGG_EINVAL, "amgg_chain_loss_grad: bad argument");
    const hipError_t e = cast_scale_rows_f64_f32(nrows, ncols, dcoeffs, row_problem, dloss, out,
                                                 static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "amgg_chain_loss_grad");
    return AMGG_OK;
}

extern "C" int amgg_validation_metric(int32_t n, const double* loss, const double* loss_jacobi, double* out,
                                      void* stream) {
    if (!loss || !loss_jacobi || !out || n < 1) return fail(AMGG_EINVAL, "amgg_validation_metric: bad argument");
    const hipError_t e = mean_difference(n, loss, loss_jacobi, out, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "amgg_validation_metric");
    return AMGG_OK;
}

extern "C" int amgg_cast_scale_f64_f32(const double* in, float* out, int64_t n, double scale, void* stream) {
    if (!in || !out || n < 0) return fail(AMGG_EINVAL, "amgg_cast_scale_f64_f32: bad argument");
    const hipError_t e = cast_scale_f64_f32(n, in, scale, out, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "amgg_cast_scale_f64_f32");
    return AMGG_OK;
}
