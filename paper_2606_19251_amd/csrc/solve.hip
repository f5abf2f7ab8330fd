// Outer FP64 loops around the V-cycle (paper Sec. 4: V-cycles iterated until the
// relative residual reaches the tolerance, at most 500 iterations; Sec. 4.2: FP32 on the
// unstructured sets, FP64 where FP32 stagnates):
//   * stationary  u <- V(u, f)                              (FP64 cycle)
//   * iterative refinement  x <- x + V(0, b - A x)          (FP64 residual, FP32/FP64 cycle)
//   * flexible CG with z = V(0, r) as preconditioner        (FP64 vectors, FP32/FP64 cycle)
// The FP32 cycle receives r / ||r|| so that its input is O(1) whatever the residual
// level; the correction is scaled back in FP64. Scalars live on the device; the host
// reads one small block of them per iteration to decide on convergence, one iteration late
// while convergence is not in sight: iteration k + 1 is already enqueued while the host waits
// for iteration k's block, and the guarded steps leave x unchanged once the device has seen
// convergence, divergence or a breakdown, so an extra iteration is a no-op for the result.
//
// One outer iteration of IR or flexible CG is a fixed sequence of ~50 kernels (most of
// them on small coarse levels, where launch latency dominates). With opts.graphs the
// sequence is captured once per configuration into a HIP graph on the context's private
// stream and replayed on the caller's stream, one graph launch per iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <string>
#include <vector>

#include "amggnn.h"
#include "ctx.hpp"
#include "errors.hpp"
#include "kernels.hpp"

using namespace amgg;

namespace {

struct Runner {
    amgg_ctx* c;
    int nu1, nu2, prec;
    hipError_t e = hipSuccess;
    // FP32 cycles: the kernel that forms each residual also writes the next cycle's FP32
    // right-hand side (iterative refinement: csr_resid_cast, which does not store the FP64
    // residual; flexible CG: fcg_update_xr) instead of a separate cast pass; off with the fused
    // kernels (amgg_set_fusion) and, for iterative refinement, on matrices the CSR-stream
    // kernels do not serve. Both forms give bitwise the same iterates.
    bool cast_fused = false;

    void ok(hipError_t r) {
        if (r != hipSuccess && e == hipSuccess) e = r;
    }

    // z = V(0, r) on the fine level. FP64: returns the pointer holding z. FP32: the cycle's
    // FP32 result pointer is left in `last32` (the caller casts it back, scaled by ||r||).
    // r scaled by s[slot] into the fine level's FP32 right-hand side; a diagonal first smoothing
    // step u = qd f is formed by the cast itself
    void cast_rhs(const double* r, int slot, hipStream_t st) {
        Level& L0 = c->lv[0];
        const bool ready = takes_ready_u(c, 0, nu1);
        ok(cast_scaled_f64_f32(L0.n, r, c->scal + slot, L0.f32, st, ready ? L0.qd32 : nullptr,
                               ready ? L0.u32 : nullptr));
    }

    // z = V(0, r). FP32: r is cast scaled by s[slot], unless r is null (the FP32 right-hand side
    // is already in place).
    const double* precondition(const double* r, hipStream_t st, int slot = kInvNorm) {
        Level& L0 = c->lv[0];
        if (prec == 64) {
            double* res = nullptr;
            ok(vcycle_level<double>(c, 0, r, L0.u64, L0.t64, true, nu1, nu2, st, &res));
            return res;
        }
        float* res = nullptr;
        const bool ready = takes_ready_u(c, 0, nu1);
        if (r) cast_rhs(r, slot, st);
        ok(vcycle_level<float>(c, 0, L0.f32, L0.u32, L0.t32, true, nu1, nu2, st, &res, false, ready));
        last32 = res;
        return nullptr;
    }
    float* last32 = nullptr;

    // Flexible CG: precondition the latest residual `cur` (prev = the one before, unused on a
    // (re)start), update p, then q = A p, alpha, x += alpha p and the next residual into `prev`.
    // (Forming p inside the product, from z and the previous p, saves a pass but gathers from
    // two vectors: slower once the vectors no longer fit the last-level cache, 8M rows.)
    void fcg_iteration(bool first, double* x, double* cur, double* prev, hipStream_t st) {
        Level& L0 = c->lv[0];
        const int32_t n = L0.n;
        double* s = c->scal;
        const double* z = precondition(cast_fused ? nullptr : cur, st, kScaleCast);
        if (prec == 32) {
            // z = (double)u32 / scale is formed where it is used (the dots, then p), not stored
            ok(fcg_castback_dots(n, last32, s, cur, first ? nullptr : prev, nullptr, c->partial2, st));
        } else {
            ok(fcg_dots64(n, z, cur, first ? nullptr : prev, c->partial2, st));
        }
        ok(fcg_finish_beta(c->partial2, s, first ? 1 : 0, st));
        if (prec == 32)
            ok(fcg_update_p32(n, last32, c->p, s, first ? 1 : 0, st));
        else
            ok(fcg_update_p(n, z, c->p, s, first ? 1 : 0, st));
        int cnt = 0;
        ok(csr_spmv_dot(L0.A(), L0.val, c->p, c->q, c->partial, &cnt, st));
        ok(fcg_finish_pq(c->partial, cnt, s, st));
        Cast32 cs;
        if (cast_fused) {
            const bool ready = takes_ready_u(c, 0, nu1);
            cs.f = L0.f32;
            cs.qd = ready ? L0.qd32 : nullptr;
            cs.u = ready ? L0.u32 : nullptr;
        }
        ok(fcg_update_xr(n, x, c->p, cur, c->q, prev, s, c->partial, st, cs));
        ok(fcg_finish_rr_guarded(c->partial, kReduceBlocks, s, st));
    }

    // Iterative refinement: x += V(0, r); r = b - A x. FP32 cycles take r scaled by a power of two
    // (kScaleCast) and their output is scaled back exactly (kUnscale).
    void ir_iteration(double* x, const double* bb, double* r, hipStream_t st) {
        Level& L0 = c->lv[0];
        const int32_t n = L0.n;
        const double* e64 = precondition(cast_fused ? nullptr : r, st, kScaleCast);
        if (prec == 64)
            ok(ir_update_f64(n, x, e64, c->scal, st));
        else
            ok(ir_update_f32(n, x, last32, c->scal, st));
        int cnt = 0;
        if (cast_fused) {
            const bool ready = takes_ready_u(c, 0, nu1);
            Cast32 cs;
            cs.f = L0.f32;
            cs.qd = ready ? L0.qd32 : nullptr;
            cs.u = ready ? L0.u32 : nullptr;
            cs.scale = c->scal + kScaleNext;
            ok(csr_resid_cast(L0.A(), L0.val, x, bb, cs, c->partial, &cnt, st));
        } else {
            ok(csr_resid_norm(L0.A(), L0.val, x, bb, r, c->partial, &cnt, st));
        }
        ok(fcg_finish_rr_guarded(c->partial, cnt, c->scal, st));
    }

    bool read_scalars(hipStream_t st) {
        ok(hipMemcpyAsync(c->host_scal, c->scal, sizeof(double) * kSlots, hipMemcpyDeviceToHost, st));
        ok(hipStreamSynchronize(st));
        return e == hipSuccess;
    }
};

void set_all_jacobi(amgg_ctx* c, hipStream_t st) {
    for (int l = 0; l + 1 < c->nlevels; ++l) amgg_set_smoother_jacobi(c, l, 2.0 / 3.0, st);
}

std::string graph_key(const amgg_ctx* c, const char* what, int prec, int nu1, int nu2, const void* a, const void* b,
                      const void* d) {
    std::string k = std::string(what) + ":" + std::to_string(prec) + ":" + std::to_string(nu1) + ":" +
                    std::to_string(nu2) + ":" + std::to_string(reinterpret_cast<uintptr_t>(a)) + ":" +
                    std::to_string(reinterpret_cast<uintptr_t>(b)) + ":" +
                    std::to_string(reinterpret_cast<uintptr_t>(d)) + ":";
    for (int l = 0; l + 1 < c->nlevels; ++l) k += static_cast<char>('0' + c->lv[l].smoother);
    return k;
}

// Run `body(stream)` either directly on `st` or through a cached graph captured on the
// context's private stream.
template <class F>
hipError_t run_body(amgg_ctx* c, bool use_graph, const std::string& key, hipStream_t st, Runner& R, F&& body) {
    if (!use_graph) {
        body(st);
        return R.e;
    }
    for (auto& g : c->graphs)
        if (g.key == key) return hipGraphLaunch(g.exec, st);
    hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    body(c->cap_stream);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(c->cap_stream, &graph);
    if (R.e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return R.e;
    }
    if (e != hipSuccess) return e;
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return e;
    c->graphs.push_back({key, exec});
    return hipGraphLaunch(exec, st);
}

}  // namespace

extern "C" int amgg_solve(amgg_ctx* c, const amgg_solve_opts* o, const double* b, double* x, amgg_solve_info* info,
                          double* history, int history_cap, void* stream) {
    return guarded([&]() -> int {
        int rc = check_ready(c, "amgg_solve");
        if (rc) return rc;
        if (c->nblk > 0)
            return fail(AMGG_ESTATE, "amgg_solve: not available on a block-diagonal (batched) hierarchy");
        if (!o || !b || !x) return fail(AMGG_EINVAL, "amgg_solve: null argument");
        if (o->outer < AMGG_OUTER_STATIONARY || o->outer > AMGG_OUTER_FCG)
            return fail(AMGG_EINVAL, "amgg_solve: unknown outer method");
        if (o->inner_precision != 64 && o->inner_precision != 32)
            return fail(AMGG_EINVAL, "amgg_solve: inner precision must be 64 or 32");
        if (o->outer == AMGG_OUTER_STATIONARY && o->inner_precision != 64)
            return fail(AMGG_EINVAL, "amgg_solve: the stationary iteration runs FP64 cycles only");
        if (o->nu1 < 0 || o->nu1 > 8 || o->nu2 < 0 || o->nu2 > 8 || o->maxit < 1 || !(o->tol > 0.0))
            return fail(AMGG_EINVAL, "amgg_solve: nu, maxit or tol out of range");
        const double div_factor = o->div_factor > 0 ? o->div_factor : 1e3;
        const double stag_ratio = o->stag_ratio > 0 ? o->stag_ratio : 0.99;
        const int stag_window = o->stag_window > 0 ? o->stag_window : 10;
        const bool use_graph = o->graphs != 0 && o->outer != AMGG_OUTER_STATIONARY;

        hipStream_t st = static_cast<hipStream_t>(stream);
        Runner R{c, o->nu1, o->nu2, o->inner_precision};
        R.ok(hipSetDevice(c->device));
        Level& L0 = c->lv[0];
        const int32_t n = L0.n;
        const CsrView A = L0.A();
        R.cast_fused = o->inner_precision == 32 && L0.fuse &&
                       (o->outer == AMGG_OUTER_FCG || (o->outer == AMGG_OUTER_IR && stream_rows_for(n, L0.nnz) > 0));
        double* s = c->scal;
        double* hs = c->host_scal;
        int vcycles = 0;

        // right-hand side, projected to zero mean for a singular (all-Neumann) hierarchy
        const double* bb = b;
        if (c->singular) {
            R.ok(partial_sum(n, b, c->partial, st));
            R.ok(finish_sum(c->partial, s + kSum, st));
            R.ok(sub_mean(n, b, s + kSum, c->bproj, st));
            bb = c->bproj;
        }
        R.ok(vec_zero_bytes(s, sizeof(double) * kSlots, st));
        R.ok(vec_zero_bytes(x, sizeof(double) * n, st));
        R.ok(vec_copy<double>(n, bb, c->ra, st));
        R.ok(partial_dot(n, bb, bb, c->partial, st));
        R.ok(fcg_finish_rr(c->partial, kReduceBlocks, s, st));
        if (!R.read_scalars(st)) return hip_fail(R.e, "amgg_solve");
        const double nb = std::sqrt(hs[kRR]);
        std::vector<double> hist{1.0};
        amgg_solve_info inf{};
        auto finish = [&](int status, double rel, int iters) {
            inf.status = status;
            inf.relres = rel;
            inf.iterations = iters;
            inf.vcycles = vcycles;
            if (info) *info = inf;
            if (history)
                for (int k = 0; k < history_cap && k < static_cast<int>(hist.size()); ++k) history[k] = hist[k];
            return status;
        };
        if (!std::isfinite(nb)) return fail(AMGG_ENONFINITE, "amgg_solve: non-finite right-hand side");
        if (nb == 0.0) return finish(0, 0.0, 0);

        double* cur = c->ra;   // latest residual
        double* prev = c->rb;  // the one before (flexible CG)
        bool first = true;     // (re)start of the recurrence
        size_t stag_base = 0;  // stagnation is judged on the history since the last (re)start
        int k = 0;             // iterations processed
        if (o->outer == AMGG_OUTER_STATIONARY) {
            for (;;) {
                double* res = nullptr;
                R.ok(vec_copy<double>(n, x, L0.u64, st));
                R.ok(vcycle_level<double>(c, 0, bb, L0.u64, L0.t64, first, o->nu1, o->nu2, st, &res));
                R.ok(vec_copy<double>(n, res, x, st));
                int cnt = 0;
                R.ok(csr_resid_norm(A, L0.val, x, bb, cur, c->partial, &cnt, st));
                R.ok(fcg_finish_rr(c->partial, cnt, s, st));
                first = false;
                ++vcycles;
                ++k;
                if (!R.read_scalars(st)) return hip_fail(R.e, "amgg_solve");
                const double rel = std::sqrt(hs[kRR]) / nb;
                hist.push_back(rel);
                if (rel <= o->tol && std::isfinite(rel)) return finish(0, rel, k);
                int outcome = 0;
                if (!std::isfinite(rel) || rel > div_factor)
                    outcome = AMGG_DIVERGED;
                else if (hist.size() - stag_base > static_cast<size_t>(stag_window) &&
                         rel > stag_ratio * hist[hist.size() - 1 - stag_window])
                    outcome = AMGG_STAGNATED;
                if (outcome == 0) {
                    if (k >= o->maxit) return finish(AMGG_MAXIT, rel, k);
                    continue;
                }
                bool learned = false;
                for (int l = 0; l + 1 < c->nlevels; ++l) learned |= !c->lv[l].baseline;
                if (!o->fallback || inf.fell_back || !learned || k >= o->maxit) return finish(outcome, rel, k);
                // Jacobi fallback from the current x (from zero if it is not finite)
                inf.fell_back = 1;
                set_all_jacobi(c, st);
                first = !std::isfinite(rel);
                if (first) R.ok(vec_zero_bytes(x, sizeof(double) * n, st));
                stag_base = hist.size() - 1;
                if (R.e != hipSuccess) return hip_fail(R.e, "amgg_solve");
            }
        }

        // IR and flexible CG: each iteration is enqueued (a graph launch) together with an
        // asynchronous copy of the scalar block into one of kPipeline pinned slots; the host keeps
        // up to kPipeline - 1 iterations in flight behind the one it inspects.
        R.ok(fcg_set_limits(s, o->tol, div_factor, st));
        if (R.cast_fused) R.cast_rhs(c->ra, kScaleCast, st);  // the first cycle's right-hand side: b
        struct InFlight {
            double* cu;
            double* pv;
        };
        std::vector<InFlight> q;  // enqueued, not yet inspected (at most kPipeline)
        int launched = 0;
        bool more = true;  // false once a stop is decided and only the in-flight one remains
        auto launch = [&]() -> hipError_t {
            double* cu = cur;
            double* pv = prev;
            const bool f0 = first;
            hipError_t e;
            if (o->outer == AMGG_OUTER_IR) {
                e = run_body(c, use_graph, graph_key(c, "ir", R.prec, o->nu1, o->nu2, x, bb, cu), st, R,
                             [&](hipStream_t qs) { R.ir_iteration(x, bb, cu, qs); });
            } else {
                e = run_body(c, use_graph, graph_key(c, f0 ? "fcg0" : "fcg", R.prec, o->nu1, o->nu2, x, cu, pv), st,
                             R, [&](hipStream_t qs) { R.fcg_iteration(f0, x, cu, pv, qs); });
                std::swap(cur, prev);
            }
            first = false;
            if (e != hipSuccess) return e;
            const int slot = launched % kPipeline;
            if ((e = hipMemcpyAsync(hs + (1 + slot) * kSlots, s, sizeof(double) * kSlots, hipMemcpyDeviceToHost,
                                    st)) != hipSuccess ||
                (e = hipEventRecord(c->ev[slot], st)) != hipSuccess)
                return e;
            q.push_back({cu, pv});
            ++launched;
            return hipSuccess;
        };
        // back to a state where nothing is in flight (a masked or superseded iteration is dropped)
        auto settle = [&]() -> bool {
            q.clear();
            launched = k;
            R.ok(hipStreamSynchronize(st));
            return R.e == hipSuccess;
        };
        // Enqueue ahead only while the in-flight iterations are not expected to converge (the
        // residual after the last of them, predicted from the last ratio, stays above twice the
        // tolerance): an iteration enqueued after the converging one would run its whole cycle for
        // nothing.
        auto ahead = [&]() {
            if (hist.size() < 3) return true;
            const double last = hist[hist.size() - 1], ratio = std::min(1.0, last / hist[hist.size() - 2]);
            double pred = last;
            for (size_t m = 0; m < q.size(); ++m) pred *= ratio;
            return pred > 2.0 * o->tol;
        };
        for (;;) {
            hipError_t e = hipSuccess;
            if (q.empty()) e = launch();
            while (e == hipSuccess && more && q.size() < static_cast<size_t>(kPipeline) && launched < o->maxit &&
                   ahead())
                e = launch();
            if (e != hipSuccess) return hip_fail(e, "amgg_solve");
            const int slot = k % kPipeline;
            if ((e = hipEventSynchronize(c->ev[slot])) != hipSuccess) return hip_fail(e, "amgg_solve");
            const double* hk = hs + (1 + slot) * kSlots;
            const InFlight it = q.front();
            q.erase(q.begin());
            ++k;
            ++vcycles;
            double rel = std::sqrt(hk[kRR]) / nb;
            const bool breakdown = hk[kFlag] != 0.0;
            const bool halted = hk[kHalt] != 0.0;  // converged or diverged, as the device saw it
            int outcome = 0;
            if (!std::isfinite(rel) || rel > div_factor || (halted && !(rel <= o->tol * (1.0 + 1e-9)))) {
                outcome = AMGG_DIVERGED;
            } else if (breakdown) {
                outcome = AMGG_BREAKDOWN;
            } else if (halted) {
                // converged: the in-flight iteration (if any) left x unchanged
                if (!settle()) return hip_fail(R.e, "amgg_solve");
                if (o->outer == AMGG_OUTER_FCG) {
                    // The CG residual is updated by recurrence and drifts from b - A x on badly
                    // conditioned problems: confirm with the true residual; if it is still above
                    // the tolerance, restart the recurrence from it.
                    cur = it.pv;
                    prev = it.cu;
                    int cnt = 0;
                    R.ok(csr_resid_norm(A, L0.val, x, bb, cur, c->partial, &cnt, st));
                    R.ok(fcg_finish_rr(c->partial, cnt, s, st));
                    if (!R.read_scalars(st)) return hip_fail(R.e, "amgg_solve");
                    rel = std::sqrt(hs[kRR]) / nb;
                    hist.push_back(rel);
                    if (rel <= o->tol) return finish(0, rel, k);
                    if (k >= o->maxit) return finish(AMGG_MAXIT, rel, k);
                    R.ok(fcg_clear_halt(s, st));
                    R.ok(ir_set_scales(s, st));
                    if (R.cast_fused) R.cast_rhs(cur, kScaleCast, st);
                    first = true;
                    more = true;
                    continue;
                }
                hist.push_back(rel);
                return finish(0, rel, k);
            }
            hist.push_back(rel);
            if (outcome == 0 && hist.size() - stag_base > static_cast<size_t>(stag_window) &&
                rel > stag_ratio * hist[hist.size() - 1 - stag_window]) {
                if (!q.empty()) {  // judge again on the iteration already in flight
                    more = false;
                    continue;
                }
                outcome = AMGG_STAGNATED;
            }
            if (outcome == 0) {
                if (k >= o->maxit && q.empty()) return finish(AMGG_MAXIT, rel, k);
                more = true;
                continue;
            }
            // divergence, breakdown or stagnation
            if (!settle()) return hip_fail(R.e, "amgg_solve");
            bool learned = false;
            for (int l = 0; l + 1 < c->nlevels; ++l) learned |= !c->lv[l].baseline;
            if (!o->fallback || inf.fell_back || !learned || k >= o->maxit) return finish(outcome, rel, k);
            // Jacobi fallback: the cycle stays a linear operator, so the iteration may
            // continue from the current x with the paper's baseline smoother.
            inf.fell_back = 1;
            set_all_jacobi(c, st);
            R.ok(fcg_clear_halt(s, st));
            if (!std::isfinite(rel)) R.ok(vec_zero_bytes(x, sizeof(double) * n, st));
            int cnt = 0;
            R.ok(csr_resid_norm(A, L0.val, x, bb, c->ra, c->partial, &cnt, st));
            R.ok(fcg_finish_rr(c->partial, cnt, s, st));
            R.ok(ir_set_scales(s, st));
            if (R.cast_fused) R.cast_rhs(c->ra, kScaleCast, st);
            cur = c->ra;
            prev = c->rb;
            first = true;
            more = true;
            stag_base = hist.size() - 1;
            if (R.e != hipSuccess) return hip_fail(R.e, "amgg_solve");
        }
    });
}

// ------------------------------------------------------------------------------------------
// Judge of the learned smoother: the plain omega-Jacobi AMG decides, on the matrix at hand,
// whether the learned coefficients pay for themselves in solve time (the paper measures the
// acceleration as the Jacobi solve time over the learned one, Sec. 4).
// ------------------------------------------------------------------------------------------
namespace {

// Runs `iters` iterations of `o` (fallback off, graphs captured beforehand by a two-iteration
// run) and measures the wall-clock time of the synchronous iterations. The residual history
// gives the final relative residual and the reduction per iteration over the second half of
// the run (the first iterations remove the error components the cycle damps best and fall
// faster than the rest of the solve will).
struct Probe {
    int iterations = 0, status = 0;
    double log10_rel = 0.0, log10_rate = 0.0, ms_per_iter = 0.0;
};

int probe_smoother(amgg_ctx* c, const amgg_solve_opts* o, int iters, const double* b, double* x, hipStream_t st,
                   Probe* out) {
    amgg_solve_opts p = *o;
    p.fallback = 0;
    std::vector<double> hist(static_cast<size_t>(iters) + 1, 1.0);
    amgg_solve_info info{};
    if (p.graphs && p.outer != AMGG_OUTER_STATIONARY) {
        p.maxit = std::min(2, iters);
        const int rc = amgg_solve(c, &p, b, x, &info, nullptr, 0, st);
        if (rc < 0) return rc;
    }
    p.maxit = iters;
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "amgg_judge_smoother");
    const auto t0 = std::chrono::steady_clock::now();
    const int rc = amgg_solve(c, &p, b, x, &info, hist.data(), iters + 1, st);
    e = hipStreamSynchronize(st);
    const auto t1 = std::chrono::steady_clock::now();
    if (rc < 0) return rc;
    if (e != hipSuccess) return hip_fail(e, "amgg_judge_smoother");
    const int k = std::min(info.iterations, iters);
    out->iterations = info.iterations;
    out->status = rc;
    out->ms_per_iter = std::chrono::duration<double, std::milli>(t1 - t0).count() / std::max(k, 1);
    auto lg = [](double v) { return v > 0.0 ? std::log10(v) : (v == 0.0 ? -INFINITY : NAN); };
    out->log10_rel = k > 0 ? lg(hist[k]) : 0.0;
    const int h = k / 2;
    out->log10_rate = k > 0 ? (out->log10_rel - lg(hist[h])) / (k - h) : 0.0;
    return AMGG_OK;
}

// Predicted solve time to tol: the probe's own iterations when it reached tol, else the probe's
// iterations plus the remaining reduction at the second-half rate.
double predicted_ms(const Probe& p, double tol) {
    if (p.status == 0) return p.ms_per_iter * p.iterations;
    if (p.status != AMGG_MAXIT || !(p.log10_rate < 0.0) || !std::isfinite(p.log10_rel)) return INFINITY;
    return p.ms_per_iter * (p.iterations + (std::log10(tol) - p.log10_rel) / p.log10_rate);
}

}  // namespace

extern "C" int amgg_judge_smoother(amgg_ctx* c, const amgg_solve_opts* o, int iters, int degree,
                                   const float* coeffs_dev, int diag_levels, const double* b, double* x,
                                   amgg_judge_info* out, void* stream) {
    return guarded([&]() -> int {
        if (!c) return fail(AMGG_EINVAL, "amgg_judge_smoother: null context");
        if (!c->finalized) return fail(AMGG_ESTATE, "amgg_judge_smoother: hierarchy not finalized");
        int rc = AMGG_OK;
        if (c->nblk > 0) return fail(AMGG_ESTATE, "amgg_judge_smoother: not available on a block-diagonal hierarchy");
        if (!o || !coeffs_dev || !b || !x || !out) return fail(AMGG_EINVAL, "amgg_judge_smoother: null argument");
        if (iters < 1 || iters > 100) return fail(AMGG_EINVAL, "amgg_judge_smoother: iters must be in [1, 100]");
        if (degree < 1 || degree > AMGG_MAX_DEGREE || diag_levels < 0)
            return fail(AMGG_EINVAL, "amgg_judge_smoother: bad degree or diag_levels");
        const hipStream_t st = static_cast<hipStream_t>(stream);
        const int nc = 2 * degree + 1;
        auto set_learned = [&]() -> int {
            for (int l = 0; l < c->nlevels; ++l) {
                const int r = amgg_set_smoother_coeffs_device_form(c, l, degree, coeffs_dev + static_cast<int64_t>(l) * nc,
                                                                   l < diag_levels ? 1 : 0, stream);
                if (r) return r;
            }
            return AMGG_OK;
        };
        amgg_judge_info j{};
        Probe pr[2];
        if ((rc = set_learned())) return rc;
        if ((rc = probe_smoother(c, o, iters, b, x, st, &pr[0]))) return rc;
        for (int l = 0; l < c->nlevels; ++l)
            if ((rc = amgg_set_smoother_jacobi(c, l, 2.0 / 3.0, stream))) return rc;
        if ((rc = probe_smoother(c, o, iters, b, x, st, &pr[1]))) return rc;
        for (int s = 0; s < 2; ++s) {
            j.iterations[s] = pr[s].iterations;
            j.status[s] = pr[s].status;
            j.log10_relres[s] = pr[s].log10_rel;
            j.log10_rate[s] = pr[s].log10_rate;
            j.ms_per_iter[s] = pr[s].ms_per_iter;
            j.predicted_ms[s] = predicted_ms(pr[s], o->tol);
        }
        j.learned_wins = j.predicted_ms[0] < j.predicted_ms[1] ? 1 : 0;
        if (j.learned_wins && (rc = set_learned())) return rc;
        *out = j;
        return AMGG_OK;
    });
}
