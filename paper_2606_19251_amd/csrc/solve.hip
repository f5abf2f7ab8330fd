// Outer FP64 loops around the V-cycle (paper Sec. 4: V-cycles iterated until the
// relative residual reaches the tolerance, at most 500 iterations; Sec. 3.4 and App. B:
// FP32 training and tests on unstructured meshes, FP64 where FP32 stagnates):
//   * stationary  u <- V(u, f)                              (FP64 cycle)
//   * iterative refinement  x <- x + V(0, b - A x)          (FP64 residual, FP32/FP64 cycle)
//   * flexible CG with z = V(0, r) as preconditioner        (FP64 vectors, FP32/FP64 cycle)
// The FP32 cycle receives r / ||r|| so that its input is O(1) whatever the residual
// level; the correction is scaled back in FP64. Scalars live on the device; the host
// reads one small block of them per iteration to decide on convergence.
#include <hip/hip_runtime.h>

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
    hipStream_t st;
    int nu1, nu2, prec;
    hipError_t e = hipSuccess;
    int vcycles = 0;

    void ok(hipError_t r) {
        if (r != hipSuccess && e == hipSuccess) e = r;
    }

    // z = V(0, r) on the fine level; returns the device pointer holding z (FP64).
    // For FP32 the FCG variant also forms the dots z.r_new, z.r_old in the cast-back pass.
    const double* precondition(const double* r, double* zbuf) {
        Level& L0 = c->lv[0];
        ++vcycles;
        if (prec == 64) {
            double* res = nullptr;
            ok(vcycle_level<double>(c, 0, r, L0.u64, L0.t64, true, nu1, nu2, st, &res));
            return res;
        }
        float* res = nullptr;
        ok(cast_scaled_f64_f32(L0.n, r, c->scal + kInvNorm, L0.f32, st));
        ok(vcycle_level<float>(c, 0, L0.f32, L0.u32, L0.t32, true, nu1, nu2, st, &res));
        last32 = res;
        (void)zbuf;
        return nullptr;
    }
    float* last32 = nullptr;

    bool read_scalars() {
        ok(hipMemcpyAsync(c->host_scal, c->scal, sizeof(double) * kSlots, hipMemcpyDeviceToHost, st));
        ok(hipStreamSynchronize(st));
        return e == hipSuccess;
    }
};

void set_all_jacobi(amgg_ctx* c, hipStream_t st) {
    for (int l = 0; l + 1 < c->nlevels; ++l) amgg_set_smoother_jacobi(c, l, 2.0 / 3.0, st);
}

}  // namespace

extern "C" int amgg_solve(amgg_ctx* c, const amgg_solve_opts* o, const double* b, double* x, amgg_solve_info* info,
                          double* history, int history_cap, void* stream) {
    return guarded([&]() -> int {
        int rc = check_ready(c, "amgg_solve");
        if (rc) return rc;
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

        hipStream_t st = static_cast<hipStream_t>(stream);
        Runner R{c, st, o->nu1, o->nu2, o->inner_precision};
        R.ok(hipSetDevice(c->device));
        Level& L0 = c->lv[0];
        const int32_t n = L0.n;
        const CsrView A = L0.A();
        double* s = c->scal;
        double* hs = c->host_scal;

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
        R.ok(fcg_finish_rr(c->partial, s, st));
        if (!R.read_scalars()) return hip_fail(R.e, "amgg_solve");
        const double nb = std::sqrt(hs[kRR]);
        std::vector<double> hist{1.0};
        amgg_solve_info inf{};
        auto finish = [&](int status, double rel, int iters) {
            inf.status = status;
            inf.relres = rel;
            inf.iterations = iters;
            inf.vcycles = R.vcycles;
            if (info) *info = inf;
            if (history)
                for (int k = 0; k < history_cap && k < static_cast<int>(hist.size()); ++k) history[k] = hist[k];
            return status;
        };
        if (!std::isfinite(nb)) return fail(AMGG_ENONFINITE, "amgg_solve: non-finite right-hand side");
        if (nb == 0.0) return finish(0, 0.0, 0);

        double* r = c->ra;   // current residual
        double* rn = c->rb;  // next residual
        bool first = true;   // (re)start of the Krylov recurrence
        size_t stag_base = 0;  // stagnation is judged on the history since the last (re)start
        int k = 0;
        for (;;) {
            // ---- one outer iteration ------------------------------------------------
            int outcome = 0;
            if (o->outer == AMGG_OUTER_STATIONARY) {
                double* res = nullptr;
                R.ok(vec_copy<double>(n, x, L0.u64, st));
                ++R.vcycles;
                R.ok(vcycle_level<double>(c, 0, bb, L0.u64, L0.t64, first, o->nu1, o->nu2, st, &res));
                R.ok(vec_copy<double>(n, res, x, st));
                R.ok(csr_resid_norm(A, L0.val, x, bb, r, c->partial, st));
                R.ok(fcg_finish_rr(c->partial, s, st));
                first = false;
            } else if (o->outer == AMGG_OUTER_IR) {
                const double* e64 = R.precondition(r, nullptr);
                if (R.prec == 64)
                    R.ok(ir_update_f64(n, x, e64, st));
                else
                    R.ok(ir_update_f32(n, x, R.last32, s, st));
                R.ok(csr_resid_norm(A, L0.val, x, bb, r, c->partial, st));
                R.ok(fcg_finish_rr(c->partial, s, st));
            } else {
                if (first) {
                    // z0 = M r0, p0 = z0, gamma = z0.r0
                    const double* z = R.precondition(r, c->z);
                    if (R.prec == 32) {
                        R.ok(fcg_castback_dots(n, R.last32, s, r, nullptr, c->z, c->partial2, st));
                        z = c->z;
                    } else {
                        R.ok(fcg_dots64(n, z, r, nullptr, c->partial2, st));
                    }
                    R.ok(fcg_finish_beta(c->partial2, s, 1, st));
                    R.ok(fcg_update_p(n, z, c->p, s, 1, st));
                    first = false;
                }
                R.ok(csr_spmv_dot(A, L0.val, c->p, c->q, c->partial, st));
                R.ok(fcg_finish_pq(c->partial, s, st));
                R.ok(fcg_update_xr(n, x, c->p, r, c->q, rn, s, c->partial, st));
                R.ok(fcg_finish_rr(c->partial, s, st));
            }
            ++k;
            if (!R.read_scalars()) return hip_fail(R.e, "amgg_solve");
            const double rel = std::sqrt(hs[kRR]) / nb;
            hist.push_back(rel);
            const bool breakdown = hs[kFlag] != 0.0;
            if (rel <= o->tol && std::isfinite(rel) && !breakdown) {
                if (o->outer == AMGG_OUTER_FCG) std::swap(r, rn);
                return finish(0, rel, k);
            }
            if (!std::isfinite(rel) || rel > div_factor)
                outcome = AMGG_DIVERGED;
            else if (breakdown)
                outcome = AMGG_BREAKDOWN;
            else if (hist.size() - stag_base > static_cast<size_t>(stag_window) &&
                     rel > stag_ratio * hist[hist.size() - 1 - stag_window])
                outcome = AMGG_STAGNATED;
            if (outcome == 0 && k >= o->maxit) return finish(AMGG_MAXIT, rel, k);
            if (outcome != 0) {
                bool learned = false;
                for (int l = 0; l + 1 < c->nlevels; ++l) learned |= !c->lv[l].baseline;
                if (!o->fallback || inf.fell_back || !learned || k >= o->maxit) return finish(outcome, rel, k);
                // Jacobi fallback: the cycle stays a linear operator, so the iteration may
                // continue from the current x with the paper's baseline smoother.
                inf.fell_back = 1;
                set_all_jacobi(c, st);
                R.ok(vec_zero_bytes(s + kFlag, sizeof(double), st));
                if (!std::isfinite(rel)) R.ok(vec_zero_bytes(x, sizeof(double) * n, st));
                R.ok(csr_resid_norm(A, L0.val, x, bb, c->ra, c->partial, st));
                R.ok(fcg_finish_rr(c->partial, s, st));
                r = c->ra;
                rn = c->rb;
                first = true;
                stag_base = hist.size() - 1;
                continue;
            }
            if (o->outer == AMGG_OUTER_FCG) {
                // z = M r_new; beta = z.(r_new - r_old)/gamma; p = z + beta p
                const double* z = R.precondition(rn, c->z);
                if (R.prec == 32) {
                    R.ok(fcg_castback_dots(n, R.last32, s, rn, r, c->z, c->partial2, st));
                    z = c->z;
                } else {
                    R.ok(fcg_dots64(n, z, rn, r, c->partial2, st));
                }
                R.ok(fcg_finish_beta(c->partial2, s, 0, st));
                R.ok(fcg_update_p(n, z, c->p, s, 0, st));
                std::swap(r, rn);
            }
            if (R.e != hipSuccess) return hip_fail(R.e, "amgg_solve");
        }
    });
}
