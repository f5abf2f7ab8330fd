// Host-side classical Ruge-Stueben setup: strength, first-pass C/F splitting, direct
// interpolation and the Galerkin product (paper Sec. 2.2; Sec. 4: classical RS with
// strength threshold 0.25; App. B.1, Tab. 7: at most 10 levels; Alg. 1, step 2).
//
// Floating-point results must not depend on the compiler: this file is built with
// -ffp-contract=off and without fast-math, and every sum is accumulated left to right
// in ascending column order so that two independent implementations following the same
// statement of the method agree bit for bit.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "amggnn.h"
#include "errors.hpp"

namespace {

struct Csr {
    int32_t nrows = 0, ncols = 0;
    std::vector<int32_t> ptr, idx;
    std::vector<double> val;
    int32_t nnz() const { return static_cast<int32_t>(idx.size()); }
};

struct RsLevel {
    Csr A, P;
    std::vector<int8_t> cf;
};

// S_i = { j != i : -a_ij >= theta * max_{k != i}(-a_ik) }, empty when that max is <= 0.
Csr strong_couplings(const Csr& A, double theta) {
    Csr S;
    S.nrows = S.ncols = A.nrows;
    S.ptr.assign(A.nrows + 1, 0);
    S.idx.reserve(A.idx.size());
    for (int32_t i = 0; i < A.nrows; ++i) {
        double big = -INFINITY;
        bool any_off = false;
        for (int32_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) {
            if (A.idx[p] == i) continue;
            any_off = true;
            big = std::max(big, -A.val[p]);
        }
        if (any_off && big > 0.0) {
            const double cut = theta * big;
            for (int32_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p)
                if (A.idx[p] != i && -A.val[p] >= cut) S.idx.push_back(A.idx[p]);
        }
        S.ptr[i + 1] = static_cast<int32_t>(S.idx.size());
    }
    return S;
}

// Pattern transpose by counting sort; rows of the result come out in ascending order.
Csr pattern_transpose(const Csr& S) {
    Csr T;
    T.nrows = S.ncols;
    T.ncols = S.nrows;
    T.ptr.assign(T.nrows + 1, 0);
    for (int32_t j : S.idx) T.ptr[j + 1]++;
    for (int32_t c = 0; c < T.nrows; ++c) T.ptr[c + 1] += T.ptr[c];
    T.idx.resize(S.idx.size());
    if (!S.val.empty()) T.val.resize(S.idx.size());
    std::vector<int32_t> fill(T.ptr.begin(), T.ptr.end() - 1);
    for (int32_t i = 0; i < S.nrows; ++i)
        for (int32_t p = S.ptr[i]; p < S.ptr[i + 1]; ++p) {
            const int32_t dst = fill[S.idx[p]]++;
            T.idx[dst] = i;
            if (!S.val.empty()) T.val[dst] = S.val[p];
        }
    return T;
}

// Max tournament tree over the undecided points, 8 children per node (a node's children are one
// 64-byte line, and an 8M-point level is 8 levels deep instead of 23). A node holds the packed
// maximum (measure << 32 | ~index) of its range, so the root answers "largest lambda, smallest
// index" without looking anything up, and an update stops climbing as soon as a node keeps its
// value. Every level is padded to a multiple of 8 entries with the empty value.
class ArgmaxTree {
  public:
    explicit ArgmaxTree(const std::vector<int64_t>& key) {
        size_t count = key.size();
        std::vector<int64_t> leaf(pad8(count), kEmpty);
        for (size_t i = 0; i < count; ++i) leaf[i] = pack(key[i], static_cast<int32_t>(i));
        level_.push_back(std::move(leaf));
        while (count > 1) {
            count = (count + 7) / 8;
            const std::vector<int64_t>& below = level_.back();
            std::vector<int64_t> up(pad8(count), kEmpty);
            for (size_t v = 0; v < count; ++v) up[v] = max8(&below[8 * v]);
            level_.push_back(std::move(up));
        }
    }
    static constexpr int64_t kDecided = INT64_MIN;
    int32_t top() const {
        const int64_t t = level_.back()[0];
        return t == kEmpty ? -1 : static_cast<int32_t>(~static_cast<uint32_t>(t & 0xFFFFFFFFu));
    }
    void set(int32_t i, int64_t k) {
        size_t v = static_cast<size_t>(i);
        level_[0][v] = pack(k, i);
        for (size_t l = 1; l < level_.size(); ++l) {
            v >>= 3;
            const int64_t m = max8(&level_[l - 1][8 * v]);
            if (level_[l][v] == m) break;
            level_[l][v] = m;
        }
    }

  private:
    // measures are counts (|lambda| < 2^31); a decided point is below every measure
    static constexpr int64_t kEmpty = INT64_MIN;
    static int64_t pack(int64_t k, int32_t i) {
        if (k == kDecided) return kEmpty;
        return static_cast<int64_t>(static_cast<uint64_t>(k) << 32) | static_cast<int64_t>(~static_cast<uint32_t>(i));
    }
    static size_t pad8(size_t n) { return n <= 8 ? 8 : (n + 7) / 8 * 8; }  // the root level is never empty
    static int64_t max8(const int64_t* c) {
        const int64_t a = std::max(std::max(c[0], c[1]), std::max(c[2], c[3]));
        const int64_t b = std::max(std::max(c[4], c[5]), std::max(c[6], c[7]));
        return std::max(a, b);
    }
    std::vector<std::vector<int64_t>> level_;
};

// Ruge-Stueben first pass. Returns cf[i] = 1 for C points, 0 for F points.
std::vector<int8_t> first_pass_split(const Csr& S) {
    const int32_t n = S.nrows;
    const Csr ST = pattern_transpose(S);
    constexpr int8_t kUndecided = -1;
    std::vector<int8_t> mark(n, kUndecided);
    std::vector<int64_t> lambda(n);
    for (int32_t i = 0; i < n; ++i) {
        const int32_t out_deg = S.ptr[i + 1] - S.ptr[i];
        const int32_t in_deg = ST.ptr[i + 1] - ST.ptr[i];
        lambda[i] = in_deg;
        if (out_deg == 0 && in_deg == 0) mark[i] = 0;  // isolated: F without interpolation
    }
    std::vector<int64_t> key(n);
    for (int32_t i = 0; i < n; ++i) key[i] = mark[i] == kUndecided ? lambda[i] : ArgmaxTree::kDecided;
    ArgmaxTree tree(key);
    std::vector<int32_t> fresh;
    for (int32_t i = tree.top(); i >= 0; i = tree.top()) {
        mark[i] = 1;
        tree.set(i, ArgmaxTree::kDecided);
        fresh.clear();
        for (int32_t p = ST.ptr[i]; p < ST.ptr[i + 1]; ++p) {
            const int32_t j = ST.idx[p];
            if (mark[j] == kUndecided) {
                mark[j] = 0;
                tree.set(j, ArgmaxTree::kDecided);
                fresh.push_back(j);
            }
        }
        for (int32_t j : fresh)
            for (int32_t p = S.ptr[j]; p < S.ptr[j + 1]; ++p) {
                const int32_t k = S.idx[p];
                if (mark[k] == kUndecided) tree.set(k, ++lambda[k]);
            }
        for (int32_t p = S.ptr[i]; p < S.ptr[i + 1]; ++p) {
            const int32_t k = S.idx[p];
            if (mark[k] == kUndecided) tree.set(k, --lambda[k]);
        }
    }
    std::vector<int8_t> cf(n);
    for (int32_t i = 0; i < n; ++i) cf[i] = mark[i] == 1 ? 1 : 0;
    return cf;
}

// Direct interpolation with positive couplings lumped on the diagonal.
Csr direct_interp(const Csr& A, const Csr& S, const std::vector<int8_t>& cf) {
    const int32_t n = A.nrows;
    std::vector<int32_t> coarse_id(n, -1);
    int32_t nc = 0;
    for (int32_t i = 0; i < n; ++i)
        if (cf[i]) coarse_id[i] = nc++;
    Csr P;
    P.nrows = n;
    P.ncols = nc;
    P.ptr.assign(n + 1, 0);
    P.idx.reserve(S.idx.size() + n);
    P.val.reserve(S.idx.size() + n);
    std::vector<char> in_ci(n, 0);
    for (int32_t i = 0; i < n; ++i) {
        if (cf[i]) {
            P.idx.push_back(coarse_id[i]);
            P.val.push_back(1.0);
            P.ptr[i + 1] = P.nnz();
            continue;
        }
        bool any = false;
        for (int32_t p = S.ptr[i]; p < S.ptr[i + 1]; ++p)
            if (cf[S.idx[p]]) {
                in_ci[S.idx[p]] = 1;
                any = true;
            }
        if (any) {
            double a_ii = 0.0;
            for (int32_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p)
                if (A.idx[p] == i) a_ii = A.val[p];
            double lumped = a_ii, neg_sum = 0.0, strong_c_sum = 0.0;
            for (int32_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) {
                const int32_t k = A.idx[p];
                if (k == i) continue;
                const double a = A.val[p];
                if (a > 0.0) lumped = lumped + a;
                if (a < 0.0) neg_sum = neg_sum + a;
                if (in_ci[k]) strong_c_sum = strong_c_sum + a;
            }
            const double ratio = neg_sum / strong_c_sum;
            for (int32_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) {
                const int32_t k = A.idx[p];
                if (!in_ci[k]) continue;
                P.idx.push_back(coarse_id[k]);
                P.val.push_back(-(ratio * A.val[p]) / lumped);
            }
            for (int32_t p = S.ptr[i]; p < S.ptr[i + 1]; ++p) in_ci[S.idx[p]] = 0;
        }
        P.ptr[i + 1] = P.nnz();
    }
    return P;
}

// C = L * Rm, one row at a time with a dense accumulator: for row i walk L's entries in
// ascending column order and, for each, Rm's row in ascending order; every structurally
// generated entry is kept.
Csr multiply_rowwise(const Csr& L, const Csr& Rm) {
    Csr C;
    C.nrows = L.nrows;
    C.ncols = Rm.ncols;
    C.ptr.assign(L.nrows + 1, 0);
    std::vector<double> acc(Rm.ncols, 0.0);
    std::vector<int32_t> seen(Rm.ncols, -1);
    std::vector<int32_t> cols;
    for (int32_t i = 0; i < L.nrows; ++i) {
        cols.clear();
        for (int32_t p = L.ptr[i]; p < L.ptr[i + 1]; ++p) {
            const int32_t j = L.idx[p];
            const double a = L.val[p];
            for (int32_t q = Rm.ptr[j]; q < Rm.ptr[j + 1]; ++q) {
                const int32_t k = Rm.idx[q];
                if (seen[k] != i) {
                    seen[k] = i;
                    acc[k] = 0.0;
                    cols.push_back(k);
                }
                acc[k] = acc[k] + a * Rm.val[q];
            }
        }
        std::sort(cols.begin(), cols.end());
        for (int32_t k : cols) {
            C.idx.push_back(k);
            C.val.push_back(acc[k]);
        }
        C.ptr[i + 1] = C.nnz();
    }
    return C;
}

Csr galerkin_product(const Csr& A, const Csr& P) {
    const Csr AP = multiply_rowwise(A, P);
    const Csr R = pattern_transpose(P);
    const Csr G = multiply_rowwise(R, AP);
    Csr Ac;
    Ac.nrows = G.nrows;
    Ac.ncols = G.ncols;
    Ac.ptr.assign(G.nrows + 1, 0);
    for (int32_t i = 0; i < G.nrows; ++i) {
        for (int32_t p = G.ptr[i]; p < G.ptr[i + 1]; ++p)
            if (G.val[p] != 0.0 || G.idx[p] == i) {
                Ac.idx.push_back(G.idx[p]);
                Ac.val.push_back(G.val[p]);
            }
        Ac.ptr[i + 1] = Ac.nnz();
    }
    return Ac;
}

bool check_pattern(const int32_t* rowptr, const int32_t* col, const double* val, int32_t n, std::string* why) {
    if (rowptr[0] != 0) return *why = "rowptr[0] != 0", false;
    for (int32_t i = 0; i < n; ++i) {
        if (rowptr[i + 1] < rowptr[i]) return *why = "rowptr not monotone", false;
        bool diag = false;
        for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            if (col[p] < 0 || col[p] >= n) return *why = "column out of range", false;
            if (p > rowptr[i] && col[p] <= col[p - 1]) return *why = "columns not strictly ascending", false;
            if (!std::isfinite(val[p])) return *why = "non-finite value", false;
            if (col[p] == i) {
                diag = true;
                if (!(val[p] > 0.0)) return *why = "diagonal must be positive", false;
            }
        }
        if (!diag) return *why = "diagonal entry missing in row " + std::to_string(i), false;
    }
    return true;
}

}  // namespace

struct amgg_rs {
    std::vector<RsLevel> levels;
    int singular = 0;
    double theta = 0.25;
    int max_levels = 1;
    int32_t max_coarse = 1;
    bool open = false;   // the last level has P and awaits its Galerkin product
    bool done = false;   // coarsening stopped: the last level is the coarsest
    bool split = false;  // the last level has its C/F split (amgg_rs_split) and awaits P
};

namespace {

int begin_impl(const char* who, const int32_t* rowptr, const int32_t* col, const double* val, int32_t n,
               double theta, int max_levels, int32_t max_coarse, amgg_rs** out) {
    const std::string w(who);
    if (!out || !rowptr || n <= 0 || (!col && rowptr[n] > 0) || (!val && rowptr[n] > 0))
        return amgg::fail(AMGG_EINVAL, w + ": null argument or n <= 0");
    if (!(theta > 0.0 && theta < 1.0) || max_levels < 1 || max_levels > AMGG_MAX_LEVELS || max_coarse < 1)
        return amgg::fail(AMGG_EINVAL, w + ": theta, max_levels or max_coarse out of range");
    std::string why;
    if (!check_pattern(rowptr, col, val, n, &why)) return amgg::fail(AMGG_EINVAL, w + ": " + why);
    auto* h = new amgg_rs();
    h->theta = theta;
    h->max_levels = max_levels;
    h->max_coarse = max_coarse;
    RsLevel top;
    top.A.nrows = top.A.ncols = n;
    top.A.ptr.assign(rowptr, rowptr + n + 1);
    top.A.idx.assign(col, col + rowptr[n]);
    top.A.val.assign(val, val + rowptr[n]);
    // all-Neumann detection: every row sums to zero relative to its diagonal
    h->singular = 1;
    for (int32_t i = 0; i < n && h->singular; ++i) {
        double s = 0.0, d = 0.0;
        for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            s += val[p];
            if (col[p] == i) d = val[p];
        }
        if (!(std::fabs(s) <= 1e-12 * d)) h->singular = 0;
    }
    h->levels.push_back(std::move(top));
    *out = h;
    return AMGG_OK;
}

// The stopping rules that do not need the split: level count and size.
bool may_coarsen(const amgg_rs* h) {
    return static_cast<int>(h->levels.size()) < h->max_levels && h->levels.back().A.nrows > h->max_coarse;
}

// ... and the ones that do: no C point, or too few rows dropped.
bool split_pays(const std::vector<int8_t>& cf) {
    int64_t nc = 0;
    for (int8_t c : cf) nc += c;
    return nc > 0 && 10 * nc <= 9 * static_cast<int64_t>(cf.size());
}

// Strength, C/F split and interpolation of the last level, or the decision to stop there.
bool coarsen_last(amgg_rs* h) {
    RsLevel& cur = h->levels.back();
    if (!may_coarsen(h)) return false;
    Csr S = strong_couplings(cur.A, h->theta);
    std::vector<int8_t> cf = first_pass_split(S);
    if (!split_pays(cf)) return false;
    cur.P = direct_interp(cur.A, S, cf);
    cur.cf = std::move(cf);
    return true;
}

// S of a matrix from one strength flag per stored entry (in stored order).
Csr couplings_from_flags(const Csr& A, const uint8_t* strong) {
    Csr S;
    S.nrows = S.ncols = A.nrows;
    S.ptr.assign(static_cast<size_t>(A.nrows) + 1, 0);
    int32_t cnt = 0;
    for (int32_t i = 0; i < A.nrows; ++i) {
        for (int32_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) cnt += strong[p] ? 1 : 0;
        S.ptr[i + 1] = cnt;
    }
    S.idx.resize(static_cast<size_t>(cnt));
    int32_t q = 0;
    for (int32_t p = 0; p < A.nnz(); ++p)
        if (strong[p]) S.idx[q++] = A.idx[p];
    return S;
}

}  // namespace

extern "C" int amgg_rs_setup(const int32_t* rowptr, const int32_t* col, const double* val, int32_t n,
                             double theta, int max_levels, int32_t max_coarse, amgg_rs** out) {
    return amgg::guarded([&]() -> int {
        amgg_rs* h = nullptr;
        const int rc = begin_impl("amgg_rs_setup", rowptr, col, val, n, theta, max_levels, max_coarse, &h);
        if (rc != AMGG_OK) return rc;
        try {
            while (coarsen_last(h)) {
                RsLevel next;
                next.A = galerkin_product(h->levels.back().A, h->levels.back().P);
                h->levels.push_back(std::move(next));
            }
        } catch (...) {
            delete h;
            throw;
        }
        h->done = true;
        *out = h;
        return AMGG_OK;
    });
}

extern "C" int amgg_rs_begin(const int32_t* rowptr, const int32_t* col, const double* val, int32_t n,
                             double theta, int max_levels, int32_t max_coarse, amgg_rs** out) {
    return amgg::guarded(
        [&]() -> int { return begin_impl("amgg_rs_begin", rowptr, col, val, n, theta, max_levels, max_coarse, out); });
}

extern "C" int amgg_rs_coarsen(amgg_rs* h, int* more) {
    return amgg::guarded([&]() -> int {
        if (!h || !more) return amgg::fail(AMGG_EINVAL, "amgg_rs_coarsen: null argument");
        if (h->open) return amgg::fail(AMGG_ESTATE, "amgg_rs_coarsen: the last level still needs its coarse matrix");
        if (h->split) return amgg::fail(AMGG_ESTATE, "amgg_rs_coarsen: the last level awaits its interpolation");
        if (h->done) {
            *more = 0;
            return AMGG_OK;
        }
        h->open = coarsen_last(h);
        h->done = !h->open;
        *more = h->open ? 1 : 0;
        return AMGG_OK;
    });
}

extern "C" int amgg_rs_split(amgg_rs* h, const uint8_t* strong, int8_t* cf_out, int* more) {
    return amgg::guarded([&]() -> int {
        if (!h || !more) return amgg::fail(AMGG_EINVAL, "amgg_rs_split: null argument");
        if (h->open) return amgg::fail(AMGG_ESTATE, "amgg_rs_split: the last level still needs its coarse matrix");
        if (h->split) return amgg::fail(AMGG_ESTATE, "amgg_rs_split: the last level awaits its interpolation");
        *more = 0;
        if (h->done) return AMGG_OK;
        if (!may_coarsen(h)) {
            h->done = true;
            return AMGG_OK;
        }
        if (!strong) {  // query: the level is to be coarsened, its strength flags are wanted
            *more = 1;
            return AMGG_OK;
        }
        if (!cf_out) return amgg::fail(AMGG_EINVAL, "amgg_rs_split: null cf");
        RsLevel& cur = h->levels.back();
        std::vector<int8_t> cf = first_pass_split(couplings_from_flags(cur.A, strong));
        if (!split_pays(cf)) {
            h->done = true;
            return AMGG_OK;
        }
        std::memcpy(cf_out, cf.data(), cf.size());
        cur.cf = std::move(cf);
        h->split = true;
        *more = 1;
        return AMGG_OK;
    });
}

extern "C" int amgg_rs_push_interp(amgg_rs* h, int32_t nc, const int32_t* rowptr, const int32_t* col,
                                   const double* val) {
    return amgg::guarded([&]() -> int {
        if (!h || !rowptr) return amgg::fail(AMGG_EINVAL, "amgg_rs_push_interp: null argument");
        if (!h->split) return amgg::fail(AMGG_ESTATE, "amgg_rs_push_interp: no level awaits its interpolation");
        RsLevel& cur = h->levels.back();
        const int32_t n = cur.A.nrows;
        int32_t want = 0;
        for (int8_t c : cur.cf) want += c;
        if (nc != want) return amgg::fail(AMGG_EINVAL, "amgg_rs_push_interp: column count differs from the C points");
        const int32_t nnz = rowptr[n];
        if (rowptr[0] != 0 || nnz < 0 || ((!col || !val) && nnz > 0))
            return amgg::fail(AMGG_EINVAL, "amgg_rs_push_interp: bad row pointers or null col / val");
        for (int32_t i = 0; i < n; ++i) {
            if (rowptr[i + 1] < rowptr[i]) return amgg::fail(AMGG_EINVAL, "amgg_rs_push_interp: decreasing row pointers");
            for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p)
                if (col[p] < 0 || col[p] >= nc || (p > rowptr[i] && col[p] <= col[p - 1]))
                    return amgg::fail(AMGG_EINVAL, "amgg_rs_push_interp: columns out of range or not ascending");
        }
        cur.P.nrows = n;
        cur.P.ncols = nc;
        cur.P.ptr.assign(rowptr, rowptr + n + 1);
        cur.P.idx.assign(col, col + nnz);
        cur.P.val.assign(val, val + nnz);
        h->split = false;
        h->open = true;
        return AMGG_OK;
    });
}

extern "C" int amgg_rs_galerkin(amgg_rs* h) {
    return amgg::guarded([&]() -> int {
        if (!h) return amgg::fail(AMGG_EINVAL, "amgg_rs_galerkin: null handle");
        if (!h->open) return amgg::fail(AMGG_ESTATE, "amgg_rs_galerkin: no level awaits its coarse matrix");
        RsLevel next;
        next.A = galerkin_product(h->levels.back().A, h->levels.back().P);
        h->levels.push_back(std::move(next));
        h->open = false;
        return AMGG_OK;
    });
}

extern "C" int amgg_rs_push_level(amgg_rs* h, int32_t n, const int32_t* rowptr, const int32_t* col,
                                  const double* val) {
    return amgg::guarded([&]() -> int {
        if (!h || !rowptr || n <= 0) return amgg::fail(AMGG_EINVAL, "amgg_rs_push_level: null argument or n <= 0");
        if (!h->open) return amgg::fail(AMGG_ESTATE, "amgg_rs_push_level: no level awaits its coarse matrix");
        if (n != h->levels.back().P.ncols)
            return amgg::fail(AMGG_EINVAL, "amgg_rs_push_level: row count differs from the coarse point count");
        const int32_t nnz = rowptr[n];
        if ((!col || !val) && nnz > 0) return amgg::fail(AMGG_EINVAL, "amgg_rs_push_level: null col or val");
        std::string why;
        if (!check_pattern(rowptr, col, val, n, &why)) return amgg::fail(AMGG_EINVAL, "amgg_rs_push_level: " + why);
        RsLevel next;
        next.A.nrows = next.A.ncols = n;
        next.A.ptr.assign(rowptr, rowptr + n + 1);
        next.A.idx.assign(col, col + nnz);
        next.A.val.assign(val, val + nnz);
        h->levels.push_back(std::move(next));
        h->open = false;
        return AMGG_OK;
    });
}

extern "C" int amgg_rs_info(const amgg_rs* h, int* nlevels, int* singular) {
    if (!h) return amgg::fail(AMGG_EINVAL, "amgg_rs_info: null handle");
    if (nlevels) *nlevels = static_cast<int>(h->levels.size());
    if (singular) *singular = h->singular;
    return AMGG_OK;
}

extern "C" int amgg_rs_level_size(const amgg_rs* h, int lvl, int32_t* n, int32_t* nnz, int32_t* p_ncols,
                                  int32_t* p_nnz) {
    if (!h || lvl < 0 || lvl >= static_cast<int>(h->levels.size()))
        return amgg::fail(AMGG_EINVAL, "amgg_rs_level_size: bad handle or level");
    const RsLevel& L = h->levels[lvl];
    if (n) *n = L.A.nrows;
    if (nnz) *nnz = L.A.nnz();
    if (p_ncols) *p_ncols = L.P.ncols;
    if (p_nnz) *p_nnz = L.P.nnz();
    return AMGG_OK;
}

extern "C" int amgg_rs_copy_level(const amgg_rs* h, int lvl, int32_t* rowptr, int32_t* col, double* val,
                                  int32_t* p_rowptr, int32_t* p_col, double* p_val, int8_t* cf) {
    if (!h || lvl < 0 || lvl >= static_cast<int>(h->levels.size()))
        return amgg::fail(AMGG_EINVAL, "amgg_rs_copy_level: bad handle or level");
    const RsLevel& L = h->levels[lvl];
    if (rowptr) std::memcpy(rowptr, L.A.ptr.data(), sizeof(int32_t) * L.A.ptr.size());
    if (col) std::memcpy(col, L.A.idx.data(), sizeof(int32_t) * L.A.idx.size());
    if (val) std::memcpy(val, L.A.val.data(), sizeof(double) * L.A.val.size());
    const bool has_p = !L.P.ptr.empty();
    if (has_p) {
        if (p_rowptr) std::memcpy(p_rowptr, L.P.ptr.data(), sizeof(int32_t) * L.P.ptr.size());
        if (p_col) std::memcpy(p_col, L.P.idx.data(), sizeof(int32_t) * L.P.idx.size());
        if (p_val) std::memcpy(p_val, L.P.val.data(), sizeof(double) * L.P.val.size());
    }
    if (cf) {
        if (has_p)
            std::memcpy(cf, L.cf.data(), L.cf.size());
        else
            std::memset(cf, 0, L.A.nrows);
    }
    return AMGG_OK;
}

extern "C" void amgg_rs_free(amgg_rs* h) { delete h; }

extern "C" int amgg_rs_setup_query(const int32_t* rowptr, const int32_t* col, const double* val, int32_t n,
                                   double theta, int max_levels, int32_t max_coarse, amgg_hier_sizes* sizes_out) {
    return amgg::guarded([&]() -> int {
        if (!sizes_out) return amgg::fail(AMGG_EINVAL, "amgg_rs_setup_query: null sizes");
        amgg_rs* h = nullptr;
        const int rc = amgg_rs_setup(rowptr, col, val, n, theta, max_levels, max_coarse, &h);
        if (rc != AMGG_OK) return rc;
        amgg_hier_sizes z{};
        z.nlevels = static_cast<int>(h->levels.size());
        z.singular = h->singular;
        for (int l = 0; l < z.nlevels; ++l) {
            const RsLevel& L = h->levels[l];
            z.n[l] = L.A.nrows;
            z.nnz[l] = L.A.nnz();
            z.p_ncols[l] = L.P.ncols;
            z.p_nnz[l] = L.P.nnz();
        }
        *sizes_out = z;
        amgg_rs_free(h);
        return AMGG_OK;
    });
}

extern "C" int amgg_rs_setup_fill(const int32_t* rowptr, const int32_t* col, const double* val, int32_t n,
                                  double theta, int max_levels, int32_t max_coarse, const amgg_hier_host* out) {
    return amgg::guarded([&]() -> int {
        if (!out) return amgg::fail(AMGG_EINVAL, "amgg_rs_setup_fill: null output");
        amgg_rs* h = nullptr;
        const int rc = amgg_rs_setup(rowptr, col, val, n, theta, max_levels, max_coarse, &h);
        if (rc != AMGG_OK) return rc;
        const int nl = static_cast<int>(h->levels.size());
        for (int l = 0; l < nl; ++l) {
            const bool coarsest = l + 1 == nl;
            if (!out->rowptr[l] || !out->col[l] || !out->val[l] ||
                (!coarsest && (!out->p_rowptr[l] || !out->p_col[l] || !out->p_val[l]))) {
                amgg_rs_free(h);
                return amgg::fail(AMGG_EINVAL, "amgg_rs_setup_fill: null array for level " + std::to_string(l));
            }
            amgg_rs_copy_level(h, l, out->rowptr[l], out->col[l], out->val[l], coarsest ? nullptr : out->p_rowptr[l],
                               coarsest ? nullptr : out->p_col[l], coarsest ? nullptr : out->p_val[l], out->cf[l]);
        }
        amgg_rs_free(h);
        return AMGG_OK;
    });
}
