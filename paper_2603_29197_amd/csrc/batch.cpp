// Batches of problems on one sparsity pattern (qg_setup_batch): the k
// problems are stacked into one separable problem whose KKT matrix is a
// symmetric permutation of diag(K_1, ..., K_k), and the analysis of one
// problem (paper Sec. 2.2, reused when only values change, Sec. 3.2) is
// replicated k times instead of being recomputed on the stack.
//
// Stacked index layout: x = (x_1, .., x_k), y = (y_1, .., y_k); the cone rows
// keep the orthant first, so z holds the orthant rows of every problem
// (problem by problem), then the cone rows of every problem.
#include "batch.hpp"

#include <algorithm>

namespace qg {

int64_t StackMap::kkt(int32_t i, int32_t v) const {
    if (v < n) return (int64_t)i * n + v;
    if (v < n + p) return (int64_t)k * n + (int64_t)i * p + (v - n);
    return (int64_t)k * (n + p) + zrow(i, v - n - p);
}

int64_t StackMap::zrow(int32_t i, int32_t w) const {
    if (w < l) return (int64_t)i * l + w;
    return (int64_t)k * l + (int64_t)i * (m - l) + (w - l);
}

// Copy i of column t of one problem's analysis is column i N1 + t of the stack
// (the stack's pivot order takes the problems one after another).
void replicate_symbolic(const Symbolic &a, const StackMap &mp, Symbolic &out) {
    const int32_t k = mp.k, N1 = a.N;
    const int32_t ns1 = a.super_ptr.empty() ? 0 : (int32_t)a.super_ptr.size() - 1;
    out = Symbolic();
    out.N = k * N1;
    if (!a.perm.empty()) {
        out.perm.resize((size_t)out.N);
        out.iperm.resize((size_t)out.N);
        for (int32_t i = 0; i < k; ++i)
            for (int32_t t = 0; t < N1; ++t) {
                const int32_t v = (int32_t)mp.kkt(i, a.perm[t]);
                out.perm[(size_t)i * N1 + t] = v;
                out.iperm[(size_t)v] = i * N1 + t;
            }
    }
    if (!a.parent.empty()) {
        out.parent.resize((size_t)out.N);
        for (int32_t i = 0; i < k; ++i)
            for (int32_t t = 0; t < N1; ++t)
                out.parent[(size_t)i * N1 + t] = a.parent[t] < 0 ? -1 : i * N1 + a.parent[t];
    }
    if (!a.colcount.empty())
        for (int32_t i = 0; i < k; ++i) out.colcount.insert(out.colcount.end(), a.colcount.begin(), a.colcount.end());
    auto tile_ptr = [&](const std::vector<int32_t> &v, std::vector<int32_t> &o) {
        if (v.empty()) return;
        for (int32_t i = 0; i < k; ++i)
            for (size_t t = 0; t + 1 < v.size(); ++t) o.push_back(v[t] + i * N1);
        o.push_back(k * N1);
    };
    tile_ptr(a.super_fund, out.super_fund);
    tile_ptr(a.super_ptr, out.super_ptr);
    if (!a.rows_ptr.empty()) {
        const int64_t nr = a.rows_ptr.back();
        for (int32_t i = 0; i < k; ++i)
            for (int32_t s = 0; s < ns1; ++s) out.rows_ptr.push_back(a.rows_ptr[s] + i * nr);
        out.rows_ptr.push_back(k * nr);
        out.rows.reserve((size_t)(k * nr));
        for (int32_t i = 0; i < k; ++i)
            for (int32_t v : a.rows) out.rows.push_back(v + i * N1);
    }
    for (int32_t i = 0; i < k; ++i)
        for (int32_t s = 0; s < (int32_t)a.sn_parent.size(); ++s)
            out.sn_parent.push_back(a.sn_parent[s] < 0 ? -1 : a.sn_parent[s] + i * ns1);
    for (int32_t i = 0; i < k; ++i) out.sn_level.insert(out.sn_level.end(), a.sn_level.begin(), a.sn_level.end());
    out.nlevels = a.nlevels;
    out.nnz_L = a.nnz_L * k;
    out.flops = a.flops * k;
}

// Block-diagonal stack of one CSC pattern with k value sets (vals: k x nnz, problem by problem);
// row i of copy c becomes rowmap(c, i), column j becomes c ncol + j.
template <typename RowMap>
static void stack_csc(const qg_csc &M, int32_t k, int32_t nrow_out, RowMap rowmap, StackedCsc &out) {
    const int64_t nnz = M.colptr[M.ncol];
    out.colptr.assign((size_t)k * M.ncol + 1, 0);
    out.rowind.resize((size_t)(k * nnz));
    out.val.resize((size_t)(k * nnz));
    int64_t pos = 0;
    for (int32_t c = 0; c < k; ++c)
        for (int32_t j = 0; j < M.ncol; ++j) {
            for (int64_t t = M.colptr[j]; t < M.colptr[j + 1]; ++t) {
                out.rowind[(size_t)pos] = (int32_t)rowmap(c, M.rowind[t]);
                out.val[(size_t)pos] = M.val[(size_t)(c * nnz + t)];
                ++pos;
            }
            out.colptr[(size_t)c * M.ncol + j + 1] = pos;
        }
    out.csc = {nrow_out, k * M.ncol, out.colptr.data(), out.rowind.data(), out.val.data()};
}

void stack_problem(const StackMap &mp, const qg_csc *P, const qg_csc *A, const qg_csc *G, StackedCsc &Ps,
                   StackedCsc &As, StackedCsc &Gs) {
    const int32_t k = mp.k;
    if (P) stack_csc(*P, k, k * mp.n, [&](int32_t c, int32_t i) { return (int64_t)c * mp.n + i; }, Ps);
    if (A) stack_csc(*A, k, k * mp.p, [&](int32_t c, int32_t i) { return (int64_t)c * mp.p + i; }, As);
    if (G) stack_csc(*G, k, k * mp.m, [&](int32_t c, int32_t i) { return mp.zrow(c, i); }, Gs);
}

}  // namespace qg
