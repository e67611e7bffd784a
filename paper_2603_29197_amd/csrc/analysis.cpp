// Host analysis of the KKT pattern (paper Sec. 2.2: reordering, permutation
// and symbolic factorization, executed once per sparsity pattern and reused
// while only values change, Sec. 3.2).
//
// The integers produced here follow one fully specified rule so that an
// independent implementation can reproduce them bit for bit:
//  1. graph = off-diagonal pattern of K (eq. 2), both triangles;
//  2. nodes of degree > max(16, floor(10 sqrt(N))) are ordered last, by index;
//  3. minimum degree on the quotient graph with supervariables (merged into
//     the smallest index when their variable and element lists coincide
//     among the pivot's neighbours), mass elimination, element absorption,
//     and the approximate external degree bound of Amestoy, Davis and Duff
//     (no aggressive absorption); pivot = least (degree, index);
//  4. postorder of the elimination tree of that order (children and roots
//     by increasing index), composed with it;
//  5. elimination tree and column counts of the final order;
//  6. fundamental supernodes (parent[j] = j+1, colcount[j] = colcount[j+1]+1,
//     j the only child of j+1);
//  7. relaxed supernodes: a group G absorbs the next supernode T when T holds
//     G's parent column and the merged block has zeros <= 0.1 stored or
//     (width <= 8 and zeros <= 64), stored = w r - w(w-1)/2 with
//     r = width(G) + colcount[first(T)];
//  8. row list of a supernode = its columns followed by the rows below it.
#include "analysis.hpp"
#include "workpool.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <numeric>
#include <set>
#include <stdexcept>
#include <utility>

namespace qg {

static int check_csc(const qg_csc *M, int32_t nrow, int32_t ncol, bool upper, bool need_values,
                     CscData &out) {
    out.nrow = nrow;
    out.ncol = ncol;
    out.colptr.assign((size_t)ncol + 1, 0);
    out.rowind.clear();
    out.val.clear();
    if (M == nullptr) return QG_OK;
    if (M->nrow != nrow || M->ncol != ncol) return QG_ERR_ARG;
    if (ncol > 0 && (M->colptr == nullptr)) return QG_ERR_ARG;
    if (ncol == 0) return QG_OK;
    if (M->colptr[0] != 0) return QG_ERR_PATTERN;
    for (int32_t j = 0; j < ncol; ++j)
        if (M->colptr[j + 1] < M->colptr[j]) return QG_ERR_PATTERN;
    int64_t nnz = M->colptr[ncol];
    if (nnz > 0 && M->rowind == nullptr) return QG_ERR_ARG;
    if (nnz > 0 && need_values && M->val == nullptr) return QG_ERR_ARG;
    for (int32_t j = 0; j < ncol; ++j) {
        for (int64_t t = M->colptr[j]; t < M->colptr[j + 1]; ++t) {
            int32_t i = M->rowind[t];
            if (i < 0 || i >= nrow) return QG_ERR_PATTERN;
            if (t > M->colptr[j] && i <= M->rowind[t - 1]) return QG_ERR_PATTERN;
            if (upper && i > j) return QG_ERR_PATTERN;
            if (need_values && !std::isfinite(M->val[t])) return QG_ERR_NONFINITE;
        }
    }
    out.colptr.assign(M->colptr, M->colptr + ncol + 1);
    out.rowind.assign(M->rowind, M->rowind + nnz);
    if (need_values && nnz > 0) out.val.assign(M->val, M->val + nnz);
    else out.val.assign((size_t)nnz, 0.0);
    return QG_OK;
}

int build_problem_pattern(ProblemPattern &pp, int32_t n, int32_t m, int32_t p,
                          const qg_csc *P, const qg_csc *A, const qg_csc *G,
                          int32_t l, int32_t nsoc, const int32_t *q, bool need_values) {
    if (n <= 0 || m < 0 || p < 0 || l < 0 || nsoc < 0) return QG_ERR_ARG;
    if (nsoc > 0 && q == nullptr) return QG_ERR_ARG;
    if (p > 0 && A == nullptr) return QG_ERR_ARG;
    if (m > 0 && G == nullptr) return QG_ERR_ARG;
    int64_t tot = l;
    for (int32_t k = 0; k < nsoc; ++k) {
        if (q[k] < 1) return QG_ERR_ARG;
        tot += q[k];
    }
    if (tot != m) return QG_ERR_ARG;
    if ((int64_t)n + p + m > (int64_t)INT32_MAX / 2) return QG_ERR_ARG;
    pp.n = n; pp.m = m; pp.p = p; pp.l = l; pp.nsoc = nsoc;
    pp.q.assign(q, q + nsoc);
    pp.soc_off.assign((size_t)nsoc + 1, l);
    for (int32_t k = 0; k < nsoc; ++k) pp.soc_off[k + 1] = pp.soc_off[k] + q[k];
    int rc;
    if ((rc = check_csc(P, n, n, true, need_values, pp.P)) != QG_OK) return rc;
    if ((rc = check_csc(A, p, n, false, need_values, pp.A)) != QG_OK) return rc;
    if ((rc = check_csc(G, m, n, false, need_values, pp.G)) != QG_OK) return rc;
    return QG_OK;
}

// Row-wise (transposed) structure of a CSC matrix: for each row, its columns
// (increasing) and the CSC position of each entry.
static void transpose_index(const CscData &M, std::vector<int64_t> &rp, std::vector<int32_t> &rc,
                            std::vector<int64_t> &rpos) {
    rp.assign((size_t)M.nrow + 1, 0);
    for (int32_t i : M.rowind) rp[i + 1]++;
    for (int32_t i = 0; i < M.nrow; ++i) rp[i + 1] += rp[i];
    rc.resize(M.rowind.size());
    rpos.resize(M.rowind.size());
    std::vector<int64_t> fill(rp.begin(), rp.end() - 1);
    for (int32_t j = 0; j < M.ncol; ++j)
        for (int64_t t = M.colptr[j]; t < M.colptr[j + 1]; ++t) {
            int64_t d = fill[M.rowind[t]]++;
            rc[d] = j;
            rpos[d] = t;
        }
}

void build_kkt_pattern(const ProblemPattern &pp, KktPattern &kp) {
    const int32_t n = pp.n, p = pp.p, m = pp.m, N = n + p + m;
    kp.N = N;
    kp.Kp.assign((size_t)N + 1, 0);
    kp.Ki.clear();
    kp.posP.assign(pp.P.rowind.size(), -1);
    kp.posA.assign(pp.A.rowind.size(), -1);
    kp.posG.assign(pp.G.rowind.size(), -1);
    kp.diag.assign((size_t)N, -1);
    kp.blk33.clear();
    kp.blk33_off.assign((size_t)pp.nsoc + 1, 0);
    std::vector<int64_t> Arp, Grp, Apos, Gpos;
    std::vector<int32_t> Arc, Grc;
    transpose_index(pp.A, Arp, Arc, Apos);
    transpose_index(pp.G, Grp, Grc, Gpos);
    // columns 0..n-1: P's upper column, then the diagonal if P lacks it
    for (int32_t j = 0; j < n; ++j) {
        bool has_diag = false;
        for (int64_t t = pp.P.colptr[j]; t < pp.P.colptr[j + 1]; ++t) {
            int32_t i = pp.P.rowind[t];
            kp.posP[t] = (int64_t)kp.Ki.size();
            if (i == j) { has_diag = true; kp.diag[j] = (int64_t)kp.Ki.size(); }
            kp.Ki.push_back(i);
        }
        if (!has_diag) { kp.diag[j] = (int64_t)kp.Ki.size(); kp.Ki.push_back(j); }
        kp.Kp[j + 1] = (int64_t)kp.Ki.size();
    }
    // columns n..n+p-1: row i of A (transposed), then the diagonal
    for (int32_t i = 0; i < p; ++i) {
        int32_t j = n + i;
        for (int64_t t = Arp[i]; t < Arp[i + 1]; ++t) {
            kp.posA[Apos[t]] = (int64_t)kp.Ki.size();
            kp.Ki.push_back(Arc[t]);
        }
        kp.diag[j] = (int64_t)kp.Ki.size();
        kp.Ki.push_back(j);
        kp.Kp[j + 1] = (int64_t)kp.Ki.size();
    }
    // columns n+p..: row i of G, then the (3,3) block column
    std::vector<int64_t> soc_pos;   // per SOC, per local column b: start of its a = 0..b entries
    int32_t cone = 0;
    for (int32_t i = 0; i < m; ++i) {
        int32_t j = n + p + i;
        for (int64_t t = Grp[i]; t < Grp[i + 1]; ++t) {
            kp.posG[Gpos[t]] = (int64_t)kp.Ki.size();
            kp.Ki.push_back(Grc[t]);
        }
        if (i < pp.l) {
            kp.diag[j] = (int64_t)kp.Ki.size();
            kp.Ki.push_back(j);
        } else {
            while (i >= pp.soc_off[cone + 1]) ++cone;
            int32_t off = pp.soc_off[cone];
            for (int32_t a = off; a <= i; ++a) {
                if (a == i) kp.diag[j] = (int64_t)kp.Ki.size();
                kp.Ki.push_back(n + p + a);
            }
        }
        kp.Kp[j + 1] = (int64_t)kp.Ki.size();
    }
    // (3,3) positions in the documented order
    for (int32_t i = 0; i < pp.l; ++i) kp.blk33.push_back(kp.diag[n + p + i]);
    for (int32_t k = 0; k < pp.nsoc; ++k) {
        kp.blk33_off[k] = (int64_t)kp.blk33.size() - pp.l;
        for (int32_t b = pp.soc_off[k]; b < pp.soc_off[k + 1]; ++b) {
            int64_t colstart = kp.Kp[n + p + b + 1] - (b - pp.soc_off[k] + 1);
            for (int32_t a = 0; a <= b - pp.soc_off[k]; ++a) kp.blk33.push_back(colstart + a);
        }
    }
    kp.blk33_off[pp.nsoc] = (int64_t)kp.blk33.size() - pp.l;
}

// ---------------------------------------------------------------------------
// ordering: approximate-degree minimum degree on the quotient graph
// ---------------------------------------------------------------------------
namespace {

enum : int8_t { VAR = 0, MERGED = 1, ELEMENT = 2, ABSORBED = 3 };

struct QuotientGraph {
    int32_t N;
    std::vector<std::vector<int32_t>> A, E, Lel;
    std::vector<int64_t> nv, deg, wtot, wcur;
    std::vector<int8_t> status;
    std::vector<int32_t> head, next, tail;  // member chains
    std::vector<int64_t> mark;
    int64_t stamp = 0;
};

inline uint64_t mix(uint64_t h, uint64_t v) {
    h ^= v + 0x9e3779b97f4a7c15ULL + (h << 6) + (h >> 2);
    return h;
}

// Min-heap of variables keyed by (degree, index), with each variable's
// position kept so that its key can be changed or it can be removed in
// O(log N) on a flat array.  The key order is total, so the minimum -- the
// next pivot -- is the same as with any other priority queue on that order.
struct DegreeHeap {
    std::vector<int32_t> heap;     // variables
    std::vector<int32_t> pos;      // position of each variable in heap, -1 if absent
    const std::vector<int64_t> *key = nullptr;
    bool less(int32_t a, int32_t b) const {
        const int64_t ka = (*key)[a], kb = (*key)[b];
        return ka < kb || (ka == kb && a < b);
    }
    void place(size_t k, int32_t v) { heap[k] = v; pos[v] = (int32_t)k; }
    void up(size_t k) {
        const int32_t v = heap[k];
        while (k > 0) {
            const size_t par = (k - 1) / 2;
            if (!less(v, heap[par])) break;
            place(k, heap[par]);
            k = par;
        }
        place(k, v);
    }
    void down(size_t k) {
        const int32_t v = heap[k];
        const size_t n = heap.size();
        for (;;) {
            size_t c = 2 * k + 1;
            if (c >= n) break;
            if (c + 1 < n && less(heap[c + 1], heap[c])) ++c;
            if (!less(heap[c], v)) break;
            place(k, heap[c]);
            k = c;
        }
        place(k, v);
    }
    void push(int32_t v) { heap.push_back(v); up(heap.size() - 1); }
    // Remove every variable of vs that is in the heap (in bulk: filter and
    // rebuild when vs is a large part of the heap, one by one otherwise).
    void remove_many(const std::vector<int32_t> &vs) {
        if (vs.size() * 8 < heap.size()) {
            for (int32_t v : vs) if (contains(v)) remove(v);
            return;
        }
        for (int32_t v : vs) if (contains(v)) pos[v] = -2;     // marked for removal
        size_t k = 0;
        for (int32_t v : heap) if (pos[v] != -2) heap[k++] = v;
        heap.resize(k);
        for (int32_t v : vs) if (pos[v] == -2) pos[v] = -1;
        rebuild();
    }
    // Insert every variable of vs with its current key.
    void push_many(const std::vector<int32_t> &vs) {
        if (vs.size() * 8 < heap.size()) {
            for (int32_t v : vs) push(v);
            return;
        }
        heap.insert(heap.end(), vs.begin(), vs.end());
        rebuild();
    }
    // Restore the heap order over the whole array (Floyd), positions included.
    void rebuild() {
        for (size_t k = 0; k < heap.size(); ++k) pos[heap[k]] = (int32_t)k;
        for (size_t k = heap.size() / 2; k-- > 0;) down(k);
    }
    bool contains(int32_t v) const { return pos[v] >= 0; }
    void remove(int32_t v) {
        const size_t k = (size_t)pos[v];
        pos[v] = -1;
        const int32_t last = heap.back();
        heap.pop_back();
        if (last == v) return;
        place(k, last);
        up(k);
        down((size_t)pos[last]);
    }
    int32_t pop() {
        const int32_t v = heap[0];
        remove(v);
        return v;
    }
};

}  // namespace

void min_degree_order(int32_t N, const std::vector<int64_t> &Gp, const std::vector<int32_t> &Gi,
                      std::vector<int32_t> &order) {
    QuotientGraph g;
    g.N = N;
    g.A.resize(N); g.E.resize(N); g.Lel.resize(N);
    g.nv.assign(N, 1); g.deg.assign(N, 0); g.wtot.assign(N, 0); g.wcur.assign(N, 0);
    g.status.assign(N, VAR);
    g.head.resize(N); g.next.assign(N, -1); g.tail.resize(N);
    g.mark.assign(N, 0);
    std::iota(g.head.begin(), g.head.end(), 0);
    std::iota(g.tail.begin(), g.tail.end(), 0);
    DegreeHeap pq;
    pq.key = &g.deg;
    pq.pos.assign(N, -1);
    pq.heap.reserve(N);
    for (int32_t i = 0; i < N; ++i) {
        auto &a = g.A[i];
        for (int64_t t = Gp[i]; t < Gp[i + 1]; ++t) if (Gi[t] != i) a.push_back(Gi[t]);
        std::sort(a.begin(), a.end());
        g.deg[i] = (int64_t)a.size();
        pq.push(i);
    }
    order.clear();
    order.reserve(N);
    int64_t rem = N;
    std::vector<int32_t> Lp, members, rest, merged_buf;
    std::vector<std::pair<uint64_t, int32_t>> keyed;
    std::vector<uint64_t> hslot, hashes;     // hash count table (open addressing) and Lp's hashes
    std::vector<int32_t> hcount;
    std::vector<size_t> run_end;
    std::vector<int32_t> elist;              // live elements adjacent to Lp (degree update)
    std::vector<int64_t> estamp((size_t)N, 0);
    int64_t estamp_id = 0;
    std::mutex elist_mu;
    // Loops over Lp whose iterations are independent run on the pool when Lp is long (the
    // dense final phase, where Lp holds most of the remaining variables).
    // The pool's threads are started at the first long pivot step only: small graphs (the pieces of
    // a nested dissection, thousands of calls) never start them.
    std::unique_ptr<WorkPool> pool_;
    auto pool = [&]() -> WorkPool & {
        if (!pool_) pool_.reset(new WorkPool(WorkPool::default_threads()));
        return *pool_;
    };
    constexpr size_t PAR_MIN = 2048;
    auto for_lp = [&](const std::function<void(int64_t, int64_t)> &fn) {
        if (Lp.size() >= PAR_MIN) pool().run((int64_t)Lp.size(), fn);
        else fn(0, (int64_t)Lp.size());
    };
    while (!pq.heap.empty()) {
        const int32_t p = pq.pop();
        // members of p in increasing order
        members.clear();
        for (int32_t v = g.head[p]; v != -1; v = g.next[v]) members.push_back(v);
        std::sort(members.begin(), members.end());
        order.insert(order.end(), members.begin(), members.end());
        // Lp = (A_p U union L_e) \ {p}, sorted: A_p and every L_e are sorted lists, so Lp is
        // formed as sorted runs and merged (the longest run with the sorted rest)
        ++g.stamp;
        const int64_t lpmark = g.stamp;
        g.mark[p] = lpmark;
        Lp.clear();
        run_end.clear();
        for (int32_t v : g.A[p])
            if (g.status[v] == VAR && g.mark[v] != lpmark) { g.mark[v] = lpmark; Lp.push_back(v); }
        run_end.push_back(Lp.size());
        for (int32_t e : g.E[p]) {
            for (int32_t v : g.Lel[e])
                if (g.status[v] == VAR && g.mark[v] != lpmark) { g.mark[v] = lpmark; Lp.push_back(v); }
            run_end.push_back(Lp.size());
        }
        {
            size_t b0 = 0, e0 = 0, prev = 0;
            for (size_t r : run_end) {
                if (r - prev > e0 - b0) { b0 = prev; e0 = r; }
                prev = r;
            }
            if (e0 - b0 < Lp.size()) {
                rest.clear();
                rest.insert(rest.end(), Lp.begin(), Lp.begin() + (std::ptrdiff_t)b0);
                rest.insert(rest.end(), Lp.begin() + (std::ptrdiff_t)e0, Lp.end());
                std::sort(rest.begin(), rest.end());
                merged_buf.resize(Lp.size());
                std::merge(Lp.begin() + (std::ptrdiff_t)b0, Lp.begin() + (std::ptrdiff_t)e0, rest.begin(),
                           rest.end(), merged_buf.begin());
                Lp.swap(merged_buf);
            }
        }
        for (int32_t e : g.E[p]) {
            g.status[e] = ABSORBED;
            std::vector<int32_t>().swap(g.Lel[e]);
        }
        g.status[p] = ELEMENT;
        rem -= g.nv[p];
        std::vector<int32_t>().swap(g.A[p]);
        std::vector<int32_t>().swap(g.E[p]);
        int64_t wlp = 0;
        for (int32_t i : Lp) wlp += g.nv[i];
        g.Lel[p] = Lp;
        g.wtot[p] = wlp;
        pq.remove_many(Lp);
        // list updates: each variable's own lists, from shared read-only marks and states
        for_lp([&](int64_t t0, int64_t t1) {
            for (int64_t t = t0; t < t1; ++t) {
                const int32_t i = Lp[(size_t)t];
                auto &Ei = g.E[i];
                size_t k = 0;
                for (int32_t e : Ei) if (g.status[e] == ELEMENT) Ei[k++] = e;
                Ei.erase(Ei.begin() + (std::ptrdiff_t)k, Ei.end());
                Ei.insert(std::lower_bound(Ei.begin(), Ei.end(), p), p);
                auto &Ai = g.A[i];
                k = 0;
                for (int32_t v : Ai) if (g.mark[v] != lpmark) Ai[k++] = v;
                Ai.erase(Ai.begin() + (std::ptrdiff_t)k, Ai.end());
            }
        });
        // supervariable detection among Lp: hash, then confirm by full equality.  Only a hash
        // shared by two or more variables can lead to a merge: those are found with an
        // open-addressing count table, and only they are sorted by (hash, index)
        hashes.resize(Lp.size());
        for_lp([&](int64_t t0, int64_t t1) {
            for (int64_t t = t0; t < t1; ++t) {
                const int32_t i = Lp[(size_t)t];
                uint64_t h = mix(mix(0, g.A[i].size()), g.E[i].size());
                for (int32_t v : g.A[i]) h = mix(h, (uint64_t)v);
                h = mix(h, 0xabcdefULL);
                for (int32_t e : g.E[i]) h = mix(h, (uint64_t)e);
                hashes[(size_t)t] = h;
            }
        });
        keyed.clear();
        size_t cap = 16;
        while (cap < 2 * Lp.size()) cap <<= 1;
        if (hslot.size() < cap) { hslot.resize(cap); hcount.resize(cap); }
        std::fill(hcount.begin(), hcount.begin() + (std::ptrdiff_t)cap, 0);
        auto slot_of = [&](uint64_t h) {
            size_t k = (size_t)((h * 0x9e3779b97f4a7c15ULL) >> 20) & (cap - 1);
            while (hcount[k] != 0 && hslot[k] != h) k = (k + 1) & (cap - 1);
            return k;
        };
        for (size_t t = 0; t < Lp.size(); ++t) {
            const size_t k = slot_of(hashes[t]);
            hslot[k] = hashes[t];
            ++hcount[k];
        }
        for (size_t t = 0; t < Lp.size(); ++t)
            if (hcount[slot_of(hashes[t])] > 1) keyed.push_back({hashes[t], Lp[t]});
        std::sort(keyed.begin(), keyed.end());
        for (size_t a = 0; a < keyed.size();) {
            size_t b = a;
            while (b < keyed.size() && keyed[b].first == keyed[a].first) ++b;
            for (size_t u = a; u < b; ++u) {
                int32_t r = keyed[u].second;
                if (g.status[r] != VAR) continue;
                for (size_t w = u + 1; w < b; ++w) {
                    int32_t j = keyed[w].second;
                    if (g.status[j] != VAR) continue;
                    if (g.A[j] != g.A[r] || g.E[j] != g.E[r]) continue;
                    // merge j into r (r < j: keyed is sorted by (hash, index))
                    g.nv[r] += g.nv[j];
                    g.next[g.tail[r]] = g.head[j];
                    g.tail[r] = g.tail[j];
                    for (int32_t v : g.A[j]) {
                        auto &Av = g.A[v];
                        Av.erase(std::find(Av.begin(), Av.end(), j));
                    }
                    for (int32_t e : g.E[j]) {
                        auto &Le = g.Lel[e];
                        Le.erase(std::find(Le.begin(), Le.end(), j));
                    }
                    std::vector<int32_t>().swap(g.A[j]);
                    std::vector<int32_t>().swap(g.E[j]);
                    g.status[j] = MERGED;
                    g.nv[j] = 0;
                }
            }
            a = b;
        }
        // approximate degrees: w_e = W(L_e \ Lp) = total weight of e minus the weight of its
        // variables in Lp, for every live element e != p of a variable of Lp (integer sums: the
        // same whichever way they are formed)
        ++estamp_id;
        if (Lp.size() < PAR_MIN) {
            // from the variables' side: each element starts from its total at its first visit
            for (int32_t i : Lp) {
                if (g.status[i] != VAR) continue;
                for (int32_t e : g.E[i]) {
                    if (e == p) continue;
                    if (estamp[e] != estamp_id) { estamp[e] = estamp_id; g.wcur[e] = g.wtot[e]; }
                    g.wcur[e] -= g.nv[i];
                }
            }
        } else {
            // from the elements' side, in parallel: the elements are collected once each (the
            // per-pivot stamp), then each sum is formed by one thread from the element's own
            // list (the incidence of live elements and variables is symmetric: e is in E_i
            // exactly when i is in L_e)
            elist.clear();
            for_lp([&](int64_t t0, int64_t t1) {
                std::vector<int32_t> mine;
                for (int64_t t = t0; t < t1; ++t) {
                    const int32_t i = Lp[(size_t)t];
                    if (g.status[i] != VAR) continue;
                    for (int32_t e : g.E[i]) {
                        if (e == p || __atomic_load_n(&estamp[e], __ATOMIC_RELAXED) == estamp_id) continue;
                        if (__atomic_exchange_n(&estamp[e], estamp_id, __ATOMIC_RELAXED) != estamp_id)
                            mine.push_back(e);
                    }
                }
                std::lock_guard<std::mutex> lk(elist_mu);
                elist.insert(elist.end(), mine.begin(), mine.end());
            });
            pool().run((int64_t)elist.size(), [&](int64_t t0, int64_t t1) {
                for (int64_t t = t0; t < t1; ++t) {
                    const int32_t e = elist[(size_t)t];
                    int64_t w = g.wtot[e];
                    // eliminated variables are dropped from the list on the way (every reader
                    // of element lists skips them)
                    auto &Le = g.Lel[e];
                    size_t k = 0;
                    for (int32_t v : Le) {
                        if (g.status[v] != VAR) continue;
                        if (g.mark[v] == lpmark) w -= g.nv[v];
                        Le[k++] = v;
                    }
                    Le.resize(k);
                    g.wcur[e] = w;
                }
            });
        }
        for_lp([&](int64_t t0, int64_t t1) {
            for (int64_t t = t0; t < t1; ++t) {
                const int32_t i = Lp[(size_t)t];
                if (g.status[i] != VAR) continue;
                int64_t wa = 0, we = 0;
                for (int32_t v : g.A[i]) wa += g.nv[v];
                for (int32_t e : g.E[i]) if (e != p) we += g.wcur[e];
                const int64_t lpi = wlp - g.nv[i];
                int64_t d = std::min(rem - g.nv[i], g.deg[i] + lpi);
                d = std::min(d, wa + lpi + we);
                g.deg[i] = d;
            }
        });
        size_t k = 0;
        for (int32_t i : Lp) if (g.status[i] == VAR) Lp[k++] = i;
        Lp.resize(k);
        pq.push_many(Lp);
    }
}

// ---------------------------------------------------------------------------
// nested dissection (the alternative to step 3)
// ---------------------------------------------------------------------------
// Automatic nested dissection by breadth-first level structures (George and
// Liu, "Computer Solution of Large Sparse Positive Definite Systems", 1981,
// ch. 8), with minimum degree on the small pieces.  For a node set S of the
// graph (ascending), ND(S) is:
//  a. |S| <= ND_LEAF: the minimum-degree order of the subgraph induced by S
//     (local node i = i-th least node of S);
//  b. the subgraph induced by S is not connected: ND of each of its
//     components, in increasing order of their least node;
//  c. connected: the level structure (BFS levels within S) rooted at the
//     least node of S; then repeatedly the node of the last level with least
//     (degree within S, index) roots a new level structure, which replaces
//     the current one while it has more levels (pseudo-peripheral root);
//  d. with h levels: h < 3 is case a; else the separator is the set of
//     nodes of level m = floor(h/2) with a neighbour in level m + 1, A the
//     levels below m plus the rest of level m, B the levels above m; the
//     order is ND(A), ND(B), then the separator by increasing index.
// Removing the separator disconnects A from B (BFS levels only touch
// adjacent levels), so the separator's columns are eliminated last and the
// elimination trees of A and B hang below them: the tree depth grows with
// the number of dissection levels, not with the length of the graph.
namespace {

constexpr int32_t ND_LEAF = 256;

struct Dissector {
    int32_t N;
    const std::vector<int64_t> &Gp;
    const std::vector<int32_t> &Gi;
    std::vector<int32_t> stamp, lev, loc, queue;
    int32_t cur = 0;
    std::vector<int32_t> &out;

    Dissector(int32_t n, const std::vector<int64_t> &gp, const std::vector<int32_t> &gi,
              std::vector<int32_t> &o)
        : N(n), Gp(gp), Gi(gi), stamp(n, -1), lev(n, -1), loc(n, -1), queue(n), out(o) {}

    // mark S as the current set (a fresh stamp)
    void mark(const std::vector<int32_t> &S) {
        ++cur;
        for (int32_t v : S) { stamp[v] = cur; lev[v] = -1; }
    }
    // BFS within the marked set from root; fills queue[0, count) in level order and the level
    // boundaries; returns the number of nodes reached
    int32_t bfs(int32_t root, std::vector<int32_t> &bounds) {
        bounds.assign(1, 0);
        int32_t head = 0, tail = 0;
        queue[tail++] = root;
        lev[root] = 0;
        int32_t lv_end = 1;
        bounds.push_back(1);
        while (head < tail) {
            const int32_t v = queue[head++];
            for (int64_t t = Gp[v]; t < Gp[v + 1]; ++t) {
                const int32_t u = Gi[t];
                if (stamp[u] == cur && lev[u] < 0) { lev[u] = lev[v] + 1; queue[tail++] = u; }
            }
            if (head == lv_end && tail > lv_end) { lv_end = tail; bounds.push_back(tail); }
        }
        return tail;
    }
    void reset_levels(int32_t count) {
        for (int32_t i = 0; i < count; ++i) lev[queue[i]] = -1;
    }
    int32_t degree_in_set(int32_t v) const {
        int32_t d = 0;
        for (int64_t t = Gp[v]; t < Gp[v + 1]; ++t) d += stamp[Gi[t]] == cur;
        return d;
    }
    // minimum degree on the subgraph induced by the marked set S
    void leaf(const std::vector<int32_t> &S) {
        const int32_t ns = (int32_t)S.size();
        for (int32_t i = 0; i < ns; ++i) loc[S[i]] = i;
        std::vector<int64_t> lp((size_t)ns + 1, 0);
        std::vector<int32_t> li;
        for (int32_t i = 0; i < ns; ++i) {
            const int32_t v = S[i];
            for (int64_t t = Gp[v]; t < Gp[v + 1]; ++t)
                if (stamp[Gi[t]] == cur) li.push_back(loc[Gi[t]]);
            lp[i + 1] = (int64_t)li.size();
            std::sort(li.begin() + lp[i], li.end());
        }
        std::vector<int32_t> o;
        min_degree_order(ns, lp, li, o);
        for (int32_t i : o) out.push_back(S[i]);
    }

    struct Item {
        bool emit;                   // true: append nodes as they are
        std::vector<int32_t> nodes;  // ascending
    };

    void run(std::vector<int32_t> all) {
        std::vector<Item> stack;
        stack.push_back({false, std::move(all)});
        std::vector<int32_t> bounds, bounds2;
        while (!stack.empty()) {
            Item it = std::move(stack.back());
            stack.pop_back();
            std::vector<int32_t> &S = it.nodes;
            if (it.emit) { out.insert(out.end(), S.begin(), S.end()); continue; }
            if (S.empty()) continue;
            mark(S);
            if ((int32_t)S.size() <= ND_LEAF) { leaf(S); continue; }
            int32_t reached = bfs(S[0], bounds);
            if (reached < (int32_t)S.size()) {
                // b: components in increasing order of their least node (S is ascending)
                std::vector<std::vector<int32_t>> comps;
                std::vector<int32_t> c(queue.begin(), queue.begin() + reached);
                std::sort(c.begin(), c.end());
                comps.push_back(std::move(c));
                for (int32_t v : S) {
                    if (lev[v] >= 0) continue;
                    const int32_t cnt = bfs(v, bounds);
                    std::vector<int32_t> cc(queue.begin(), queue.begin() + cnt);
                    std::sort(cc.begin(), cc.end());
                    comps.push_back(std::move(cc));
                }
                for (size_t i = comps.size(); i-- > 0;) stack.push_back({false, std::move(comps[i])});
                continue;
            }
            // c: pseudo-peripheral root
            int32_t root = S[0];
            while (true) {
                const int32_t l0 = bounds[bounds.size() - 2], l1 = bounds.back();
                int32_t best = -1, bdeg = 0;
                for (int32_t i = l0; i < l1; ++i) {
                    const int32_t v = queue[i], dv = degree_in_set(v);
                    if (best < 0 || dv < bdeg || (dv == bdeg && v < best)) { best = v; bdeg = dv; }
                }
                reset_levels(reached);
                bfs(best, bounds2);
                if (bounds2.size() > bounds.size()) {
                    root = best;
                    bounds.swap(bounds2);
                    continue;
                }
                reset_levels(reached);
                bfs(root, bounds);
                break;
            }
            const int32_t h = (int32_t)bounds.size() - 1;
            if (h < 3) { leaf(S); continue; }
            const int32_t m = h / 2;
            std::vector<int32_t> A, B, sep;
            for (int32_t i = 0; i < bounds[m]; ++i) A.push_back(queue[i]);
            for (int32_t i = bounds[m]; i < bounds[m + 1]; ++i) {
                const int32_t v = queue[i];
                bool touches = false;
                for (int64_t t = Gp[v]; t < Gp[v + 1] && !touches; ++t)
                    touches = stamp[Gi[t]] == cur && lev[Gi[t]] == m + 1;
                (touches ? sep : A).push_back(v);
            }
            for (int32_t i = bounds[m + 1]; i < reached; ++i) B.push_back(queue[i]);
            std::sort(A.begin(), A.end());
            std::sort(B.begin(), B.end());
            std::sort(sep.begin(), sep.end());
            stack.push_back({true, std::move(sep)});
            stack.push_back({false, std::move(B)});
            stack.push_back({false, std::move(A)});
        }
    }
};

}  // namespace

void nd_order(int32_t N, const std::vector<int64_t> &Gp, const std::vector<int32_t> &Gi,
              std::vector<int32_t> &order) {
    order.clear();
    order.reserve(N);
    std::vector<int32_t> all(N);
    std::iota(all.begin(), all.end(), 0);
    Dissector d(N, Gp, Gi, order);
    d.run(std::move(all));
}

// ---------------------------------------------------------------------------
// elimination tree, postorder, column counts, supernodes
// ---------------------------------------------------------------------------
namespace {

// Upper triangle pattern (CSC) of the permuted matrix, rows sorted.
void permuted_upper(const KktPattern &kp, const std::vector<int32_t> &iperm,
                    std::vector<int64_t> &Up, std::vector<int32_t> &Ui) {
    const int32_t N = kp.N;
    Up.assign((size_t)N + 1, 0);
    for (int32_t j = 0; j < N; ++j)
        for (int64_t t = kp.Kp[j]; t < kp.Kp[j + 1]; ++t) {
            int32_t a = iperm[kp.Ki[t]], b = iperm[j];
            Up[std::max(a, b) + 1]++;
        }
    for (int32_t j = 0; j < N; ++j) Up[j + 1] += Up[j];
    Ui.resize(kp.Ki.size());
    std::vector<int64_t> fill(Up.begin(), Up.end() - 1);
    for (int32_t j = 0; j < N; ++j)
        for (int64_t t = kp.Kp[j]; t < kp.Kp[j + 1]; ++t) {
            int32_t a = iperm[kp.Ki[t]], b = iperm[j];
            Ui[fill[std::max(a, b)]++] = std::min(a, b);
        }
    for (int32_t j = 0; j < N; ++j) std::sort(Ui.begin() + Up[j], Ui.begin() + Up[j + 1]);
}

void etree_of(int32_t N, const std::vector<int64_t> &Up, const std::vector<int32_t> &Ui,
              std::vector<int32_t> &parent) {
    parent.assign(N, -1);
    std::vector<int32_t> root(N, -1);   // path-compressed ancestor
    for (int32_t k = 0; k < N; ++k) {
        for (int64_t t = Up[k]; t < Up[k + 1]; ++t) {
            int32_t i = Ui[t];
            while (i != -1 && i < k) {
                int32_t up = root[i];
                root[i] = k;
                if (up == -1) { parent[i] = k; break; }
                i = up;
            }
        }
    }
}

void postorder_of(const std::vector<int32_t> &parent, std::vector<int32_t> &post) {
    const int32_t N = (int32_t)parent.size();
    std::vector<int32_t> first(N, -1), sib(N, -1);
    // children lists in increasing order: insert from the highest index down
    for (int32_t j = N - 1; j >= 0; --j)
        if (parent[j] >= 0) { sib[j] = first[parent[j]]; first[parent[j]] = j; }
    post.clear();
    post.reserve(N);
    std::vector<int32_t> stack;
    for (int32_t r = 0; r < N; ++r) {
        if (parent[r] != -1) continue;
        stack.push_back(r);
        while (!stack.empty()) {
            int32_t v = stack.back();
            if (first[v] != -1) {
                int32_t c = first[v];
                first[v] = sib[c];   // consume the child
                stack.push_back(c);
            } else {
                stack.pop_back();
                post.push_back(v);
            }
        }
    }
}

}  // namespace

void analyze_pattern(const KktPattern &kp, Symbolic &sym, int ordering) {
    const int32_t N = kp.N;
    sym.N = N;
    // 1. symmetric graph without the diagonal
    std::vector<int64_t> deg(N, 0);
    for (int32_t j = 0; j < N; ++j)
        for (int64_t t = kp.Kp[j]; t < kp.Kp[j + 1]; ++t)
            if (kp.Ki[t] != j) { deg[j]++; deg[kp.Ki[t]]++; }
    // 2. dense nodes
    const int64_t cut = std::max<int64_t>(16, (int64_t)std::floor(10.0 * std::sqrt((double)N)));
    std::vector<int32_t> local(N, -1), keep;
    for (int32_t i = 0; i < N; ++i)
        if (deg[i] <= cut) { local[i] = (int32_t)keep.size(); keep.push_back(i); }
    const int32_t Ns = (int32_t)keep.size();
    std::vector<int64_t> Gp((size_t)Ns + 1, 0);
    for (int32_t j = 0; j < N; ++j)
        for (int64_t t = kp.Kp[j]; t < kp.Kp[j + 1]; ++t) {
            int32_t i = kp.Ki[t];
            if (i == j || local[i] < 0 || local[j] < 0) continue;
            Gp[local[i] + 1]++; Gp[local[j] + 1]++;
        }
    for (int32_t i = 0; i < Ns; ++i) Gp[i + 1] += Gp[i];
    std::vector<int32_t> Gi(Gp[Ns]);
    {
        std::vector<int64_t> fill(Gp.begin(), Gp.end() - 1);
        for (int32_t j = 0; j < N; ++j)
            for (int64_t t = kp.Kp[j]; t < kp.Kp[j + 1]; ++t) {
                int32_t i = kp.Ki[t];
                if (i == j || local[i] < 0 || local[j] < 0) continue;
                Gi[fill[local[i]]++] = local[j];
                Gi[fill[local[j]]++] = local[i];
            }
    }
    // 3. minimum degree, or nested dissection with minimum degree on its pieces
    std::vector<int32_t> md_local, md;
    if (ordering == QG_ORDER_ND) nd_order(Ns, Gp, Gi, md_local);
    else min_degree_order(Ns, Gp, Gi, md_local);
    md.reserve(N);
    for (int32_t v : md_local) md.push_back(keep[v]);
    for (int32_t i = 0; i < N; ++i) if (local[i] < 0) md.push_back(i);
    // 4. postorder of the etree of the minimum-degree order
    std::vector<int32_t> inv(N);
    for (int32_t k = 0; k < N; ++k) inv[md[k]] = k;
    std::vector<int64_t> Up;
    std::vector<int32_t> Ui, par, post;
    permuted_upper(kp, inv, Up, Ui);
    etree_of(N, Up, Ui, par);
    postorder_of(par, post);
    sym.perm.resize(N);
    for (int32_t k = 0; k < N; ++k) sym.perm[k] = md[post[k]];
    sym.iperm.resize(N);
    for (int32_t k = 0; k < N; ++k) sym.iperm[sym.perm[k]] = k;
    // 5. etree and column counts of the final order (row subtrees)
    permuted_upper(kp, sym.iperm, Up, Ui);
    etree_of(N, Up, Ui, sym.parent);
    sym.colcount.assign(N, 1);
    {
        std::vector<int32_t> visited(N, -1);
        for (int32_t k = 0; k < N; ++k) {
            visited[k] = k;
            for (int64_t t = Up[k]; t < Up[k + 1]; ++t) {
                for (int32_t i = Ui[t]; visited[i] != k; i = sym.parent[i]) {
                    visited[i] = k;
                    sym.colcount[i]++;
                }
            }
        }
    }
    sym.nnz_L = 0;
    sym.flops = 0.0;
    for (int32_t j = 0; j < N; ++j) {
        sym.nnz_L += sym.colcount[j];
        double c = (double)(sym.colcount[j] - 1);
        sym.flops += c * c + 3.0 * c;
    }
    // 6. fundamental supernodes
    std::vector<int32_t> nchild(N, 0);
    for (int32_t j = 0; j < N; ++j) if (sym.parent[j] >= 0) nchild[sym.parent[j]]++;
    sym.super_fund.clear();
    if (N > 0) sym.super_fund.push_back(0);
    for (int32_t j = 0; j + 1 < N; ++j) {
        bool joins = sym.parent[j] == j + 1 && sym.colcount[j] == sym.colcount[j + 1] + 1 &&
                     nchild[j + 1] == 1;
        if (!joins) sym.super_fund.push_back(j + 1);
    }
    sym.super_fund.push_back(N);
    // 7. relaxed supernodes
    sym.super_ptr.clear();
    {
        const int32_t nf = (int32_t)sym.super_fund.size() - 1;
        int32_t gf = sym.super_fund[0], gl = sym.super_fund[1] - 1;
        int64_t gsum = 0;
        for (int32_t c = gf; c <= gl; ++c) gsum += sym.colcount[c];
        for (int32_t s = 1; s < nf; ++s) {
            const int32_t tf = sym.super_fund[s], tl = sym.super_fund[s + 1] - 1;
            int64_t tsum = 0;
            for (int32_t c = tf; c <= tl; ++c) tsum += sym.colcount[c];
            bool merge = false;
            if (sym.parent[gl] == tf) {
                const int64_t w = tl - gf + 1;
                const int64_t r = (gl - gf + 1) + sym.colcount[tf];
                const int64_t stored = w * r - w * (w - 1) / 2;
                const int64_t zeros = stored - (gsum + tsum);
                merge = ((double)zeros <= 0.1 * (double)stored) || (w <= 8 && zeros <= 64);
            }
            if (merge) {
                gl = tl;
                gsum += tsum;
            } else {
                sym.super_ptr.push_back(gf);
                gf = tf; gl = tl; gsum = tsum;
            }
        }
        if (N > 0) sym.super_ptr.push_back(gf);
        sym.super_ptr.push_back(N);
    }
    // 8. row lists by the union recursion over the supernodal tree: rows below
    //    a supernode = (its columns' K rows U its children's rows below) beyond
    //    its last column
    const int32_t ns = (int32_t)sym.super_ptr.size() - 1;
    std::vector<int32_t> col2sn(N);
    for (int32_t s = 0; s < ns; ++s)
        for (int32_t c = sym.super_ptr[s]; c < sym.super_ptr[s + 1]; ++c) col2sn[c] = s;
    sym.sn_parent.assign(ns, -1);
    for (int32_t s = 0; s < ns; ++s) {
        int32_t pc = sym.parent[sym.super_ptr[s + 1] - 1];
        sym.sn_parent[s] = pc >= 0 ? col2sn[pc] : -1;
    }
    // lower structure of the permuted matrix: for column c, rows i > c
    std::vector<int64_t> Lop((size_t)N + 1, 0);
    for (int32_t j = 0; j < N; ++j)
        for (int64_t t = Up[j]; t < Up[j + 1]; ++t) if (Ui[t] < j) Lop[Ui[t] + 1]++;
    for (int32_t j = 0; j < N; ++j) Lop[j + 1] += Lop[j];
    std::vector<int32_t> Loi(Lop[N]);
    {
        std::vector<int64_t> fill(Lop.begin(), Lop.end() - 1);
        for (int32_t j = 0; j < N; ++j)
            for (int64_t t = Up[j]; t < Up[j + 1]; ++t) if (Ui[t] < j) Loi[fill[Ui[t]]++] = j;
    }
    std::vector<std::vector<int32_t>> below(ns);
    std::vector<int32_t> cfirst(ns, -1), csib(ns, -1);
    for (int32_t s = ns - 1; s >= 0; --s)
        if (sym.sn_parent[s] >= 0) { csib[s] = cfirst[sym.sn_parent[s]]; cfirst[sym.sn_parent[s]] = s; }
    std::vector<int32_t> seen(N, -1), buf;
    sym.rows_ptr.assign((size_t)ns + 1, 0);
    sym.rows.clear();
    sym.sn_level.assign(ns, 0);
    for (int32_t s = 0; s < ns; ++s) {
        const int32_t f = sym.super_ptr[s], l = sym.super_ptr[s + 1] - 1;
        buf.clear();
        for (int32_t c = f; c <= l; ++c)
            for (int64_t t = Lop[c]; t < Lop[c + 1]; ++t) {
                int32_t i = Loi[t];
                if (i > l && seen[i] != s) { seen[i] = s; buf.push_back(i); }
            }
        for (int32_t c = cfirst[s]; c != -1; c = csib[c]) {
            for (int32_t i : below[c])
                if (i > l && seen[i] != s) { seen[i] = s; buf.push_back(i); }
            std::vector<int32_t>().swap(below[c]);
            sym.sn_level[s] = std::max(sym.sn_level[s], sym.sn_level[c] + 1);
        }
        std::sort(buf.begin(), buf.end());
        for (int32_t c = f; c <= l; ++c) sym.rows.push_back(c);
        sym.rows.insert(sym.rows.end(), buf.begin(), buf.end());
        sym.rows_ptr[s + 1] = (int64_t)sym.rows.size();
        if (sym.sn_parent[s] >= 0) below[s] = buf;
        // consistency with the column counts: rows below = structure of the last column
        if ((int64_t)buf.size() + 1 != sym.colcount[l])
            throw std::logic_error("row list does not match the column count");
    }
    sym.nlevels = 0;
    for (int32_t s = 0; s < ns; ++s) sym.nlevels = std::max(sym.nlevels, sym.sn_level[s] + 1);
}

}  // namespace qg
