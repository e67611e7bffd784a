// Builds the supernodal multifrontal plan from the analysis: front layout,
// per-column assembly lists (K entries and child contributions through
// relative indices), level schedule, and uploads it with the static data.
#include <algorithm>
#include <cstring>

#include "kernels.hpp"
#include "solver.hpp"

#include <cmath>

namespace qg {

int hip_fail(qg_handle *h, hipError_t e) {
    if (h) h->last_hip = (int)e;
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? QG_ERR_OOM : QG_ERR_HIP;
}

// Device memory of the handle: through the caller's allocator when one was
// given to qg_setup, else hipMalloc.  A buffer that already has the requested
// length is kept (value updates re-upload into the same memory).
void *dmem_alloc(qg_handle *h, size_t bytes) {
    if (h->alloc) {
        void *p = h->alloc(h->alloc_ctx, bytes);
        h->alloc_refused = (p == nullptr);
        return p;
    }
    void *p = nullptr;
    const hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) { h->last_hip = (int)e; (void)hipGetLastError(); return nullptr; }
    return p;
}

void dmem_free(qg_handle *h, void *p) {
    if (!p) return;
    if (h->alloc) { if (h->free_fn) h->free_fn(h->alloc_ctx, p); }
    else (void)hipFree(p);
}

template <typename T>
int dalloc(qg_handle *h, DBuf<T> &b, size_t n) {
    if (n == 0) n = 1;
    if (b.p && b.n == n) return QG_OK;
    if (b.p) { dmem_free(h, b.p); b.p = nullptr; b.n = 0; }
    b.p = (T *)dmem_alloc(h, n * sizeof(T));
    if (!b.p) return QG_ERR_OOM;
    b.n = n;
    return QG_OK;
}

template <typename T>
int dupload(qg_handle *h, DBuf<T> &b, const std::vector<T> &v) {
    int rc = dalloc(h, b, v.size());
    if (rc) return rc;
    if (!v.empty())
        QG_HIP(h, hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, h->stream));
    return QG_OK;
}

template int dalloc<double>(qg_handle *, DBuf<double> &, size_t);
template int dalloc<float>(qg_handle *, DBuf<float> &, size_t);
template int dalloc<int32_t>(qg_handle *, DBuf<int32_t> &, size_t);
template int dalloc<int64_t>(qg_handle *, DBuf<int64_t> &, size_t);
template int dalloc<int8_t>(qg_handle *, DBuf<int8_t> &, size_t);
template int dalloc<unsigned long long>(qg_handle *, DBuf<unsigned long long> &, size_t);
template int dupload<double>(qg_handle *, DBuf<double> &, const std::vector<double> &);
template int dupload<int32_t>(qg_handle *, DBuf<int32_t> &, const std::vector<int32_t> &);
template int dupload<int64_t>(qg_handle *, DBuf<int64_t> &, const std::vector<int64_t> &);
template int dupload<int8_t>(qg_handle *, DBuf<int8_t> &, const std::vector<int8_t> &);

template <typename T>
static void dfree_(qg_handle *h, DBuf<T> &b) {
    dmem_free(h, b.p);
    b.p = nullptr;
    b.n = 0;
}

void dfree_all(qg_handle *h) {
    Device &d = h->d;
    // FP32 factor buffers are views into the FP64 ones (a factor is in one precision at a time)
    d.front32 = {}; d.dinv32 = {}; d.sinv32 = {}; d.w32 = {};
    dfree_(h, d.kval); dfree_(h, d.blk33); dfree_(h, d.blk_off); dfree_(h, d.soc_off); dfree_(h, d.big_cones); dfree_(h, d.big_chunk_cone); dfree_(h, d.big_chunk_start); dfree_(h, d.bigsc); dfree_(h, d.kr_ptr);
    dfree_(h, d.kr_col); dfree_(h, d.kr_val); dfree_(h, d.c); dfree_(h, d.b); dfree_(h, d.h); dfree_(h, d.craw); dfree_(h, d.braw); dfree_(h, d.hraw); dfree_(h, d.rz_dsc); dfree_(h, d.rz_rsc); dfree_(h, d.Pp); dfree_(h, d.Pi);
    dfree_(h, d.Ap); dfree_(h, d.Ai); dfree_(h, d.Gp); dfree_(h, d.Gi); dfree_(h, d.posG);
    dfree_(h, d.perm); dfree_(h, d.iperm);
    dfree_(h, d.sn_first); dfree_(h, d.sn_rows); dfree_(h, d.task_sn); dfree_(h, d.task_col);
    dfree_(h, d.ctb_src); dfree_(h, d.ch_ptr); dfree_(h, d.ch_list);
    dfree_(h, d.lvl_small_sn); dfree_(h, d.sn_rptr); dfree_(h, d.fr_off); dfree_(h, d.task_ptr);
    dfree_(h, d.ctb_ptr); dfree_(h, d.uv_off); dfree_(h, d.reg_sign);
    dfree_(h, d.ent_dst); dfree_(h, d.ent_sptr); dfree_(h, d.ent_src); dfree_(h, d.ent_reg); dfree_(h, d.zseg_off);
    dfree_(h, d.zseg_len); dfree_(h, d.chain_comp_ptr); dfree_(h, d.chain_grp_ptr); dfree_(h, d.chain_sn);
    dfree_(h, d.ent_front);
    dfree_(h, d.front64); dfree_(h, d.uvec); dfree_(h, d.dinv64);
    dfree_(h, d.sinv64); dfree_(h, d.w64); dfree_(h, d.ubuf);
    dfree_(h, d.vbuf); dfree_(h, d.col2sn); dfree_(h, d.nreg); dfree_(h, d.vwork); dfree_(h, d.task0);
    dfree_(h, d.x); dfree_(h, d.y); dfree_(h, d.s); dfree_(h, d.z); dfree_(h, d.rx); dfree_(h, d.ry); dfree_(h, d.rz);
    dfree_(h, d.kx); dfree_(h, d.rhs); dfree_(h, d.sol); dfree_(h, d.res); dfree_(h, d.corr); dfree_(h, d.xp);
    dfree_(h, d.dsa); dfree_(h, d.ds); dfree_(h, d.t); dfree_(h, d.lam); dfree_(h, d.w); dfree_(h, d.wbar); dfree_(h, d.beta);
    dfree_(h, d.scal); dfree_(h, d.scal_inst); dfree_(h, d.amin); dfree_(h, d.mu); dfree_(h, d.partials); dfree_(h, d.zcone); dfree_(h, d.alpha); dfree_(h, d.flag);
}

// Fronts of the device factorization.  The analysis' supernodes are kept,
// except that a child supernode with at most MERGE_K columns whose own front
// would be large (r > SMALL_R) is factored inside its parent's front: its
// columns move to just before the parent's columns and become leading
// pivots of that front.  Moving a column to just before its elimination-tree
// ancestor keeps every column after all of its descendants, so this is a
// renaming of rows and columns under which L keeps its values; the merged
// front stores the zeros of the child's column explicitly.  It replaces the
// r x r update matrix such a child would form and its parent would assemble
// by a few extra dense pivots in the parent front.  The extra columns per
// front are capped at max(MERGE_K, r / 16).
constexpr int32_t MERGE_K = 16;

int group_fronts(const Symbolic &sym, Symbolic &g) {
    const int32_t N = sym.N;
    const int32_t ns = (int32_t)sym.super_ptr.size() - 1;
    auto kof = [&](int32_t s) { return sym.super_ptr[s + 1] - sym.super_ptr[s]; };
    auto rof = [&](int32_t s) { return (int32_t)(sym.rows_ptr[s + 1] - sym.rows_ptr[s]); };
    std::vector<int32_t> head(ns), extra(ns, 0);
    for (int32_t s = 0; s < ns; ++s) head[s] = s;
    for (int32_t s = ns - 1; s >= 0; --s) {     // parents before children
        const int32_t P = sym.sn_parent[s];
        if (P < 0) continue;
        const int32_t H = head[P];
        const int32_t cap = std::max(MERGE_K, rof(H) / 16);
        if (rof(s) > SMALL_R && kof(s) <= MERGE_K && rof(H) > SMALL_R && extra[H] + kof(s) <= cap) {
            head[s] = H;
            extra[H] += kof(s);
        }
    }
    std::vector<std::vector<int32_t>> members(ns);
    for (int32_t s = 0; s < ns; ++s) if (head[s] != s) members[head[s]].push_back(s);   // increasing index
    std::vector<int32_t> new_of_old(N), gidx(ns, -1);
    g.N = N;
    g.super_ptr.assign(1, 0);
    int32_t pos = 0, ng = 0;
    for (int32_t s = 0; s < ns; ++s) {
        if (head[s] != s) continue;
        for (int32_t m : members[s])
            for (int32_t c = sym.super_ptr[m]; c < sym.super_ptr[m + 1]; ++c) new_of_old[c] = pos++;
        for (int32_t c = sym.super_ptr[s]; c < sym.super_ptr[s + 1]; ++c) new_of_old[c] = pos++;
        g.super_ptr.push_back(pos);
        gidx[s] = ng++;
    }
    if (pos != N) return QG_ERR_PATTERN;
    g.perm.assign(N, 0);
    g.iperm.assign(N, 0);
    for (int32_t c = 0; c < N; ++c) {
        g.perm[new_of_old[c]] = sym.perm[c];
        g.iperm[sym.perm[c]] = new_of_old[c];
    }
    // rows: the group's columns, then the head's rows below its columns (renamed, sorted)
    g.rows_ptr.assign(1, 0);
    g.rows.clear();
    g.sn_parent.assign(ng, -1);
    std::vector<int32_t> tail;
    for (int32_t s = 0; s < ns; ++s) {
        if (head[s] != s) continue;
        const int32_t G = gidx[s];
        const int32_t f = g.super_ptr[G], kg = g.super_ptr[G + 1] - f;
        for (int32_t c = 0; c < kg; ++c) g.rows.push_back(f + c);
        tail.clear();
        for (int64_t t = sym.rows_ptr[s] + kof(s); t < sym.rows_ptr[s + 1]; ++t) tail.push_back(new_of_old[sym.rows[t]]);
        std::sort(tail.begin(), tail.end());
        if (!tail.empty() && tail[0] < f + kg) return QG_ERR_PATTERN;
        g.rows.insert(g.rows.end(), tail.begin(), tail.end());
        g.rows_ptr.push_back((int64_t)g.rows.size());
        // every merged child's column structure must lie in the merged front
        const int32_t *gr = g.rows.data() + g.rows_ptr[G], *ge = g.rows.data() + g.rows_ptr[G + 1];
        for (int32_t m : members[s])
            for (int64_t t = sym.rows_ptr[m]; t < sym.rows_ptr[m + 1]; ++t)
                if (!std::binary_search(gr, ge, new_of_old[sym.rows[t]])) return QG_ERR_PATTERN;
        const int32_t P = sym.sn_parent[s];
        if (P >= 0) g.sn_parent[G] = gidx[head[P]];
    }
    // levels (children precede parents in group order)
    g.sn_level.assign(ng, 0);
    g.nlevels = ng > 0 ? 1 : 0;
    for (int32_t G = 0; G < ng; ++G) {
        const int32_t P = g.sn_parent[G];
        if (P >= 0) {
            if (P <= G) return QG_ERR_PATTERN;
            g.sn_level[P] = std::max(g.sn_level[P], g.sn_level[G] + 1);
            g.nlevels = std::max(g.nlevels, g.sn_level[P] + 1);
        }
    }
    g.nnz_L = sym.nnz_L;
    g.flops = sym.flops;
    return QG_OK;
}

// Chains: the narrow upper levels of deep elimination trees.  From the first
// level L0 with fewer than CHAIN_LEVEL_MIN fronts on, each tree's fronts at
// levels >= L0 form one component; when every component's fronts have at most CHAIN_R
// rows and at most CHAIN_WIDTH_MAX fronts per level on average, each component
// is factored and solved by one workgroup that walks its levels with workgroup barriers, instead of one launch per level (the
// levels below L0, wide enough to fill the device, keep the level launches).
// A component depends only on fronts below L0 (its own tree), and nothing
// else depends on it except those fronts, in the backward solve.  Each level
// lists its chain fronts after the others, so that the level kernels' entry
// and segment ranges can stop before them.
static void select_chains(Plan &pl, const Symbolic &sym, bool enabled) {
    const int32_t ns = pl.ns;
    pl.in_chain.assign((size_t)ns, 0);
    pl.chain_comp_ptr.assign(1, 0);
    pl.chain_grp_ptr.assign(1, 0);
    pl.chain_sn.clear();
    pl.chain_maxr = 0;
    pl.chain_L0 = pl.nlevels;
    if (!enabled) return;
    for (int32_t L = 0; L < pl.nlevels; ++L)
        if (pl.lvl_ptr[L + 1] - pl.lvl_ptr[L] < CHAIN_LEVEL_MIN) { pl.chain_L0 = L; break; }
    if (pl.chain_L0 >= pl.nlevels) return;
    // root of each front's tree; component eligibility per root
    std::vector<int32_t> root((size_t)ns);
    for (int32_t f = ns - 1; f >= 0; --f) {       // parents have larger indices
        const int32_t P = sym.sn_parent[f];
        root[f] = P < 0 ? f : root[P];
    }
    std::vector<int8_t> ok((size_t)ns, 1);
    std::vector<int32_t> members((size_t)ns, 0), top((size_t)ns, -1);
    for (int32_t f = 0; f < ns; ++f) {
        if (sym.sn_level[f] < pl.chain_L0) continue;
        const int64_t r = pl.sn_rptr[f + 1] - pl.sn_rptr[f];
        if (r > CHAIN_R) ok[root[f]] = 0;
        members[root[f]]++;
        top[root[f]] = std::max(top[root[f]], sym.sn_level[f]);
    }
    // a wide component (more than CHAIN_WIDTH_MAX fronts per level on average, as in the upper
    // levels of a nested-dissection tree) would be taken a few fronts at a time by one workgroup;
    // and chains pay only when they replace the level launches from L0 up, so one component that
    // does not qualify keeps every level launch (no chains at all)
    for (int32_t R = 0; R < ns; ++R)
        if (members[R] > 0 && (!ok[R] || members[R] > (int64_t)CHAIN_WIDTH_MAX * (top[R] - pl.chain_L0 + 1))) {
            pl.chain_L0 = pl.nlevels;
            return;
        }
    // components in root order; inside, fronts by level then index
    std::vector<std::vector<int32_t>> comp_of((size_t)ns);
    for (int32_t t = pl.lvl_ptr[pl.chain_L0]; t < pl.lvl_ptr[pl.nlevels]; ++t) {
        const int32_t f = pl.lvl_sn[t];
        if (ok[root[f]] && members[root[f]] > 0) comp_of[root[f]].push_back(f);
    }
    for (int32_t R = 0; R < ns; ++R) {
        if (comp_of[R].empty()) continue;
        int32_t prev = -1;
        for (int32_t f : comp_of[R]) {
            if (sym.sn_level[f] != prev && prev >= 0) pl.chain_grp_ptr.push_back((int32_t)pl.chain_sn.size());
            prev = sym.sn_level[f];
            pl.chain_sn.push_back(f);
            pl.in_chain[f] = 1;
            pl.chain_maxr = std::max<int32_t>(pl.chain_maxr, (int32_t)(pl.sn_rptr[f + 1] - pl.sn_rptr[f]));
        }
        pl.chain_grp_ptr.push_back((int32_t)pl.chain_sn.size());
        pl.chain_comp_ptr.push_back((int32_t)pl.chain_grp_ptr.size() - 1);
    }
    // each level: its other fronts first, then its chain fronts
    for (int32_t L = pl.chain_L0; L < pl.nlevels; ++L)
        std::stable_partition(pl.lvl_sn.begin() + pl.lvl_ptr[L], pl.lvl_sn.begin() + pl.lvl_ptr[L + 1],
                              [&](int32_t f) { return !pl.in_chain[f]; });
}

// The chain partition as the kernels rely on it: every front is handled once
// (level lists or a chain); a chain front's children are earlier fronts of its
// own component or fronts below the chain levels; no other front has a chain
// child; the level kernels' entry ranges stop before the chain fronts' entries.
static bool check_chains(const Plan &pl, const Symbolic &sym) {
    const int32_t ns = pl.ns;
    std::vector<int32_t> seen((size_t)ns, 0), comp((size_t)ns, -1), grp((size_t)ns, -1);
    for (int32_t s : pl.lvl_small_sn) seen[s]++;
    for (int32_t s : pl.lvl_large_sn) seen[s]++;
    const int32_t nc = (int32_t)pl.chain_comp_ptr.size() - 1;
    for (int32_t c = 0; c < nc; ++c)
        for (int32_t g = pl.chain_comp_ptr[c]; g < pl.chain_comp_ptr[c + 1]; ++g)
            for (int32_t t = pl.chain_grp_ptr[g]; t < pl.chain_grp_ptr[g + 1]; ++t) {
                const int32_t s = pl.chain_sn[t];
                seen[s]++;
                comp[s] = c;
                grp[s] = g;
                if (!pl.in_chain[s] || pl.sn_rptr[s + 1] - pl.sn_rptr[s] > CHAIN_R) return false;
            }
    for (int32_t s = 0; s < ns; ++s) {
        if (seen[s] != 1) return false;
        const int32_t L = sym.sn_level[s];
        for (int32_t u = pl.ch_ptr[s]; u < pl.ch_ptr[s + 1]; ++u) {
            const int32_t c = pl.ch_list[u];
            if (pl.in_chain[s]) {
                if (pl.in_chain[c] ? (comp[c] != comp[s] || grp[c] >= grp[s]) : sym.sn_level[c] >= pl.chain_L0)
                    return false;
            } else if (pl.in_chain[c]) {
                return false;
            }
        }
        if (pl.in_chain[s]) {
            if (pl.ent_front[2 * (size_t)s] < pl.ent_lvl_mid[L] || pl.ent_front[2 * (size_t)s + 1] > pl.ent_lvl_ptr[L + 1])
                return false;
        } else if (pl.ent_front[2 * (size_t)s + 1] > pl.ent_lvl_mid[L]) {
            return false;
        }
    }
    return true;
}

// Assembly map of the numeric factorization (the extend-add of the paper's
// multifrontal factorization, Sec. 2.2): per level, the front entries that
// receive a value, each with its sources in the order the sum is formed -- the
// entry of K, then (after the static regularization of a pivot diagonal) the
// children's update-matrix entries in child order -- so the device forms every
// entry independently and the result does not depend on scheduling.  Also the
// segments of front storage cleared first (the whole front for small fronts,
// the lower part of each column for large ones), in chunks of ZCHUNK entries.
static bool build_assembly_map(Plan &pl, const std::vector<int64_t> &task_base, int64_t nnzK) {
    constexpr int64_t ZCHUNK = 8192;
    pl.ent_lvl_ptr.assign((size_t)pl.nlevels + 1, 0);
    pl.zseg_lvl_ptr.assign((size_t)pl.nlevels + 1, 0);
    pl.ent_lvl_mid.assign((size_t)pl.nlevels, 0);
    pl.zseg_lvl_mid.assign((size_t)pl.nlevels, 0);
    pl.ent_front.assign(2 * (size_t)pl.ns, 0);
    pl.ent_dst.clear(); pl.ent_reg.clear(); pl.ent_src.clear(); pl.zseg_off.clear(); pl.zseg_len.clear();
    pl.ent_sptr.assign(1, 0);
    std::vector<int32_t> cnt((size_t)pl.max_r + 1, 0);
    std::vector<int64_t> pos((size_t)pl.max_r + 1, 0);
    std::vector<uint8_t> live((size_t)pl.max_r + 1, 0);
    std::vector<int32_t> touched;
    auto zseg = [&](int64_t off, int64_t len) {
        for (int64_t c = 0; c < len; c += ZCHUNK) {
            pl.zseg_off.push_back(off + c);
            pl.zseg_len.push_back((int32_t)std::min(ZCHUNK, len - c));
        }
    };
    for (int32_t L = 0; L < pl.nlevels; ++L) {
        pl.ent_lvl_mid[L] = -1;
        for (int32_t t = pl.lvl_ptr[L]; t < pl.lvl_ptr[L + 1]; ++t) {
            const int32_t s = pl.lvl_sn[t];
            const int64_t r = pl.sn_rptr[s + 1] - pl.sn_rptr[s];
            const int32_t k = pl.sn_first[s + 1] - pl.sn_first[s];
            if (pl.in_chain[s] && pl.ent_lvl_mid[L] < 0) {   // the level's chain fronts start here
                pl.ent_lvl_mid[L] = (int64_t)pl.ent_dst.size();
                pl.zseg_lvl_mid[L] = (int64_t)pl.zseg_off.size();
            }
            pl.ent_front[2 * (size_t)s] = (int64_t)pl.ent_dst.size();
            if (pl.in_chain[s]) {
                // assembled in LDS: no segments to clear
            } else if (r <= SMALL_R) {
                zseg(pl.fr_off[s], r * r);
            } else {
                for (int64_t j = 0; j < r; ++j) zseg(pl.fr_off[s] + j * r + j, r - j);
            }
            for (int32_t j = 0; j < (int32_t)r; ++j) {
                const int64_t task = task_base[s] + j;
                touched.clear();
                auto touch = [&](int32_t row, int n) {
                    if (!live[row]) { live[row] = 1; touched.push_back(row); }
                    cnt[row] += n;
                };
                for (int64_t a = pl.asm_ptr[task]; a < pl.asm_ptr[task + 1]; ++a) touch(pl.asm_row[a], 1);
                if (j < k) touch(j, 0);
                for (int64_t u = pl.ctb_ptr[task]; u < pl.ctb_ptr[task + 1]; ++u) {
                    const int32_t c = pl.ctb_child[u], jc = pl.ctb_col[u];
                    const int32_t mc = (int32_t)(pl.rel_ptr[c + 1] - pl.rel_ptr[c]);
                    const int32_t *rl = pl.rel.data() + pl.rel_ptr[c];
                    for (int32_t i = jc; i < mc; ++i) touch(rl[i], 1);
                }
                std::sort(touched.begin(), touched.end());
                for (int32_t row : touched) {
                    pos[row] = pl.ent_sptr.back();
                    pl.ent_dst.push_back(pl.fr_off[s] + (int64_t)j * r + row);
                    pl.ent_reg.push_back(j < k && row == j ? pl.reg_sign[pl.sn_first[s] + j] : (int8_t)-1);
                    pl.ent_sptr.push_back(pl.ent_sptr.back() + cnt[row]);
                }
                pl.ent_src.resize((size_t)pl.ent_sptr.back());
                for (int64_t a = pl.asm_ptr[task]; a < pl.asm_ptr[task + 1]; ++a)
                    pl.ent_src[pos[pl.asm_row[a]]++] = -pl.asm_src[a] - 1;
                for (int64_t u = pl.ctb_ptr[task]; u < pl.ctb_ptr[task + 1]; ++u) {
                    const int32_t c = pl.ctb_child[u], jc = pl.ctb_col[u];
                    const int64_t rc = pl.sn_rptr[c + 1] - pl.sn_rptr[c];
                    const int64_t kc = pl.sn_first[c + 1] - pl.sn_first[c];
                    const int32_t mc = (int32_t)(rc - kc);
                    const int32_t *rl = pl.rel.data() + pl.rel_ptr[c];
                    const int64_t ucol = pl.fr_off[c] + (kc + jc) * rc + kc;   // update block column jc
                    for (int32_t i = jc; i < mc; ++i) pl.ent_src[pos[rl[i]]++] = ucol + i;
                }
                for (int32_t row : touched) { live[row] = 0; cnt[row] = 0; }
            }
            pl.ent_front[2 * (size_t)s + 1] = (int64_t)pl.ent_dst.size();
        }
        pl.ent_lvl_ptr[L + 1] = (int64_t)pl.ent_dst.size();
        pl.zseg_lvl_ptr[L + 1] = (int64_t)pl.zseg_off.size();
        if (pl.ent_lvl_mid[L] < 0) {
            pl.ent_lvl_mid[L] = pl.ent_lvl_ptr[L + 1];
            pl.zseg_lvl_mid[L] = pl.zseg_lvl_ptr[L + 1];
        }
    }
    // every index the device will follow stays inside the front buffer / the K values
    for (int64_t d : pl.ent_dst) if (d < 0 || d >= pl.front_total) return false;
    for (int64_t v : pl.ent_src) if (v >= pl.front_total || (v < 0 && -v - 1 >= nnzK)) return false;
    for (size_t z = 0; z < pl.zseg_off.size(); ++z)
        if (pl.zseg_off[z] < 0 || pl.zseg_off[z] + pl.zseg_len[z] > pl.front_total) return false;
    return true;
}

int build_plan(qg_handle *h) {
    // a batch arrives with its device fronts formed copy by copy (qg_setup_batch)
    if (h->ncopy == 1) {
        int rc0 = group_fronts(h->sym, h->fronts);
        if (rc0) return rc0;
    }
    const Symbolic &sym = h->fronts;
    const KktPattern &kp = h->kp;
    Plan &pl = h->plan;
    const int32_t N = sym.N;
    const int32_t ns = (int32_t)sym.super_ptr.size() - 1;
    pl.ns = ns;
    pl.nlevels = sym.nlevels;
    pl.sn_first = sym.super_ptr;
    pl.sn_rptr = sym.rows_ptr;
    pl.sn_rows = sym.rows;
    pl.fr_off.assign((size_t)ns + 1, 0);
    pl.uv_off.assign((size_t)ns + 1, 0);
    pl.max_r = 0;
    for (int32_t s = 0; s < ns; ++s) {
        const int64_t r = pl.sn_rptr[s + 1] - pl.sn_rptr[s];
        const int64_t k = pl.sn_first[s + 1] - pl.sn_first[s];
        pl.fr_off[s + 1] = pl.fr_off[s] + r * r;
        pl.uv_off[s + 1] = pl.uv_off[s] + (r - k);
        pl.max_r = std::max<int32_t>(pl.max_r, (int32_t)r);
    }
    if (pl.max_r > MAX_FRONT_R) return QG_ERR_SIZE;
    pl.front_total = pl.fr_off[ns];
    pl.uv_total = pl.uv_off[ns];
    pl.dinv_off.assign((size_t)ns + 1, 0);
    for (int32_t s = 0; s < ns; ++s) {
        const int64_t r = pl.sn_rptr[s + 1] - pl.sn_rptr[s];
        const int64_t k = pl.sn_first[s + 1] - pl.sn_first[s];
        pl.dinv_off[s + 1] = pl.dinv_off[s] + (r > SMALL_R ? ((k + NB - 1) / NB) * NB * NB : 0);
    }
    pl.dinv_total = pl.dinv_off[ns];
    pl.sinv_off.assign((size_t)ns + 1, 0);
    for (int32_t s = 0; s < ns; ++s) {
        const int64_t r = pl.sn_rptr[s + 1] - pl.sn_rptr[s];
        const int64_t k = pl.sn_first[s + 1] - pl.sn_first[s];
        int64_t sz = 0;
        if (r > SMALL_R)
            for (int64_t J0 = 0; J0 < k; J0 += SB) {
                const int64_t ld = (std::min<int64_t>(SB, k - J0) + NB - 1) / NB * NB;
                sz += 2 * ld * ld;
            }
        pl.sinv_off[s + 1] = pl.sinv_off[s] + sz;
    }
    pl.sinv_total = pl.sinv_off[ns];
    // W_J = L(rows below the super-block, J) X_J per super-block of a large front
    pl.w_off.assign((size_t)ns + 1, 0);
    for (int32_t s = 0; s < ns; ++s) {
        const int64_t r = pl.sn_rptr[s + 1] - pl.sn_rptr[s];
        const int64_t k = pl.sn_first[s + 1] - pl.sn_first[s];
        int64_t sz = 0;
        if (r > SMALL_R)
            for (int64_t J0 = 0; J0 < k; J0 += SB) {
                const int64_t J1 = std::min<int64_t>(k, J0 + SB);
                sz += (r - J1) * (J1 - J0);
            }
        pl.w_off[s + 1] = pl.w_off[s] + sz;
    }
    pl.w_total = pl.w_off[ns];
    // levels
    pl.lvl_ptr.assign((size_t)pl.nlevels + 1, 0);
    for (int32_t s = 0; s < ns; ++s) pl.lvl_ptr[sym.sn_level[s] + 1]++;
    for (int32_t L = 0; L < pl.nlevels; ++L) pl.lvl_ptr[L + 1] += pl.lvl_ptr[L];
    pl.lvl_sn.assign(ns, 0);
    {
        std::vector<int32_t> fill(pl.lvl_ptr.begin(), pl.lvl_ptr.end() - 1);
        for (int32_t s = 0; s < ns; ++s) pl.lvl_sn[fill[sym.sn_level[s]]++] = s;
    }
    select_chains(pl, sym, h->st.chains != 0);
    pl.lvl_small_maxr.assign((size_t)pl.nlevels, 0);
    pl.lvl_small_rsum.assign((size_t)pl.nlevels, 0);
    pl.lvl_tiny_cnt.assign((size_t)pl.nlevels, 0);
    pl.lvl_tiny8_cnt.assign((size_t)pl.nlevels, 0);
    pl.lvl_small_ptr.assign((size_t)pl.nlevels + 1, 0);
    pl.lvl_large_ptr.assign((size_t)pl.nlevels + 1, 0);
    pl.lvl_small_sn.clear();
    pl.lvl_large_sn.clear();
    pl.large_flops = 0.0;
    for (int32_t L = 0; L < pl.nlevels; ++L) {
        for (int32_t t = pl.lvl_ptr[L]; t < pl.lvl_ptr[L + 1]; ++t) {
            const int32_t s = pl.lvl_sn[t];
            const int64_t r = pl.sn_rptr[s + 1] - pl.sn_rptr[s];
            if (pl.in_chain[s]) continue;          // factored and solved by the chain kernels
            if (r <= SMALL_R) {
                pl.lvl_small_sn.push_back(s);
                pl.lvl_small_maxr[L] = std::max<int32_t>(pl.lvl_small_maxr[L], (int32_t)r);
                pl.lvl_small_rsum[L] += r;
            } else {
                pl.lvl_large_sn.push_back(s);
                const double rr = (double)r, kk = (double)(pl.sn_first[s + 1] - pl.sn_first[s]);
                // sum over the k pivots j of (r - j - 1)^2
                pl.large_flops += kk * (rr - 1) * (rr - 1) - (rr - 1) * kk * (kk - 1) + (kk - 1) * kk * (2 * kk - 1) / 6;
            }
        }
        pl.lvl_small_ptr[L + 1] = (int32_t)pl.lvl_small_sn.size();
        pl.lvl_large_ptr[L + 1] = (int32_t)pl.lvl_large_sn.size();
        // fronts of at most TINY_R rows first; a level with at least TINY_MIN of them runs them on lane
        // groups (the order of a level's small fronts does not matter: they are independent)
        auto b = pl.lvl_small_sn.begin() + pl.lvl_small_ptr[L], e = pl.lvl_small_sn.begin() + pl.lvl_small_ptr[L + 1];
        auto mid = std::stable_partition(b, e, [&](int32_t f) { return pl.sn_rptr[f + 1] - pl.sn_rptr[f] <= TINY_R; });
        const int32_t nt = (int32_t)(mid - b);
        pl.lvl_tiny_cnt[L] = (h->st.tiny_groups && nt >= TINY_MIN) ? nt : 0;
        if (pl.lvl_tiny_cnt[L] > 0) {   // the row sum then covers the other small fronts only
            for (auto it = b; it != mid; ++it) pl.lvl_small_rsum[L] -= pl.sn_rptr[*it + 1] - pl.sn_rptr[*it];
            // and the fronts of at most TINY_R8 rows first among them (factored in smaller tiles)
            auto mid8 = std::stable_partition(b, mid, [&](int32_t f) { return pl.sn_rptr[f + 1] - pl.sn_rptr[f] <= TINY_R8; });
            pl.lvl_tiny8_cnt[L] = (int32_t)(mid8 - b);
        }
    }
    // children (increasing index)
    pl.ch_ptr.assign((size_t)ns + 1, 0);
    for (int32_t s = 0; s < ns; ++s) if (sym.sn_parent[s] >= 0) pl.ch_ptr[sym.sn_parent[s] + 1]++;
    for (int32_t s = 0; s < ns; ++s) pl.ch_ptr[s + 1] += pl.ch_ptr[s];
    pl.ch_list.assign(pl.ch_ptr[ns], 0);
    {
        std::vector<int32_t> fill(pl.ch_ptr.begin(), pl.ch_ptr.end() - 1);
        for (int32_t s = 0; s < ns; ++s)
            if (sym.sn_parent[s] >= 0) pl.ch_list[fill[sym.sn_parent[s]]++] = s;
    }
    // relative indices of each supernode's update rows in its parent's row list
    pl.rel_ptr.assign((size_t)ns + 1, 0);
    pl.rel.clear();
    for (int32_t s = 0; s < ns; ++s) {
        const int32_t k = pl.sn_first[s + 1] - pl.sn_first[s];
        const int32_t ps = sym.sn_parent[s];
        const int32_t *rs = pl.sn_rows.data() + pl.sn_rptr[s];
        const int64_t r = pl.sn_rptr[s + 1] - pl.sn_rptr[s];
        if (ps >= 0) {
            const int32_t *rp = pl.sn_rows.data() + pl.sn_rptr[ps];
            const int32_t *re = pl.sn_rows.data() + pl.sn_rptr[ps + 1];
            const int32_t *cur = rp;
            for (int64_t i = k; i < r; ++i) {
                cur = std::lower_bound(cur, re, rs[i]);
                if (cur == re || *cur != rs[i]) return QG_ERR_PATTERN;   // inconsistent analysis
                pl.rel.push_back((int32_t)(cur - rp));
            }
        } else if (r != k) {
            return QG_ERR_PATTERN;
        }
        pl.rel_ptr[s + 1] = (int64_t)pl.rel.size();
    }
    // column tasks, level by level
    std::vector<int64_t> task_base(ns, 0);
    pl.task_ptr.assign((size_t)pl.nlevels + 1, 0);
    pl.task_sn.clear();
    pl.task_col.clear();
    for (int32_t L = 0; L < pl.nlevels; ++L) {
        for (int32_t t = pl.lvl_ptr[L]; t < pl.lvl_ptr[L + 1]; ++t) {
            const int32_t s = pl.lvl_sn[t];
            const int32_t r = (int32_t)(pl.sn_rptr[s + 1] - pl.sn_rptr[s]);
            task_base[s] = (int64_t)pl.task_sn.size();
            for (int32_t j = 0; j < r; ++j) { pl.task_sn.push_back(s); pl.task_col.push_back(j); }
        }
        pl.task_ptr[L + 1] = (int64_t)pl.task_sn.size();
    }
    const int64_t ntask = (int64_t)pl.task_sn.size();
    pl.task0 = task_base;
    // K entries per task
    std::vector<int32_t> col2sn(N);
    for (int32_t s = 0; s < ns; ++s)
        for (int32_t c = pl.sn_first[s]; c < pl.sn_first[s + 1]; ++c) col2sn[c] = s;
    const int64_t nnzK = (int64_t)kp.Ki.size();
    std::vector<int64_t> ent_task(nnzK);
    std::vector<int32_t> ent_row(nnzK);
    pl.asm_ptr.assign((size_t)ntask + 1, 0);
    for (int32_t j = 0; j < N; ++j)
        for (int64_t t = kp.Kp[j]; t < kp.Kp[j + 1]; ++t) {
            const int32_t a = sym.iperm[kp.Ki[t]], b = sym.iperm[j];
            const int32_t c = std::min(a, b), r = std::max(a, b);
            const int32_t s = col2sn[c];
            const int32_t *rs = pl.sn_rows.data() + pl.sn_rptr[s];
            const int32_t *re = pl.sn_rows.data() + pl.sn_rptr[s + 1];
            const int32_t *it = std::lower_bound(rs, re, r);
            if (it == re || *it != r) return QG_ERR_PATTERN;
            ent_task[t] = task_base[s] + (c - pl.sn_first[s]);
            ent_row[t] = (int32_t)(it - rs);
            pl.asm_ptr[ent_task[t] + 1]++;
        }
    for (int64_t t = 0; t < ntask; ++t) pl.asm_ptr[t + 1] += pl.asm_ptr[t];
    pl.asm_src.assign(nnzK, 0);
    pl.asm_row.assign(nnzK, 0);
    {
        std::vector<int64_t> fill(pl.asm_ptr.begin(), pl.asm_ptr.end() - 1);
        for (int64_t t = 0; t < nnzK; ++t) {
            const int64_t d = fill[ent_task[t]]++;
            pl.asm_src[d] = t;
            pl.asm_row[d] = ent_row[t];
        }
    }
    // child contributions per task, in child order
    pl.ctb_ptr.assign((size_t)ntask + 1, 0);
    for (int32_t s = 0; s < ns; ++s)
        for (int32_t u = pl.ch_ptr[s]; u < pl.ch_ptr[s + 1]; ++u) {
            const int32_t c = pl.ch_list[u];
            for (int64_t i = pl.rel_ptr[c]; i < pl.rel_ptr[c + 1]; ++i)
                pl.ctb_ptr[task_base[s] + pl.rel[i] + 1]++;
        }
    for (int64_t t = 0; t < ntask; ++t) pl.ctb_ptr[t + 1] += pl.ctb_ptr[t];
    pl.ctb_child.assign(pl.ctb_ptr[ntask], 0);
    pl.ctb_col.assign(pl.ctb_ptr[ntask], 0);
    pl.ctb_src.assign(pl.ctb_ptr[ntask], 0);
    {
        std::vector<int64_t> fill(pl.ctb_ptr.begin(), pl.ctb_ptr.end() - 1);
        for (int32_t s = 0; s < ns; ++s)
            for (int32_t u = pl.ch_ptr[s]; u < pl.ch_ptr[s + 1]; ++u) {
                const int32_t c = pl.ch_list[u];
                for (int64_t i = pl.rel_ptr[c]; i < pl.rel_ptr[c + 1]; ++i) {
                    const int64_t d = fill[task_base[s] + pl.rel[i]]++;
                    pl.ctb_child[d] = c;
                    pl.ctb_col[d] = (int32_t)(i - pl.rel_ptr[c]);
                    pl.ctb_src[d] = task_base[c] + (pl.sn_first[c + 1] - pl.sn_first[c]) + (i - pl.rel_ptr[c]);
                }
            }
    }
    // kind of each permuted column: 0 primal x, 1 equality y, 2 cone z
    pl.reg_sign.assign(N, 0);
    for (int32_t c = 0; c < N; ++c) {
        const int32_t o = sym.perm[c];
        pl.reg_sign[c] = (int8_t)(o < h->n ? 0 : (o < h->n + h->p ? 1 : 2));
    }
    if (!build_assembly_map(pl, task_base, nnzK)) return QG_ERR_PATTERN;
    if (!check_chains(pl, sym)) return QG_ERR_PATTERN;
    // copies of a batch: every offset of copy z is copy 0's plus z times a fixed distance per front
    pl.ncopy = h->ncopy;
    if (ns % pl.ncopy) return QG_ERR_PATTERN;
    pl.ns1 = ns / pl.ncopy;
    pl.copy_stride.assign((size_t)pl.ns1, CopyStride());
    if (pl.ncopy > 1) {
        for (int32_t s = 0; s < pl.ns1; ++s) {
            CopyStride &c = pl.copy_stride[s];
            const int32_t t = s + pl.ns1;
            c.f = pl.fr_off[t] - pl.fr_off[s];
            c.dinv = pl.dinv_off[t] - pl.dinv_off[s];
            c.sinv = pl.sinv_off[t] - pl.sinv_off[s];
            c.w = pl.w_off[t] - pl.w_off[s];
            c.task = pl.task0[t] - pl.task0[s];
            c.col = pl.sn_first[t] - pl.sn_first[s];
            c.front = pl.ns1;
            for (int32_t z = 1; z < pl.ncopy; ++z) {
                const int32_t u = s + z * pl.ns1;
                if (pl.fr_off[u] != pl.fr_off[s] + z * c.f || pl.dinv_off[u] != pl.dinv_off[s] + z * c.dinv ||
                    pl.sinv_off[u] != pl.sinv_off[s] + z * c.sinv || pl.w_off[u] != pl.w_off[s] + z * c.w ||
                    pl.task0[u] != pl.task0[s] + z * c.task || pl.sn_first[u] != pl.sn_first[s] + z * c.col ||
                    pl.sn_rptr[u + 1] - pl.sn_rptr[u] != pl.sn_rptr[s + 1] - pl.sn_rptr[s] ||
                    pl.sn_first[u + 1] - pl.sn_first[u] != pl.sn_first[s + 1] - pl.sn_first[s])
                    return QG_ERR_PATTERN;
            }
        }
    }
    return QG_OK;
}

// Ruiz equilibration of the data (a setup-time preprocessing; the paper states none): D (n), E (p) and
// F (m), each pass dividing every column of the data matrix [P A' G'; A 0 0; G 0 0] (x columns, P taken
// symmetric) and every row of A and of G by the square root of its largest magnitude (1 for an empty
// one), the rows of one second-order cone by a common factor (the largest over the cone's rows, so
// that the scaled cone is the same cone); then the objective scaling k = 1 / max(1, |D c|_inf).  The
// scaled problem is  k D P D, k D c, E A D, E b, F G D, F h  with  x = D x^, y = E y^ / k,
// z = F z^ / k, s = s^ / F.
static void ruiz_scaling(const ProblemPattern &pp, const std::vector<double> &c, int passes, double &k,
                         std::vector<double> &dsc) {
    const int32_t n = pp.n, p = pp.p, m = pp.m;
    dsc.assign((size_t)n + p + m, 1.0);
    double *D = dsc.data(), *E = D + n, *F = E + p;
    std::vector<double> cx((size_t)n), rw((size_t)p + m);
    for (int it = 0; it < passes; ++it) {
        std::fill(cx.begin(), cx.end(), 0.0);
        std::fill(rw.begin(), rw.end(), 0.0);
        for (int32_t j = 0; j < n; ++j) {
            for (int64_t t = pp.P.colptr[j]; t < pp.P.colptr[j + 1]; ++t) {
                const int32_t i = pp.P.rowind[t];
                const double v = std::fabs(D[i] * pp.P.val[t] * D[j]);
                cx[j] = std::max(cx[j], v);
                cx[i] = std::max(cx[i], v);
            }
            for (int64_t t = pp.A.colptr[j]; t < pp.A.colptr[j + 1]; ++t) {
                const int32_t i = pp.A.rowind[t];
                const double v = std::fabs(E[i] * pp.A.val[t] * D[j]);
                cx[j] = std::max(cx[j], v);
                rw[i] = std::max(rw[i], v);
            }
            for (int64_t t = pp.G.colptr[j]; t < pp.G.colptr[j + 1]; ++t) {
                const int32_t i = pp.G.rowind[t];
                const double v = std::fabs(F[i] * pp.G.val[t] * D[j]);
                cx[j] = std::max(cx[j], v);
                rw[p + i] = std::max(rw[p + i], v);
            }
        }
        for (int32_t k2 = 0; k2 < pp.nsoc; ++k2) {
            double mx = 0.0;
            for (int32_t i = pp.soc_off[k2]; i < pp.soc_off[k2 + 1]; ++i) mx = std::max(mx, rw[p + i]);
            for (int32_t i = pp.soc_off[k2]; i < pp.soc_off[k2 + 1]; ++i) rw[p + i] = mx;
        }
        auto f = [](double v) { return v > 0.0 ? 1.0 / std::sqrt(v) : 1.0; };
        for (int32_t j = 0; j < n; ++j) D[j] *= f(cx[j]);
        for (int32_t i = 0; i < p + m; ++i) E[i] *= f(rw[i]);   // E and F are contiguous
    }
    double cn = 0.0;
    for (int32_t j = 0; j < n; ++j) cn = std::max(cn, std::fabs(D[j] * c[j]));
    k = 1.0 / std::max(1.0, cn);
}

int upload_static_values(qg_handle *h, bool vectors) {
    const ProblemPattern &pp = h->pp;
    const KktPattern &kp = h->kp;
    const int32_t n = h->n, p = h->p, N = h->N;
    int rc;
    // K upper values without the (3,3) block (zeros there); with Ruiz equilibration the scaled data
    h->kval_static.assign(kp.Ki.size(), 0.0);
    if (h->ruiz > 0) {
        // the objective scaling takes the current c (at setup the host copy, later the device one)
        std::vector<double> c;
        if (vectors) {
            c = h->hc;
        } else {
            c.resize((size_t)n);
            if (n > 0)
                QG_HIP(h, hipMemcpyAsync(c.data(), h->d.craw.p, sizeof(double) * n, hipMemcpyDeviceToHost,
                                         h->stream));
            QG_HIP(h, hipStreamSynchronize(h->stream));
        }
        ruiz_scaling(pp, c, h->ruiz, h->ruiz_k, h->ruiz_dsc);
        const double *D = h->ruiz_dsc.data(), *E = D + n, *F = E + p;
        const double k = h->ruiz_k;
        for (int32_t j = 0; j < n; ++j) {
            for (int64_t t = pp.P.colptr[j]; t < pp.P.colptr[j + 1]; ++t)
                h->kval_static[kp.posP[t]] = k * D[pp.P.rowind[t]] * pp.P.val[t] * D[j];
            for (int64_t t = pp.A.colptr[j]; t < pp.A.colptr[j + 1]; ++t)
                h->kval_static[kp.posA[t]] = E[pp.A.rowind[t]] * pp.A.val[t] * D[j];
            for (int64_t t = pp.G.colptr[j]; t < pp.G.colptr[j + 1]; ++t)
                h->kval_static[kp.posG[t]] = F[pp.G.rowind[t]] * pp.G.val[t] * D[j];
        }
        std::vector<double> rsc((size_t)N);
        for (int32_t j = 0; j < n; ++j) rsc[j] = 1.0 / (k * D[j]);
        for (int32_t i = n; i < N; ++i) rsc[i] = 1.0 / D[i];
        if ((rc = dupload(h, h->d.rz_dsc, h->ruiz_dsc))) return rc;
        if ((rc = dupload(h, h->d.rz_rsc, rsc))) return rc;
    } else {
        for (size_t t = 0; t < pp.P.val.size(); ++t) h->kval_static[kp.posP[t]] = pp.P.val[t];
        for (size_t t = 0; t < pp.A.val.size(); ++t) h->kval_static[kp.posA[t]] = pp.A.val[t];
        for (size_t t = 0; t < pp.G.val.size(); ++t) h->kval_static[kp.posG[t]] = pp.G.val[t];
    }
    rc = dupload(h, h->d.kval, h->kval_static);
    if (rc) return rc;
    // full symmetric CSR of the static part (both triangles; the (3,3) block excluded)
    std::vector<int64_t> rp((size_t)N + 1, 0);
    auto in33 = [&](int32_t i, int32_t j) { return i >= n + p && j >= n + p; };
    for (int32_t j = 0; j < N; ++j)
        for (int64_t t = kp.Kp[j]; t < kp.Kp[j + 1]; ++t) {
            const int32_t i = kp.Ki[t];
            if (in33(i, j)) continue;
            rp[i + 1]++;
            if (i != j) rp[j + 1]++;
        }
    for (int32_t i = 0; i < N; ++i) rp[i + 1] += rp[i];
    std::vector<int32_t> rc_(rp[N]);
    std::vector<double> rv(rp[N]);
    {
        std::vector<int64_t> fill(rp.begin(), rp.end() - 1);
        // rows receive entries in increasing column order: first the upper
        // part of row i (columns j > i come from columns j of the upper CSC),
        // so build per row and sort
        for (int32_t j = 0; j < N; ++j)
            for (int64_t t = kp.Kp[j]; t < kp.Kp[j + 1]; ++t) {
                const int32_t i = kp.Ki[t];
                if (in33(i, j)) continue;
                const double v = h->kval_static[t];
                rc_[fill[i]] = j; rv[fill[i]++] = v;
                if (i != j) { rc_[fill[j]] = i; rv[fill[j]++] = v; }
            }
        std::vector<std::pair<int32_t, double>> tmp;
        for (int32_t i = 0; i < N; ++i) {
            tmp.clear();
            for (int64_t t = rp[i]; t < rp[i + 1]; ++t) tmp.push_back({rc_[t], rv[t]});
            std::sort(tmp.begin(), tmp.end());
            for (int64_t t = rp[i]; t < rp[i + 1]; ++t) { rc_[t] = tmp[t - rp[i]].first; rv[t] = tmp[t - rp[i]].second; }
        }
    }
    h->kr_nnz = rp[N];
    if ((rc = dupload(h, h->d.kr_ptr, rp))) return rc;
    if ((rc = dupload(h, h->d.kr_col, rc_))) return rc;
    if ((rc = dupload(h, h->d.kr_val, rv))) return rc;
    if (vectors && h->ruiz > 0) {
        // the caller's vectors are kept; the scaled ones are formed on the device
        if ((rc = dupload(h, h->d.craw, h->hc))) return rc;
        if ((rc = dupload(h, h->d.braw, h->hb))) return rc;
        if ((rc = dupload(h, h->d.hraw, h->hh))) return rc;
        if ((rc = dalloc(h, h->d.c, h->hc.size()))) return rc;
        if ((rc = dalloc(h, h->d.b, h->hb.size()))) return rc;
        if ((rc = dalloc(h, h->d.h, h->hh.size()))) return rc;
    } else if (vectors) {
        if ((rc = dupload(h, h->d.c, h->hc))) return rc;
        if ((rc = dupload(h, h->d.b, h->hb))) return rc;
        if ((rc = dupload(h, h->d.h, h->hh))) return rc;
    }
    if (h->ruiz > 0) return launch_scale_vectors(h);   // new scalings or new vectors
    return QG_OK;
}

}  // namespace qg
