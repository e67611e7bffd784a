// Host analysis of the KKT pattern: the reordering, permutation and symbolic
// factorization that the paper runs once per sparsity pattern (Sec. 2.2),
// plus the maps the device kernels use every iteration.
#pragma once

#include <cstdint>
#include <vector>

#include "qg.h"

namespace qg {

// Validated problem pattern (+ values) in canonical form.
struct CscData {
    int32_t nrow = 0, ncol = 0;
    std::vector<int64_t> colptr;   // ncol + 1
    std::vector<int32_t> rowind;
    std::vector<double> val;
};

struct ProblemPattern {
    int32_t n = 0, m = 0, p = 0, l = 0, nsoc = 0;
    std::vector<int32_t> q;        // SOC dimensions
    std::vector<int32_t> soc_off;  // nsoc + 1: row offsets within z (starting at l)
    CscData P, A, G;               // P: upper triangle
};

// Upper-CSC pattern of K (eq. 2) in the original ordering, and where each
// piece of data lands in its value array.
struct KktPattern {
    int32_t N = 0;
    std::vector<int64_t> Kp;       // N + 1
    std::vector<int32_t> Ki;
    std::vector<int64_t> posP, posA, posG;   // per input entry (CSC order of P, A, G)
    std::vector<int64_t> diag;     // N: position of each diagonal entry
    std::vector<int64_t> blk33;    // (3,3) block: orthant diagonals (l), then per SOC the
                                   // upper triangle column by column (b = 0..q-1, a = 0..b)
    std::vector<int64_t> blk33_off;  // nsoc + 1: offsets of each SOC's entries in blk33 (after l)
};

struct Symbolic {
    int32_t N = 0;
    std::vector<int32_t> perm, iperm, parent;
    std::vector<int64_t> colcount;
    std::vector<int32_t> super_fund, super_ptr;
    std::vector<int64_t> rows_ptr;
    std::vector<int32_t> rows;
    // supernodal tree (relaxed partition)
    std::vector<int32_t> sn_parent;          // parent supernode (-1 root)
    std::vector<int32_t> sn_level;           // 0 for leaves
    int32_t nlevels = 0;
    int64_t nnz_L = 0;
    double flops = 0.0;
};

int build_problem_pattern(ProblemPattern &pp, int32_t n, int32_t m, int32_t p,
                          const qg_csc *P, const qg_csc *A, const qg_csc *G,
                          int32_t l, int32_t nsoc, const int32_t *q, bool need_values);
void build_kkt_pattern(const ProblemPattern &pp, KktPattern &kp);

// The ordering rule and every step after it (see analysis.cpp); ordering is
// QG_ORDER_MD or QG_ORDER_ND (step 3).
void analyze_pattern(const KktPattern &kp, Symbolic &sym, int ordering = QG_ORDER_MD);

// Exposed for tests of the ordering alone: order of the graph (both
// triangles, no self loops), approximate-degree rule with merging.
void min_degree_order(int32_t N, const std::vector<int64_t> &Gp, const std::vector<int32_t> &Gi,
                      std::vector<int32_t> &order);
// Nested dissection of the same kind of graph (rule in analysis.cpp).
void nd_order(int32_t N, const std::vector<int64_t> &Gp, const std::vector<int32_t> &Gi,
              std::vector<int32_t> &order);

}  // namespace qg
