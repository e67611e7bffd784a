// Batches of problems on one sparsity pattern: stacking of the data and
// replication of one problem's analysis (see batch.cpp).
#pragma once

#include <cstdint>
#include <vector>

#include "analysis.hpp"
#include "qg.h"

namespace qg {

// Sizes of one problem and the batch size; maps indices of problem i into the stack.
struct StackMap {
    int32_t k = 1, n = 0, p = 0, m = 0, l = 0;
    int64_t kkt(int32_t i, int32_t v) const;    // KKT index v (x, y, z order) of problem i
    int64_t zrow(int32_t i, int32_t w) const;   // cone row w of problem i
};

struct StackedCsc {
    std::vector<int64_t> colptr;
    std::vector<int32_t> rowind;
    std::vector<double> val;
    qg_csc csc{};
};

void replicate_symbolic(const Symbolic &a, const StackMap &mp, Symbolic &out);
void stack_problem(const StackMap &mp, const qg_csc *P, const qg_csc *A, const qg_csc *G, StackedCsc &Ps,
                   StackedCsc &As, StackedCsc &Gs);

}  // namespace qg
