// Host-side sparse structure of the hierarchy: row split and pattern of the auxiliary smoothed
// prolongation (Def. def:aux_sp), symbolic Galerkin product, transposes, colouring.
#pragma once

#include <cstdint>
#include <vector>

#include "coarsen.hpp"

namespace eamg {

// Block sparsity pattern, column indices ascending within each row.
struct Pattern {
  int n_rows = 0, n_cols = 0;
  std::vector<int64_t> rp;
  std::vector<int> col;
  int64_t nnz() const { return rp.empty() ? 0 : rp.back(); }
};

enum RowType : int { ROW_S = 0, ROW_A = 1, ROW_D = 2 };

// Everything the device needs to assemble P_s numerically.
struct ProlongPlan {
  std::vector<int> type;          // per fine row
  Pattern P;                      // P_s pattern
  std::vector<int64_t> F_ptr;     // per fine row, into F_vtx / F_edge (A rows only)
  std::vector<int> F_vtx, F_edge; // filtered neighbour l and the aux edge {i, l}
};

// Row types and P_s pattern.  cap_S / cap_A: column caps of real-matrix / edge-matrix rows.
//  * cols_S(i) = {agg(i)} U {agg(j) : A_ij structurally nonzero, j not in D}; S row iff
//    |cols_S(i)| <= cap_S, else an edge-matrix (A) row.
//  * F^i: edge neighbours l not in D grouped by agg(l); the group agg(i) and the cap_A - 1 other
//    groups with the largest sum of tr E^il are kept, picked one at a time; sums within the
//    relative band tie_rtol of the largest tie and the smaller coarse id wins.
ProlongPlan plan_prolongation(const Pattern &A, const AuxLevel &aux, const std::vector<int> &agg_of,
                              const std::vector<char> &dmask, int cap_S, int cap_A, double tie_rtol);

// Structural pattern of A * B.
Pattern spgemm_symbolic(const Pattern &A, const Pattern &B);

// Transposed pattern; src[q] = index in P of entry q of the transpose.
Pattern transpose_pattern(const Pattern &P, std::vector<int64_t> &src);

// Greedy colouring in smallest-last order (vertices removed by minimum remaining degree, lowest
// id on ties; coloured in reverse removal order with the smallest colour unused by neighbours).
std::vector<int> greedy_coloring(int n, const int64_t *rp, const int *col, int &n_colors);
inline std::vector<int> greedy_coloring(const Pattern &A, int &n_colors) {
  return greedy_coloring(A.n_rows, A.rp.data(), A.col.data(), n_colors);
}

// Symmetric permutation of a square pattern: row/col v -> inv[v].  Columns re-sorted;
// src[q] = index in A of entry q of the result.
Pattern permute_pattern(const Pattern &A, const std::vector<int> &perm, const std::vector<int> &inv,
                        std::vector<int64_t> &src);

// Rows permuted by the fine permutation, columns renumbered by the coarse one (re-sorted).
Pattern permute_rect(const Pattern &P, const std::vector<int> &perm_rows,
                     const std::vector<int> &inv_cols, std::vector<int64_t> &src);

}  // namespace eamg
