// Host symbolic analysis for the ER solver: everything about a circuit that
// depends only on its sparsity, computed once per distinct pattern.
//
// The paper factorises only the conductance Jacobian G_k (Algorithm 2, one
// LU_decompose(G_k) per step, reused when h is reduced).  Its pattern is the
// union of G_lin and the MOSFET stamp positions; it is fixed for the whole
// run, so ordering, fill, level schedules and scatter maps are built here and
// only numbers change on the GPU.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "layout.hpp"

namespace expri {

struct PatternInput {
  int32_t n = 0;
  // G_lin, C: n x n CSR;  B: n x n_src CSR  (0-based, sorted, no duplicates)
  const int32_t *g_rowptr = nullptr, *g_col = nullptr;
  const int32_t *c_rowptr = nullptr, *c_col = nullptr;
  const int32_t *b_rowptr = nullptr, *b_col = nullptr;
  int32_t n_src = 0;
  int32_t n_dev = 0;
  const int32_t *dev_d = nullptr, *dev_g = nullptr, *dev_s = nullptr;  // node ids, -1 GND, -2 VDD
};

// Symbolic data shared by every instance with the same pattern.  All node ids
// are in the permuted ("internal") numbering unless stated otherwise.
struct Symbolic {
  int32_t n = 0, n_src = 0, n_dev = 0;
  std::vector<int32_t> perm;      // perm[new] = old
  std::vector<int32_t> iperm;     // iperm[old] = new

  // combined L\U pattern in CSR by rows (strict lower = L, diag + upper = U)
  std::vector<int32_t> lu_rowptr, lu_col, lu_diag;
  // level schedules: forward (L solve and the row-wise refactor) and
  // backward (U solve)
  std::vector<int32_t> lev_ptr, lev_rows, ulev_ptr, ulev_rows;
  // refactor: per row i the pivot groups (one per k in L(i,:), increasing k)
  std::vector<int32_t> row_grp;   // [n+1]
  std::vector<int32_t> grp_pos;   // position of l_ik in row i
  std::vector<int32_t> grp_diag;  // position of u_kk
  std::vector<int32_t> grp_ptr;   // range into the update pairs
  std::vector<int32_t> pair_src, pair_dst;  // a[dst] -= l_ik * a[src]

  // assembly of G_k into the LU storage: value index of G_lin (or -1) and
  // the device-derivative contributions of each LU position
  std::vector<int32_t> lu_gidx;   // [nnz_lu]
  std::vector<int32_t> jac_ptr;   // [nnz_lu + 1]
  std::vector<int32_t> jac_code;  // (dev << 4) | (cross << 3) | (eq << 2) | var
  // device current gather per node: (dev << 1) | eq  (eq 0 = drain, 1 = source)
  std::vector<int32_t> node_ptr, node_code;
  // permuted G_lin, C, B patterns (rows and columns permuted); *_src maps a
  // permuted nonzero back to its index in the caller's value array
  std::vector<int32_t> g_rowptr, g_col, g_src;
  std::vector<int32_t> c_rowptr, c_col, c_src;
  std::vector<int32_t> b_rowptr, b_col, b_src;
  // devices: terminals in the internal numbering (rails keep -1 / -2)
  std::vector<int32_t> dev_node;  // [3 * n_dev]  d, g, s
  // DC blocks: strongly connected components of the DC dependency graph
  std::vector<int32_t> block_of;  // [n] internal ids
  int32_t n_blocks = 0;

  int64_t flops = 0;              // multiply-adds of one refactor
  int32_t max_row = 0;
  uint64_t hash = 0;
  std::string error;
};

// Builds the symbolic data; returns false (with sym.error) on bad input.
bool analyse(const PatternInput &in, Symbolic &sym);

// Hash of a pattern (for sharing symbolic data across instances).
uint64_t pattern_hash(const PatternInput &in);

// Flattened schedule of one triangular solve for block size bs (lower = L
// solve, else U solve); appends to the slot / row arrays.  All levels of one
// direction share one slot count P per lane.
bool build_solve_schedule(const Symbolic &S, int bs, bool lower, std::vector<SolveLevel> &sched,
                          std::vector<int32_t> &slot_pos, std::vector<int32_t> &slot_col,
                          std::vector<int32_t> &row_of, int force_p = 0);

// The passes of a schedule in execution order, one code each:
// (active << 16) | (log2(G) << 8) | kPassSync on the last pass of a level,
// where lanes t < active hold the pass's rows (rows in the pass times G).
std::vector<int32_t> pass_codes(const std::vector<SolveLevel> &sched, int bs);

// ELL layout of C's (permuted) pattern: entry k of row i at k * ld + i
// (ld = n when 0), -1 = padding; returns the ELL width.
int32_t build_c_ell(const Symbolic &S, std::vector<int32_t> &col, int ld = 0);

// Validates a 0-based CSR pattern (sorted, no duplicates, in range).
bool check_csr_pattern(int32_t rows, int32_t cols, const int32_t *rp, const int32_t *ci, const char *name,
                       std::string &err);

// Fill-reducing order of a symmetric graph (adjacency without self loops) by
// recursive BFS-level bisection (nested dissection).  Exposed for tests.
std::vector<int32_t> nested_dissection(int32_t n, const std::vector<int32_t> &adj_ptr,
                                       const std::vector<int32_t> &adj);

}  // namespace expri
