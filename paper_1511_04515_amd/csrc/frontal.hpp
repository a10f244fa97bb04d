// Host symbolic analysis of one large circuit for the multifrontal engine.
//
// The step factorises only G_k = G_lin + J_dev(x_k) (Algorithm 2,
// LU_decompose(G_k), once per accepted step and reused when h shrinks).  For a
// circuit too large for one workgroup, the factorisation is organised as a
// tree of dense frontal matrices: a nested-dissection order of the symmetrised
// pattern of G_k gives a separator tree; every tree node (a leaf subdomain or
// a separator) is one front whose pivot columns are contiguous in the new
// order.  The front of node s is the dense matrix on the index set
// I_s = cols(s) ∪ R_s, where R_s holds the later rows that the pivot columns of
// s (and the update matrices of its children) reach.  Its partial LU gives the
// factors of the pivot columns and the Schur complement on R_s, which is
// added into the parent's front (extend-add).  Every array here depends only
// on the pattern; the GPU fills the numbers.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "symbolic.hpp"

namespace expri {

struct FrontalSym {
  int32_t n = 0, n_src = 0, n_dev = 0;
  std::vector<int32_t> perm, iperm;  // perm[new] = old, iperm[old] = new
  int32_t n_front = 0;
  // fronts in postorder (children before parents)
  std::vector<int32_t> c0, nc;       // pivot columns [c0, c0 + nc) in the new order
  std::vector<int32_t> fsz;          // f_s = nc + |R_s|
  std::vector<int32_t> parent;       // -1 at a root
  std::vector<int32_t> height;       // 0 at a leaf, 1 + max over children
  std::vector<int32_t> r_ptr, r_idx; // R_s, increasing new indices (>= c0 + nc)
  std::vector<int32_t> rel;          // [r_ptr]: local index in the parent's front of R_s[a]
  std::vector<int64_t> f_off;        // offset (doubles) of front s, column-major f_s x f_s
  int64_t front_doubles = 0;
  std::vector<int32_t> u_off;        // offset of the solve update vector of s (|R_s| doubles)
  int64_t upd_doubles = 0;
  std::vector<int32_t> owner;        // [n] the front whose pivot columns hold node (new id)
  // fronts by height (the fronts of one height are independent)
  std::vector<int32_t> lev_ptr, lev_front;
  std::vector<int32_t> ch_ptr, ch;   // children of each front
  // assembly of G_k into the fronts: one entry per distinct front position
  std::vector<int64_t> ent_pos;      // position (doubles) in the fronts buffer
  std::vector<int32_t> ent_row;      // row of G_k (new order) of the entry
  std::vector<int32_t> ent_g;        // index into the permuted G_lin values, or -1
  std::vector<int32_t> ent_jptr;     // [n_ent + 1]
  std::vector<int32_t> ent_jcode;    // (dev << 3) | (eq << 2) | var; eq 0 = drain row, 1 = source row
  // permuted G_lin, C, B (rows and columns in the new order); *_src maps a
  // permuted nonzero to its index in the caller's value array
  std::vector<int32_t> g_rowptr, g_col, g_src;
  std::vector<int32_t> c_rowptr, c_col, c_src;
  std::vector<int32_t> b_rowptr, b_col, b_src;
  std::vector<int32_t> dev_node;     // [3 n_dev] d, g, s in the new order (rails keep -1 / -2)
  // device current gather per node: (dev << 1) | eq
  std::vector<int32_t> node_ptr, node_code;
  int64_t lu_entries = 0;            // stored factor entries: sum nc (2 f - nc)
  double flops = 0.0;                // flops of one numeric factorisation
  int32_t max_front = 0, max_nc = 0;
  std::string error;
};

// Builds the analysis; leaf = largest subdomain kept as one front.
bool analyse_frontal(const PatternInput &in, FrontalSym &fs, int32_t leaf = 32);

}  // namespace expri
