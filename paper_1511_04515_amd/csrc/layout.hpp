// Plain-old-data structures shared by the host runtime and the gfx950 kernels.
// One InstDesc describes one circuit instance: device pointers to its
// (possibly shared) symbolic arrays, its own values, its workspace and its
// run state.  Every node id inside is in the internal (permuted) numbering.
#pragma once

#include <stdint.h>

namespace expri {

constexpr int kMaxKrylov = 60;        // hard upper bound on m
constexpr int kHLd = kMaxKrylov + 1;  // leading dimension of stored Hessenbergs

// Rows of a length-n vector one thread of a bs-thread workgroup keeps in
// registers (rows t + e bs, e < E).  The basis columns and C's ELL columns
// are padded with zeros to E bs rows so that these rows load without a
// bound test.  n <= max_rows_per_thread(bs) bs: 18 rows at 512 threads, 9
// otherwise.  The transient kernel is compiled for a bound EM on E (9, or 18
// at 512 threads): the smaller bound keeps it to the registers of two
// workgroups per compute unit.
constexpr int max_rows_per_thread(int bs) { return bs == 512 ? 18 : 9; }
constexpr int rows_per_thread(int n, int bs) {
  return n <= 4 * bs ? 4 : n <= 6 * bs ? 6 : n <= 9 * bs ? 9 : n <= 12 * bs ? 12 : 18;
}
constexpr int kRecFixed = 16;         // fixed doubles per trace record (8 + 8 step features)
constexpr int kFeat = 8;              // step features seen by the learned controller
constexpr int kPhases = 6;            // profiled phases of a step
// status codes (mirror expri_status of the public header)
constexpr int kOK = 0, kEINVAL = -1, kENOMEM = -2, kESINGULAR = -3, kEKRYLOV = -4,
              kESTEPMIN = -5, kENONFINITE = -6, kEHIP = -7, kEPATTERN = -8, kENOCONV = -9;

struct Opts {
  double E_rr;        // step error budget (V, infinity norm)
  double eps_K;       // Krylov residual tolerance (V)
  double alpha;       // step reduction after a rejection
  double beta;        // step growth
  double h_init, h_min, h_max;
  double breakdown;   // happy-breakdown threshold, relative to max |H|
  double piv_tol;     // small-pivot threshold, relative to the row's max |G_k|
  int32_t grow_if_rejects_lt;
  int32_t m_max;
  int32_t controller; // 1: the learned controller proposes h and the first residual test
  int32_t erc;        // 1: ER-C correction of x_{k+1}
  double gamma;       // ER-C factor
  double ctrl_safety;         // factor on the predicted step
  const uint16_t *ctrl_w;     // bfloat16 network parameters (inference layout)
  const float *ctrl_norm;     // input / output standardisation
};

// Run state of one instance; lives in device memory between launches.
struct InstState {
  double t;           // current time
  double h_prop;      // proposed step
  int32_t bp_idx;     // first breakpoint strictly after t
  int32_t steps;      // accepted steps so far in this run
  int32_t status;     // 0 running/ok, <0 error code
  int32_t done;       // 1 when t reached T (or error)
  int32_t lu_count;   // numeric factorisations in this run
  int32_t rejects;    // total rejected trials
  int32_t arnoldi;    // total Arnoldi iterations
  int32_t lu_valid;   // factors of G_k are current (linear circuits keep them)
  int32_t trials;     // step trials (accepted + rejected)
  int32_t m_err_prev; // Krylov size of the previous accepted step's error MEVP
  int64_t mgs_terms;  // inner products of modified Gram-Schmidt (sum of j+1)
  int64_t comb_terms; // basis columns combined into x_{k+1} and e_rr
  // wall-clock ticks per phase: factor, rhs, arnoldi solve, mgs, phi, trial
  double ph[kPhases];
  // the previous accepted step, as seen by the step features
  double h_prev, rho_prev, err_prev;
  int32_t m_prev, rej_prev;
};

// One level of a flattened triangular-solve schedule: rows of the level are
// handled by groups of G lanes (G a power of two), each lane multiplying P
// stored entries (P is the same for every level of one direction); the
// level's rows need `passes` sweeps of the block.
struct SolveLevel {
  int32_t G, P, passes, rows;  // rows: rows of the level
  int32_t slot_base;  // into slot_pos / slot_col: index (q * P + j) * BS + t
  int32_t row_base;   // into row_of: index q * BS + t / G
};
constexpr int kPassSync = 1;  // pass code flag: last pass of its level

struct InstDesc {
  int32_t n, n_dev, n_src, n_bp;
  int32_t nnz_lu, n_lev, n_ulev, n_probe;
  int32_t has_dev, max_row;  // max_row: longest row of L\U
  // solve passes that one wave holds (at most 64 active lanes): the last
  // l_narrow L passes and the first u_narrow U passes
  int32_t l_narrow, u_narrow;
  double vdd, T, h_max;

  // symbolic (shared by instances of one pattern)
  const int32_t *lu_rowptr, *lu_col, *lu_diag;
  const int32_t *lev_ptr, *lev_rows, *ulev_ptr, *ulev_rows;
  const int32_t *row_grp, *grp_pos, *grp_diag, *grp_ptr, *pair_src, *pair_dst;
  const int32_t *lu_gidx, *jac_ptr, *jac_code, *node_ptr, *node_code;
  const int32_t *g_rowptr, *g_col, *c_rowptr, *c_col, *b_rowptr, *b_col;
  const int32_t *dev_node;      // 3 per device
  // flattened solve schedules (built for the launch block size): the L
  // passes then the U passes, one code each ((active << 16) | (log2 G << 8) |
  // kPassSync; lanes t >= active have no row in the pass); pass q of
  // a direction reads slots base + (q * P + j) * BS + t and row slots
  // base + q * BS + t / G
  const int32_t *pass_code;
  const int32_t *slot_pos, *slot_col, *row_of;
  const int32_t *rdv_pos;             // per row slot of the U passes: position of u_ii (-1: none)
  // the repacking's work lists: slots holding an entry (slot, L\U position)
  // and U row slots holding a row (row slot, position of u_ii); every other
  // slot keeps the 0 (value) or 1 (pivot) written when the workspace is bound
  const int32_t *pk_slot, *pk_pos, *rd_slot, *rd_pos;
  int32_t n_pk, n_rd;
  const int32_t *jpos;                // L\U positions that receive device derivatives
  int32_t n_jpos, pad5;
  int32_t n_lpass, n_upass, pl, pu;   // passes and slots per lane of L and U
  int32_t u_slot_base, u_row_base;    // where the U passes start
  int32_t n_slots, n_srows;           // sizes of slot_pos / row_of
  // C in ELL layout: entry k of row i at k * c_ell_ld + i (column -1 and
  // value 0 on padding, rows n .. c_ell_ld - 1 included)
  const int32_t *c_ell_col;
  int32_t c_ell_k, c_ell_ld;
  const int32_t *perm;          // perm[internal] = caller's node id
  const int32_t *probe;         // internal ids of the probed nodes

  // values (per instance, permuted to the internal numbering)
  const double *g_val, *c_val, *b_val;
  const double *g_lu;           // G_lin scattered to the L\U positions (0 elsewhere)
  const double *c_ell_val;
  const double *dev_par;        // 4 per device: type (+1/-1), K = k' W/L, V_th, lambda
  const int32_t *src_ptr;       // n_src + 1
  const double *src_t, *src_v;  // PWL corners
  const double *bp;             // breakpoints in (0, T), then T

  // workspace (per instance)
  double *xk, *x1, *w, *p, *z, *tmp, *e;
  double *devI, *devD, *devI1;  // per device: I(x_k), dI/d(d,g,s)(x_k), I(x_{k+1})
  double *Ik;                   // node currents at x_k
  double *lu;                   // L\U values
  double *sval;                 // L\U values in solve-slot order (0 on padding)
  double *rdv;                  // 1 / u_ii per U row slot (1 where the slot has no row)
  double *V, *Ve;               // Krylov bases, n x (m_max + 1), column j at j * ldv
  double *H, *He;               // Hessenbergs, kHLd x kMaxKrylov column-major
  double *mat;                  // small dense matrices when they do not fit in LDS
  int64_t ldv;                  // column stride of V / Ve (>= E BS, multiple of 32; rows n.. are 0)
  InstState *state;
  double *trace;                // records of kRecFixed + n_probe doubles
  int32_t trace_cap;            // records available
  int32_t vcols;                // columns of V and of Ve (m_max + 1)
};

}  // namespace expri
