// The multifrontal engine: Algorithm 2 (with Algorithm 1 inside) for one
// circuit too large for one workgroup.  The host drives the step: it launches
// the kernels of grid.hip on one stream and reads back the few numbers that
// decide the control flow (the Krylov residual, happy breakdown, the error
// norm, a singular pivot).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "frontal.hpp"
#include "layout.hpp"

namespace expri {

// the circuit values in the caller's numbering (host arrays, copied)
struct GridValues {
  const double *g_val, *c_val, *b_val;     // CSR values of G_lin, C, B
  const double *kind, *kp, *wl, *vth, *lam;  // per device (kind: +1 NMOS, -1 PMOS)
  int32_t n_src;
  const int32_t *npts;                      // PWL points per source
  const double *const *t;                   // PWL times per source
  const double *const *v;                   // PWL values per source
  double vdd, T;
};

struct GridOpts {
  double E_rr, eps_K, alpha, beta, h_init, h_min, h_max, breakdown, piv_tol;
  int32_t grow_if_rejects_lt, m_max, trace_cap;
};

// One accepted step as recorded in the trace (the layout of the transient
// kernel's records: t, h, h_try, m, m_err, rejects, err, rho, eight feature
// slots, then the probed voltages).
struct GridStepRec {
  double t, h, h_try, err, rho;
  int32_t m, m_err, rejects;
};

struct GridEngine {
  FrontalSym fs;
  GridOpts o{};
  hipStream_t stream = nullptr;
  int32_t n_probe = 0;
  double vdd = 1.0, T = 0.0, h_max = 0.0;
  std::vector<double> bps;  // source corners in (0, T), then T
  std::string err;

  // device memory (owned)
  std::vector<void *> allocs;
  // symbolic
  int32_t *d_perm = nullptr, *d_c0 = nullptr, *d_nc = nullptr, *d_fsz = nullptr, *d_parent = nullptr;
  int32_t *d_r_ptr = nullptr, *d_r_idx = nullptr, *d_rel = nullptr, *d_u_off = nullptr;
  int32_t *d_ch_ptr = nullptr, *d_ch = nullptr, *d_lev_front = nullptr;
  int64_t *d_f_off = nullptr, *d_ent_pos = nullptr;
  int32_t *d_ent_row = nullptr, *d_ent_g = nullptr, *d_ent_jptr = nullptr, *d_ent_jcode = nullptr;
  int32_t *d_g_rowptr = nullptr, *d_g_col = nullptr, *d_c_rowptr = nullptr, *d_c_col = nullptr;
  int32_t *d_b_rowptr = nullptr, *d_b_col = nullptr, *d_dev_node = nullptr, *d_node_ptr = nullptr;
  int32_t *d_node_code = nullptr, *d_src_ptr = nullptr, *d_probe = nullptr;
  // per-step work lists: extend-add passes, panel fronts and update tiles
  struct Step {
    int32_t k0, chunk, n_diag, n_panel, n_tiles;
    int32_t *diag = nullptr, *panel = nullptr, *tiles = nullptr;
  };
  struct Level {
    int32_t first, count;  // into lev_front
    int32_t n_small_parents = 0;  // fronts with children whose update matrices are <= 32 x 32
    int32_t *small_parents = nullptr;
    std::vector<std::pair<int32_t, int32_t *>> extend;  // (items, device list) per pass
    int32_t n_small = 0, n_big = 0;  // solve: fronts with f <= 64 (a wave each) and the rest
    int32_t *small = nullptr, *big = nullptr;
    int32_t big_maxp = 0;  // the most pivots of a front in big
    // workgroup size of the pivot-block solves with one right-hand side: 512
    // threads once a block's update rows outnumber 256 threads (the few large
    // fronts near the root)
    int tri_bs() const { return big_maxp > 256 + 32 ? 512 : 256; }
    int32_t n_fwd = 0, n_bwd = 0;  // solve GEMV items (front, 64-row chunk)
    int32_t *fwd = nullptr, *bwd = nullptr;
    int32_t n_lu32 = 0, n_lu64 = 0;  // fronts factored whole by one wave (f <= 32, f <= 64)
    int32_t *lu32 = nullptr, *lu64 = nullptr;
    int32_t n_trmv = 0;        // (front, 64-row chunk) of the fronts with inverted pivot blocks
    int32_t *trmv = nullptr;
    std::vector<Step> steps;
  };
  std::vector<Level> levels;
  // values
  double *d_g_val = nullptr, *d_c_val = nullptr, *d_b_val = nullptr, *d_par = nullptr;
  double *d_src_t = nullptr, *d_src_v = nullptr;
  // numeric
  double *d_F = nullptr, *d_upd = nullptr;
  // pivot blocks with more than kInvPivots pivots are inverted after each
  // factorisation (L11^{-1} and U11^{-1} in one p x p array per front), and
  // their triangular solves become grid-wide products
  int64_t *d_inv_off = nullptr;  // per front: offset into d_Finv, -1 if not inverted
  double *d_Finv = nullptr, *d_tmp = nullptr;
  int32_t n_inv_items = 0, max_p_inv = 0;
  int32_t *d_inv_items = nullptr;
  unsigned long long *d_rowmax = nullptr;
  int32_t *d_bad = nullptr;
  double *d_xk = nullptr, *d_x1 = nullptr, *d_w = nullptr, *d_p = nullptr, *d_z = nullptr, *d_r = nullptr;
  double *d_bs = nullptr, *d_u = nullptr, *d_sl = nullptr, *d_e = nullptr, *d_y = nullptr;
  double *d_devI0 = nullptr, *d_devI1 = nullptr, *d_devD = nullptr, *d_devD1 = nullptr;
  double *d_V = nullptr, *d_Ve = nullptr, *d_H = nullptr, *d_He = nullptr, *d_mat = nullptr;
  double *d_part = nullptr, *d_h1 = nullptr, *d_h2 = nullptr;
  double *d_scm = nullptr, *d_sce = nullptr;  // per basis: beta, ||w||^2, breakdown, 1/||w||
  double *d_out = nullptr;                    // hess_phi1 output: d, d2, rho
  double *d_oute = nullptr;
  double *d_red = nullptr;                    // reduction results
  // the learned step controller (bfloat16 network and standardisation owned
  // by the context; null: the paper's alpha / beta control)
  const uint16_t *ctrl_w = nullptr;
  const float *ctrl_norm = nullptr;
  double ctrl_safety = 1.0;
  float *d_feat = nullptr, *d_cout = nullptr;  // one feature vector, (m, log10 h)
  int64_t ldv = 0;
  bool factored = false;

  // counters of the last call
  int64_t lu_count = 0, arnoldi = 0, trials = 0, mgs_terms = 0, comb_terms = 0, rejects = 0;
  double phase_s[6] = {0, 0, 0, 0, 0, 0};
  std::vector<double> trace;  // records of the last transient call
  double t_reached = 0.0, next_h = 0.0;
  int32_t steps = 0;
  double kernel_s = 0.0;

  ~GridEngine();
  // returns an expri status code; err holds the message
  int setup(const PatternInput &pin, const GridValues &val, const int32_t *probe, int32_t n_probe,
            const GridOpts &opts, hipStream_t s, int32_t leaf);
  int factor(const double *x_caller);
  int solve(const double *b_caller, double *y_caller);
  int mevp(const double *v_caller, double *out_caller, double h, double eps, int32_t *m, double *rho);
  int dc(double *x_caller, double t0);
  // adaptive run to T (grid == nullptr) or replay of the given accepted times
  int run(double *x_caller, double t0, const double *grid, int32_t n_grid, int32_t max_steps, double E_rr,
          double eps_K, double h0, GridStepRec *last);
  // diagnostic timings (seconds per repetition): 0 solve pair, 7 refactor
  int diag(int what, int reps, double *sec);

 private:
  template <class T>
  T *dalloc(size_t count);
  template <class T>
  T *dupload(const std::vector<T> &v);
  int fail(int code, const std::string &msg);
  int hip(hipError_t e, const char *what);
  int factor_internal(const double *x);
  int solve_internal(double *b, int nr = 1);  // in place, new order; nr = 2: b and b + n
  struct Basis {
    double *V, *H, *sc, *out;
    int m;
    bool exact;
  };
  int basis_start(Basis &B, const double *v);
  int converge(Basis &B, double h, double eps, double *rho, int want2, int m_first);
  int arnoldi_step(Basis &B);
  int read_scalars(const double *d, double *h, size_t count);
};

}  // namespace expri
