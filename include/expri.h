/*
 * expri -- exponential Rosenbrock-Euler transient solver with the invert-Krylov
 * matrix-exponential-vector product, for gfx950 (MI355X).
 *
 * Method: Zhuang, Yu, Kang, Wang, Cheng, "An Algorithmic Framework for
 * Efficient Large-Scale Circuit Simulation Using Exponential Integrators",
 * DAC 2015.  The circuit is the DAE of the paper's background section,
 *     C x' = -G_lin x - I_dev(x) + B u(t),
 * with C symmetric positive semi-definite (it may be singular), G_lin the
 * linear conductances, I_dev the MOSFET currents (level-1 model) and u
 * piecewise linear.  Each step (Algorithm 2) linearises at x_k, factorises
 * only G_k = G_lin + dI_dev/dx (one LU per accepted step, reused when the step
 * is reduced), evaluates the phi-function products on the invert Krylov
 * subspace K_m(-G_k^{-1} C, v) (Algorithm 1, MEVP_IKS) and accepts the step
 * when the local nonlinear error estimate (section "Local Nonlinear Error
 * Estimator") is within E_rr.
 *
 * Conventions for every entry point
 *   - Units are SI (V, A, S, F, s).  Node ids are 0-based; EXPRI_GND and
 *     EXPRI_VDD denote the ideal rails.
 *   - Host input arrays are copied during the call; the caller may free them
 *     on return.  Arguments documented as "device" are device pointers that the
 *     caller owns (e.g. PyTorch tensors) and that must stay valid for the call.
 *   - Work is queued on the HIP stream given to expri_setup; every entry point
 *     that produces results synchronises that stream before returning.  A
 *     batch whose instances need different block sizes (see expri_setup)
 *     runs its transient kernel as one launch per block size, concurrently:
 *     the first on that stream, the others on streams the context creates
 *     (default priority), forked from and joined back to it with events.
 *   - Every call returns an expri_status; nothing throws, aborts or prints.
 *     expri_last_error() gives a message for the last failure.  After an error
 *     in a transient call the caller's state vectors hold the last accepted
 *     state.
 *   - A batch: expri_setup takes n_inst circuits.  Instances with identical
 *     sparsity share their symbolic analysis; each instance is integrated
 *     independently (its own time grid, status and trace).  Per-instance
 *     device vectors are passed as a host array of n_inst device pointers.
 */
#ifndef EXPRI_H
#define EXPRI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EXPRI_GND (-1)
#define EXPRI_VDD (-2)

typedef struct expri_ctx expri_ctx;

typedef enum {
  EXPRI_OK = 0,
  EXPRI_EINVAL = -1,     /* bad argument or circuit description */
  EXPRI_ENOMEM = -2,     /* device or host allocation failed */
  EXPRI_ESINGULAR = -3,  /* |u_ii| <= piv_tol * max_j |G_k(i,j)| in the LU of G_k */
  EXPRI_EKRYLOV = -4,    /* m_max Arnoldi steps without residual <= eps_krylov */
  EXPRI_ESTEPMIN = -5,   /* the step fell below h_min */
  EXPRI_ENONFINITE = -6, /* NaN or Inf in the state or the small exponential */
  EXPRI_EHIP = -7,       /* a HIP runtime call failed */
  EXPRI_EPATTERN = -8,   /* instance data inconsistent with its pattern */
  EXPRI_ENOCONV = -9     /* DC Newton iteration did not converge */
} expri_status;

/* CSR matrix, 0-based, column indices sorted and unique within a row. */
typedef struct {
  int32_t n_rows, n_cols, nnz;
  const int32_t *rowptr; /* n_rows + 1 */
  const int32_t *colidx; /* nnz */
  const double *val;     /* nnz */
} expri_csr;

/* Level-1 (Shichman-Hodges) MOSFETs with channel-length modulation:
 * triode I = K (V_ov V_ds - V_ds^2/2)(1 + lam V_ds), saturation
 * I = K V_ov^2 / 2 (1 + lam V_ds), K = kp * wl; PMOS is the mirror image. */
typedef struct {
  int32_t n;
  const int8_t *type;                /* +1 NMOS, -1 PMOS */
  const int32_t *d, *g, *s;          /* terminals: node id, EXPRI_GND or EXPRI_VDD */
  const double *kp, *wl, *vth, *lam; /* A/V^2, -, V (magnitude), 1/V */
} expri_mosfets;

/* Piecewise-linear waveform: value v[i] at t[i], linear between corners,
 * constant outside [t[0], t[npts-1]]; t strictly increasing. */
typedef struct {
  int32_t npts;
  const double *t, *v;
} expri_pwl;

/* One circuit instance. */
typedef struct {
  int32_t n;          /* unknowns (node voltages) */
  expri_csr G;        /* n x n linear conductance matrix */
  expri_csr C;        /* n x n capacitance matrix, symmetric PSD */
  expri_csr B;        /* n x n_src source incidence */
  expri_mosfets dev;  /* nonlinear devices */
  int32_t n_src;
  const expri_pwl *src; /* n_src waveforms, one per column of B */
  double vdd;         /* value of the EXPRI_VDD rail */
  double T;           /* end of the transient */
  int32_t n_probe;    /* nodes recorded in each trace record */
  const int32_t *probe;
} expri_circuit;

/* Solver options (Algorithm 2 parameters and the readings documented in the
 * design notes).  expri_default_opts fills: E_rr = 1e-6 V, eps_krylov =
 * 0.1 E_rr, alpha = 0.5, beta = 2, grow_if_rejects_lt = 5, h_init = 1e-13 s,
 * h_min = 1e-18 s, h_max = 0 (meaning T / 20 per instance), m_max = 60,
 * breakdown = 1e-13, piv_tol = 1e-13, block_size = 0 (automatic),
 * trace_cap = 4096 records per instance and launch. */
typedef struct {
  double E_rr, eps_krylov, alpha, beta, h_init, h_min, h_max, breakdown, piv_tol;
  int32_t grow_if_rejects_lt, m_max, block_size, trace_cap;
  /* ER-C (the modified correction term, Algorithm 2 with O_pt_c): when erc is
   * 1, every trial's x_{k+1} is corrected by -gamma h phi_2(hJ) C^{-1} dF,
   * evaluated on the error estimate's Krylov basis; acceptance uses the
   * estimate of the uncorrected x_{k+1}.  Default erc = 0, gamma = 0.1. */
  int32_t erc;
  /* slots per lane of the flattened triangular-solve passes (1, 2, 4 or 8;
   * 0 = chosen per direction from the pass count and the padding; a value
   * that the longest row of a level does not fit in 64 lanes falls back to
   * the automatic choice) */
  int32_t solve_slots;
  /* at most this many workgroups of the transient kernel resident on the GPU
   * at a time, each taking the batch's instances in turn (0 = one per compute
   * unit; fewer leave compute units to other work) */
  int32_t max_workgroups;
  /* engine: 0 = automatic (a single circuit with n > 9216 goes to the
   * multifrontal engine, everything else to the one-workgroup engine),
   * 1 = one-workgroup engine only, 2 = the multifrontal engine (one circuit;
   * no ER-C, no expri_set_values / bind_workspace /
   * run_noalloc / lu_pattern) */
  int32_t engine;
  double gamma;
  /* 1: every instance gets its own copy of the symbolic data even when it
   * shares its pattern with another (a measurement aid: the same batch with
   * and without one shared copy of the index arrays); default 0 */
  int32_t private_patterns;
  /* 1: the launch configuration of every distinct pattern (block size and
   * rows-per-thread bound, solve slots) is measured instead of taken from
   * the rule: each candidate runs the pattern's first instance for a short
   * transient from its DC point on this GPU and the fastest per accepted
   * step is kept (the rule's choice unless another is 3 % faster).  The
   * choice is cached for the life of the process by pattern hash, so a
   * pattern is measured once; expri_instance_config reports it.  The trial
   * runs make expri_setup take longer (seconds for tens of patterns) and
   * allocate device memory.  Default 0 (the rule; block_size and
   * solve_slots as given). */
  int32_t autotune;
} expri_opts;

/* The launch configuration of instance inst: cfg[0] block size, cfg[1] the
 * transient kernel's rows-per-thread bound, cfg[2] and cfg[3] the slots per
 * lane of the L and U solve passes.  EINVAL for a bad index or a context of
 * the multifrontal engine. */
expri_status expri_instance_config(const expri_ctx *ctx, int32_t inst, int32_t cfg[4]);

/* Number of trial contexts the autotuner has run in this process (each
 * measures one candidate configuration on a set of patterns). */
int64_t expri_autotune_runs(void);

/* Counters of the last transient or DC call of one instance. */
typedef struct {
  double t;          /* time reached */
  int32_t steps;     /* accepted steps (DC: Newton iterations) */
  int32_t lu_count;  /* numeric factorisations of G_k */
  int32_t rejects;   /* rejected trials */
  int32_t arnoldi;   /* Arnoldi iterations (both MEVPs) */
  int32_t status;    /* expri_status of this instance */
  /* device time per phase of the step loop (seconds, from the GPU wall
   * clock): 0 device stamp + LU refactor, 1 right-hand-side solves, 2 Arnoldi
   * SpMV + triangular solves, 3 modified Gram-Schmidt, 4 Hessenberg
   * exponential and residual, 5 trial update, re-stamp, error set-up */
  double phase_s[6];
  int32_t trials;     /* step trials (accepted + rejected) */
  int64_t mgs_terms;  /* Gram-Schmidt inner products (sum over Arnoldi steps of j+1) */
  int64_t comb_terms; /* Krylov basis columns combined into x_{k+1} and e_rr */
} expri_run_info;

/* Result of one adaptive step (expri_step) of one instance. */
typedef struct {
  double t;          /* time reached: t + h_used (or the source corner / T it landed on) */
  double h_used;     /* size of the accepted trial (0 if no step was taken: t >= T) */
  double h_next;     /* proposed size of the next step (alpha / beta rule) */
  double err_inf;    /* ||e_rr||_inf of the accepted trial (V) */
  double krylov_res; /* residual rho_m(h_used) of the step's MEVP (V) */
  int32_t m;         /* Krylov dimension of the step's MEVP */
  int32_t m_err;     /* Krylov dimension of the error estimate's MEVP */
  int32_t n_reject;  /* rejected trials before the accepted one */
  int32_t status;    /* expri_status of this instance */
} expri_step_info;

/* Trace record layout (doubles): t, h, h_try (the first trial before
 * clipping to a source corner or T), m, m_err, rejects, err_inf,
 * krylov_residual, the eight step features (below), then the n_probe probed
 * voltages at t.  The features of step k are computed before its step size
 * is chosen: log10 ||r_k||_inf (A), m_{k-1} / 60, log10 h_{k-1} (the
 * nominal size of step k-1: its h_try when it landed on a corner at the
 * first try, else its h),
 * log10 rho_{k-1}, log10(1 + max |du/dt| * 1 ns), log10 ||F_k(x_k)||_inf
 * (F_k(x) = J_dev(x_k) x - I_dev(x), A), log10(err_{k-1} / E_rr) and the
 * rejections of step k-1 (logarithms of values below 1e-30 are clamped). */
#define EXPRI_REC_FIXED 16

/* Fill o with the defaults listed above. */
expri_status expri_default_opts(expri_opts *o);

/* Analyse and upload n_inst circuits (host data, copied): the inputs of
 * Algorithm 2, i.e. the circuit DAE of the paper's background section
 * (C, G_lin, B, the devices behind F and the PWL sources u), with the error
 * budget E_rr and the MEVP tolerance of the options.  Builds the
 * symbolic analysis of G_k's pattern (fill-reducing order, L\U pattern, level
 * schedules, refactor update lists, stamp maps) once per distinct pattern.
 * Each instance runs in one workgroup of 256 threads when n <= 2048 and
 * 512 up to n = 9216 (or opts.block_size, which must then satisfy
 * n <= 18 x 512 at 512 threads and n <= 9 block_size otherwise); the
 * instances of one block size and one rows-per-thread bound of the transient
 * kernel (9, or 18 at 512 threads when n > 4608) form a launch class.
 * hip_stream: the hipStream_t all work is queued on (NULL = default stream).
 * EINVAL for malformed input; ENOMEM / EHIP on allocation failure. */
expri_status expri_setup(expri_ctx **ctx, const expri_circuit *ckt, int32_t n_inst,
                         const expri_opts *o, void *hip_stream);

/* Replace the values of instance `inst` (0 <= inst < n_inst) by those of
 * *ckt, keeping its symbolic analysis: the circuit data of the system
 * C x' = -G x + F(x) + B u (Section 3) for one more point of a sweep over
 * one topology.  *ckt must have the instance's sparsity pattern (n, G, C and
 * B patterns, device terminals, number of sources), its number of probes and
 * its total number of PWL corners; every value may change: G, C, B, the
 * device parameters, the PWL corners (times and values), vdd and T.  Host
 * arrays are copied before the call returns.  Waits for the context's
 * streams, so no kernel of the context reads the old values.  Every later
 * run, step and DC call factorises afresh; expri_solve and expri_mevp
 * return EINVAL until expri_factor runs again.  EPATTERN if the pattern
 * differs, EINVAL for other mismatches or malformed values (the instance
 * keeps its old values then). */
expri_status expri_set_values(expri_ctx *ctx, int32_t inst, const expri_circuit *ckt);

/* Device workspace the context needs (bytes, 256-byte aligned use). */
expri_status expri_workspace_size(const expri_ctx *ctx, size_t *bytes);

/* Give the context a caller-owned device workspace of at least
 * expri_workspace_size bytes (must outlive the context's use).  Without it
 * the first compute call allocates one.  Queues a kernel on the context's
 * stream that initialises the entries the kernels read but never write (the
 * padding rows of the Krylov basis storage, the empty solve slots), so the
 * caller need not clear the workspace.  EINVAL if too small or misaligned. */
expri_status expri_bind_workspace(expri_ctx *ctx, void *dev_ptr, size_t bytes);

/* DC operating point at time t0 (Algorithm 2, x(0) = DC_solution): x[i]
 * (device, n values each, caller numbering) is the starting guess on entry and
 * the solution on return.  Newton on B u - G_lin x - I_dev(x) = 0 with the
 * gate couplings between strongly connected blocks dropped until the update
 * is below 1e-9 V, then full Newton to 1e-12 V.  ENOCONV / ESINGULAR. */
expri_status expri_dc(expri_ctx *ctx, double *const *x, double t0);

/* Stamp the devices at x (device vectors) and factorise G_k on the GPU
 * (Algorithm 2, LU_decompose(G_k)).  The factors stay in the context for
 * expri_solve / expri_mevp.  ESINGULAR on a small pivot. */
expri_status expri_factor(expri_ctx *ctx, const double *const *x);

/* y[i] = G_k^{-1} b[i] with the factors of the last expri_factor (device
 * vectors, caller numbering; y may not alias b). */
expri_status expri_solve(expri_ctx *ctx, const double *const *b, double *const *y);

/* Algorithm 1 on the factors of the last expri_factor: out[i] =
 * (I - e^{hJ}) v[i], J = -C^{-1} G_k, from the invert Krylov basis grown
 * until the residual norm rho_m(h) <= eps.  m[i] and rho[i] (host arrays of
 * n_inst, may be NULL) receive the basis size and residual.  EKRYLOV. */
expri_status expri_mevp(expri_ctx *ctx, const double *const *v, double *const *out, double h,
                        double eps, int32_t *m, double *rho);

/* Adaptive ER transient of every instance from t0 to its T (Algorithm 2 with
 * step control).  x[i] (device, caller numbering) holds the initial state and
 * receives the final one.  Each accepted step appends one trace record
 * (retrieve with expri_trace).  max_steps_per_launch bounds the work of one
 * kernel launch (<= trace_cap); the call loops until all instances finish. */
expri_status expri_run(expri_ctx *ctx, double *const *x, double t0, int32_t max_steps_per_launch);

/* Replay (parity against a reference time grid): step instance i through
 * the given accepted times t_seq[i][0..n_steps[i]) (host arrays, increasing,
 * > t0), accepting every first trial.  Each step is Algorithm 2's body
 * (stamp, LU_decompose(G_k), MEVP_IKS of Algorithm 1, update), and the error
 * estimate of the local nonlinear error estimator section is still computed
 * and recorded.  The grid is only read during the call; later calls use the
 * instances' source corners again.  Errors as expri_run. */
expri_status expri_run_schedule(expri_ctx *ctx, double *const *x, double t0,
                                const double *const *t_seq, const int32_t *n_steps);

/* One adaptive step of Algorithm 2 for every instance, from (t, x[i]) with
 * proposed size h and error budget tol (V; 0 = the context's E_rr; the Krylov
 * tolerance is tol / 10): the step is clipped to the next source corner and to
 * the instance's T (u stays linear on the step, as the ER step assumes),
 * G_k is factorised once, and trials shrink by alpha, reusing the factors and
 * the Krylov basis, until ||e_rr||_inf <= tol (the trial loop of Algorithm 2;
 * the paper's step control, never the learned controller).  x[i] (device,
 * caller numbering) receives x_{k+1}; info (host array of n_inst, may be
 * NULL) receives the time reached, the accepted size, the next proposed size
 * (beta h after fewer than 5 rejections), the error, the Krylov sizes and the
 * rejections.  An instance with t >= T takes no step (h_used = 0).
 * ESTEPMIN / EKRYLOV / ESINGULAR / ENONFINITE keep x[i] at its input. */
expri_status expri_step(expri_ctx *ctx, double *const *x, double t, double h, double tol,
                        expri_step_info *info);

/* One step of exactly h from (t, x) for every instance: expri_run_schedule
 * with a grid of one point t + h (the first trial is accepted whatever its
 * error estimate); info (host array of n_inst, may be NULL) receives the
 * counters.  For replays of a given grid. */
expri_status expri_step_fixed(expri_ctx *ctx, double *const *x, double t, double h,
                              expri_run_info *info);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): expri_run
 * with the context's workspace placed in a static device array of the
 * library (64 MiB per GPU, held until the process ends) instead of memory the
 * library allocates or the caller binds.  The call itself allocates no device
 * memory.  Results equal expri_run's.  The context's own workspace, if it has
 * one, is left untouched (factors kept for expri_solve / expri_mevp).  Every
 * call on one GPU shares that GPU's array and overwrites it (the padding the
 * kernels read is re-initialised by each call): calls that overlap on one GPU,
 * from any context or thread, race.  EINVAL if expri_workspace_size exceeds
 * 64 MiB; otherwise errors as expri_run. */
expri_status expri_run_noalloc(expri_ctx *ctx, double *const *x, double t0, int32_t max_steps_per_launch);

/* Copy up to cap trace records of instance inst (host buffer of
 * cap * (EXPRI_REC_FIXED + n_probe) doubles); *n_rec = records available. */
expri_status expri_trace(const expri_ctx *ctx, int32_t inst, double *out, int64_t cap, int64_t *n_rec);

/* Summed device duration (HIP events on the context's stream, around the
 * concurrent launches of all launch classes) of the transient-kernel launches
 * of the last expri_run / expri_run_schedule / expri_step call, and their
 * number. */
expri_status expri_kernel_time(const expri_ctx *ctx, double *seconds, int32_t *launches);

/* The launch classes, (block size, rows-per-thread bound of the transient
 * kernel) descending: *n_classes receives their number; for the first
 * min(cap, n) classes block_size[q], max_rows[q] (the bound: 9, or 18 for the
 * 512-thread kernel of circuits with n > 4608; 0 for the multifrontal
 * engine), n_inst[q], workgroups[q] (the transient kernel's grid; its
 * workgroups take the class's instances in turn) and kernel_s[q] (the summed
 * duration of that class's transient-kernel launches in the last transient
 * call, HIP events on the stream it runs on) are written where the array is
 * not NULL, and inst_class (host, n_inst entries, may be NULL) receives the
 * class of every instance. */
expri_status expri_launch_classes(const expri_ctx *ctx, int32_t cap, int32_t *block_size, int32_t *max_rows,
                                  int32_t *n_inst, int32_t *workgroups, double *kernel_s, int32_t *inst_class,
                                  int32_t *n_classes);

/* Diagnostic: device time (seconds per repetition, GPU wall clock) of one
 * building block of the step on instance 0's current factors:
 * what = 0 full G_k solve, 1 L solve, 2 U solve, 3 one Arnoldi step
 * j = arg (C SpMV, solve, Gram-Schmidt against arg + 1 vectors), 4 workgroup
 * reduction, 5 one barrier per solve pass and nothing else, 6 the Hessenberg
 * exponential and residual for m = arg on a synthetic H, 7 assembly and
 * refactor of G_k (with the slot repacking) at the last stamp, 8 the
 * assembly alone, 9 the slot repacking alone, 10 the device stamp alone,
 * 11 the first arg levels of the refactor and the repacking.  It overwrites
 * instance 0's basis, Hessenbergs and solve vector with synthetic data.
 * EXPRI_EINVAL unless 0 <= arg < m_max (and arg >= 1 for what = 6). */
expri_status expri_diag_time(expri_ctx *ctx, int32_t what, int32_t reps, int32_t arg, double *seconds);

/* Threads per workgroup of the first launch class (the largest block size
 * in the batch; one workgroup per instance). */
expri_status expri_block_size(const expri_ctx *ctx, int32_t *bs);

/* Counters of the last transient / DC call of instance inst. */
expri_status expri_get_run_info(const expri_ctx *ctx, int32_t inst, expri_run_info *info);

/* Symbolic data of instance inst (host buffers may be NULL to query sizes):
 * L\U CSR in the internal order (rowptr n+1, col nnz), perm[internal] =
 * caller node id, level counts of the L and U solves and the multiply-adds of
 * one refactor. */
expri_status expri_lu_pattern(const expri_ctx *ctx, int32_t inst, int32_t *rowptr, int32_t *col,
                              int32_t *perm, int64_t *nnz, int32_t *n_lev, int32_t *n_ulev,
                              int64_t *flops);

/* L\U values of instance inst after expri_factor (host buffer of nnz). */
expri_status expri_lu_values(const expri_ctx *ctx, int32_t inst, double *out);

/* Host-only diagnostics of the symbolic analysis (no GPU is touched):
 * expri_symbolic_create analyses one circuit's pattern; expri_symbolic_array
 * copies one of its integer arrays by name ("perm", "lu_rowptr", "lu_col",
 * "lu_diag", "lev_ptr", "lev_rows", "ulev_ptr", "ulev_rows", "row_grp",
 * "grp_pos", "grp_diag", "grp_ptr", "pair_src", "pair_dst", "lu_gidx",
 * "jac_ptr", "jac_code", "node_ptr", "node_code", "g_rowptr", "g_col",
 * "g_src", "c_rowptr", "c_col", "c_src", "b_rowptr", "b_col", "b_src",
 * "dev_node", "block_of"): up to cap values into out (may be NULL), *len =
 * full length.  EINVAL for an unknown name. */
typedef struct expri_symbolic expri_symbolic;
expri_status expri_symbolic_create(expri_symbolic **sym, const expri_circuit *ckt);
/* Build the flattened solve schedules for block size bs (256, 512, 1024)
 * and slots per lane solve_slots (as expri_opts.solve_slots; a value that a
 * row does not fit falls back to the automatic choice), exposed as arrays
 * "lsched" / "usched" (6 ints per level: G, P, passes, rows, slot_base,
 * row_base), "slot_pos", "slot_col", "row_of", "pass_code" (one per pass, L
 * then U: (active << 16) | (log2 G << 8) | 1 on a level's last pass, lanes
 * t >= active holding no row) and "c_ell_col" (ELL pattern of C, followed by
 * its width).  EXPRI_EINVAL for a bad bs or solve_slots, or
 * when a row of L or U has more than 512 off-diagonal entries. */
expri_status expri_symbolic_schedule(expri_symbolic *sym, int32_t bs, int32_t solve_slots);
expri_status expri_symbolic_array(const expri_symbolic *sym, const char *name, int32_t *out, int64_t cap,
                                  int64_t *len);
void expri_symbolic_destroy(expri_symbolic *sym);

/* Host-only diagnostics of the multifrontal analysis used for one large
 * circuit (no GPU is touched): the nested-dissection separator tree of G_k's
 * pattern as a tree of dense fronts (LU_decompose(G_k) of Algorithm 2 organised
 * by fronts).  leaf = the largest subdomain kept as one front.
 * expri_frontal_array copies a named array as int64 (perm, c0, nc, fsz,
 * parent, height, r_ptr, r_idx, rel, f_off, u_off, owner, lev_ptr,
 * lev_front, ch_ptr, ch, ent_pos, ent_row, ent_g, ent_jptr, ent_jcode, g_rowptr,
 * g_col, g_src, c_rowptr, c_col, c_src, b_rowptr, b_col, b_src, dev_node,
 * node_ptr, node_code); expri_frontal_stats writes 8 doubles: fronts, front
 * storage (doubles), stored factor entries, flops of one factorisation,
 * largest front, largest pivot block, heights, update-vector storage. */
typedef struct expri_frontal expri_frontal;
expri_status expri_frontal_create(expri_frontal **f, const expri_circuit *ckt, int32_t leaf);
expri_status expri_frontal_array(const expri_frontal *f, const char *name, int64_t *out, int64_t cap,
                                 int64_t *len);
expri_status expri_frontal_stats(const expri_frontal *f, double *out);
void expri_frontal_destroy(expri_frontal *f);

/* Message of the last failure ("" if none). */
const char *expri_last_error(const expri_ctx *ctx);

/* Release everything the context owns (not a bound workspace). */
void expri_destroy(expri_ctx *ctx);

/* ---------------------------------------------------------------------------
 * Learned step controller (not part of the paper; an addition to Algorithm
 * 2's step control, whose error test still decides acceptance).  A multilayer
 * perceptron 8 -> 64 -> 64 -> 2 with ReLU hidden layers maps eight features
 * of the step to (m, log10 h).  Parameters are EXPRI_MLP_PARAMS floats in the
 * order W1 (64 x 8, row-major), b1 (64), W2 (64 x 64), b2 (64), W3 (2 x 64),
 * b3 (2).  Inputs and targets are standardised with EXPRI_MLP_NORM floats:
 * input mean (8), input std (8), target mean (2), target std (2).  The loss
 * is half the mean squared error over a minibatch.
 *
 * Samples: X is n x 8 and T (targets) n x 2 float32, row-major, device
 * pointers owned by the caller.  Work runs on the stream given at creation;
 * calls that return host results synchronise it.
 * ------------------------------------------------------------------------- */
#define EXPRI_MLP_PARAMS 4866
#define EXPRI_MLP_NORM 20

typedef struct expri_mlp expri_mlp;

/* Training state on the device: float32 parameters (copied from the host
 * array params), zero Adam moments, unit standardisation.  EINVAL for NULL
 * arguments, EHIP/ENOMEM when device memory cannot be had. */
expri_status expri_mlp_create(expri_mlp **m, const float *params, void *hip_stream);
/* Standardisation from the host (EXPRI_MLP_NORM floats; EINVAL unless every
 * std is > 0), or fitted on the device to the population mean and standard
 * deviation of n samples (a constant column gets std 1). */
expri_status expri_mlp_set_norm(expri_mlp *m, const float *norm);
expri_status expri_mlp_fit_norm(expri_mlp *m, const float *X, const float *T, int32_t n);
/* Copy the parameters and/or the standardisation to host arrays (either may
 * be NULL, not both). */
expri_status expri_mlp_get(const expri_mlp *m, float *params, float *norm);
/* Loss and gradient (float32 forward and backward passes on the device,
 * workgroup partial sums added in a fixed order) over n >= 1 samples; loss
 * and grad (EXPRI_MLP_PARAMS floats) are host outputs, either may be NULL. */
expri_status expri_mlp_grad(expri_mlp *m, const float *X, const float *T, int32_t n, float *loss, float *grad);
/* One Adam step (Kingma & Ba; beta1 0.9, beta2 0.999, eps 1e-8, bias
 * corrected) with learning rate lr > 0 on the minibatch; the loss before the
 * update goes to *loss when loss is not NULL. */
expri_status expri_mlp_adam_step(expri_mlp *m, const float *X, const float *T, int32_t n, float lr, float *loss);
/* Inference: Y (device, n x 2, de-standardised) = net(X) with float32
 * weights (bf16 = 0) or with bfloat16 weights, inputs and hidden
 * activations and float32 sums (bf16 = 1), one wavefront per sample. */
expri_status expri_mlp_forward(expri_mlp *m, const float *X, float *Y, int32_t n, int32_t bf16);
const char *expri_mlp_last_error(const expri_mlp *m);
void expri_mlp_destroy(expri_mlp *m);

/* Use a trained network (host arrays: EXPRI_MLP_PARAMS parameters and
 * EXPRI_MLP_NORM standardisation floats) as the step controller of expri_run
 * on ctx; params = NULL restores the paper's alpha/beta rule.  The
 * parameters are rounded to bfloat16 and evaluated in the transient kernel
 * (bfloat16 inference, float32 sums) on the step features.  For each step
 * the network's h, times safety (0 < safety <= 1), bounded to
 * [alpha, beta] x the previous step's nominal size and to h_max, is the
 * first trial; it lands on the next source corner (or T) when that is within
 * 1.25 h and takes half the gap when the gap is shorter than 2 h; the residual test of the first MEVP
 * starts at the predicted m minus one.  The error estimate still accepts or
 * rejects every trial, and rejections halve h as in Algorithm 2.  When a
 * learned trial's MEVP does not converge within m_max, the step restarts
 * once from the paper's own proposal (keeping the basis).  Replays
 * (expri_run_schedule, expri_step_fixed) and expri_step ignore the
 * controller.  The multifrontal engine takes the same network and rules in
 * expri_run (features reduced on the device, the network evaluated by one
 * wave).  EINVAL for a
 * non-finite parameter, a std <= 0 or safety outside (0, 1]. */
expri_status expri_controller_load(expri_ctx *ctx, const float *params, const float *norm, double safety);

#ifdef __cplusplus
}
#endif

#endif /* EXPRI_H */
