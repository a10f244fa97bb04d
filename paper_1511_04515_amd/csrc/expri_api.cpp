// C-ABI of the ER solver (include/expri.h): context, host-side validation,
// upload of symbolic data and values, workspace layout and the host loops
// that drive the gfx950 kernels of engine.hip.
#include "../../include/expri.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "layout.hpp"
#include "mlp.hpp"
#include "grid_engine.hpp"
#include "symbolic.hpp"

// Workspace of expri_run_noalloc: a file-scope device array, so that the
// call needs no allocation.  Each GPU holds its own copy for the life of the
// process.  In host code `scratch` only names the array: its device address
// comes from hipGetSymbolAddress (scratch_ptr below).
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace expri {
// launchers (engine.hip)
size_t lds_bytes(int bs, int R);
hipError_t set_lds_limits(size_t bytes);
hipError_t launch_begin(const InstDesc *d, int n_inst, const double *const *xin, double t0, double h0,
                        hipStream_t s);
hipError_t launch_end(const InstDesc *d, int n_inst, double *const *xout, hipStream_t s);
hipError_t launch_init_workspace(const InstDesc *d, int n_inst, hipStream_t s);
hipError_t launch_run(const InstDesc *d, const int *order, int n_inst, int grid, int *next, const Opts &o,
                      int max_steps, int replay, int bs, int em, int R, int NX, hipStream_t s);
hipError_t launch_zero_counters(int *next, int n, hipStream_t s);
hipError_t launch_dc(const InstDesc *d, const int *order, int n_inst, const Opts &o, double t0, int max_it,
                     int bs, int R, int NX, hipStream_t s);
hipError_t launch_factor(const InstDesc *d, const int *order, int n_inst, const Opts &o, int bs, int R, int NX,
                         hipStream_t s);
hipError_t launch_solve(const InstDesc *d, const int *order, int n_inst, const double *const *b,
                        double *const *y, int bs, int R, int NX, hipStream_t s);
hipError_t launch_mevp(const InstDesc *d, const int *order, int n_inst, const Opts &o, const double *const *v,
                       double *const *out, double h, double eps, int bs, int R, int NX, hipStream_t s);
hipError_t launch_mlp_pack(const float *p, void *out, bool bf16, hipStream_t s);
hipError_t launch_diag(const InstDesc *d, int what, int reps, int arg, long long *out, int bs, int R, int NX,
                       hipStream_t s);
}  // namespace expri

using namespace expri;

namespace {

constexpr size_t kAlign = 256;
constexpr int64_t kMaxRunSteps = 4000000;  // accepted steps per instance and call

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Appends arrays into one byte image with 256-byte alignment.
struct Packer {
  std::vector<char> img;
  template <class T>
  size_t add(const T *p, size_t count) {
    size_t off = align_up(img.size());
    img.resize(off + std::max<size_t>(count * sizeof(T), 1), 0);
    if (count) std::memcpy(img.data() + off, p, count * sizeof(T));
    return off;
  }
  template <class T>
  size_t add(const std::vector<T> &v) { return add(v.data(), v.size()); }
};

struct PatternDev {
  Symbolic sym;
  uint64_t hash = 0;
  int bs = 512;  // block size of its launch class
  bool tuned = false;  // bs and slots come from the autotuner
  int slots = 0;       // solve slots asked of the schedule builder (0: its cost model)
  // flattened solve schedules and C ELL pattern (depend on the block size)
  std::vector<SolveLevel> lsched, usched;
  std::vector<int32_t> slot_pos, slot_col, row_of, c_ell_col, pass_code, rdv_pos, jpos;
  std::vector<int32_t> pk_slot, pk_pos, rd_slot, rd_pos;  // repacking work lists
  int32_t c_ell_k = 0, n_lpass = 0, n_upass = 0, pl = 1, pu = 1, u_slot_base = 0, u_row_base = 0;
  int32_t l_narrow = 0, u_narrow = 0, c_ell_ld = 0;
  size_t o_pass_code, o_slot_pos, o_slot_col, o_row_of, o_c_ell_col, o_rdv_pos, o_jpos;
  size_t o_pk_slot, o_pk_pos, o_rd_slot, o_rd_pos;
  size_t lu_rowptr, lu_col, lu_diag, lev_ptr, lev_rows, ulev_ptr, ulev_rows, row_grp, grp_pos,
      grp_diag, grp_ptr, pair_src, pair_dst, lu_gidx, jac_ptr, jac_code, node_ptr, node_code,
      g_rowptr, g_col, c_rowptr, c_col, b_rowptr, b_col, dev_node, perm;
};

struct Inst {
  int pat = 0;
  int32_t n = 0, n_dev = 0, n_src = 0, n_probe = 0, n_bp = 0;
  double vdd = 1.0, T = 0.0, h_max = 0.0;
  size_t g_val, g_lu, c_val, b_val, c_ell_val, dev_par, src_ptr, src_t, src_v, bp, probe;  // const offsets
  int32_t n_corners = 0;  // PWL corners over all sources (the breakpoint array holds n_corners + 1)
  // workspace offsets
  size_t xk, x1, w, p, z, tmp, e, Ik, devI, devD, devI1, lu, sval, rdv, V, Ve, H, He, mat, state, trace;
  int64_t ldv = 0;
  std::vector<double> trace_host;
  expri_run_info info{};
};

// The instances that share one block size (and so one LDS shape): a launch
// of the transient kernel per class, the classes concurrently on their own
// streams (class 0 on the caller's stream), larger block sizes first.
struct LaunchClass {
  int bs = 512, em = 9, R = 0, NX = 0;  // block size, rows-per-thread bound of its kernel
  int first = 0, count = 0;  // their slice of the launch order
  int grid = 1;              // workgroups of its transient launch (each takes instances in turn)
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipEvent_t e0 = nullptr, e1 = nullptr;  // around its k_run launch, on its stream
  double kernel_s = 0.0;                  // summed k_run duration of the last call
};

}  // namespace

struct expri_ctx {
  hipStream_t stream = nullptr;
  expri_opts opts{};
  std::vector<PatternDev> pats;
  std::vector<Inst> inst;
  char *d_const = nullptr;
  size_t const_bytes = 0;
  char *d_ws = nullptr;
  size_t ws_bytes = 0;
  bool ws_owned = false;
  InstDesc *d_desc = nullptr;
  std::vector<InstDesc> h_desc;
  void **d_ptrs = nullptr;  // 4 * n_inst device pointers
  int *d_order = nullptr;   // instances by launch class, the largest first within a class
  std::vector<LaunchClass> cls;
  std::vector<int> inst_class;  // launch class of each instance
  int *d_next = nullptr;        // per class: the next instance a transient workgroup takes
  hipEvent_t ev_fork = nullptr;
  uint16_t *d_ctrl_w = nullptr;  // learned controller: bfloat16 parameters (inference layout)
  float *d_ctrl_norm = nullptr;   // and its standardisation; null = the paper's step control
  float *d_ctrl_tmp = nullptr;    // float32 staging for the conversion
  double ctrl_safety = 1.0;
  bool ctrl_on = false;
  int bs = 512;  // block size of class 0
  double wall_hz = 1e8;  // GPU wall-clock counter rate
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  double run_kernel_s = 0.0;  // summed duration of the k_run launches of the last call
  int32_t run_launches = 0;
  bool factors_stale = false;  // values replaced since the last expri_factor
  // one large circuit: the multifrontal engine (no launch classes, no
  // workspace of the per-instance layout)
  std::unique_ptr<GridEngine> grid;
  std::string err;
};

namespace {

expri_status fail(expri_ctx *c, expri_status s, const std::string &msg) {
  if (c) c->err = msg;
  return s;
}

expri_status hip_fail(expri_ctx *c, hipError_t e, const char *what) {
  return fail(c, EXPRI_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(ctx, call)                                \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #call); \
  } while (0)

Opts kernel_opts(const expri_opts &o) {
  Opts k{};
  k.E_rr = o.E_rr;
  k.eps_K = o.eps_krylov;
  k.alpha = o.alpha;
  k.beta = o.beta;
  k.h_init = o.h_init;
  k.h_min = o.h_min;
  k.h_max = o.h_max;
  k.breakdown = o.breakdown;
  k.piv_tol = o.piv_tol;
  k.grow_if_rejects_lt = o.grow_if_rejects_lt;
  k.m_max = o.m_max;
  k.erc = o.erc;
  k.gamma = o.gamma;
  return k;
}

bool finite_all(const double *p, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

// permuted copy of CSR values: out[e'] = val[src[e']]
std::vector<double> gather(const double *val, const std::vector<int32_t> &src) {
  std::vector<double> out(src.size());
  for (size_t e = 0; e < src.size(); ++e) out[e] = val[src[e]];
  return out;
}

PatternInput pattern_input(const expri_circuit &K) {
  PatternInput pin;
  pin.n = K.n;
  pin.g_rowptr = K.G.rowptr; pin.g_col = K.G.colidx;
  pin.c_rowptr = K.C.rowptr; pin.c_col = K.C.colidx;
  pin.b_rowptr = K.B.rowptr; pin.b_col = K.B.colidx;
  pin.n_src = K.n_src;
  pin.n_dev = K.dev.n;
  pin.dev_d = K.dev.d; pin.dev_g = K.dev.g; pin.dev_s = K.dev.s;
  return pin;
}

// The value arrays of one instance in the internal numbering: G, G scattered
// to the L\U positions, C (CSR and padded ELL), B, the device parameters, the
// PWL sources, the breakpoints (corners inside (0, T), then T; padded to
// n_corners + 1 entries) and the probed nodes.  Built by expri_setup and
// again by expri_set_values.
struct InstValues {
  std::vector<double> g, glu, c, ell, b, par, st, sv, bps;
  std::vector<int32_t> sp, pr;
  int32_t n_bp = 0;
};

InstValues inst_values(const expri_circuit &K, const PatternDev &PD) {
  const Symbolic &S = PD.sym;
  InstValues v;
  v.g = gather(K.G.val, S.g_src);
  v.glu.assign(S.lu_gidx.size(), 0.0);
  for (size_t p = 0; p < v.glu.size(); ++p)
    if (S.lu_gidx[p] >= 0) v.glu[p] = v.g[S.lu_gidx[p]];
  v.c = gather(K.C.val, S.c_src);
  v.ell.assign((size_t)std::max(PD.c_ell_k, 1) * PD.c_ell_ld, 0.0);
  for (int i = 0; i < K.n; ++i)
    for (int e = S.c_rowptr[i]; e < S.c_rowptr[i + 1]; ++e)
      v.ell[(size_t)(e - S.c_rowptr[i]) * PD.c_ell_ld + i] = v.c[e];
  v.b = gather(K.B.val, S.b_src);
  v.par.resize(4 * (size_t)K.dev.n);
  for (int i = 0; i < K.dev.n; ++i) {
    v.par[4 * i] = K.dev.type[i];
    v.par[4 * i + 1] = K.dev.kp[i] * K.dev.wl[i];
    v.par[4 * i + 2] = K.dev.vth[i];
    v.par[4 * i + 3] = K.dev.lam[i];
  }
  v.sp.assign(K.n_src + 1, 0);
  for (int q = 0; q < K.n_src; ++q) {
    v.sp[q + 1] = v.sp[q] + K.src[q].npts;
    v.st.insert(v.st.end(), K.src[q].t, K.src[q].t + K.src[q].npts);
    v.sv.insert(v.sv.end(), K.src[q].v, K.src[q].v + K.src[q].npts);
    for (int i = 0; i < K.src[q].npts; ++i)
      if (K.src[q].t[i] > 0 && K.src[q].t[i] < K.T) v.bps.push_back(K.src[q].t[i]);
  }
  std::sort(v.bps.begin(), v.bps.end());
  v.bps.erase(std::unique(v.bps.begin(), v.bps.end()), v.bps.end());
  v.bps.push_back(K.T);
  v.n_bp = (int32_t)v.bps.size();
  v.bps.resize(v.st.size() + 1, K.T);
  v.pr.resize(K.n_probe);
  for (int q = 0; q < K.n_probe; ++q) v.pr[q] = S.iperm[K.probe[q]];
  return v;
}


expri_status validate_circuit(expri_ctx *c, const expri_circuit &k, int idx) {
  const std::string w = "instance " + std::to_string(idx) + ": ";
  if (k.n <= 0) return fail(c, EXPRI_EINVAL, w + "n must be positive");
  auto mat_ok = [&](const expri_csr &m, int32_t r, int32_t cc, const char *nm) -> bool {
    if (m.n_rows != r || m.n_cols != cc) { c->err = w + nm + ": wrong shape"; return false; }
    if (!m.rowptr || (m.nnz > 0 && (!m.colidx || !m.val))) { c->err = w + nm + ": null array"; return false; }
    if (m.rowptr[0] != 0 || m.rowptr[r] != m.nnz) { c->err = w + nm + ": rowptr/nnz mismatch"; return false; }
    if (!finite_all(m.val, m.nnz)) { c->err = w + nm + ": non-finite value"; return false; }
    return true;
  };
  if (!mat_ok(k.G, k.n, k.n, "G") || !mat_ok(k.C, k.n, k.n, "C") || !mat_ok(k.B, k.n, k.n_src, "B"))
    return EXPRI_EINVAL;
  if (k.n_src < 0 || (k.n_src > 0 && !k.src)) return fail(c, EXPRI_EINVAL, w + "bad sources");
  for (int s = 0; s < k.n_src; ++s) {
    const expri_pwl &p = k.src[s];
    if (p.npts < 1 || !p.t || !p.v) return fail(c, EXPRI_EINVAL, w + "empty PWL source");
    if (!finite_all(p.t, p.npts) || !finite_all(p.v, p.npts))
      return fail(c, EXPRI_EINVAL, w + "non-finite PWL corner");
    for (int i = 1; i < p.npts; ++i)
      if (!(p.t[i] > p.t[i - 1])) return fail(c, EXPRI_EINVAL, w + "PWL times not increasing");
  }
  if (k.dev.n < 0 || (k.dev.n > 0 && (!k.dev.type || !k.dev.d || !k.dev.g || !k.dev.s || !k.dev.kp ||
                                      !k.dev.wl || !k.dev.vth || !k.dev.lam)))
    return fail(c, EXPRI_EINVAL, w + "bad device table");
  for (int i = 0; i < k.dev.n; ++i) {
    if (k.dev.type[i] != 1 && k.dev.type[i] != -1) return fail(c, EXPRI_EINVAL, w + "device type must be +-1");
    const double v[4] = {k.dev.kp[i], k.dev.wl[i], k.dev.vth[i], k.dev.lam[i]};
    if (!finite_all(v, 4)) return fail(c, EXPRI_EINVAL, w + "non-finite device parameter");
  }
  if (!(k.T > 0) || !std::isfinite(k.T) || !std::isfinite(k.vdd)) return fail(c, EXPRI_EINVAL, w + "bad T / vdd");
  if (k.n_probe < 0 || (k.n_probe > 0 && !k.probe)) return fail(c, EXPRI_EINVAL, w + "bad probes");
  for (int i = 0; i < k.n_probe; ++i)
    if (k.probe[i] < 0 || k.probe[i] >= k.n) return fail(c, EXPRI_EINVAL, w + "probe out of range");
  return EXPRI_OK;
}

// workspace layout; returns total bytes
size_t layout_workspace(expri_ctx *c) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + std::max<size_t>(bytes, 8));
    return o;
  };
  const int mm = c->opts.m_max;
  for (auto &I : c->inst) {
    const auto &S = c->pats[I.pat].sym;
    const size_t n = I.n, nd = std::max(I.n_dev, 1);
    // every thread loads E rows of a basis column without a bound test, the
    // rows past n holding zeros
    const int bsp = c->pats[I.pat].bs;
    const size_t rows = std::max(n, (size_t)rows_per_thread((int)n, bsp) * bsp);
    I.ldv = (int64_t)((rows + 31) / 32 * 32);
    I.xk = take(8 * n); I.x1 = take(8 * n); I.w = take(8 * n); I.p = take(8 * n);
    I.z = take(8 * n); I.tmp = take(8 * n); I.e = take(8 * n); I.Ik = take(8 * n);
    I.devI = take(8 * nd); I.devD = take(24 * nd); I.devI1 = take(8 * nd);
    I.lu = take(8 * (size_t)S.lu_rowptr[n]);
    I.sval = take(8 * c->pats[I.pat].slot_pos.size());
    I.rdv = take(8 * c->pats[I.pat].row_of.size());
    I.V = take(8 * (size_t)I.ldv * (mm + 1));
    I.Ve = take(8 * (size_t)I.ldv * (mm + 1));
    I.H = take(8 * (size_t)kHLd * kMaxKrylov);
    I.He = take(8 * (size_t)kHLd * kMaxKrylov);
    I.mat = take(8 * (size_t)7 * kHLd * kHLd);
    I.state = take(sizeof(InstState));
    I.trace = take(8 * (size_t)c->opts.trace_cap * (kRecFixed + I.n_probe));
  }
  return off;
}

void fill_descs(expri_ctx *c) {
  c->h_desc.resize(c->inst.size());
  for (size_t k = 0; k < c->inst.size(); ++k) {
    const Inst &I = c->inst[k];
    const PatternDev &P = c->pats[I.pat];
    const Symbolic &S = P.sym;
    InstDesc d{};
    auto ci = [&](size_t off) { return reinterpret_cast<const int32_t *>(c->d_const + off); };
    auto cd = [&](size_t off) { return reinterpret_cast<const double *>(c->d_const + off); };
    auto wd = [&](size_t off) { return reinterpret_cast<double *>(c->d_ws + off); };
    d.n = I.n;
    d.n_dev = I.n_dev;
    d.n_src = I.n_src;
    d.n_bp = I.n_bp;
    d.nnz_lu = S.lu_rowptr[I.n];
    d.n_lev = (int32_t)S.lev_ptr.size() - 1;
    d.n_ulev = (int32_t)S.ulev_ptr.size() - 1;
    d.n_probe = I.n_probe;
    d.has_dev = I.n_dev > 0;
    d.max_row = S.max_row;
    d.vdd = I.vdd;
    d.T = I.T;
    d.h_max = I.h_max;
    d.lu_rowptr = ci(P.lu_rowptr); d.lu_col = ci(P.lu_col); d.lu_diag = ci(P.lu_diag);
    d.lev_ptr = ci(P.lev_ptr); d.lev_rows = ci(P.lev_rows);
    d.ulev_ptr = ci(P.ulev_ptr); d.ulev_rows = ci(P.ulev_rows);
    d.row_grp = ci(P.row_grp); d.grp_pos = ci(P.grp_pos); d.grp_diag = ci(P.grp_diag);
    d.grp_ptr = ci(P.grp_ptr); d.pair_src = ci(P.pair_src); d.pair_dst = ci(P.pair_dst);
    d.lu_gidx = ci(P.lu_gidx); d.jac_ptr = ci(P.jac_ptr); d.jac_code = ci(P.jac_code);
    d.node_ptr = ci(P.node_ptr); d.node_code = ci(P.node_code);
    d.g_rowptr = ci(P.g_rowptr); d.g_col = ci(P.g_col);
    d.c_rowptr = ci(P.c_rowptr); d.c_col = ci(P.c_col);
    d.b_rowptr = ci(P.b_rowptr); d.b_col = ci(P.b_col);
    d.dev_node = ci(P.dev_node); d.perm = ci(P.perm);
    d.pass_code = ci(P.o_pass_code);
    d.n_lpass = P.n_lpass; d.n_upass = P.n_upass; d.pl = P.pl; d.pu = P.pu;
    d.l_narrow = P.l_narrow; d.u_narrow = P.u_narrow;
    d.u_slot_base = P.u_slot_base; d.u_row_base = P.u_row_base;
    d.n_slots = (int32_t)P.slot_pos.size(); d.n_srows = (int32_t)P.row_of.size();
    d.slot_pos = ci(P.o_slot_pos); d.slot_col = ci(P.o_slot_col); d.row_of = ci(P.o_row_of);
    d.c_ell_col = ci(P.o_c_ell_col); d.c_ell_k = P.c_ell_k; d.c_ell_ld = P.c_ell_ld;
    d.c_ell_val = cd(I.c_ell_val);
    d.probe = ci(I.probe);
    d.g_val = cd(I.g_val); d.c_val = cd(I.c_val); d.b_val = cd(I.b_val); d.g_lu = cd(I.g_lu);
    d.rdv_pos = ci(P.o_rdv_pos); d.jpos = ci(P.o_jpos); d.n_jpos = (int32_t)P.jpos.size();
    d.pk_slot = ci(P.o_pk_slot); d.pk_pos = ci(P.o_pk_pos); d.n_pk = (int32_t)P.pk_slot.size();
    d.rd_slot = ci(P.o_rd_slot); d.rd_pos = ci(P.o_rd_pos); d.n_rd = (int32_t)P.rd_slot.size();
    d.dev_par = cd(I.dev_par); d.src_ptr = ci(I.src_ptr); d.src_t = cd(I.src_t);
    d.src_v = cd(I.src_v); d.bp = cd(I.bp);
    d.xk = wd(I.xk); d.x1 = wd(I.x1); d.w = wd(I.w); d.p = wd(I.p); d.z = wd(I.z);
    d.tmp = wd(I.tmp); d.e = wd(I.e); d.devI = wd(I.devI); d.devD = wd(I.devD);
    d.devI1 = wd(I.devI1); d.Ik = wd(I.Ik); d.lu = wd(I.lu); d.sval = wd(I.sval); d.rdv = wd(I.rdv);
    d.V = wd(I.V); d.Ve = wd(I.Ve);
    d.H = wd(I.H); d.He = wd(I.He); d.mat = wd(I.mat);
    d.ldv = I.ldv;
    d.state = reinterpret_cast<InstState *>(c->d_ws + I.state);
    d.trace = wd(I.trace);
    d.trace_cap = c->opts.trace_cap;
    d.vcols = c->opts.m_max + 1;
    c->h_desc[k] = d;
  }
}

expri_status ensure_ws(expri_ctx *c) {
  if (c->d_ws) return EXPRI_OK;
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, c->ws_bytes);
  if (e != hipSuccess) return fail(c, EXPRI_ENOMEM, std::string("workspace allocation: ") + hipGetErrorString(e));
  c->d_ws = static_cast<char *>(p);
  c->ws_owned = true;
  fill_descs(c);
  HIPCHK(c, hipMemcpyAsync(c->d_desc, c->h_desc.data(), sizeof(InstDesc) * c->h_desc.size(),
                           hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, launch_init_workspace(c->d_desc, (int)c->inst.size(), c->stream));
  return EXPRI_OK;
}

// point every descriptor's step-end table at the instance's own source
// corners (expri_run_schedule points it at a replay grid for one call)
void restore_corners(expri_ctx *c) {
  for (size_t k = 0; k < c->inst.size(); ++k) {
    const Inst &I = c->inst[k];
    c->h_desc[k].bp = reinterpret_cast<const double *>(c->d_const + I.bp);
    c->h_desc[k].n_bp = I.n_bp;
  }
}

expri_status upload_descs(expri_ctx *c) {
  HIPCHK(c, hipMemcpyAsync(c->d_desc, c->h_desc.data(), sizeof(InstDesc) * c->h_desc.size(),
                           hipMemcpyHostToDevice, c->stream));
  return EXPRI_OK;
}

// copy a host array of n_inst device pointers into d_ptrs[slot * n_inst ...]
expri_status put_ptrs(expri_ctx *c, int slot, const void *const *ptrs) {
  const size_t n = c->inst.size();
  for (size_t i = 0; i < n; ++i)
    if (!ptrs[i]) return fail(c, EXPRI_EINVAL, "null device vector");
  HIPCHK(c, hipMemcpyAsync(c->d_ptrs + slot * n, ptrs, sizeof(void *) * n, hipMemcpyHostToDevice, c->stream));
  return EXPRI_OK;
}

expri_status read_states(expri_ctx *c, std::vector<InstState> &st) {
  st.resize(c->inst.size());
  for (size_t k = 0; k < c->inst.size(); ++k)
    HIPCHK(c, hipMemcpyAsync(&st[k], c->d_ws + c->inst[k].state, sizeof(InstState), hipMemcpyDeviceToHost,
                             c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return EXPRI_OK;
}

expri_status first_error(expri_ctx *c, const std::vector<InstState> &st, const char *what) {
  for (size_t k = 0; k < st.size(); ++k)
    if (st[k].status != kOK) {
      static const char *names[] = {"ok", "invalid argument", "out of memory", "singular pivot in LU(G_k)",
                                    "Krylov residual not reached at m_max", "step below h_min",
                                    "non-finite value", "HIP error", "pattern mismatch",
                                    "Newton iteration did not converge"};
      const int s = -st[k].status;
      return fail(c, (expri_status)st[k].status,
                  std::string(what) + ": instance " + std::to_string(k) + ": " +
                      ((s >= 0 && s <= 9) ? names[s] : "error"));
    }
  return EXPRI_OK;
}

// one k_run launch per launch class, the classes concurrently (fork / join
// on the caller's stream); ev0 / ev1 bracket the whole on the caller's stream
expri_status launch_run_classes(expri_ctx *c, const Opts &ko, int max_steps, int replay) {
  HIPCHK(c, hipEventRecord(c->ev0, c->stream));
  HIPCHK(c, launch_zero_counters(c->d_next, (int)c->cls.size(), c->stream));
  HIPCHK(c, hipEventRecord(c->ev_fork, c->stream));
  for (size_t q = 0; q < c->cls.size(); ++q) {
    LaunchClass &K = c->cls[q];
    if (K.stream != c->stream) HIPCHK(c, hipStreamWaitEvent(K.stream, c->ev_fork, 0));
    HIPCHK(c, hipEventRecord(K.e0, K.stream));
    HIPCHK(c, launch_run(c->d_desc, c->d_order + K.first, K.count, K.grid, c->d_next + q, ko, max_steps, replay,
                         K.bs, K.em, K.R, K.NX, K.stream));
    HIPCHK(c, hipEventRecord(K.e1, K.stream));
  }
  for (auto &K : c->cls)
    if (K.stream != c->stream) HIPCHK(c, hipStreamWaitEvent(c->stream, K.e1, 0));
  HIPCHK(c, hipEventRecord(c->ev1, c->stream));
  return EXPRI_OK;
}

// drive k_run until every instance is done (adaptive or replay)
expri_status drive(expri_ctx *c, double *const *x, double t0, int max_steps, int replay) {
  const int n = (int)c->inst.size();
  if (max_steps < 1 || max_steps > c->opts.trace_cap)
    return fail(c, EXPRI_EINVAL, "max_steps_per_launch must be in [1, trace_cap]");
  expri_status s;
  if ((s = upload_descs(c)) != EXPRI_OK) return s;
  if ((s = put_ptrs(c, 0, reinterpret_cast<const void *const *>(x))) != EXPRI_OK) return s;
  Opts ko = kernel_opts(c->opts);
  if (c->ctrl_on && !replay) {
    ko.controller = 1;
    ko.ctrl_w = c->d_ctrl_w;
    ko.ctrl_norm = c->d_ctrl_norm;
    ko.ctrl_safety = c->ctrl_safety;
  }
  HIPCHK(c, launch_begin(c->d_desc, n, reinterpret_cast<const double *const *>(c->d_ptrs), t0, c->opts.h_init,
                         c->stream));
  for (auto &I : c->inst) I.trace_host.clear();
  c->run_kernel_s = 0.0;
  c->run_launches = 0;
  for (auto &K : c->cls) K.kernel_s = 0.0;
  std::vector<int32_t> prev(n, 0);
  std::vector<InstState> st;
  const int64_t max_launches = kMaxRunSteps / max_steps + 1;
  for (int64_t launches = 0;; ++launches) {
    if (launches >= max_launches)
      return fail(c, EXPRI_ESTEPMIN, "step budget of " + std::to_string(kMaxRunSteps) + " accepted steps exhausted");
    if ((s = launch_run_classes(c, ko, max_steps, replay)) != EXPRI_OK) return s;
    if ((s = read_states(c, st)) != EXPRI_OK) return s;
    float ms = 0.0f;
    HIPCHK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
    c->run_kernel_s += 1e-3 * ms;
    for (auto &K : c->cls) {
      HIPCHK(c, hipEventElapsedTime(&ms, K.e0, K.e1));
      K.kernel_s += 1e-3 * ms;
    }
    ++c->run_launches;
    bool all = true;
    for (int k = 0; k < n; ++k) {
      Inst &I = c->inst[k];
      const int32_t add = st[k].steps - prev[k];
      if (add > 0) {
        const size_t rec = kRecFixed + I.n_probe;
        const size_t old = I.trace_host.size();
        I.trace_host.resize(old + (size_t)add * rec);
        HIPCHK(c, hipMemcpyAsync(I.trace_host.data() + old, c->d_ws + I.trace, sizeof(double) * add * rec,
                                 hipMemcpyDeviceToHost, c->stream));
      }
      prev[k] = st[k].steps;
      if (!st[k].done) all = false;
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (all) break;
  }
  HIPCHK(c, launch_end(c->d_desc, n, reinterpret_cast<double *const *>(c->d_ptrs), c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int k = 0; k < n; ++k) {
    expri_run_info &in = c->inst[k].info;
    in.t = st[k].t;
    in.steps = st[k].steps;
    in.lu_count = st[k].lu_count;
    in.rejects = st[k].rejects;
    in.arnoldi = st[k].arnoldi;
    in.status = st[k].status;
    for (int p = 0; p < 6; ++p) in.phase_s[p] = st[k].ph[p] / c->wall_hz;
    in.trials = st[k].trials;
    in.mgs_terms = st[k].mgs_terms;
    in.comb_terms = st[k].comb_terms;
  }
  return first_error(c, st, "transient");
}

// Address of the scratch array on each device, taken once per device with
// that device current.
std::mutex g_scratch_mu;
char *g_scratch_dev[64] = {};

expri_status scratch_ptr(expri_ctx *c, char **out) {
  int dev = 0;
  HIPCHK(c, hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(c, EXPRI_EINVAL, "run_noalloc: device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(c, EXPRI_EHIP, std::string("run_noalloc: scratch address: ") + hipGetErrorString(e));
    g_scratch_dev[dev] = static_cast<char *>(p);
  }
  *out = g_scratch_dev[dev];
  return EXPRI_OK;
}

// The largest circuit the one-workgroup engine holds (18 rows per thread at
// 512 threads); beyond it a single circuit goes to the multifrontal engine.
constexpr int32_t kMaxWorkgroupRows = 9216;

expri_status grid_status(expri_ctx *c, int st) {
  if (st != 0) c->err = c->grid->err;
  return (expri_status)st;
}

// the run summary and trace of the multifrontal engine's last call
void grid_info(expri_ctx *c, int st) {
  GridEngine &G = *c->grid;
  Inst &I = c->inst[0];
  I.info = expri_run_info{};
  I.info.t = G.t_reached;
  I.info.steps = G.steps;
  I.info.lu_count = (int32_t)G.lu_count;
  I.info.rejects = (int32_t)G.rejects;
  I.info.arnoldi = (int32_t)G.arnoldi;
  I.info.status = st;
  I.info.trials = (int32_t)G.trials;
  I.info.mgs_terms = G.mgs_terms;
  I.info.comb_terms = G.comb_terms;
  I.trace_host = G.trace;
  c->run_kernel_s = G.kernel_s;
  c->run_launches = 1;
}

// ---- autotuning of the per-pattern launch configuration ----

// the block size the rule gives a circuit of n rows
int rule_block_size(int n) { return n <= 2048 ? 256 : n <= max_rows_per_thread(512) * 512 ? 512 : 1024; }

// Patterns analysed before (by hash); set only while the autotuner creates
// its trial contexts, so that they copy the analysis instead of redoing it.
thread_local const std::map<uint64_t, const Symbolic *> *t_presym = nullptr;

struct TuneChoice {
  int bs = 0, slots = 0;
};
std::mutex g_tune_mu;                       // one autotuning at a time in the process
std::map<uint64_t, TuneChoice> g_tune_cache;  // pattern hash -> measured choice
int64_t g_tune_runs = 0;

// slots per lane the schedule builder takes for (bs, slots) in each direction
bool effective_slots(const Symbolic &S, int bs, int slots, int &pl, int &pu) {
  std::vector<SolveLevel> ls, us;
  std::vector<int32_t> a, b, r;
  if (!build_solve_schedule(S, bs, true, ls, a, b, r, slots)) return false;
  if (!build_solve_schedule(S, bs, false, us, a, b, r, slots)) return false;
  pl = ls.empty() ? 1 : ls[0].P;
  pu = us.empty() ? 1 : us[0].P;
  return true;
}

// Per-instance device time per accepted step (wall-clock ticks) of a trial
// context: the instances start from x at t = 0, run k_steps accepted steps
// untimed (caches and step sizes settle), then k_steps more, measured by the
// kernel's own phase clocks.  Infinite for an instance that fails.
expri_status trial_cost(expri_ctx *t, double *const *x, int k_steps, std::vector<double> &cost) {
  const int n = (int)t->inst.size();
  cost.assign(n, INFINITY);
  expri_status s;
  if ((s = ensure_ws(t)) != EXPRI_OK) return s;
  if ((s = upload_descs(t)) != EXPRI_OK) return s;
  if ((s = put_ptrs(t, 0, reinterpret_cast<const void *const *>(x))) != EXPRI_OK) return s;
  const Opts ko = kernel_opts(t->opts);
  HIPCHK(t, launch_begin(t->d_desc, n, reinterpret_cast<const double *const *>(t->d_ptrs), 0.0, t->opts.h_init,
                         t->stream));
  std::vector<InstState> st0, st1;
  if ((s = launch_run_classes(t, ko, k_steps, 0)) != EXPRI_OK) return s;
  if ((s = read_states(t, st0)) != EXPRI_OK) return s;
  if ((s = launch_run_classes(t, ko, k_steps, 0)) != EXPRI_OK) return s;
  if ((s = read_states(t, st1)) != EXPRI_OK) return s;
  for (int k = 0; k < n; ++k) {
    if (st1[k].status != kOK) continue;
    double ticks = 0.0;
    for (int p = 0; p < kPhases; ++p) ticks += st1[k].ph[p] - st0[k].ph[p];
    int steps = st1[k].steps - st0[k].steps;
    if (steps <= 0) {  // finished within the first launch: its whole run
      ticks = 0.0;
      for (int p = 0; p < kPhases; ++p) ticks += st1[k].ph[p];
      steps = st1[k].steps;
    }
    if (steps > 0) cost[k] = ticks / steps;
  }
  return EXPRI_OK;
}

// Chooses (block size, solve slots) for every pattern of c: from the
// process-wide cache, else by trial contexts, one per candidate
// configuration, each holding the first instance of every pattern that
// configuration applies to.
expri_status autotune(expri_ctx *c, const expri_circuit *ckt, int32_t n_inst) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  const int np = (int)c->pats.size();
  std::vector<int> rep(np, -1);
  for (int k = 0; k < n_inst; ++k)
    if (rep[c->inst[k].pat] < 0) rep[c->inst[k].pat] = k;
  // candidates of the patterns not in the cache: every feasible block size
  // with each slot count that gives a distinct schedule
  std::map<std::pair<int, int>, std::vector<int>> trials;  // (bs, slots) -> patterns
  std::vector<std::map<std::pair<int, int>, double>> cost(np);
  std::map<uint64_t, const Symbolic *> presym;
  for (int p = 0; p < np; ++p) {
    PatternDev &P = c->pats[p];
    const auto hit = g_tune_cache.find(P.hash);
    if (hit != g_tune_cache.end()) {
      P.bs = hit->second.bs;
      P.slots = hit->second.slots;
      P.tuned = true;
      continue;
    }
    presym[P.hash] = &P.sym;
    const int n = P.sym.n;
    for (int bs : {256, 512, 1024}) {
      if (n > max_rows_per_thread(bs) * bs || (bs == 1024 && n <= 2048)) continue;
      std::vector<std::pair<int, int>> seen;
      for (int slots : {0, 1, 2, 4, 8}) {
        int pl = 0, pu = 0;
        if (!effective_slots(P.sym, bs, slots, pl, pu)) continue;
        if (std::find(seen.begin(), seen.end(), std::make_pair(pl, pu)) != seen.end()) continue;
        seen.push_back({pl, pu});
        trials[{bs, slots}].push_back(p);
      }
    }
  }
  constexpr int kTuneSteps = 24;
  for (const auto &tr : trials) {
    const std::vector<int> &pats = tr.second;
    std::vector<expri_circuit> cs;
    for (int p : pats) cs.push_back(ckt[rep[p]]);
    expri_opts o2 = c->opts;
    o2.autotune = 0;
    o2.block_size = tr.first.first;
    o2.solve_slots = tr.first.second;
    o2.private_patterns = 0;
    o2.max_workgroups = 0;
    o2.trace_cap = kTuneSteps;
    expri_ctx *t = nullptr;
    t_presym = &presym;
    expri_status s = expri_setup(&t, cs.data(), (int32_t)cs.size(), &o2, c->stream);
    t_presym = nullptr;
    ++g_tune_runs;
    std::vector<double *> xs(cs.size(), nullptr);
    std::vector<double> tc;
    bool ok = s == EXPRI_OK;
    for (size_t q = 0; q < cs.size() && ok; ++q)
      ok = hipMalloc(reinterpret_cast<void **>(&xs[q]), sizeof(double) * cs[q].n) == hipSuccess &&
           hipMemsetAsync(xs[q], 0, sizeof(double) * cs[q].n, c->stream) == hipSuccess;
    if (ok) ok = expri_dc(t, xs.data(), 0.0) == EXPRI_OK;
    if (ok) ok = trial_cost(t, xs.data(), kTuneSteps, tc) == EXPRI_OK;
    for (double *x : xs)
      if (x) (void)hipFree(x);
    expri_destroy(t);
    if (!ok) continue;  // this configuration stays unmeasured (infinite cost)
    for (size_t q = 0; q < pats.size(); ++q) cost[pats[q]][tr.first] = tc[q];
  }
  // the rule's configuration unless another is 3 % faster
  for (int p = 0; p < np; ++p) {
    PatternDev &P = c->pats[p];
    if (P.tuned) continue;
    TuneChoice ch{rule_block_size(P.sym.n), c->opts.solve_slots};
    double best = INFINITY;
    for (const auto &kv : cost[p])
      if (kv.first.first == ch.bs && kv.first.second == ch.slots) best = kv.second;
    if (!(best < INFINITY)) {  // the rule's slot count may have been folded into another candidate
      int pl0 = 0, pu0 = 0;
      if (effective_slots(P.sym, ch.bs, ch.slots, pl0, pu0))
        for (const auto &kv : cost[p]) {
          int pl = 0, pu = 0;
          if (kv.first.first == ch.bs && effective_slots(P.sym, ch.bs, kv.first.second, pl, pu) && pl == pl0 &&
              pu == pu0)
            best = kv.second;
        }
    }
    for (const auto &kv : cost[p])
      if (kv.second < 0.97 * best) {
        best = kv.second;
        ch = TuneChoice{kv.first.first, kv.first.second};
      }
    P.bs = ch.bs;
    P.slots = ch.slots;
    P.tuned = true;
    g_tune_cache[P.hash] = ch;
  }
  return EXPRI_OK;
}

expri_status setup_grid(expri_ctx *c, const expri_circuit *ckt, int32_t n_inst) {
  const expri_opts &op = c->opts;
  if (n_inst != 1) return fail(c, EXPRI_EINVAL, "the multifrontal engine takes one circuit");
  if (op.erc != 0) return fail(c, EXPRI_EINVAL, "ER-C is not available in the multifrontal engine");
  expri_status s;
  if ((s = validate_circuit(c, ckt[0], 0)) != EXPRI_OK) return s;
  const expri_circuit &K = ckt[0];
  const PatternInput pin = pattern_input(K);
  std::vector<double> kind(K.dev.n);
  for (int i = 0; i < K.dev.n; ++i) kind[i] = K.dev.type[i];
  std::vector<int32_t> npts(K.n_src);
  std::vector<const double *> ts(K.n_src), vs(K.n_src);
  for (int q = 0; q < K.n_src; ++q) {
    npts[q] = K.src[q].npts;
    ts[q] = K.src[q].t;
    vs[q] = K.src[q].v;
  }
  GridValues val{K.G.val, K.C.val, K.B.val, kind.data(), K.dev.kp, K.dev.wl, K.dev.vth, K.dev.lam,
                 K.n_src, npts.data(), ts.data(), vs.data(), K.vdd, K.T};
  GridOpts go{op.E_rr, op.eps_krylov, op.alpha, op.beta, op.h_init, op.h_min, op.h_max, op.breakdown, op.piv_tol,
              op.grow_if_rejects_lt, op.m_max, op.trace_cap};
  c->grid.reset(new (std::nothrow) GridEngine());
  if (!c->grid) return fail(c, EXPRI_ENOMEM, "engine allocation");
  const int st = c->grid->setup(pin, val, K.probe, K.n_probe, go, c->stream, 16);
  if (st != 0) return grid_status(c, st);
  Inst I;
  I.n = K.n;
  I.n_dev = K.dev.n;
  I.n_src = K.n_src;
  I.n_probe = K.n_probe;
  I.vdd = K.vdd;
  I.T = K.T;
  I.h_max = c->grid->h_max;
  c->inst.push_back(std::move(I));
  c->h_desc.resize(1);
  return EXPRI_OK;
}

}  // namespace

extern "C" {

expri_status expri_default_opts(expri_opts *o) {
  if (!o) return EXPRI_EINVAL;
  o->E_rr = 1e-6;
  o->eps_krylov = 1e-7;
  o->alpha = 0.5;
  o->beta = 2.0;
  o->h_init = 1e-13;
  o->h_min = 1e-18;
  o->h_max = 0.0;
  o->breakdown = 1e-13;
  o->piv_tol = 1e-13;
  o->grow_if_rejects_lt = 5;
  o->m_max = 60;
  o->block_size = 0;
  o->trace_cap = 4096;
  o->erc = 0;
  o->solve_slots = 0;
  o->max_workgroups = 0;
  o->engine = 0;
  o->private_patterns = 0;
  o->autotune = 0;
  o->gamma = 0.1;
  return EXPRI_OK;
}

namespace {
expri_status setup_impl(expri_ctx **out, const expri_circuit *ckt, int32_t n_inst, const expri_opts *o,
                        void *hip_stream);
}

expri_status expri_setup(expri_ctx **out, const expri_circuit *ckt, int32_t n_inst, const expri_opts *o,
                         void *hip_stream) {
  expri_status s = setup_impl(out, ckt, n_inst, o, hip_stream);
  // automatic engine choice: a single circuit that the one-workgroup engine
  // cannot hold (rows of L or U too long for its solve passes, or too large
  // for its LDS) goes to the multifrontal engine
  const int engine = o ? o->engine : 0;
  if (s == EXPRI_EINVAL && engine == 0 && n_inst == 1 && out && *out && !(*out)->grid) {
    const std::string &msg = (*out)->err;
    if (msg.find("longer than the triangular solve handles") != std::string::npos ||
        msg.find("too large for the one-workgroup engine") != std::string::npos) {
      expri_opts o2;
      if (o) o2 = *o; else expri_default_opts(&o2);
      o2.engine = 2;
      expri_destroy(*out);
      *out = nullptr;
      s = setup_impl(out, ckt, n_inst, &o2, hip_stream);
    }
  }
  return s;
}

namespace {
expri_status setup_impl(expri_ctx **out, const expri_circuit *ckt, int32_t n_inst, const expri_opts *o,
                        void *hip_stream) {
  if (!out) return EXPRI_EINVAL;
  *out = nullptr;
  std::unique_ptr<expri_ctx> c(new (std::nothrow) expri_ctx());
  if (!c) return EXPRI_ENOMEM;
  if (!ckt || n_inst <= 0) return EXPRI_EINVAL;
  c->stream = static_cast<hipStream_t>(hip_stream);
  if (o) c->opts = *o; else expri_default_opts(&c->opts);
  const expri_opts &op = c->opts;
  if (!(op.E_rr > 0) || !(op.eps_krylov > 0) || !(op.alpha > 0 && op.alpha < 1) || !(op.beta >= 1) ||
      !(op.h_init > 0) || !(op.h_min > 0) || !(op.h_max >= 0) || !(op.breakdown >= 0) ||
      !(op.piv_tol >= 0) || op.m_max < 1 || op.m_max > kMaxKrylov || op.trace_cap < 1 ||
      (op.erc != 0 && op.erc != 1) || !std::isfinite(op.gamma) ||
      (op.solve_slots != 0 && op.solve_slots != 1 && op.solve_slots != 2 && op.solve_slots != 4 &&
       op.solve_slots != 8) ||
      op.max_workgroups < 0 || op.engine < 0 || op.engine > 2 || (op.private_patterns != 0 && op.private_patterns != 1) ||
      (op.autotune != 0 && op.autotune != 1) ||
      (op.block_size != 0 && op.block_size != 256 && op.block_size != 512 && op.block_size != 1024)) {
    *out = c.release();
    (*out)->err = "invalid options";
    return EXPRI_EINVAL;
  }
  expri_status s;
  if (op.engine == 2 || (op.engine == 0 && n_inst == 1 && ckt[0].n > kMaxWorkgroupRows)) {
    if ((s = setup_grid(c.get(), ckt, n_inst)) != EXPRI_OK) {
      *out = c.release();
      return s;
    }
    *out = c.release();
    return EXPRI_OK;
  }
  std::map<uint64_t, int> by_hash;
  for (int k = 0; k < n_inst; ++k) {
    if ((s = validate_circuit(c.get(), ckt[k], k)) != EXPRI_OK) {
      *out = c.release();
      return s;
    }
    const expri_circuit &K = ckt[k];
    const PatternInput pin = pattern_input(K);
    const uint64_t h = pattern_hash(pin);
    int pid;
    auto it = op.private_patterns ? by_hash.end() : by_hash.find(h);
    if (it != by_hash.end()) {
      pid = it->second;
      const Symbolic &S = c->pats[pid].sym;
      // guard against a hash collision: compare the sizes and the G pattern
      bool same = S.n == K.n && S.n_dev == K.dev.n && S.n_src == K.n_src &&
                  (int32_t)S.g_col.size() == K.G.nnz && (int32_t)S.c_col.size() == K.C.nnz;
      if (!same) { *out = c.release(); (*out)->err = "pattern hash collision"; return EXPRI_EPATTERN; }
    } else {
      PatternDev P;
      P.hash = h;
      const auto pre = t_presym ? t_presym->find(h) : std::map<uint64_t, const Symbolic *>::const_iterator();
      if (t_presym && pre != t_presym->end()) {
        P.sym = *pre->second;
      } else if (!analyse(pin, P.sym)) {
        *out = c.release();
        (*out)->err = "instance " + std::to_string(k) + ": " + P.sym.error;
        return EXPRI_EINVAL;
      }
      pid = (int)c->pats.size();
      c->pats.push_back(std::move(P));
      by_hash[h] = pid;
    }
    Inst I;
    I.pat = pid;
    I.n = K.n;
    I.n_dev = K.dev.n;
    I.n_src = K.n_src;
    I.n_probe = K.n_probe;
    I.vdd = K.vdd;
    I.T = K.T;
    I.h_max = op.h_max > 0 ? op.h_max : K.T / 20;
    c->inst.push_back(std::move(I));
  }

  // ---- launch shape ----
  int dev = 0;
  hipDeviceProp_t prop;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) { *out = c.release(); return hip_fail(*out, e, "device query"); }
  int wall_khz = 0;
  if (hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && wall_khz > 0)
    c->wall_hz = 1e3 * wall_khz;
  // ---- launch classes.  A thread keeps at most max_rows_per_thread(bs)
  // rows of a vector in registers (18 at 512 threads, 9 otherwise): a
  // pattern takes 256 threads up to n = 2048 and 512 up to 18 x 512 = 9216
  // (or the block size the options force); the instances of one block size
  // and one rows-per-thread bound of the transient kernel form a launch
  // class ----
  if (op.autotune) {
    if ((s = autotune(c.get(), ckt, n_inst)) != EXPRI_OK) {
      *out = c.release();
      return s;
    }
  }
  for (auto &P : c->pats) {
    if (!P.tuned) {
      P.bs = op.block_size ? op.block_size : rule_block_size(P.sym.n);
      P.slots = op.solve_slots;
    }
    if (P.sym.n > max_rows_per_thread(P.bs) * P.bs) {
      *out = c.release();
      (*out)->err = "block size " + std::to_string(P.bs) + " too small for n = " + std::to_string(P.sym.n);
      return EXPRI_EINVAL;
    }
  }
  const size_t limit = prop.sharedMemPerBlock;
  // the transient kernel's rows-per-thread bound: 18 at 512 threads beyond
  // 9 x 512 rows, else 9; the classes are (block size, bound), larger first
  auto row_bound = [](int bs, int n) { return (bs == 512 && n > 9 * 512) ? 18 : 9; };
  for (const auto &key : {std::pair<int, int>{1024, 9}, {512, 18}, {512, 9}, {256, 9}}) {
    const int bs = key.first, em = key.second;
    int nm = 0;
    for (const auto &I : c->inst)
      if (c->pats[I.pat].bs == bs && row_bound(bs, c->pats[I.pat].sym.n) == em) nm = std::max(nm, I.n);
    if (nm == 0) continue;
    // LDS: the vector area (solve vector / current Arnoldi basis vector, NX
    // doubles) and behind it the small dense matrices of the Hessenberg
    // exponential: five 32 x 33 matrices cover m <= 31 (larger m use global
    // scratch)
    const size_t extras = lds_bytes(bs, 0);
    const size_t NX = ((size_t)nm + 63) / 64 * 64;
    size_t RD = std::max<size_t>(5 * 32 * 33, NX < 8192 ? 8192 - NX : 0);
    if (8 * (NX + RD) + extras > limit && 8 * NX + extras < limit) RD = (limit - extras) / 8 - NX;
    if (8 * (NX + RD) + extras > limit || RD < 5 * 16 * 17) {
      *out = c.release();
      (*out)->err = "circuit too large for the one-workgroup engine (n = " + std::to_string(nm) + ")";
      return EXPRI_EINVAL;
    }
    LaunchClass K;
    K.bs = bs;
    K.em = em;
    K.NX = (int)NX;
    K.R = (int)(NX + RD);
    c->cls.push_back(K);
  }
  c->bs = c->cls[0].bs;
  c->inst_class.resize(n_inst);
  for (int k = 0; k < n_inst; ++k)
    for (size_t q = 0; q < c->cls.size(); ++q)
      if (c->cls[q].bs == c->pats[c->inst[k].pat].bs &&
          c->cls[q].em == row_bound(c->cls[q].bs, c->pats[c->inst[k].pat].sym.n))
        c->inst_class[k] = (int)q;
  // flattened solve schedules and the C ELL pattern for the pattern's block size
  for (auto &P : c->pats) {
    P.u_slot_base = -1;
    if (build_solve_schedule(P.sym, P.bs, true, P.lsched, P.slot_pos, P.slot_col, P.row_of, P.slots)) {
      P.u_slot_base = (int32_t)P.slot_pos.size();
      P.u_row_base = (int32_t)P.row_of.size();
      if (!build_solve_schedule(P.sym, P.bs, false, P.usched, P.slot_pos, P.slot_col, P.row_of, P.slots))
        P.u_slot_base = -1;
    }
    if (P.u_slot_base < 0) {
      *out = c.release();
      (*out)->err = "a row of L or U is longer than the triangular solve handles (512 entries)";
      return EXPRI_EINVAL;
    }
    P.pass_code = pass_codes(P.lsched, P.bs);
    P.n_lpass = (int32_t)P.pass_code.size();
    const std::vector<int32_t> up = pass_codes(P.usched, P.bs);
    P.n_upass = (int32_t)up.size();
    P.pass_code.insert(P.pass_code.end(), up.begin(), up.end());
    // passes one wave holds: the trailing L passes and leading U passes with
    // at most 64 active lanes
    P.l_narrow = 0;
    while (P.l_narrow < P.n_lpass && (P.pass_code[P.n_lpass - 1 - P.l_narrow] >> 16) <= 64) ++P.l_narrow;
    P.u_narrow = 0;
    while (P.u_narrow < P.n_upass && (P.pass_code[P.n_lpass + P.u_narrow] >> 16) <= 64) ++P.u_narrow;
    P.pl = P.lsched.empty() ? 1 : P.lsched[0].P;
    P.pu = P.usched.empty() ? 1 : P.usched[0].P;
    // C's ELL columns padded to E BS rows (see the basis column stride)
    P.c_ell_ld = std::max(P.sym.n, rows_per_thread(P.sym.n, P.bs) * P.bs);
    P.c_ell_k = build_c_ell(P.sym, P.c_ell_col, P.c_ell_ld);
    // pivot positions for the U passes' row slots; positions with device terms
    P.rdv_pos.assign(P.row_of.size(), -1);
    for (size_t r = (size_t)P.u_row_base; r < P.row_of.size(); ++r)
      if (P.row_of[r] >= 0) P.rdv_pos[r] = P.sym.lu_diag[P.row_of[r]];
    P.pk_slot.clear(); P.pk_pos.clear(); P.rd_slot.clear(); P.rd_pos.clear();
    for (size_t k = 0; k < P.slot_pos.size(); ++k)
      if (P.slot_pos[k] >= 0) { P.pk_slot.push_back((int32_t)k); P.pk_pos.push_back(P.slot_pos[k]); }
    for (size_t r = 0; r < P.rdv_pos.size(); ++r)
      if (P.rdv_pos[r] >= 0) { P.rd_slot.push_back((int32_t)r); P.rd_pos.push_back(P.rdv_pos[r]); }
    P.jpos.clear();
    for (size_t p = 0; p + 1 < P.sym.jac_ptr.size(); ++p)
      if (P.sym.jac_ptr[p + 1] > P.sym.jac_ptr[p]) P.jpos.push_back((int32_t)p);
  }
  // ---- pack constant data ----
  Packer pk;
  for (auto &P : c->pats) {
    const Symbolic &S = P.sym;
    P.lu_rowptr = pk.add(S.lu_rowptr); P.lu_col = pk.add(S.lu_col); P.lu_diag = pk.add(S.lu_diag);
    P.lev_ptr = pk.add(S.lev_ptr); P.lev_rows = pk.add(S.lev_rows);
    P.ulev_ptr = pk.add(S.ulev_ptr); P.ulev_rows = pk.add(S.ulev_rows);
    P.row_grp = pk.add(S.row_grp); P.grp_pos = pk.add(S.grp_pos); P.grp_diag = pk.add(S.grp_diag);
    P.grp_ptr = pk.add(S.grp_ptr); P.pair_src = pk.add(S.pair_src); P.pair_dst = pk.add(S.pair_dst);
    P.lu_gidx = pk.add(S.lu_gidx); P.jac_ptr = pk.add(S.jac_ptr); P.jac_code = pk.add(S.jac_code);
    P.node_ptr = pk.add(S.node_ptr); P.node_code = pk.add(S.node_code);
    P.g_rowptr = pk.add(S.g_rowptr); P.g_col = pk.add(S.g_col);
    P.c_rowptr = pk.add(S.c_rowptr); P.c_col = pk.add(S.c_col);
    P.b_rowptr = pk.add(S.b_rowptr); P.b_col = pk.add(S.b_col);
    P.dev_node = pk.add(S.dev_node); P.perm = pk.add(S.perm);
    P.o_pass_code = pk.add(P.pass_code);
    P.o_rdv_pos = pk.add(P.rdv_pos);
    P.o_pk_slot = pk.add(P.pk_slot); P.o_pk_pos = pk.add(P.pk_pos);
    P.o_rd_slot = pk.add(P.rd_slot); P.o_rd_pos = pk.add(P.rd_pos);
    P.o_jpos = pk.add(P.jpos);
    P.o_slot_pos = pk.add(P.slot_pos); P.o_slot_col = pk.add(P.slot_col); P.o_row_of = pk.add(P.row_of);
    P.o_c_ell_col = pk.add(P.c_ell_col);
  }
  for (int k = 0; k < n_inst; ++k) {
    Inst &I = c->inst[k];
    const InstValues v = inst_values(ckt[k], c->pats[I.pat]);
    I.g_val = pk.add(v.g);
    I.g_lu = pk.add(v.glu);
    I.c_val = pk.add(v.c);
    I.c_ell_val = pk.add(v.ell);
    I.b_val = pk.add(v.b);
    I.dev_par = pk.add(v.par);
    I.n_bp = v.n_bp;
    I.n_corners = (int32_t)v.st.size();
    I.src_ptr = pk.add(v.sp);
    I.src_t = pk.add(v.st);
    I.src_v = pk.add(v.sv);
    I.bp = pk.add(v.bps);
    I.probe = pk.add(v.pr);
  }
  c->const_bytes = pk.img.size();
  void *p = nullptr;
  e = hipMalloc(&p, c->const_bytes);
  if (e != hipSuccess) { *out = c.release(); (*out)->err = "constant upload allocation failed"; return EXPRI_ENOMEM; }
  c->d_const = static_cast<char *>(p);
  e = hipMemcpy(c->d_const, pk.img.data(), c->const_bytes, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&c->d_desc), sizeof(InstDesc) * n_inst);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&c->d_ptrs), sizeof(void *) * 4 * n_inst);
  if (e == hipSuccess) {
    // by launch class; within a class longest-processing-time-first: larger
    // instances (more nodes, then more devices) are launched first so they do
    // not wait for a free compute unit
    std::vector<int> order(n_inst);
    for (int k = 0; k < n_inst; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
      if (c->inst_class[a] != c->inst_class[b]) return c->inst_class[a] < c->inst_class[b];
      if (ckt[a].n != ckt[b].n) return ckt[a].n > ckt[b].n;
      return ckt[a].dev.n > ckt[b].dev.n;
    });
    for (int k = 0; k < n_inst; ++k) {
      LaunchClass &K = c->cls[c->inst_class[order[k]]];
      if (K.count == 0) K.first = k;
      ++K.count;
    }
    // transient grids: the first class (largest block size) one workgroup per
    // instance; the compute units it leaves go to the other classes by the
    // compute units their instances need (two workgroups per compute unit for
    // the 9-row kernels at 256 and 512 threads, whose register bound allows
    // it, one otherwise): every instance gets a workgroup when they all fit,
    // else the shares are in proportion to the need (at least one workgroup
    // each), so that every workgroup of every class finds a place at once.
    // With max_workgroups the first class is capped as well and the others
    // get one workgroup per compute unit.
    const int ncls = (int)c->cls.size();
    const int cus = op.max_workgroups > 0 ? op.max_workgroups : std::max(prop.multiProcessorCount, 1);
    c->cls[0].grid = op.max_workgroups > 0 ? std::min(c->cls[0].count, std::max(1, cus - (ncls - 1)))
                                           : c->cls[0].count;
    const long long left = std::max(cus - c->cls[0].grid, 0);
    auto per_cu = [&](const LaunchClass &K) { return (op.max_workgroups == 0 && K.bs <= 512 && K.em <= 9) ? 2 : 1; };
    long long need = 0;
    for (int q = 1; q < ncls; ++q) need += (c->cls[q].count + per_cu(c->cls[q]) - 1) / per_cu(c->cls[q]);
    for (int q = 1; q < ncls; ++q) {
      LaunchClass &K = c->cls[q];
      const int pc = per_cu(K);
      const long long nq = (K.count + pc - 1) / pc;
      K.grid = need <= left ? K.count
                            : std::max(1, std::min(K.count, (int)(pc * (left * nq / std::max(need, 1LL)))));
    }
    e = hipMalloc(reinterpret_cast<void **>(&c->d_next), sizeof(int) * c->cls.size());
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&c->d_order), sizeof(int) * n_inst);
    if (e == hipSuccess) e = hipMemcpy(c->d_order, order.data(), sizeof(int) * n_inst, hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) { *out = c.release(); return hip_fail(*out, e, "setup upload"); }

  e = hipEventCreate(&c->ev0);
  if (e == hipSuccess) e = hipEventCreate(&c->ev1);
  if (e == hipSuccess) e = hipEventCreate(&c->ev_fork);
  for (size_t q = 0; q < c->cls.size() && e == hipSuccess; ++q) {
    LaunchClass &K = c->cls[q];
    e = hipEventCreate(&K.e0);
    if (e == hipSuccess) e = hipEventCreate(&K.e1);
    if (e == hipSuccess && q == 0) K.stream = c->stream;
    if (e == hipSuccess && q > 0) {
      e = hipStreamCreateWithFlags(&K.stream, hipStreamNonBlocking);
      K.own_stream = e == hipSuccess;
    }
  }
  if (e != hipSuccess) { *out = c.release(); return hip_fail(*out, e, "event / stream create"); }
  // the per-kernel LDS ceiling is process-wide: allow the device maximum and
  // pass each launch its own size
  e = set_lds_limits(limit);
  if (e != hipSuccess) { *out = c.release(); return hip_fail(*out, e, "LDS limit"); }
  c->ws_bytes = layout_workspace(c.get());
  *out = c.release();
  return EXPRI_OK;
}
}  // namespace

expri_status expri_set_values(expri_ctx *c, int32_t inst, const expri_circuit *ckt) {
  if (!c) return EXPRI_EINVAL;
  if (c->grid) return fail(c, EXPRI_EINVAL, "set_values: not available in the multifrontal engine");
  if (!ckt || inst < 0 || inst >= (int32_t)c->inst.size())
    return fail(c, EXPRI_EINVAL, "set_values: instance out of range or null circuit");
  expri_status s;
  if ((s = validate_circuit(c, *ckt, inst)) != EXPRI_OK) return s;
  const expri_circuit &K = *ckt;
  Inst &I = c->inst[inst];
  const PatternDev &P = c->pats[I.pat];
  const Symbolic &S = P.sym;
  const std::string w = "set_values: instance " + std::to_string(inst) + ": ";
  const bool same = pattern_hash(pattern_input(K)) == S.hash && S.n == K.n && S.n_dev == K.dev.n &&
                    S.n_src == K.n_src && (int32_t)S.g_col.size() == K.G.nnz &&
                    (int32_t)S.c_col.size() == K.C.nnz && (int32_t)S.b_col.size() == K.B.nnz;
  if (!same) return fail(c, EXPRI_EPATTERN, w + "the circuit's sparsity pattern differs from the instance's");
  if (K.n_probe != I.n_probe) return fail(c, EXPRI_EINVAL, w + "the number of probes differs");
  const InstValues v = inst_values(K, P);
  if ((int32_t)v.st.size() != I.n_corners) return fail(c, EXPRI_EINVAL, w + "the number of PWL corners differs");
  // no kernel of this context may still read the old values
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (const auto &Q : c->cls)
    if (Q.stream && Q.stream != c->stream) HIPCHK(c, hipStreamSynchronize(Q.stream));
  auto put = [&](size_t off, const void *src, size_t bytes) -> hipError_t {
    return bytes ? hipMemcpy(c->d_const + off, src, bytes, hipMemcpyHostToDevice) : hipSuccess;
  };
  const std::pair<size_t, std::pair<const void *, size_t>> parts[] = {
      {I.g_val, {v.g.data(), 8 * v.g.size()}},        {I.g_lu, {v.glu.data(), 8 * v.glu.size()}},
      {I.c_val, {v.c.data(), 8 * v.c.size()}},        {I.c_ell_val, {v.ell.data(), 8 * v.ell.size()}},
      {I.b_val, {v.b.data(), 8 * v.b.size()}},        {I.dev_par, {v.par.data(), 8 * v.par.size()}},
      {I.src_ptr, {v.sp.data(), 4 * v.sp.size()}},    {I.src_t, {v.st.data(), 8 * v.st.size()}},
      {I.src_v, {v.sv.data(), 8 * v.sv.size()}},      {I.bp, {v.bps.data(), 8 * v.bps.size()}},
      {I.probe, {v.pr.data(), 4 * v.pr.size()}}};
  for (const auto &q : parts) HIPCHK(c, put(q.first, q.second.first, q.second.second));
  I.vdd = K.vdd;
  I.T = K.T;
  I.h_max = c->opts.h_max > 0 ? c->opts.h_max : K.T / 20;
  I.n_bp = v.n_bp;
  c->factors_stale = true;
  if (c->d_ws) {
    fill_descs(c);
    if ((s = upload_descs(c)) != EXPRI_OK) return s;
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return EXPRI_OK;
}

expri_status expri_workspace_size(const expri_ctx *c, size_t *bytes) {
  if (!c || !bytes) return EXPRI_EINVAL;
  *bytes = c->ws_bytes;
  return EXPRI_OK;
}

expri_status expri_bind_workspace(expri_ctx *c, void *dev_ptr, size_t bytes) {
  if (!c) return EXPRI_EINVAL;
  if (c->grid) return fail(c, EXPRI_EINVAL, "bind_workspace: the multifrontal engine owns its memory");
  if (!dev_ptr || bytes < c->ws_bytes) return fail(c, EXPRI_EINVAL, "workspace too small");
  if (reinterpret_cast<uintptr_t>(dev_ptr) % kAlign) return fail(c, EXPRI_EINVAL, "workspace not 256-byte aligned");
  if (c->d_ws && c->ws_owned) (void)hipFree(c->d_ws);
  c->d_ws = static_cast<char *>(dev_ptr);
  c->ws_owned = false;
  fill_descs(c);
  expri_status s = upload_descs(c);
  if (s != EXPRI_OK) return s;
  // entries read but never written (basis padding, empty solve slots)
  HIPCHK(c, launch_init_workspace(c->d_desc, (int)c->inst.size(), c->stream));
  return EXPRI_OK;
}

expri_status expri_dc(expri_ctx *c, double *const *x, double t0) {
  if (!c || !x) return EXPRI_EINVAL;
  if (c->grid) {
    const int st = c->grid->dc(x[0], t0);
    grid_info(c, st);
    return grid_status(c, st);
  }
  expri_status s;
  if ((s = ensure_ws(c)) != EXPRI_OK) return s;
  const int n = (int)c->inst.size();
  if ((s = upload_descs(c)) != EXPRI_OK) return s;
  if ((s = put_ptrs(c, 0, reinterpret_cast<const void *const *>(x))) != EXPRI_OK) return s;
  HIPCHK(c, launch_begin(c->d_desc, n, reinterpret_cast<const double *const *>(c->d_ptrs), t0, c->opts.h_init, c->stream));
  for (const auto &K : c->cls)
    HIPCHK(c, launch_dc(c->d_desc, c->d_order + K.first, K.count, kernel_opts(c->opts), t0, 20000, K.bs, K.R, K.NX,
                        c->stream));
  std::vector<InstState> st;
  if ((s = read_states(c, st)) != EXPRI_OK) return s;
  // write back only instances that converged (x keeps its input otherwise)
  for (int k = 0; k < n; ++k) {
    c->inst[k].info = expri_run_info{t0, st[k].steps, st[k].steps, 0, 0, st[k].status, {0, 0, 0, 0, 0, 0},
                                     0, 0, 0};
  }
  if ((s = first_error(c, st, "DC")) != EXPRI_OK) return s;
  HIPCHK(c, launch_end(c->d_desc, n, reinterpret_cast<double *const *>(c->d_ptrs), c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return EXPRI_OK;
}

expri_status expri_factor(expri_ctx *c, const double *const *x) {
  if (!c || !x) return EXPRI_EINVAL;
  if (c->grid) return grid_status(c, c->grid->factor(x[0]));
  expri_status s;
  if ((s = ensure_ws(c)) != EXPRI_OK) return s;
  const int n = (int)c->inst.size();
  if ((s = upload_descs(c)) != EXPRI_OK) return s;
  if ((s = put_ptrs(c, 0, reinterpret_cast<const void *const *>(x))) != EXPRI_OK) return s;
  HIPCHK(c, launch_begin(c->d_desc, n, reinterpret_cast<const double *const *>(c->d_ptrs), 0.0, c->opts.h_init, c->stream));
  for (const auto &K : c->cls)
    HIPCHK(c, launch_factor(c->d_desc, c->d_order + K.first, K.count, kernel_opts(c->opts), K.bs, K.R, K.NX,
                            c->stream));
  std::vector<InstState> st;
  if ((s = read_states(c, st)) != EXPRI_OK) return s;
  if ((s = first_error(c, st, "factor")) != EXPRI_OK) return s;
  c->factors_stale = false;
  return EXPRI_OK;
}

expri_status expri_solve(expri_ctx *c, const double *const *b, double *const *y) {
  if (!c || !b || !y) return EXPRI_EINVAL;
  if (c->grid) return grid_status(c, c->grid->solve(b[0], y[0]));
  if (c->factors_stale) return fail(c, EXPRI_EINVAL, "solve: values replaced since the last expri_factor");
  expri_status s;
  if ((s = ensure_ws(c)) != EXPRI_OK) return s;
  const int n = (int)c->inst.size();
  if ((s = upload_descs(c)) != EXPRI_OK) return s;
  if ((s = put_ptrs(c, 0, reinterpret_cast<const void *const *>(b))) != EXPRI_OK) return s;
  if ((s = put_ptrs(c, 1, reinterpret_cast<const void *const *>(y))) != EXPRI_OK) return s;
  for (const auto &K : c->cls)
    HIPCHK(c, launch_solve(c->d_desc, c->d_order + K.first, K.count,
                           reinterpret_cast<const double *const *>(c->d_ptrs),
                           reinterpret_cast<double *const *>(c->d_ptrs + n), K.bs, K.R, K.NX, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return EXPRI_OK;
}

expri_status expri_mevp(expri_ctx *c, const double *const *v, double *const *out, double h, double eps,
                        int32_t *m, double *rho) {
  if (!c || !v || !out || !(h > 0) || !(eps > 0)) return EXPRI_EINVAL;
  if (c->grid) {
    const int st = c->grid->mevp(v[0], out[0], h, eps, m, rho);
    c->inst[0].info = expri_run_info{};
    c->inst[0].info.arnoldi = (int32_t)c->grid->arnoldi;
    c->inst[0].info.status = st;
    return grid_status(c, st);
  }
  if (c->factors_stale) return fail(c, EXPRI_EINVAL, "mevp: values replaced since the last expri_factor");
  expri_status s;
  if ((s = ensure_ws(c)) != EXPRI_OK) return s;
  const int n = (int)c->inst.size();
  if ((s = put_ptrs(c, 0, reinterpret_cast<const void *const *>(v))) != EXPRI_OK) return s;
  if ((s = put_ptrs(c, 1, reinterpret_cast<const void *const *>(out))) != EXPRI_OK) return s;
  for (const auto &K : c->cls)
    HIPCHK(c, launch_mevp(c->d_desc, c->d_order + K.first, K.count, kernel_opts(c->opts),
                          reinterpret_cast<const double *const *>(c->d_ptrs),
                          reinterpret_cast<double *const *>(c->d_ptrs + n), h, eps, K.bs, K.R, K.NX, c->stream));
  std::vector<InstState> st;
  if ((s = read_states(c, st)) != EXPRI_OK) return s;
  for (int k = 0; k < n; ++k) {
    if (m) m[k] = st[k].arnoldi;
    if (rho) rho[k] = st[k].t;
    expri_run_info &in = c->inst[k].info;
    in = expri_run_info{};
    in.arnoldi = st[k].arnoldi;
    in.status = st[k].status;
    for (int p = 0; p < 6; ++p) in.phase_s[p] = st[k].ph[p] / c->wall_hz;
  }
  return first_error(c, st, "mevp");
}

expri_status expri_run(expri_ctx *c, double *const *x, double t0, int32_t max_steps_per_launch) {
  if (!c || !x) return EXPRI_EINVAL;
  if (c->grid) {
    const int st = c->grid->run(x[0], t0, nullptr, 0, INT32_MAX, c->opts.E_rr, c->opts.eps_krylov, c->opts.h_init,
                                nullptr);
    grid_info(c, st);
    return grid_status(c, st);
  }
  expri_status s;
  if ((s = ensure_ws(c)) != EXPRI_OK) return s;
  restore_corners(c);
  return drive(c, x, t0, max_steps_per_launch, 0);
}

expri_status expri_run_schedule(expri_ctx *c, double *const *x, double t0, const double *const *t_seq,
                                const int32_t *n_steps) {
  if (!c || !x || !t_seq || !n_steps) return EXPRI_EINVAL;
  if (c->grid) {
    for (int i = 0; i < n_steps[0]; ++i)
      if (!(t_seq[0][i] > (i ? t_seq[0][i - 1] : t0)) || !std::isfinite(t_seq[0][i]))
        return fail(c, EXPRI_EINVAL, "schedule not increasing");
    const int st = c->grid->run(x[0], t0, t_seq[0], n_steps[0], INT32_MAX, c->opts.E_rr, c->opts.eps_krylov,
                                c->opts.h_init, nullptr);
    grid_info(c, st);
    return grid_status(c, st);
  }
  expri_status s;
  if ((s = ensure_ws(c)) != EXPRI_OK) return s;
  const int n = (int)c->inst.size();
  size_t total = 0;
  int32_t most = 1;
  for (int k = 0; k < n; ++k) {
    if (n_steps[k] < 0 || (n_steps[k] > 0 && !t_seq[k])) return fail(c, EXPRI_EINVAL, "bad schedule");
    double prev = t0;
    for (int i = 0; i < n_steps[k]; ++i) {
      if (!(t_seq[k][i] > prev) || !std::isfinite(t_seq[k][i])) return fail(c, EXPRI_EINVAL, "schedule not increasing");
      prev = t_seq[k][i];
    }
    total += align_up(8 * (size_t)std::max(n_steps[k], 1));
    most = std::max(most, n_steps[k]);
  }
  char *d = nullptr;
  HIPCHK(c, hipMalloc(reinterpret_cast<void **>(&d), total));
  size_t off = 0;
  s = EXPRI_OK;
  for (int k = 0; k < n && s == EXPRI_OK; ++k) {
    if (n_steps[k] > 0 &&
        hipMemcpy(d + off, t_seq[k], 8 * (size_t)n_steps[k], hipMemcpyHostToDevice) != hipSuccess)
      s = fail(c, EXPRI_EHIP, "schedule upload");
    c->h_desc[k].bp = reinterpret_cast<const double *>(d + off);
    c->h_desc[k].n_bp = n_steps[k];
    off += align_up(8 * (size_t)std::max(n_steps[k], 1));
  }
  if (s == EXPRI_OK) s = drive(c, x, t0, std::min(most, c->opts.trace_cap), 1);
  // the descriptors point at the schedule only for this call: every later
  // call reads the source corners again
  (void)hipStreamSynchronize(c->stream);
  restore_corners(c);
  const expri_status su = upload_descs(c);
  (void)hipStreamSynchronize(c->stream);
  (void)hipFree(d);
  return s != EXPRI_OK ? s : su;
}

expri_status expri_step(expri_ctx *c, double *const *x, double t, double h, double tol, expri_step_info *info) {
  if (!c || !x || !(h > 0) || !std::isfinite(t) || !(tol >= 0)) return EXPRI_EINVAL;
  if (c->grid) {
    GridStepRec rec{};
    const double E = tol > 0 ? tol : c->opts.E_rr, eps = tol > 0 ? 0.1 * tol : c->opts.eps_krylov;
    const int st = c->grid->run(x[0], t, nullptr, 0, 1, E, eps, h, &rec);
    grid_info(c, st);
    if (info) {
      info[0] = expri_step_info{};
      info[0].t = c->grid->t_reached;
      info[0].h_next = c->grid->next_h;
      info[0].status = st;
      if (c->grid->steps > 0) {
        info[0].h_used = rec.h;
        info[0].err_inf = rec.err;
        info[0].krylov_res = rec.rho;
        info[0].m = rec.m;
        info[0].m_err = rec.m_err;
        info[0].n_reject = rec.rejects;
      }
    }
    return grid_status(c, st);
  }
  expri_status s;
  if ((s = ensure_ws(c)) != EXPRI_OK) return s;
  const int n = (int)c->inst.size();
  restore_corners(c);
  if ((s = upload_descs(c)) != EXPRI_OK) return s;
  if ((s = put_ptrs(c, 0, reinterpret_cast<const void *const *>(x))) != EXPRI_OK) return s;
  // the paper's step control at the error budget tol (eps_K = tol / 10)
  Opts ko = kernel_opts(c->opts);
  if (tol > 0) {
    ko.E_rr = tol;
    ko.eps_K = 0.1 * tol;
  }
  HIPCHK(c, launch_begin(c->d_desc, n, reinterpret_cast<const double *const *>(c->d_ptrs), t, h, c->stream));
  for (auto &I : c->inst) I.trace_host.clear();
  for (auto &K : c->cls) K.kernel_s = 0.0;
  if ((s = launch_run_classes(c, ko, 1, 0)) != EXPRI_OK) return s;
  std::vector<InstState> st;
  if ((s = read_states(c, st)) != EXPRI_OK) return s;
  float ms = 0.0f;
  HIPCHK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
  c->run_kernel_s = 1e-3 * ms;
  c->run_launches = 1;
  for (auto &K : c->cls) {
    HIPCHK(c, hipEventElapsedTime(&ms, K.e0, K.e1));
    K.kernel_s = 1e-3 * ms;
  }
  for (int k = 0; k < n; ++k) {
    Inst &I = c->inst[k];
    const size_t rec = kRecFixed + I.n_probe;
    I.trace_host.assign((size_t)st[k].steps * rec, 0.0);
    if (st[k].steps > 0)
      HIPCHK(c, hipMemcpyAsync(I.trace_host.data(), c->d_ws + I.trace, sizeof(double) * rec,
                               hipMemcpyDeviceToHost, c->stream));
  }
  HIPCHK(c, launch_end(c->d_desc, n, reinterpret_cast<double *const *>(c->d_ptrs), c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int k = 0; k < n; ++k) {
    Inst &I = c->inst[k];
    expri_run_info &in = I.info;
    in.t = st[k].t;
    in.steps = st[k].steps;
    in.lu_count = st[k].lu_count;
    in.rejects = st[k].rejects;
    in.arnoldi = st[k].arnoldi;
    in.status = st[k].status;
    for (int p = 0; p < 6; ++p) in.phase_s[p] = st[k].ph[p] / c->wall_hz;
    in.trials = st[k].trials;
    in.mgs_terms = st[k].mgs_terms;
    in.comb_terms = st[k].comb_terms;
    if (info) {
      expri_step_info &o = info[k];
      o = expri_step_info{};
      o.t = st[k].t;
      o.h_next = st[k].h_prop;
      o.n_reject = st[k].rejects;
      o.status = st[k].status;
      if (st[k].steps > 0) {
        const double *r = I.trace_host.data();
        o.h_used = r[1];
        o.m = (int32_t)r[3];
        o.m_err = (int32_t)r[4];
        o.err_inf = r[6];
        o.krylov_res = r[7];
      }
    }
  }
  return first_error(c, st, "step");
}

expri_status expri_step_fixed(expri_ctx *c, double *const *x, double t, double h, expri_run_info *info) {
  if (!c || !x || !(h > 0)) return EXPRI_EINVAL;
  const int n = (int)c->inst.size();
  std::vector<double> tn(n, t + h);
  std::vector<const double *> seq(n);
  std::vector<int32_t> cnt(n, 1);
  for (int k = 0; k < n; ++k) seq[k] = &tn[k];
  expri_status s = expri_run_schedule(c, x, t, seq.data(), cnt.data());
  if (info)
    for (int k = 0; k < n; ++k) info[k] = c->inst[k].info;
  return s;
}

expri_status expri_run_noalloc(expri_ctx *c, double *const *x, double t0, int32_t max_steps_per_launch) {
  if (!c || !x) return EXPRI_EINVAL;
  if (c->grid) return fail(c, EXPRI_EINVAL, "run_noalloc: not available in the multifrontal engine");
  if (c->ws_bytes > kScratchBytes)
    return fail(c, EXPRI_EINVAL, "run_noalloc: the context needs a workspace of " + std::to_string(c->ws_bytes) +
                                     " bytes, more than the static scratch of " + std::to_string(kScratchBytes));
  char *scr = nullptr;
  expri_status s = scratch_ptr(c, &scr);
  if (s != EXPRI_OK) return s;
  // the call's workspace is the scratch array; the context's own workspace
  // (if any) is set aside and restored afterwards, untouched
  char *own = c->d_ws;
  const bool own_owned = c->ws_owned;
  c->d_ws = scr;
  c->ws_owned = false;
  fill_descs(c);
  restore_corners(c);
  s = upload_descs(c);
  if (s == EXPRI_OK && hipSuccess != launch_init_workspace(c->d_desc, (int)c->inst.size(), c->stream))
    s = fail(c, EXPRI_EHIP, "run_noalloc: workspace initialisation");
  if (s == EXPRI_OK) s = drive(c, x, t0, max_steps_per_launch, 0);
  (void)hipStreamSynchronize(c->stream);
  c->d_ws = own;
  c->ws_owned = own_owned;
  fill_descs(c);
  const expri_status su = own ? upload_descs(c) : EXPRI_OK;
  (void)hipStreamSynchronize(c->stream);
  return s != EXPRI_OK ? s : su;
}

expri_status expri_trace(const expri_ctx *c, int32_t inst, double *out, int64_t cap, int64_t *n_rec) {
  if (!c || inst < 0 || inst >= (int32_t)c->inst.size() || !n_rec) return EXPRI_EINVAL;
  const Inst &I = c->inst[inst];
  const size_t rec = kRecFixed + I.n_probe;
  const int64_t avail = (int64_t)(I.trace_host.size() / rec);
  *n_rec = avail;
  if (out && cap > 0) std::memcpy(out, I.trace_host.data(), sizeof(double) * rec * std::min(cap, avail));
  return EXPRI_OK;
}

expri_status expri_get_run_info(const expri_ctx *c, int32_t inst, expri_run_info *info) {
  if (!c || inst < 0 || inst >= (int32_t)c->inst.size() || !info) return EXPRI_EINVAL;
  *info = c->inst[inst].info;
  return EXPRI_OK;
}

expri_status expri_lu_pattern(const expri_ctx *c, int32_t inst, int32_t *rowptr, int32_t *col, int32_t *perm,
                              int64_t *nnz, int32_t *n_lev, int32_t *n_ulev, int64_t *flops) {
  if (!c || inst < 0 || inst >= (int32_t)c->inst.size()) return EXPRI_EINVAL;
  if (c->grid) return EXPRI_EINVAL;
  const Symbolic &S = c->pats[c->inst[inst].pat].sym;
  if (rowptr) std::memcpy(rowptr, S.lu_rowptr.data(), sizeof(int32_t) * S.lu_rowptr.size());
  if (col) std::memcpy(col, S.lu_col.data(), sizeof(int32_t) * S.lu_col.size());
  if (perm) std::memcpy(perm, S.perm.data(), sizeof(int32_t) * S.perm.size());
  if (nnz) *nnz = (int64_t)S.lu_col.size();
  if (n_lev) *n_lev = (int32_t)S.lev_ptr.size() - 1;
  if (n_ulev) *n_ulev = (int32_t)S.ulev_ptr.size() - 1;
  if (flops) *flops = S.flops;
  return EXPRI_OK;
}

expri_status expri_lu_values(const expri_ctx *c, int32_t inst, double *out) {
  if (!c || !out || inst < 0 || inst >= (int32_t)c->inst.size() || !c->d_ws) return EXPRI_EINVAL;
  if (c->grid) return EXPRI_EINVAL;
  const Inst &I = c->inst[inst];
  const size_t nnz = c->pats[I.pat].sym.lu_col.size();
  if (hipMemcpy(out, c->d_ws + I.lu, sizeof(double) * nnz, hipMemcpyDeviceToHost) != hipSuccess)
    return EXPRI_EHIP;
  return EXPRI_OK;
}

expri_status expri_diag_time(expri_ctx *c, int32_t what, int32_t reps, int32_t arg, double *seconds) {
  if (!c || !seconds || what < 0 || what > 11 || reps < 1) return EXPRI_EINVAL;
  if (c->grid) return grid_status(c, c->grid->diag(what, reps, seconds));
  if (arg < 0 || arg > c->opts.m_max - 1 || (what == 6 && arg < 1)) return EXPRI_EINVAL;
  expri_status s;
  if ((s = ensure_ws(c)) != EXPRI_OK) return s;
  long long *d = nullptr;
  HIPCHK(c, hipMalloc(reinterpret_cast<void **>(&d), 2 * sizeof(long long)));
  const LaunchClass &K = c->cls[c->inst_class[0]];
  hipError_t e = launch_diag(c->d_desc, what, reps, arg, d, K.bs, K.R, K.NX, c->stream);
  long long h[2] = {0, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(h, d, sizeof(h), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  (void)hipFree(d);
  if (e != hipSuccess) return hip_fail(c, e, "diag");
  *seconds = h[0] / c->wall_hz / reps;
  return EXPRI_OK;
}

expri_status expri_block_size(const expri_ctx *c, int32_t *bs) {
  if (!c || !bs) return EXPRI_EINVAL;
  *bs = c->grid ? 256 : c->bs;
  return EXPRI_OK;
}

expri_status expri_kernel_time(const expri_ctx *c, double *seconds, int32_t *launches) {
  if (!c || !seconds || !launches) return EXPRI_EINVAL;
  *seconds = c->run_kernel_s;
  *launches = c->run_launches;
  return EXPRI_OK;
}

expri_status expri_launch_classes(const expri_ctx *c, int32_t cap, int32_t *block_size, int32_t *max_rows,
                                  int32_t *n_inst, int32_t *workgroups, double *kernel_s, int32_t *inst_class,
                                  int32_t *n_classes) {
  if (!c || !n_classes || cap < 0) return EXPRI_EINVAL;
  if (c->grid) {  // one "class": the multifrontal engine's kernels (256 threads), grid-wide launches
    *n_classes = 1;
    if (inst_class) inst_class[0] = 0;
    if (cap >= 1) {
      if (block_size) block_size[0] = 256;
      if (max_rows) max_rows[0] = 0;
      if (n_inst) n_inst[0] = 1;
      if (workgroups) workgroups[0] = 0;
      if (kernel_s) kernel_s[0] = c->run_kernel_s;
    }
    return EXPRI_OK;
  }
  *n_classes = (int32_t)c->cls.size();
  if (inst_class)
    for (size_t k = 0; k < c->inst_class.size(); ++k) inst_class[k] = c->inst_class[k];
  for (int32_t q = 0; q < std::min<int32_t>(cap, *n_classes); ++q) {
    if (block_size) block_size[q] = c->cls[q].bs;
    if (max_rows) max_rows[q] = c->cls[q].em;
    if (n_inst) n_inst[q] = c->cls[q].count;
    if (workgroups) workgroups[q] = c->cls[q].grid;
    if (kernel_s) kernel_s[q] = c->cls[q].kernel_s;
  }
  return EXPRI_OK;
}

const char *expri_last_error(const expri_ctx *c) { return c ? c->err.c_str() : "null context"; }

expri_status expri_instance_config(const expri_ctx *c, int32_t inst, int32_t cfg[4]) {
  if (!c || !cfg || c->grid || inst < 0 || inst >= (int32_t)c->inst.size()) return EXPRI_EINVAL;
  const int q = c->inst_class[inst];
  const PatternDev &P = c->pats[c->inst[inst].pat];
  cfg[0] = P.bs;
  cfg[1] = c->cls[q].em;
  cfg[2] = P.pl;
  cfg[3] = P.pu;
  return EXPRI_OK;
}

int64_t expri_autotune_runs(void) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  return g_tune_runs;
}

expri_status expri_controller_load(expri_ctx *c, const float *params, const float *norm, double safety) {
  if (!c) return EXPRI_EINVAL;
  if (!params) {
    c->ctrl_on = false;
    if (c->grid) c->grid->ctrl_w = nullptr;
    return EXPRI_OK;
  }
  if (!norm || !(safety > 0.0 && safety <= 1.0)) return fail(c, EXPRI_EINVAL, "controller: norm missing or safety not in (0, 1]");
  for (int i = 0; i < kMlpIn; ++i)
    if (!(norm[kMlpIn + i] > 0.0f)) return fail(c, EXPRI_EINVAL, "controller: input std must be > 0");
  for (int o = 0; o < kMlpOut; ++o)
    if (!(norm[2 * kMlpIn + kMlpOut + o] > 0.0f)) return fail(c, EXPRI_EINVAL, "controller: target std must be > 0");
  for (int i = 0; i < kMlpParams; ++i)
    if (!std::isfinite(params[i])) return fail(c, EXPRI_EINVAL, "controller: non-finite parameter");
  if (!c->d_ctrl_w) {
    HIPCHK(c, hipMalloc(reinterpret_cast<void **>(&c->d_ctrl_w), sizeof(uint16_t) * kMlpParams));
    HIPCHK(c, hipMalloc(reinterpret_cast<void **>(&c->d_ctrl_norm), sizeof(float) * kMlpNorm));
    HIPCHK(c, hipMalloc(reinterpret_cast<void **>(&c->d_ctrl_tmp), sizeof(float) * kMlpParams));
  }
  HIPCHK(c, hipMemcpyAsync(c->d_ctrl_tmp, params, sizeof(float) * kMlpParams, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d_ctrl_norm, norm, sizeof(float) * kMlpNorm, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, launch_mlp_pack(c->d_ctrl_tmp, c->d_ctrl_w, true, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->ctrl_on = true;
  c->ctrl_safety = safety;
  if (c->grid) {
    c->grid->ctrl_w = c->d_ctrl_w;
    c->grid->ctrl_norm = c->d_ctrl_norm;
    c->grid->ctrl_safety = safety;
  }
  return EXPRI_OK;
}

void expri_destroy(expri_ctx *c) {
  if (!c) return;
  if (c->d_ctrl_w) (void)hipFree(c->d_ctrl_w);
  if (c->d_ctrl_norm) (void)hipFree(c->d_ctrl_norm);
  if (c->d_ctrl_tmp) (void)hipFree(c->d_ctrl_tmp);
  if (c->d_ws && c->ws_owned) (void)hipFree(c->d_ws);
  if (c->d_const) (void)hipFree(c->d_const);
  if (c->d_desc) (void)hipFree(c->d_desc);
  if (c->d_ptrs) (void)hipFree(c->d_ptrs);
  if (c->d_order) (void)hipFree(c->d_order);
  if (c->d_next) (void)hipFree(c->d_next);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  for (auto &K : c->cls) {
    if (K.e0) (void)hipEventDestroy(K.e0);
    if (K.e1) (void)hipEventDestroy(K.e1);
    if (K.own_stream && K.stream) (void)hipStreamDestroy(K.stream);
  }
  delete c;
}

}  // extern "C"
