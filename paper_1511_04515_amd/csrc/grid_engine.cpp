// Host driver of the multifrontal engine (see grid_engine.hpp): set-up of
// the device data and the step loop of Algorithm 2 with Algorithm 1 inside.
#include "grid_engine.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace expri {

// kernels of grid.hip and engine.hip
hipError_t g_fill(double *p, int64_t n, double v, hipStream_t s);
hipError_t g_gather(int n, const int *map, const double *x, double *y, hipStream_t s);
hipError_t g_scatter(int n, const int *map, const double *x, double *y, hipStream_t s);
hipError_t g_stamp(int n_dev, const int *dev_node, const double *par, const double *x, double vdd, double *devI,
                   double *devD, hipStream_t s);
hipError_t g_assemble(int n_ent, const int64_t *ent_pos, const int *ent_row, const int *ent_g, const int *ent_jptr,
                      const int *ent_jcode, const double *g_val, const double *devD, double *F,
                      unsigned long long *rowmax, hipStream_t s);
hipError_t g_extend(int n_items, const int *items, const int *nc, const int *fsz, const int *parent,
                    const int64_t *f_off, const int *r_ptr, const int *rel, double *F, hipStream_t s);
hipError_t g_extend_small(int n_parents, const int *parents, const int *nc, const int *fsz, const int64_t *f_off,
                          const int *ch_ptr, const int *ch, const int *r_ptr, const int *rel, double *F, hipStream_t s);
hipError_t g_small_lu(int n32, const int *f32, int n64, const int *f64, const int *c0, const int *nc, const int *fsz,
                      const int64_t *f_off, const unsigned long long *rowmax, double piv_tol, double *F, int *bad,
                      hipStream_t s);
hipError_t g_panel(int n_fronts, const int *fronts, int n_items, const int *items, int k0, int C, int fuse,
                   const int *c0, const int *nc, const int *fsz, const int64_t *f_off,
                   const unsigned long long *rowmax, double piv_tol, double *F, int *bad, hipStream_t s);
hipError_t g_set_limits();
hipError_t g_update(int n_items, const int *items, int k0, const int *c0, const int *nc, const int *fsz,
                    const int64_t *f_off, const unsigned long long *rowmax, double piv_tol, double *F, int *bad,
                    hipStream_t s);
hipError_t g_fwd(int n_small, const int *small, int n_big, const int *big, int n_items, const int *items,
                 int max_f, int max_nc, const int *c0, const int *nc, const int *fsz, const int64_t *f_off,
                 const int *ch_ptr, const int *ch, const int *r_ptr, const int *rel, const int *u_off, const double *F,
                 double *x, int nr, int64_t ldx, double *upd, int64_t ldu, int tri_bs, int n_trmv,
                 const int *trmv, int max_p_inv, const int64_t *inv_off, const double *Finv, double *tmp,
                 hipStream_t s);
hipError_t g_bwd(int n_small, const int *small, int n_big, const int *big, int n_items, const int *items,
                 int max_f, int max_nc, const int *c0, const int *nc, const int *fsz, const int64_t *f_off,
                 const int *r_ptr, const int *r_idx, const double *F, double *x, int nr, int64_t ldx, int tri_bs,
                 int n_trmv, const int *trmv, int max_p_inv, const int64_t *inv_off, const double *Finv,
                 double *tmp, hipStream_t s);
hipError_t g_inv(int n_items, const int *items, const int *nc, const int *fsz, const int64_t *f_off,
                 const int64_t *inv_off, const double *F, double *Finv, hipStream_t s);
hipError_t g_sources(int n_src, const int *src_ptr, const double *src_t, const double *src_v, double t, double tm,
                     double *u, double *slope, hipStream_t s);
hipError_t g_rhs(int n, const int *g_rowptr, const int *g_col, const double *g_val, const int *b_rowptr,
                 const int *b_col, const double *b_val, const int *node_ptr, const int *node_code, const double *devI,
                 const double *x, const double *u, const double *sl, double *r, double *bs, hipStream_t s);
hipError_t g_spmv(int n, const int *rp, const int *ci, const double *val, const double *x, double alpha, double *y,
                  hipStream_t s);
hipError_t g_dots(int n, const double *V, int64_t ldv, int ncol, const double *w, double *partial, double *out,
                  hipStream_t s);
hipError_t g_absmax(int n, const double *x, double *partial, double *out, hipStream_t s);
hipError_t g_gemv_sub(int n, const double *V, int64_t ldv, int ncol, const double *hcoef, double *w, hipStream_t s);
hipError_t g_hcol(int j, const double *h1, const double *h2, double *H, double breakdown, double *sc, hipStream_t s);
hipError_t g_scale(int n, const double *x, const double *sc, int idx, double *out, hipStream_t s);
hipError_t g_start(int n, const double *v, double *sc, double *v1, hipStream_t s);
hipError_t g_combine(int n, const double *base, const double *p, double h, const double *V, int64_t ldv, int m,
                     const double *beta, const double *d, double *out, hipStream_t s);
hipError_t g_axpy(int n, double a, const double *x, double *y, hipStream_t s);
hipError_t g_sub(int n, const double *a, const double *b, double *out, hipStream_t s);
hipError_t g_dF(int n, const int *node_ptr, const int *node_code, const int *dev_node, const double *devD,
                const double *devI0, const double *devI1, const double *xk, const double *x1, double *out,
                hipStream_t s);
hipError_t g_fk(int n, const int *node_ptr, const int *node_code, const int *dev_node, const double *devD,
                const double *devI, const double *x, double *out, hipStream_t s);
hipError_t g_ctrl(const uint16_t *w, const float *norm, const float *feat, float *out, hipStream_t s);
hipError_t launch_hess_phi1(const double *H, int m, double h, const double *beta, int want2, double *mat,
                            double *out, hipStream_t s);

namespace {
// status codes (include/expri.h)
constexpr int kSOK = 0, kSEINVAL = -1, kSENOMEM = -2, kSESINGULAR = -3, kSEKRYLOV = -4, kSESTEPMIN = -5,
              kSENONFINITE = -6, kSEHIP = -7, kSENOCONV = -9;
constexpr int kRBlocks = 512;  // blocks of the two-pass reductions (grid.hip)
constexpr int kSc = 2 * kHLd + 8;  // offset of the basis scalars in the hess_phi1 output area
constexpr int kFuse = 64;          // trailing blocks up to this size are updated by the panel kernel
constexpr int kInvPivots = 288;    // pivot blocks with more pivots are inverted after each factorisation
}  // namespace

#define GCHK(call)                                  \
  do {                                              \
    const hipError_t e_ = (call);                   \
    if (e_ != hipSuccess) return hip(e_, #call);    \
  } while (0)
#define GRET(call)                 \
  do {                             \
    const int s_ = (call);         \
    if (s_ != kSOK) return s_;     \
  } while (0)

GridEngine::~GridEngine() {
  for (void *p : allocs) (void)hipFree(p);
}

int GridEngine::fail(int code, const std::string &msg) {
  err = msg;
  return code;
}

int GridEngine::hip(hipError_t e, const char *what) {
  err = std::string("HIP error ") + hipGetErrorString(e) + " in " + what;
  return kSEHIP;
}

template <class T>
T *GridEngine::dalloc(size_t count) {
  void *p = nullptr;
  if (hipMalloc(&p, sizeof(T) * std::max<size_t>(count, 1)) != hipSuccess) return nullptr;
  allocs.push_back(p);
  return static_cast<T *>(p);
}

template <class T>
T *GridEngine::dupload(const std::vector<T> &v) {
  T *p = dalloc<T>(v.size());
  if (p && !v.empty() && hipMemcpy(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice) != hipSuccess)
    return nullptr;
  return p;
}

int GridEngine::setup(const PatternInput &pin, const GridValues &val, const int32_t *probe, int32_t nprobe,
                      const GridOpts &opts, hipStream_t s, int32_t leaf) {
  o = opts;
  stream = s;
  GCHK(g_set_limits());
  if (!analyse_frontal(pin, fs, leaf)) return fail(kSEINVAL, "multifrontal analysis: " + fs.error);
  const int n = fs.n;
  vdd = val.vdd;
  T = val.T;
  h_max = o.h_max > 0 ? o.h_max : T / 20;
  n_probe = nprobe;
  bool ok = true;
  auto up32 = [&](const std::vector<int32_t> &v) {
    int32_t *p = dupload(v);
    ok = ok && p;
    return p;
  };
  auto up64 = [&](const std::vector<int64_t> &v) {
    int64_t *p = dupload(v);
    ok = ok && p;
    return p;
  };
  auto upd = [&](const std::vector<double> &v) {
    double *p = dupload(v);
    ok = ok && p;
    return p;
  };
  d_perm = up32(fs.perm);
  d_c0 = up32(fs.c0);
  d_nc = up32(fs.nc);
  d_fsz = up32(fs.fsz);
  d_parent = up32(fs.parent);
  d_r_ptr = up32(fs.r_ptr);
  d_r_idx = up32(fs.r_idx);
  d_rel = up32(fs.rel);
  d_u_off = up32(fs.u_off);
  d_ch_ptr = up32(fs.ch_ptr);
  d_ch = up32(fs.ch);
  d_lev_front = up32(fs.lev_front);
  d_f_off = up64(fs.f_off);
  d_ent_pos = up64(fs.ent_pos);
  d_ent_row = up32(fs.ent_row);
  d_ent_g = up32(fs.ent_g);
  d_ent_jptr = up32(fs.ent_jptr);
  d_ent_jcode = up32(fs.ent_jcode);
  d_g_rowptr = up32(fs.g_rowptr);
  d_g_col = up32(fs.g_col);
  d_c_rowptr = up32(fs.c_rowptr);
  d_c_col = up32(fs.c_col);
  d_b_rowptr = up32(fs.b_rowptr);
  d_b_col = up32(fs.b_col);
  d_dev_node = up32(fs.dev_node);
  d_node_ptr = up32(fs.node_ptr);
  d_node_code = up32(fs.node_code);
  // values in the new order
  auto gather = [](const double *v, const std::vector<int32_t> &src) {
    std::vector<double> out(src.size());
    for (size_t i = 0; i < src.size(); ++i) out[i] = v[src[i]];
    return out;
  };
  d_g_val = upd(gather(val.g_val, fs.g_src));
  d_c_val = upd(gather(val.c_val, fs.c_src));
  d_b_val = upd(gather(val.b_val, fs.b_src));
  std::vector<double> par(4 * (size_t)fs.n_dev);
  for (int k = 0; k < fs.n_dev; ++k) {
    par[4 * k] = val.kind[k];
    par[4 * k + 1] = val.kp[k] * val.wl[k];
    par[4 * k + 2] = val.vth[k];
    par[4 * k + 3] = val.lam[k];
  }
  d_par = upd(par);
  std::vector<int32_t> sp(val.n_src + 1, 0);
  std::vector<double> st, sv;
  for (int q = 0; q < val.n_src; ++q) {
    sp[q + 1] = sp[q] + val.npts[q];
    st.insert(st.end(), val.t[q], val.t[q] + val.npts[q]);
    sv.insert(sv.end(), val.v[q], val.v[q] + val.npts[q]);
    for (int i = 0; i < val.npts[q]; ++i)
      if (val.t[q][i] > 0 && val.t[q][i] < T) bps.push_back(val.t[q][i]);
  }
  std::sort(bps.begin(), bps.end());
  bps.erase(std::unique(bps.begin(), bps.end()), bps.end());
  bps.push_back(T);
  d_src_ptr = up32(sp);
  d_src_t = upd(st);
  d_src_v = upd(sv);
  std::vector<int32_t> pr(nprobe);
  for (int q = 0; q < nprobe; ++q) pr[q] = fs.iperm[probe[q]];
  d_probe = up32(pr);

  // work lists of every tree height: extend-add passes (one child per parent
  // and pass, 32 x 32 tiles of its Schur complement), panel fronts and
  // trailing-update tiles of each 32-wide pivot step
  const int H = (int)fs.lev_ptr.size() - 1;
  levels.resize(H);
  // fronts whose pivot blocks are inverted: the few large ones near the root,
  // whose one-workgroup triangular solves would otherwise set the solve time
  auto inverted = [&](int s_) { return fs.fsz[s_] > 64 && fs.nc[s_] > kInvPivots; };
  std::vector<int64_t> inv_off(fs.nc.size(), -1);
  int64_t inv_doubles = 0;
  for (size_t s_ = 0; s_ < fs.nc.size(); ++s_)
    if (inverted((int)s_)) {
      inv_off[s_] = inv_doubles;
      inv_doubles += ((int64_t)fs.nc[s_] * fs.nc[s_] + 31) / 32 * 32;
      max_p_inv = std::max(max_p_inv, fs.nc[s_]);
    }
  std::vector<int32_t> pool;
  std::vector<std::pair<size_t, int32_t **>> fix;
  for (int h = 0; h < H; ++h) {
    Level &L = levels[h];
    L.first = fs.lev_ptr[h];
    L.count = fs.lev_ptr[h + 1] - fs.lev_ptr[h];
    // fronts with f <= 64 are factored whole by one wave each (k_g_small_lu);
    // the pivot steps below are for the larger ones
    auto small_front = [&](int s_) { return fs.fsz[s_] <= 64; };
    int maxch = 0, maxnc = 0;
    for (int q = L.first; q < L.first + L.count; ++q) {
      const int s_ = fs.lev_front[q];
      maxch = std::max(maxch, fs.ch_ptr[s_ + 1] - fs.ch_ptr[s_]);
      if (!small_front(s_)) maxnc = std::max(maxnc, fs.nc[s_]);
    }
    // children with update matrices of at most 32 x 32 are added by one
    // workgroup per parent; the larger ones in passes of 32 x 32 tiles, the
    // pass-th large child of every parent in pass `pass`
    auto big_child = [&](int c) { return fs.fsz[c] - fs.nc[c] > 32; };
    {
      const size_t at = pool.size();
      for (int q = L.first; q < L.first + L.count; ++q) {
        const int s_ = fs.lev_front[q];
        bool any = false;
        for (int e = fs.ch_ptr[s_]; e < fs.ch_ptr[s_ + 1]; ++e) any = any || !big_child(fs.ch[e]);
        if (any) pool.push_back(s_);
      }
      L.n_small_parents = (int32_t)(pool.size() - at);
      fix.push_back({at, nullptr});
    }
    maxch = 0;
    for (int q = L.first; q < L.first + L.count; ++q) {
      const int s_ = fs.lev_front[q];
      int nb = 0;
      for (int e = fs.ch_ptr[s_]; e < fs.ch_ptr[s_ + 1]; ++e) nb += big_child(fs.ch[e]);
      maxch = std::max(maxch, nb);
    }
    L.extend.resize(maxch);
    for (int pass = 0; pass < maxch; ++pass) {
      const size_t at = pool.size();
      for (int q = L.first; q < L.first + L.count; ++q) {
        const int s_ = fs.lev_front[q];
        int c = -1;
        for (int e = fs.ch_ptr[s_], k = 0; e < fs.ch_ptr[s_ + 1]; ++e)
          if (big_child(fs.ch[e]) && k++ == pass) { c = fs.ch[e]; break; }
        if (c < 0) continue;
        const int r = fs.fsz[c] - fs.nc[c];
        const int nt = (r + 31) / 32;
        for (int tj = 0; tj < nt; ++tj)
          for (int ti = 0; ti < nt; ++ti) {
            pool.push_back(c);
            pool.push_back(ti | (tj << 16));
          }
      }
      L.extend[pass].first = (int32_t)((pool.size() - at) / 2);
      fix.push_back({at, &L.extend[pass].second});
    }
    // the solve's fronts: small ones (f <= 64, one wave each) and the rest
    // (one workgroup each for the pivot block, GEMV items for L21 / U12)
    {
      const size_t at_s = pool.size();
      for (int q = L.first; q < L.first + L.count; ++q)
        if (fs.fsz[fs.lev_front[q]] <= 64) pool.push_back(fs.lev_front[q]);
      L.n_small = (int32_t)(pool.size() - at_s);
      fix.push_back({at_s, nullptr});
      const size_t at_g = pool.size();
      for (int q = L.first; q < L.first + L.count; ++q)
        if (fs.fsz[fs.lev_front[q]] > 64) {
          pool.push_back(fs.lev_front[q]);
          L.big_maxp = std::max(L.big_maxp, fs.nc[fs.lev_front[q]]);
        }
      L.n_big = (int32_t)(pool.size() - at_g);
      fix.push_back({at_g, nullptr});
    }
    // solve GEMV items: (front, 64-row chunk) of L21 (forward) and of U12's
    // pivot rows (backward), large fronts with a non-empty update part only
    {
      const size_t at_f = pool.size();
      for (int q = L.first; q < L.first + L.count; ++q) {
        const int s_ = fs.lev_front[q];
        if (fs.fsz[s_] <= 64) continue;
        const int r = fs.fsz[s_] - fs.nc[s_];
        for (int c = 0; r > 0 && c < (r + 63) / 64; ++c) {
          pool.push_back(s_);
          pool.push_back(c);
        }
      }
      L.n_fwd = (int32_t)((pool.size() - at_f) / 2);
      fix.push_back({at_f, nullptr});
      const size_t at_b = pool.size();
      for (int q = L.first; q < L.first + L.count; ++q) {
        const int s_ = fs.lev_front[q];
        if (fs.fsz[s_] <= 64 || fs.fsz[s_] == fs.nc[s_]) continue;
        for (int c = 0; c < (fs.nc[s_] + 63) / 64; ++c) {
          pool.push_back(s_);
          pool.push_back(c);
        }
      }
      L.n_bwd = (int32_t)((pool.size() - at_b) / 2);
      fix.push_back({at_b, nullptr});
    }
    {
      const size_t at32 = pool.size();
      for (int q = L.first; q < L.first + L.count; ++q) {
        const int s_ = fs.lev_front[q];
        if (fs.nc[s_] > 0 && fs.fsz[s_] <= 32) pool.push_back(s_);
      }
      L.n_lu32 = (int32_t)(pool.size() - at32);
      fix.push_back({at32, nullptr});
      const size_t at64 = pool.size();
      for (int q = L.first; q < L.first + L.count; ++q) {
        const int s_ = fs.lev_front[q];
        if (fs.nc[s_] > 0 && fs.fsz[s_] > 32 && fs.fsz[s_] <= 64) pool.push_back(s_);
      }
      L.n_lu64 = (int32_t)(pool.size() - at64);
      fix.push_back({at64, nullptr});
    }
    {
      const size_t at_i = pool.size();
      for (int q = L.first; q < L.first + L.count; ++q) {
        const int s_ = fs.lev_front[q];
        if (!inverted(s_)) continue;
        for (int c = 0; c < (fs.nc[s_] + 63) / 64; ++c) {
          pool.push_back(s_);
          pool.push_back(c);
        }
      }
      L.n_trmv = (int32_t)((pool.size() - at_i) / 2);
      fix.push_back({at_i, nullptr});
    }
    // fronts whose trailing update of the previous step ran as tiles: tile
    // (0, 0) of that update has factored this step's diagonal block
    std::vector<char> tiled(fs.nc.size(), 0);
    for (int k0 = 0; k0 < maxnc; k0 += 32) {
      Step S{};
      S.k0 = k0;
      // panel chunk: the largest trailing size of the step, rounded to 8, at
      // most 128 (two chunks of rows and columns per 256 threads)
      int maxrem = 0;
      for (int q = L.first; q < L.first + L.count; ++q) {
        const int s_ = fs.lev_front[q];
        if (fs.nc[s_] > k0 && !small_front(s_))
          maxrem = std::max(maxrem, fs.fsz[s_] - k0 - std::min(32, fs.nc[s_] - k0));
      }
      S.chunk = std::min(128, std::max(8, (maxrem + 7) / 8 * 8));
      const size_t at_d = pool.size();
      for (int q = L.first; q < L.first + L.count; ++q)
        if (fs.nc[fs.lev_front[q]] > k0 && !tiled[fs.lev_front[q]] && !small_front(fs.lev_front[q]))
          pool.push_back(fs.lev_front[q]);
      S.n_diag = (int32_t)(pool.size() - at_d);
      fix.push_back({at_d, nullptr});
      const size_t at_p = pool.size();
      for (int q = L.first; q < L.first + L.count; ++q) {
        const int s_ = fs.lev_front[q];
        if (fs.nc[s_] <= k0 || small_front(s_)) continue;
        const int rem = fs.fsz[s_] - k0 - std::min(32, fs.nc[s_] - k0);
        const int nch = std::max(1, (rem + S.chunk - 1) / S.chunk);
        for (int c = 0; c < nch; ++c) {
          pool.push_back(s_);
          pool.push_back(c);
        }
      }
      S.n_panel = (int32_t)((pool.size() - at_p) / 2);
      const size_t at_t = pool.size();
      for (int q = L.first; q < L.first + L.count; ++q) {
        const int s_ = fs.lev_front[q];
        if (fs.nc[s_] <= k0 || small_front(s_)) continue;
        const int kb = std::min(32, fs.nc[s_] - k0), rem = fs.fsz[s_] - k0 - kb;
        tiled[s_] = 0;
        if (rem <= S.chunk && rem <= kFuse) continue;  // updated inside the panel kernel
        tiled[s_] = 1;
        const int nt = (rem + 63) / 64;
        for (int tj = 0; tj < nt; ++tj)
          for (int ti = 0; ti < nt; ++ti) {
            pool.push_back(s_);
            pool.push_back(ti | (tj << 16));
          }
      }
      S.n_tiles = (int32_t)((pool.size() - at_t) / 2);
      L.steps.push_back(S);
      fix.push_back({at_p, nullptr});
      fix.push_back({at_t, nullptr});
    }
  }
  // inversion items (front, 2 column block + which), the largest fronts first
  const size_t at_inv = pool.size();
  {
    std::vector<int32_t> inv_fronts;
    for (size_t s_ = 0; s_ < fs.nc.size(); ++s_)
      if (inv_off[s_] >= 0) inv_fronts.push_back((int32_t)s_);
    std::stable_sort(inv_fronts.begin(), inv_fronts.end(),
                     [&](int32_t a_, int32_t b_) { return fs.nc[a_] > fs.nc[b_]; });
    for (int32_t s_ : inv_fronts)
      for (int cb = 0; cb < (fs.nc[s_] + 31) / 32; ++cb)
        for (int u = 0; u < 2; ++u) {
          pool.push_back(s_);
          // the lower inverse's first column blocks and the upper's last ones
          // carry the longest recurrences: they go first
          pool.push_back(2 * (u == 0 ? cb : (fs.nc[s_] + 31) / 32 - 1 - cb) + u);
        }
    n_inv_items = (int32_t)((pool.size() - at_inv) / 2);
  }
  int32_t *d_pool = up32(pool);
  d_inv_off = up64(inv_off);
  if (!ok) return fail(kSENOMEM, "device allocation or upload failed (symbolic data)");
  d_inv_items = d_pool + at_inv;
  {
    size_t f = 0;
    for (int h = 0; h < H; ++h) {
      levels[h].small_parents = d_pool + fix[f++].first;
      for (auto &e : levels[h].extend) e.second = d_pool + fix[f++].first;
      levels[h].small = d_pool + fix[f++].first;
      levels[h].big = d_pool + fix[f++].first;
      levels[h].fwd = d_pool + fix[f++].first;
      levels[h].bwd = d_pool + fix[f++].first;
      levels[h].lu32 = d_pool + fix[f++].first;
      levels[h].lu64 = d_pool + fix[f++].first;
      levels[h].trmv = d_pool + fix[f++].first;
      for (auto &S : levels[h].steps) {
        S.diag = d_pool + fix[f++].first;
        S.panel = d_pool + fix[f++].first;
        S.tiles = d_pool + fix[f++].first;
      }
    }
  }
  // numeric buffers
  ldv = ((int64_t)n + 31) / 32 * 32;
  const int cols = o.m_max + 1;
  d_F = dalloc<double>(fs.front_doubles);
  d_upd = dalloc<double>(2 * fs.upd_doubles);  // update vectors of up to two right-hand sides
  d_Finv = dalloc<double>(std::max<int64_t>(inv_doubles, 1));
  d_tmp = dalloc<double>(2 * (size_t)n);        // pivot rows of inverted fronts, two right-hand sides
  d_rowmax = dalloc<unsigned long long>(n);
  d_bad = dalloc<int32_t>(1);
  // w and p side by side: they are solved together
  d_xk = dalloc<double>(n); d_x1 = dalloc<double>(n); d_w = dalloc<double>(2 * (size_t)n); d_p = d_w + n;
  d_z = dalloc<double>(n); d_r = dalloc<double>(n); d_bs = dalloc<double>(n); d_e = dalloc<double>(n);
  d_y = dalloc<double>(n);
  d_u = dalloc<double>(std::max(val.n_src, 1)); d_sl = dalloc<double>(std::max(val.n_src, 1));
  d_devI0 = dalloc<double>(fs.n_dev); d_devI1 = dalloc<double>(fs.n_dev); d_devD = dalloc<double>(3 * fs.n_dev);
  d_devD1 = dalloc<double>(3 * fs.n_dev);
  d_V = dalloc<double>(ldv * cols); d_Ve = dalloc<double>(ldv * cols);
  d_H = dalloc<double>(kHLd * kHLd); d_He = dalloc<double>(kHLd * kHLd);
  d_mat = dalloc<double>(5 * 64 * 65);
  d_part = dalloc<double>((size_t)kRBlocks * 64);
  d_h1 = dalloc<double>(kHLd); d_h2 = dalloc<double>(kHLd);
  d_out = dalloc<double>(kSc + 8); d_oute = dalloc<double>(kSc + 8);
  d_scm = d_out + kSc;
  d_sce = d_oute + kSc;
  d_red = dalloc<double>(8);
  d_feat = dalloc<float>(kFeat);
  d_cout = dalloc<float>(2);
  if (!d_feat || !d_cout || !d_F || !d_upd || !d_Finv || !d_tmp || !d_rowmax || !d_bad || !d_xk || !d_x1 || !d_w || !d_p || !d_z || !d_r || !d_bs || !d_e ||
      !d_y || !d_u || !d_sl || !d_devI0 || !d_devI1 || !d_devD || !d_devD1 || !d_V || !d_Ve || !d_H || !d_He || !d_mat ||
      !d_part || !d_h1 || !d_h2 || !d_out || !d_oute || !d_red)
    return fail(kSENOMEM, "device allocation failed (workspace)");
  GCHK(g_fill(d_H, kHLd * kHLd, 0.0, stream));
  GCHK(g_fill(d_He, kHLd * kHLd, 0.0, stream));
  GCHK(g_fill(d_out, kSc + 8, 0.0, stream));
  GCHK(g_fill(d_oute, kSc + 8, 0.0, stream));
  GCHK(hipStreamSynchronize(stream));
  return kSOK;
}

int GridEngine::read_scalars(const double *d, double *h, size_t count) {
  GCHK(hipMemcpyAsync(h, d, sizeof(double) * count, hipMemcpyDeviceToHost, stream));
  GCHK(hipStreamSynchronize(stream));
  return kSOK;
}

int GridEngine::factor_internal(const double *x) {
  const int n = fs.n;
  GCHK(g_stamp(fs.n_dev, d_dev_node, d_par, x, vdd, d_devI0, d_devD, stream));
  GCHK(g_fill(d_F, fs.front_doubles, 0.0, stream));
  GCHK(g_fill(reinterpret_cast<double *>(d_rowmax), n, 0.0, stream));
  GCHK(hipMemsetAsync(d_bad, 0, sizeof(int32_t), stream));
  GCHK(g_assemble((int)fs.ent_pos.size(), d_ent_pos, d_ent_row, d_ent_g, d_ent_jptr, d_ent_jcode, d_g_val, d_devD,
                  d_F, d_rowmax, stream));
  for (const Level &L : levels) {
    GCHK(g_extend_small(L.n_small_parents, L.small_parents, d_nc, d_fsz, d_f_off, d_ch_ptr, d_ch, d_r_ptr, d_rel, d_F,
                        stream));
    for (const auto &e : L.extend)
      GCHK(g_extend(e.first, e.second, d_nc, d_fsz, d_parent, d_f_off, d_r_ptr, d_rel, d_F, stream));
    GCHK(g_small_lu(L.n_lu32, L.lu32, L.n_lu64, L.lu64, d_c0, d_nc, d_fsz, d_f_off, d_rowmax, o.piv_tol, d_F, d_bad,
                    stream));
    for (const Step &S : L.steps) {
      GCHK(g_panel(S.n_diag, S.diag, S.n_panel, S.panel, S.k0, S.chunk, kFuse, d_c0, d_nc, d_fsz, d_f_off, d_rowmax,
                   o.piv_tol, d_F, d_bad, stream));
      GCHK(g_update(S.n_tiles, S.tiles, S.k0, d_c0, d_nc, d_fsz, d_f_off, d_rowmax, o.piv_tol, d_F, d_bad, stream));
    }
  }
  GCHK(g_inv(n_inv_items, d_inv_items, d_nc, d_fsz, d_f_off, d_inv_off, d_F, d_Finv, stream));
  int32_t bad = 0;
  GCHK(hipMemcpyAsync(&bad, d_bad, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
  GCHK(hipStreamSynchronize(stream));
  ++lu_count;
  factored = bad == 0;
  if (bad) return fail(kSESINGULAR, "singular pivot in LU(G_k) at row " + std::to_string(bad - 1));
  return kSOK;
}

int GridEngine::solve_internal(double *b, int nr) {
  // two right-hand sides (b and b + n) share the factor loads; their vectors
  // need 2 max(f) doubles of LDS in one workgroup
  if (nr == 2 && 2 * sizeof(double) * (size_t)std::max(fs.max_front, fs.max_nc) > 65536) {
    GRET(solve_internal(b, 1));
    return solve_internal(b + fs.n, 1);
  }
  for (const Level &L : levels)
    GCHK(g_fwd(L.n_small, L.small, L.n_big, L.big, L.n_fwd, L.fwd, fs.max_front, fs.max_nc, d_c0, d_nc, d_fsz,
               d_f_off, d_ch_ptr, d_ch, d_r_ptr, d_rel, d_u_off, d_F, b, nr, fs.n, d_upd, fs.upd_doubles,
               L.tri_bs(), L.n_trmv, L.trmv, max_p_inv, d_inv_off, d_Finv, d_tmp, stream));
  for (int h = (int)levels.size() - 1; h >= 0; --h) {
    const Level &L = levels[h];
    GCHK(g_bwd(L.n_small, L.small, L.n_big, L.big, L.n_bwd, L.bwd, fs.max_front, fs.max_nc, d_c0, d_nc, d_fsz,
               d_f_off, d_r_ptr, d_r_idx, d_F, b, nr, fs.n, L.tri_bs(), L.n_trmv, L.trmv, max_p_inv, d_inv_off,
               d_Finv, d_tmp, stream));
  }
  return kSOK;
}

int GridEngine::basis_start(Basis &B, const double *v) {
  const int n = fs.n;
  GCHK(g_dots(n, v, ldv, 1, v, d_part, B.sc + 1, stream));
  GCHK(g_start(n, v, B.sc, B.V, stream));
  double beta = 0.0;
  GRET(read_scalars(B.sc, &beta, 1));
  B.m = 0;
  B.exact = beta == 0.0;
  if (!std::isfinite(beta)) return fail(kSENONFINITE, "non-finite Krylov start vector");
  return kSOK;
}

// one Arnoldi step (Algorithm 1): w = -G^{-1} C v_j, two passes of classical
// Gram-Schmidt against v_1..v_j, h_{j+1,j} = ||w||, v_{j+1} = w / h_{j+1,j}
int GridEngine::arnoldi_step(Basis &B) {
  const int n = fs.n, j = B.m;
  const double *vj = B.V + (int64_t)j * ldv;
  GCHK(g_spmv(n, d_c_rowptr, d_c_col, d_c_val, vj, -1.0, d_w, stream));
  GRET(solve_internal(d_w));
  GCHK(g_dots(n, B.V, ldv, j + 1, d_w, d_part, d_h1, stream));
  GCHK(g_gemv_sub(n, B.V, ldv, j + 1, d_h1, d_w, stream));
  GCHK(g_dots(n, B.V, ldv, j + 1, d_w, d_part, d_h2, stream));
  GCHK(g_gemv_sub(n, B.V, ldv, j + 1, d_h2, d_w, stream));
  GCHK(g_dots(n, d_w, ldv, 1, d_w, d_part, B.sc + 1, stream));
  GCHK(g_hcol(j, d_h1, d_h2, B.H, o.breakdown, B.sc, stream));
  GCHK(g_scale(n, d_w, B.sc, 3, B.V + (int64_t)(j + 1) * ldv, stream));
  B.m = j + 1;
  ++arnoldi;
  mgs_terms += 2 * (j + 1);
  return kSOK;
}

// grow the basis until rho_m(h) <= eps (Algorithm 1's residual test from
// m_first on); d stays in B.out
int GridEngine::converge(Basis &B, double h, double eps, double *rho, int want2, int m_first) {
  if (B.exact && B.m == 0) {  // zero start vector
    *rho = 0.0;
    return kSOK;
  }
  for (int it = 0;; ++it) {
    if (B.m > 0 && (B.m >= m_first || B.exact)) {
      GCHK(launch_hess_phi1(B.H, B.m, h, B.sc, want2, d_mat, B.out, stream));
      double got[4];  // rho, then (at kSc) beta, ||w||^2, breakdown
      GCHK(hipMemcpyAsync(got, B.out + 2 * kHLd, sizeof(double), hipMemcpyDeviceToHost, stream));
      GCHK(hipMemcpyAsync(got + 1, B.sc, 3 * sizeof(double), hipMemcpyDeviceToHost, stream));
      GCHK(hipStreamSynchronize(stream));
      *rho = got[0];
      if (got[3] != 0.0) B.exact = true;
      if (*rho <= eps) return kSOK;
      if (B.exact) return fail(kSEKRYLOV, "invariant subspace with a non-finite exponential");
    }
    if (B.m >= o.m_max) return fail(kSEKRYLOV, "Krylov residual not reached at m_max");
    GRET(arnoldi_step(B));
    if (B.m < m_first) {
      double flag = 0.0;
      GRET(read_scalars(B.sc + 2, &flag, 1));
      if (flag != 0.0) B.exact = true;
    }
  }
}

int GridEngine::factor(const double *x_caller) {
  GCHK(g_gather(fs.n, d_perm, x_caller, d_xk, stream));
  lu_count = 0;
  return factor_internal(d_xk);
}

int GridEngine::solve(const double *b_caller, double *y_caller) {
  if (!factored) return fail(kSEINVAL, "solve: no factors (call expri_factor)");
  GCHK(g_gather(fs.n, d_perm, b_caller, d_y, stream));
  GRET(solve_internal(d_y));
  GCHK(g_scatter(fs.n, d_perm, d_y, y_caller, stream));
  GCHK(hipStreamSynchronize(stream));
  return kSOK;
}

int GridEngine::mevp(const double *v_caller, double *out_caller, double h, double eps, int32_t *m, double *rho) {
  if (!factored) return fail(kSEINVAL, "mevp: no factors (call expri_factor)");
  const int n = fs.n;
  arnoldi = 0;
  GCHK(g_gather(n, d_perm, v_caller, d_z, stream));
  Basis B{d_V, d_H, d_scm, d_out, 0, false};
  GRET(basis_start(B, d_z));
  double r = 0.0;
  GRET(converge(B, h, eps, &r, 0, 1));
  GCHK(g_combine(n, nullptr, nullptr, 0.0, B.V, ldv, B.m, B.sc, B.out, d_y, stream));
  GCHK(g_scatter(n, d_perm, d_y, out_caller, stream));
  GCHK(hipStreamSynchronize(stream));
  if (m) *m = B.m;
  if (rho) *rho = r;
  return kSOK;
}

int GridEngine::dc(double *x_caller, double t0) {
  const int n = fs.n;
  lu_count = 0;
  steps = 0;
  GCHK(g_gather(n, d_perm, x_caller, d_xk, stream));
  GCHK(g_sources(fs.n_src, d_src_ptr, d_src_t, d_src_v, t0, t0, d_u, d_sl, stream));
  for (int it = 0; it < 200; ++it) {
    GRET(factor_internal(d_xk));
    GCHK(g_rhs(n, d_g_rowptr, d_g_col, d_g_val, d_b_rowptr, d_b_col, d_b_val, d_node_ptr, d_node_code, d_devI0, d_xk,
               d_u, d_sl, d_r, d_bs, stream));
    GRET(solve_internal(d_r));
    GCHK(g_absmax(n, d_r, d_part, d_red, stream));
    double big = 0.0;
    GRET(read_scalars(d_red, &big, 1));
    if (!std::isfinite(big)) return fail(kSENONFINITE, "DC: non-finite Newton update");
    GCHK(g_axpy(n, big > 0.3 ? 0.3 / big : 1.0, d_r, d_xk, stream));
    steps = it + 1;
    if (big <= 1e-12) {
      GCHK(g_scatter(n, d_perm, d_xk, x_caller, stream));
      GCHK(hipStreamSynchronize(stream));
      t_reached = t0;
      return kSOK;
    }
  }
  return fail(kSENOCONV, "DC Newton did not converge");
}

int GridEngine::run(double *x_caller, double t0, const double *grid, int32_t n_grid, int32_t max_steps,
                    double E_rr, double eps_K, double h0, GridStepRec *last) {
  const int n = fs.n;
  const bool replay = grid != nullptr;
  const bool has_dev = fs.n_dev > 0;
  lu_count = arnoldi = trials = mgs_terms = comb_terms = rejects = 0;
  steps = 0;
  trace.clear();
  const int rec = kRecFixed + n_probe;
  hipEvent_t e0, e1;
  GCHK(hipEventCreate(&e0));
  GCHK(hipEventCreate(&e1));
  struct EvGuard {
    hipEvent_t a, b;
    ~EvGuard() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } guard{e0, e1};
  GCHK(hipEventRecord(e0, stream));
  GCHK(g_gather(n, d_perm, x_caller, d_xk, stream));
  double t = t0, h_prop = std::min(h0, h_max);
  // the learned controller proposes (m, h) from features of the step; the
  // error test still judges every trial (as in the transient kernel)
  const bool learned = ctrl_w != nullptr && !replay;
  double h_prev = h_prop, rho_prev = 0.0, err_prev = 0.0;
  int m_prev = 0, rej_prev = 0, m_err_prev = 0;
  size_t bp_idx = 0;
  while (bp_idx + 1 < bps.size() && bps[bp_idx] <= t0) ++bp_idx;
  bool lu_valid = false;
  std::vector<double> probes(n_probe);
  int status = kSOK;
  for (;;) {
    if (replay ? steps >= n_grid : !(t < T)) break;
    if (steps >= max_steps) break;
    double h_try, t_land, h_unc;
    bool land;
    if (replay) {
      t_land = grid[steps];
      h_try = h_unc = t_land - t;
      land = true;
    } else {
      t_land = bps[bp_idx];
      h_try = h_unc = std::min(h_prop, h_max);
      land = false;
      if (t + h_try * (1.0 + 1e-3) >= t_land) {
        h_try = t_land - t;
        land = true;
      }
    }
    // stamp and factor G_k at x_k (a linear circuit keeps its factors)
    if (has_dev || !lu_valid) {
      if ((status = factor_internal(d_xk)) != kSOK) break;
      lu_valid = true;
    } else {
      GCHK(g_stamp(fs.n_dev, d_dev_node, d_par, d_xk, vdd, d_devI0, d_devD, stream));
    }
    // step features (recorded in every mode, the learned controller's input):
    // log ||r_k||, m_{k-1} / 60, log h_{k-1}, log rho_{k-1}, log(1 + max |du/dt|
    // 1 ns) at the middle of the segment, log ||F_k(x_k)||, log(e_{k-1} / E_rr),
    // rejections of step k - 1
    double feat[kFeat] = {0, 0, 0, 0, 0, 0, 0, 0};
    int m_first = 1;
    if (!replay) {
      const double ts = t + 0.5 * (learned ? bps[bp_idx] - t : h_try);
      GCHK(g_sources(fs.n_src, d_src_ptr, d_src_t, d_src_v, t, ts, d_u, d_sl, stream));
      GCHK(g_rhs(n, d_g_rowptr, d_g_col, d_g_val, d_b_rowptr, d_b_col, d_b_val, d_node_ptr, d_node_code, d_devI0,
                 d_xk, d_u, d_sl, d_w, d_p, stream));
      GCHK(g_absmax(n, d_w, d_part, d_red, stream));
      GCHK(g_fk(n, d_node_ptr, d_node_code, d_dev_node, d_devD, d_devI0, d_xk, d_e, stream));
      GCHK(g_absmax(n, d_e, d_part, d_red + 1, stream));
      if (fs.n_src > 0) GCHK(g_absmax(fs.n_src, d_sl, d_part, d_red + 2, stream));
      else GCHK(g_fill(d_red + 2, 1, 0.0, stream));
      double nr[3];
      GRET(read_scalars(d_red, nr, 3));
      feat[0] = std::log10(std::max(nr[0], 1e-30));
      feat[1] = m_prev / 60.0;
      feat[2] = std::log10(h_prev);
      feat[3] = std::log10(std::max(rho_prev, 1e-30));
      feat[4] = std::log10(1.0 + nr[2] * 1e-9);
      feat[5] = std::log10(std::max(nr[1], 1e-30));
      feat[6] = std::log10(std::max(err_prev / E_rr, 1e-30));
      feat[7] = rej_prev;
      if (learned) {
        float ff[kFeat], out[2];
        for (int i = 0; i < kFeat; ++i) ff[i] = (float)feat[i];
        GCHK(hipMemcpyAsync(d_feat, ff, sizeof(ff), hipMemcpyHostToDevice, stream));
        GCHK(g_ctrl(ctrl_w, ctrl_norm, d_feat, d_cout, stream));
        GCHK(hipMemcpyAsync(out, d_cout, sizeof(out), hipMemcpyDeviceToHost, stream));
        GCHK(hipStreamSynchronize(stream));
        // the first residual test at m - 1; the step within alpha .. beta of
        // the previous accepted one, stretched by up to 25 % to land on a
        // source corner or split into halves before one
        m_first = (int)std::min(std::max(std::rint((double)out[0]) - 1.0, 1.0), (double)o.m_max);
        double hl = ctrl_safety * std::pow(10.0, (double)out[1]);
        if (!(hl == hl)) hl = h_prev;
        hl = std::min(std::max(hl, o.alpha * h_prev), o.beta * h_prev);
        t_land = bps[bp_idx];
        h_try = h_unc = std::min(hl, h_max);
        land = false;
        if (t + h_try * 1.25 >= t_land) {
          h_try = t_land - t;
          land = true;
        } else if (t + 2.0 * h_try > t_land) {
          h_try = 0.5 * (t_land - t);
        }
      }
    }
    // w = G^{-1} r, p = G^{-1} B s, z = G^{-1} C p, v = w - z
    GCHK(g_sources(fs.n_src, d_src_ptr, d_src_t, d_src_v, t, t + 0.5 * h_try, d_u, d_sl, stream));
    GCHK(g_rhs(n, d_g_rowptr, d_g_col, d_g_val, d_b_rowptr, d_b_col, d_b_val, d_node_ptr, d_node_code, d_devI0, d_xk,
               d_u, d_sl, d_w, d_p, stream));
    GRET(solve_internal(d_w, 2));  // w and p (d_p = d_w + n)
    GCHK(g_spmv(n, d_c_rowptr, d_c_col, d_c_val, d_p, 1.0, d_z, stream));
    GRET(solve_internal(d_z));
    GCHK(g_sub(n, d_w, d_z, d_r, stream));
    Basis Bm{d_V, d_H, d_scm, d_out, 0, false};
    if ((status = basis_start(Bm, d_r)) != kSOK) break;
    double h = h_try, rho = 0.0, errv = 0.0;
    int rej = 0, m_err = 0;
    bool fell_back = false;
    // a learned proposal whose MEVP misses eps_K at m_max restarts once from
    // the paper's proposal (the basis is kept)
    auto fall_back = [&]() {
      fell_back = true;
      double hp = std::min(h_prop, h_max);
      h_unc = hp;
      t_land = bps[bp_idx];
      land = false;
      if (t + hp * (1.0 + 1e-3) >= t_land) {
        hp = t_land - t;
        land = true;
      }
      h = h_try = hp;
      rej = 0;
      status = kSOK;
    };
    for (;;) {
      ++trials;
      status = converge(Bm, h, eps_K, &rho, 0, rej == 0 ? m_first : 1);
      if (status == kSEKRYLOV && learned && !fell_back) {
        fall_back();
        continue;
      }
      if (status != kSOK) break;
      GCHK(g_combine(n, d_xk, d_p, h, Bm.V, ldv, Bm.m, Bm.sc, Bm.out, d_x1, stream));
      comb_terms += Bm.m;
      errv = 0.0;
      m_err = 0;
      if (has_dev) {
        // e_rr = (I - e^{hJ}) G_k^{-1} dF on its own invert Krylov basis
        GCHK(g_stamp(fs.n_dev, d_dev_node, d_par, d_x1, vdd, d_devI1, d_devD1, stream));
        GCHK(g_dF(n, d_node_ptr, d_node_code, d_dev_node, d_devD, d_devI0, d_devI1, d_xk, d_x1, d_e, stream));
        GRET(solve_internal(d_e));
        Basis Be{d_Ve, d_He, d_sce, d_oute, 0, false};
        double rho_e = 0.0;
        if ((status = basis_start(Be, d_e)) != kSOK) break;
        status = converge(Be, h, eps_K, &rho_e, 0, learned ? std::max(1, m_err_prev - 2) : 1);
        if (status == kSEKRYLOV && learned && !fell_back) {
          fall_back();
          continue;
        }
        if (status != kSOK) break;
        m_err = Be.m;
        GCHK(g_combine(n, nullptr, nullptr, 0.0, Be.V, ldv, Be.m, Be.sc, Be.out, d_e, stream));
        comb_terms += Be.m;
        GCHK(g_absmax(n, d_e, d_part, d_red, stream));
        GRET(read_scalars(d_red, &errv, 1));
        if (!std::isfinite(errv)) {
          status = fail(kSENONFINITE, "non-finite error estimate");
          break;
        }
      }
      if (replay || errv <= E_rr) break;
      ++rej;
      h *= o.alpha;
      if (h < o.h_min) {
        status = fail(kSESTEPMIN, "step below h_min");
        break;
      }
    }
    if (status != kSOK) break;
    // accept
    const double t_new = (land && rej == 0) ? t_land : t + h;
    GCHK(hipMemcpyAsync(d_xk, d_x1, sizeof(double) * n, hipMemcpyDeviceToDevice, stream));
    if (n_probe > 0) {
      GCHK(g_gather(n_probe, d_probe, d_x1, d_y, stream));
      GRET(read_scalars(d_y, probes.data(), n_probe));
    }
    const size_t base = trace.size();
    trace.resize(base + rec, 0.0);
    double *r = trace.data() + base;
    r[0] = t_new; r[1] = h; r[2] = h_unc; r[3] = Bm.m; r[4] = m_err; r[5] = rej; r[6] = errv; r[7] = rho;
    for (int i = 0; i < kFeat; ++i) r[8 + i] = feat[i];
    for (int q = 0; q < n_probe; ++q) r[kRecFixed + q] = probes[q];
    h_prev = (land && rej == 0) ? h_unc : h;
    rho_prev = rho;
    err_prev = errv;
    m_prev = Bm.m;
    rej_prev = rej;
    m_err_prev = m_err;
    if (last) *last = GridStepRec{t_new, h, h_unc, errv, rho, Bm.m, m_err, rej};
    const double grow = rej < o.grow_if_rejects_lt ? o.beta : 1.0;
    h_prop = std::min(h_max, grow * (rej == 0 ? h_prop : h));
    t = t_new;
    if (!replay)
      while (bp_idx + 1 < bps.size() && bps[bp_idx] <= t) ++bp_idx;
    rejects += rej;
    ++steps;
  }
  t_reached = t;
  next_h = h_prop;
  GCHK(g_scatter(n, d_perm, d_xk, x_caller, stream));
  GCHK(hipEventRecord(e1, stream));
  GCHK(hipStreamSynchronize(stream));
  float ms = 0.0f;
  GCHK(hipEventElapsedTime(&ms, e0, e1));
  kernel_s = 1e-3 * ms;
  return status;
}

int GridEngine::diag(int what, int reps, double *sec) {
  if (!factored && what == 0) return fail(kSEINVAL, "diag: no factors");
  hipEvent_t e0, e1;
  GCHK(hipEventCreate(&e0));
  GCHK(hipEventCreate(&e1));
  GCHK(g_fill(d_y, fs.n, 1.0, stream));
  GCHK(hipEventRecord(e0, stream));
  for (int r = 0; r < reps; ++r) {
    if (what == 0) {  // a fresh right-hand side each time (repeated solves would overflow)
      GCHK(g_fill(d_y, fs.n, 1.0, stream));
      GRET(solve_internal(d_y));
    }
    else if (what == 7) GRET(factor_internal(d_xk));
    else if (what == 2) GCHK(g_spmv(fs.n, d_c_rowptr, d_c_col, d_c_val, d_y, 1.0, d_z, stream));
    else return fail(kSEINVAL, "diag: unknown building block");
  }
  GCHK(hipEventRecord(e1, stream));
  GCHK(hipStreamSynchronize(stream));
  float ms = 0.0f;
  GCHK(hipEventElapsedTime(&ms, e0, e1));
  *sec = 1e-3 * ms / std::max(reps, 1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return kSOK;
}

}  // namespace expri
