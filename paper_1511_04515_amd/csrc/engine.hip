// gfx950 kernels of the exponential Rosenbrock-Euler (ER) solver with the
// invert-Krylov MEVP (Zhuang et al., DAC 2015: Algorithm 1 MEVP_IKS inside
// Algorithm 2 ER).
//
// Execution model: one workgroup owns one circuit instance and runs the whole
// step on the device -- device stamp, numeric LU of G_k, the three right-hand
// sides, Arnoldi with modified Gram-Schmidt, the small Hessenberg exponential
// with its residual test, the update, the error MEVP and the accept / reject
// decision -- with no host round trip.  Many instances (a batch) are many
// workgroups of one launch.  Inside a workgroup:
//   * vector work is element-strided over the threads (coalesced);
//   * triangular solves and the refactor are level scheduled (one barrier per
//     level) with the solution vector resident in LDS;
//   * reductions are wave butterflies plus one LDS exchange, and every thread
//     ends with the bit-identical value, so control flow stays uniform;
//   * the (m+1) x (m+1) matrices of the Hessenberg exponential live in LDS
//     (reusing the solve vector's space) or, when too large, in global scratch.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "devcommon.hpp"
#include "layout.hpp"
#include "mosfet.hpp"
#include "mlp.hpp"

namespace expri {

// LDS scratch layout (dynamic shared memory):
//   region : R doubles  -- solve vector, or small dense matrices
//   slots  : 2 * NW doubles -- reduction exchange (double buffered)
//   dmain, derr : kHLd doubles each -- small vectors d of the two MEVPs
//   4 doubles unused
//   prof, hcol, derr2
template <int BS>
struct Lds {
  double *region;  // vector area: solve vector / current Arnoldi basis vector
  double *dense;   // small dense matrices of the Hessenberg exponential
  double *slots;
  double *dmain;
  double *derr;

  double *hcol; // kHLd doubles: current Hessenberg column
  double *derr2;  // kHLd doubles: ER-C coefficients on the error basis
  long long *prof;  // kPhases phase counters
  int R;   // region + dense, doubles
  int RD;  // dense, doubles
  int par;
};

template <int BS>
__device__ __forceinline__ double wg_sum(Lds<BS> &L, double v) {
  v = wave_sum(v);
  double *s = L.slots + L.par * (BS / 64);
  if ((tid() & 63) == 0) s[tid() >> 6] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int i = 0; i < BS / 64; ++i) r += s[i];
  L.par ^= 1;
  return r;
}

template <int BS>
__device__ __forceinline__ double wg_max(Lds<BS> &L, double v) {
  v = wave_max(v);
  double *s = L.slots + L.par * (BS / 64);
  if ((tid() & 63) == 0) s[tid() >> 6] = v;
  __syncthreads();
  double r = s[0];
#pragma unroll
  for (int i = 1; i < BS / 64; ++i) r = nmax(r, s[i]);
  L.par ^= 1;
  return r;
}

// the first thread's v, to every thread of the workgroup
template <int BS>
__device__ __forceinline__ double wg_bcast0(Lds<BS> &L, double v) {
  double *s = L.slots + L.par * (BS / 64);
  if (tid() == 0) s[0] = v;
  __syncthreads();
  const double r = s[0];
  L.par ^= 1;
  return r;
}

// Per-phase wall-clock accounting (every thread keeps the same counters; the
// first thread stores them).  Phases: 0 stamp + factor, 1 right-hand sides,
// 2 Arnoldi SpMV + solve, 3 modified Gram-Schmidt, 4 Hessenberg exponential,
// 5 trial update, device re-stamp and error-estimate set-up.
struct Prof {
  long long *acc;  // kPhases counters in LDS, updated by the first thread
  long long last;
  __device__ __forceinline__ void start(long long *lds) {
    acc = lds;
    if (tid() < kPhases) acc[tid()] = 0;
    last = wall_clock64();
  }
  __device__ __forceinline__ void mark(int p) {
    const long long now = wall_clock64();
    if (tid() == 0) acc[p] += now - last;
    last = now;
  }
};


__device__ __forceinline__ double node_v(const double *x, int node, double vdd) {
  return node >= 0 ? x[node] : (node == -2 ? vdd : 0.0);
}

// ---------------------------------------------------------------------------
// piecewise-linear sources
// ---------------------------------------------------------------------------

__device__ __forceinline__ int pwl_seg(const double *T, int lo, int hi, double t) {
  // largest i in [lo, hi) with T[i] <= t   (requires T[lo] <= t < T[hi])
  int a = lo, b = hi;
  while (b - a > 1) {
    const int mid = (a + b) >> 1;
    if (T[mid] <= t) a = mid; else b = mid;
  }
  return a;
}

__device__ __forceinline__ double pwl_value(const InstDesc &D, int src, double t) {
  const int lo = gbl(D.src_ptr)[src], hi = gbl(D.src_ptr)[src + 1] - 1;
  if (t <= gbl(D.src_t)[lo]) return gbl(D.src_v)[lo];
  if (t >= gbl(D.src_t)[hi]) return gbl(D.src_v)[hi];
  const int i = pwl_seg(D.src_t, lo, hi, t);
  const double slope = (D.src_v[i + 1] - gbl(D.src_v)[i]) / (D.src_t[i + 1] - gbl(D.src_t)[i]);
  return gbl(D.src_v)[i] + (t - gbl(D.src_t)[i]) * slope;
}

__device__ __forceinline__ double pwl_slope(const InstDesc &D, int src, double tm) {
  const int lo = gbl(D.src_ptr)[src], hi = gbl(D.src_ptr)[src + 1] - 1;
  if (hi <= lo || tm < gbl(D.src_t)[lo] || tm >= gbl(D.src_t)[hi]) return 0.0;
  const int i = pwl_seg(D.src_t, lo, hi, tm);
  return (D.src_v[i + 1] - gbl(D.src_v)[i]) / (D.src_t[i + 1] - gbl(D.src_t)[i]);
}

// ---------------------------------------------------------------------------
// device stamp and G_k assembly
// ---------------------------------------------------------------------------

template <int BS>
__device__ __forceinline__ void stamp_devices(const InstDesc &D, const double *x, double *devI, double *devD) {
  for (int k = tid(); k < D.n_dev; k += BS) {
    const int nd = gbl(D.dev_node)[3 * k], ng = gbl(D.dev_node)[3 * k + 1], ns = gbl(D.dev_node)[3 * k + 2];
    const GMEM double *par = gbl(D.dev_par) + 4 * k;
    double I, dd, dg, ds;
    mos_eval(par[0], node_v(x, nd, D.vdd), node_v(x, ng, D.vdd), node_v(x, ns, D.vdd), par[1],
             par[2], par[3], I, dd, dg, ds);
    devI[k] = I;
    if (devD) {
      devD[3 * k] = dd;
      devD[3 * k + 1] = dg;
      devD[3 * k + 2] = ds;
    }
  }
}

// lu <- G_lin + J_dev (drop the derivative couplings between DC blocks when
// dc_block is set) ;  Ik <- I_dev(x) per node.  G_lin comes pre-scattered to
// the L\U positions (a coalesced copy); the few positions with device terms
// are then rewritten with their sums.
template <int BS>
__device__ __forceinline__ void assemble(const InstDesc &D, bool dc_block) {
  const GMEM double *__restrict__ glu = gbl(D.g_lu);
  GMEM double *__restrict__ lu = gbl(D.lu);
  const int nz = D.nnz_lu;
  // loads at clamped indices, unconditionally: a branch around each load
  // would make the compiler wait for every load in flight at each join
  for (int p0 = tid(); p0 < nz; p0 += 8 * BS) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = glu[min(p0 + u * BS, nz - 1)];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (p0 + u * BS < nz) lu[p0 + u * BS] = v[u];
  }
  __syncthreads();
  const GMEM int *__restrict__ jpos = gbl(D.jpos), *__restrict__ jptr = gbl(D.jac_ptr), *__restrict__ jcode = gbl(D.jac_code);
  const GMEM double *__restrict__ devD = gbl(D.devD);
  for (int q = tid(); q < D.n_jpos; q += BS) {
    const int p = jpos[q];
    double v = glu[p];
    for (int c = jptr[p]; c < jptr[p + 1]; ++c) {
      const int code = jcode[c];
      if (dc_block && ((code >> 3) & 1)) continue;
      const double dv = devD[3 * (code >> 4) + (code & 3)];
      v += ((code >> 2) & 1) ? -dv : dv;
    }
    lu[p] = v;
  }
  for (int i = tid(); i < D.n; i += BS) {
    double s = 0.0;
    for (int c = gbl(D.node_ptr)[i]; c < gbl(D.node_ptr)[i + 1]; ++c) {
      const int code = gbl(D.node_code)[c];
      const double Iv = gbl(D.devI)[code >> 1];
      s += (code & 1) ? -Iv : Iv;
    }
    gbl(D.Ik)[i] = s;
  }
}

// Slot-ordered copy of the factors for the solves: sval[k] is the L\U value
// of slot k of the flattened schedules (0 on padding) and rdv[r] the
// reciprocal 1 / u_ii of the pivot of the row in row slot r of the U passes
// (1 where the slot holds no row), so that the U passes multiply.  A solve
// pass then reads its operands with coalesced loads that depend on nothing
// the solve computes, so they can be issued a pass ahead.
template <int BS>
__device__ __forceinline__ void pack_slots(const InstDesc &D) {
  const GMEM double *__restrict__ a = gbl(D.lu);
  GMEM double *__restrict__ sv = gbl(D.sval);
  GMEM double *__restrict__ rdv = gbl(D.rdv);
  // only the slots that hold an entry (the others keep their 0), eight at a
  // time with their loads issued together at clamped indices
  const GMEM int *__restrict__ ks = gbl(D.pk_slot), *__restrict__ kp = gbl(D.pk_pos);
  const int np = D.n_pk;
  for (int k0 = tid(); k0 < np; k0 += 8 * BS) {
    int s8[8], p8[8];
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = min(k0 + u * BS, np - 1);
      s8[u] = ks[k];
      p8[u] = kp[k];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = a[p8[u]];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (k0 + u * BS < np) sv[s8[u]] = v[u];
  }
  const GMEM int *__restrict__ rs = gbl(D.rd_slot), *__restrict__ rp = gbl(D.rd_pos);
  const int nr = D.n_rd;
  for (int k0 = tid(); k0 < nr; k0 += 8 * BS) {
    int s8[8], p8[8];
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = min(k0 + u * BS, nr - 1);
      s8[u] = rs[k];
      p8[u] = rp[k];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = a[p8[u]];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (k0 + u * BS < nr) rdv[s8[u]] = 1.0 / v[u];
  }
  __syncthreads();
}

// numeric refactor of the L\U storage (row-wise Doolittle, static pivots).
// Returns false when a pivot is small: |u_ii| <= piv_tol * max_j |G_k(i, j)|.
// Row i of a level takes its pivot groups in order: l_ik = a_ik / u_kk, then
// a_ij -= l_ik u_kj over the group's update pairs.  Wide levels run one row
// per thread.  Narrow levels (the separators at the top of the ordering,
// where the rows are long and the group chains deep) run one row per wave:
// the row is staged in LDS, the pivots u_kk and the u_kj of up to 64 pairs
// are loaded by the lanes at once (rows k are final), and only the chain
// over the groups is sequential, in LDS.  The update order of every entry is
// the same in both forms.
template <int BS>
__device__ __forceinline__ void refactor_row_wave(GMEM double *a, const GMEM int *rowptr, const GMEM int *row_grp,
                                                  const GMEM int *grp_pos, const GMEM int *grp_diag,
                                                  const GMEM int *grp_ptr, const GMEM int *pair_dst,
                                                  const GMEM int *pair_src, int i, int diag_i, double *rb,
                                                  double piv_tol, int lane, int &bad) {
  const int rs = rowptr[i], len = rowptr[i + 1] - rs;
  double rmx = 0.0;
  for (int q = lane; q < len; q += 64) {
    const double v = a[rs + q];
    rb[q] = v;
    rmx = fmax(rmx, fabs(v));
  }
  rmx = wave_max(rmx);
  const int g0 = row_grp[i], ng = row_grp[i + 1] - g0;
  const int p0 = grp_ptr[g0], np = grp_ptr[g0 + ng] - p0;
  wfence();
  if (ng <= 64 && np <= 64) {
    int goff = 0, glo = 0, ghi = 0, pd = 0;
    double gdg = 1.0, ps = 0.0;
    if (lane < ng) {
      goff = grp_pos[g0 + lane] - rs;
      gdg = a[grp_diag[g0 + lane]];
      glo = grp_ptr[g0 + lane] - p0;
      ghi = grp_ptr[g0 + lane + 1] - p0;
    }
    if (lane < np) {
      pd = pair_dst[p0 + lane] - rs;
      ps = a[pair_src[p0 + lane]];
    }
    for (int g = 0; g < ng; ++g) {
      const int off = __builtin_amdgcn_readlane(goff, g);
      const int lo = __builtin_amdgcn_readlane(glo, g), hi = __builtin_amdgcn_readlane(ghi, g);
      const double l = rb[off] / readlane_d(gdg, g);
      wfence();
      if (lane == 0) rb[off] = l;
      if (lane >= lo && lane < hi) rb[pd] -= l * ps;
      wfence();
    }
  } else {
    for (int g = 0; g < ng; ++g) {
      const int off = grp_pos[g0 + g] - rs;
      const double l = rb[off] / a[grp_diag[g0 + g]];
      wfence();
      if (lane == 0) rb[off] = l;
      for (int u = grp_ptr[g0 + g] + lane; u < grp_ptr[g0 + g + 1]; u += 64)
        rb[pair_dst[u] - rs] -= l * a[pair_src[u]];
      wfence();
    }
  }
  for (int q = lane; q < len; q += 64) a[rs + q] = rb[q];
  if (lane == 0 && !(fabs(rb[diag_i - rs]) > piv_tol * rmx)) bad = 1;
}

// Levels of at most this many rows per wave run one row per wave (the
// separators near the root, where the rows are long and the group chains
// deep); wider levels run one row per thread.  (16 rows per wave, and groups
// of 2 to 8 lanes per row for the wider levels, measured slower on the
// chains.)
constexpr int kWaveRowLevels = 4;
template <int BS>
__device__ __forceinline__ bool refactor(const InstDesc &D, Lds<BS> &L, double piv_tol, int max_levels = 1 << 30) {
  GMEM double *a = gbl(D.lu);
  const GMEM int *lev_ptr = gbl(D.lev_ptr), *lev_rows = gbl(D.lev_rows), *rowptr = gbl(D.lu_rowptr);
  const GMEM int *row_grp = gbl(D.row_grp), *grp_pos = gbl(D.grp_pos), *grp_diag = gbl(D.grp_diag);
  const GMEM int *grp_ptr = gbl(D.grp_ptr), *pair_dst = gbl(D.pair_dst), *pair_src = gbl(D.pair_src);
  const GMEM int *diag = gbl(D.lu_diag);
  constexpr int NW = BS / 64;
  const int t = tid(), lane = t & 63, wave = t >> 6;
  // per-wave row buffers in the LDS vector area (free while G_k is refactored)
  const bool wave_rows_fit = NW * D.max_row <= L.R;
  int bad = 0;
  for (int lv = 0; lv < min(D.n_lev, max_levels); ++lv) {
    const int q0 = lev_ptr[lv], q1 = lev_ptr[lv + 1];
    if (wave_rows_fit && q1 - q0 <= kWaveRowLevels * NW) {
      for (int q = q0 + wave; q < q1; q += NW) {
        const int i = lev_rows[q];
        refactor_row_wave<BS>(a, rowptr, row_grp, grp_pos, grp_diag, grp_ptr, pair_dst, pair_src, i, diag[i],
                              L.region + wave * D.max_row, piv_tol, lane, bad);
      }
    } else {
      for (int q = q0 + t; q < q1; q += BS) {
        const int i = lev_rows[q];
        const int r0 = rowptr[i], r1 = rowptr[i + 1];
        double rmax = 0.0;
        for (int p = r0; p < r1; p += 8) {  // eight loads in flight at clamped indices
          double v[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) v[k] = a[min(p + k, r1 - 1)];
#pragma unroll
          for (int k = 0; k < 8; ++k) rmax = fmax(rmax, fabs(v[k]));
        }
        for (int g = row_grp[i]; g < row_grp[i + 1]; ++g) {
          const int pik = grp_pos[g];
          const int u0 = grp_ptr[g], u1 = grp_ptr[g + 1];
          const double l = a[pik] / a[grp_diag[g]];
          a[pik] = l;
          // a group's pairs have distinct targets in row i and sources in
          // the (final) pivot row: four at a time, their loads issued
          // together at clamped indices
          for (int u = u0; u < u1; u += 4) {
            int dd[4];
            double dv[4], sv[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              const int uu = min(u + k, u1 - 1);
              dd[k] = pair_dst[uu];
              sv[k] = a[pair_src[uu]];
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) dv[k] = a[dd[k]];
#pragma unroll
            for (int k = 0; k < 4; ++k)
              if (u + k < u1) a[dd[k]] = dv[k] - l * sv[k];
          }
        }
        const double dii = a[diag[i]];
        if (!(fabs(dii) > piv_tol * rmax)) bad = 1;
      }
    }
    __syncthreads();
  }
  if (wg_max(L, (double)bad) != 0.0) return false;
  pack_slots<BS>(D);
  return true;
}

// Operands of one solve pass held by one lane: P slot values and columns,
// the row its group owns and that row's reciprocal pivot.  Lanes at or past
// the pass's active count (code >> 16) own no row and load nothing.
//
// The fetch first waits for every load still in flight (the previous fetch,
// issued a pass earlier).  Its own loads sit in a branch that lanes without a
// row skip, and after such a branch the compiler cannot count the loads in
// flight: the arithmetic of the pass whose operands arrived before the branch
// would otherwise wait for this fetch as well.
template <int P>
struct PassRegs {
  double v[P];
  int c[P];
  int row;
  double dv;
};

template <int BS, int P, bool UPPER>
__device__ __forceinline__ void pass_fetch(PassRegs<P> &o, const GMEM double *__restrict__ sv,
                                           const GMEM int *__restrict__ scol, const GMEM int *__restrict__ rowof,
                                           const GMEM double *__restrict__ rdv, int sbase, int rbase, int code,
                                           int t) {
  const int lg = (code >> 8) & 15;
  __builtin_amdgcn_s_waitcnt(kWaitVm0);
  if (t < (code >> 16)) {
#pragma unroll
    for (int j = 0; j < P; ++j) {
      o.v[j] = sv[sbase + j * BS + t];
      o.c[j] = scol[sbase + j * BS + t];
    }
    o.row = rowof[rbase + (t >> lg)];
    o.dv = UPPER ? rdv[rbase + (t >> lg)] : 1.0;  // 1 / pivot, used in the U solve only
  } else {
#pragma unroll
    for (int j = 0; j < P; ++j) {
      o.v[j] = 0.0;
      o.c[j] = 0;
    }
    o.row = -1;
    o.dv = 1.0;
  }
}


template <int P, bool UPPER>
__device__ __forceinline__ void pass_apply(const PassRegs<P> &o, double *xs, int code, int t) {
  const int lg = (code >> 8) & 15;
  // the group leader's own row value is read together with the gathers (a
  // row is written only by its own pass), not after the group sum
  const bool lead = (t & ((1 << lg) - 1)) == 0 && o.row >= 0;
  const double xr = lead ? xs[o.row] : 0.0;
  double acc = 0.0;
#pragma unroll
  for (int j = 0; j < P; ++j) acc += o.v[j] * xs[o.c[j]];
  acc = group_sum(acc, 1 << lg);
  if (lead) xs[o.row] = UPPER ? (xr - acc) * o.dv : xr - acc;
}

// The passes of one direction in order, each pass's loads issued while the
// previous pass computes (two register sets, alternating).  Pass q reads
// slots sbase + (q P + j) BS + t and row slot rbase + q BS + t / G; a barrier
// follows the last pass of every level.
template <int BS, int P, bool UPPER, bool WAVE0 = false>
__device__ __forceinline__ void solve_dir(const InstDesc &D, double *xs, const CMEM int *__restrict__ code,
                                          int np, int sbase, int rbase) {
  if (np == 0) return;
  const GMEM double *__restrict__ sv = gbl(D.sval);
  const GMEM int *__restrict__ scol = gbl(D.slot_col);
  const GMEM int *__restrict__ rowof = gbl(D.row_of);
  const GMEM double *__restrict__ rdv = gbl(D.rdv);
  const int t = tid();
  PassRegs<P> A, B;
  int ca = code[0], cb;
  pass_fetch<BS, P, UPPER>(A, sv, scol, rowof, rdv, sbase, rbase, ca, t);
  for (int q = 0; q < np; q += 2) {
    // the pass after q (the last pass again past the end: in range, unused)
    const int q1 = q + 1 < np ? q + 1 : np - 1;
    cb = code[q1];
    pass_fetch<BS, P, UPPER>(B, sv, scol, rowof, rdv, sbase + q1 * P * BS, rbase + q1 * BS, cb, t);
    pass_apply<P, UPPER>(A, xs, ca, t);
    if (ca & kPassSync) {
      if (WAVE0) wfence();  // one wave: its LDS accesses are in order
      else __syncthreads();
    }
    if (q + 1 >= np) break;
    const int q2 = q + 2 < np ? q + 2 : np - 1;
    ca = code[q2];
    pass_fetch<BS, P, UPPER>(A, sv, scol, rowof, rdv, sbase + q2 * P * BS, rbase + q2 * BS, ca, t);
    pass_apply<P, UPPER>(B, xs, cb, t);
    if (cb & kPassSync) {
      if (WAVE0) wfence();
      else __syncthreads();
    }
  }
}

// passes [q0, q0 + np) of one direction (slot count p)
template <int BS, bool UPPER, bool WAVE0>
__device__ __forceinline__ void solve_range(const InstDesc &D, double *xs, const CMEM int *code, int p, int q0,
                                            int np, int sbase, int rbase) {
  code += q0;
  sbase += q0 * p * BS;
  rbase += q0 * BS;
  switch (p) {
    case 1: solve_dir<BS, 1, UPPER, WAVE0>(D, xs, code, np, sbase, rbase); break;
    case 2: solve_dir<BS, 2, UPPER, WAVE0>(D, xs, code, np, sbase, rbase); break;
    case 4: solve_dir<BS, 4, UPPER, WAVE0>(D, xs, code, np, sbase, rbase); break;
    default: solve_dir<BS, 8, UPPER, WAVE0>(D, xs, code, np, sbase, rbase); break;
  }
}

// in-place solve G_k y = b with b (and then y) in the LDS vector xs: the L
// passes, then the U passes, of the flattened level schedules.  The passes
// near the root of the elimination tree (the last l_narrow L passes and the
// first u_narrow U passes, each with at most 64 active lanes) run in wave 0
// alone, ordered by its own LDS access order instead of workgroup barriers;
// a barrier on either side of that stretch orders it with the wide passes.
// Returns after a barrier: xs is complete for every thread.
template <int BS>
__device__ __forceinline__ void solve_lds(const InstDesc &D, double *xs, bool lower = true, bool upper = true) {
  const CMEM int *lcode = cst(D.pass_code);
  const CMEM int *ucode = lcode + D.n_lpass;
  const int lw = D.n_lpass - D.l_narrow;  // wide L passes
  const int uw0 = D.u_narrow;             // first wide U pass
  if (lower && lw > 0) solve_range<BS, false, false>(D, xs, lcode, D.pl, 0, lw, 0, 0);
  const bool narrow = (lower && D.l_narrow > 0) || (upper && D.u_narrow > 0);
  if (narrow) {
    __syncthreads();
    if (tid() < 64) {
      if (lower) solve_range<BS, false, true>(D, xs, lcode, D.pl, lw, D.l_narrow, 0, 0);
      if (upper) solve_range<BS, true, true>(D, xs, ucode, D.pu, 0, D.u_narrow, D.u_slot_base, D.u_row_base);
    }
    __syncthreads();
  }
  if (upper && D.n_upass > uw0)
    solve_range<BS, true, false>(D, xs, ucode, D.pu, uw0, D.n_upass - uw0, D.u_slot_base, D.u_row_base);
}

// (C v)_i from the ELL copy of C (entries in the CSR order of the row)
__device__ __forceinline__ double c_row(const InstDesc &D, const double *v, int i) {
  double s = 0.0;
  for (int k = 0; k < D.c_ell_k; ++k) {
    const int c = gbl(D.c_ell_col)[(int64_t)k * D.c_ell_ld + i];
    if (c >= 0) s += gbl(D.c_ell_val)[(int64_t)k * D.c_ell_ld + i] * v[c];
  }
  return s;
}

__device__ __forceinline__ double csr_row_dot(const int *rp, const int *ci, const double *val,
                                              const double *v, int i) {
  double s = 0.0;
  for (int e = rp[i]; e < rp[i + 1]; ++e) s += val[e] * v[ci[e]];
  return s;
}

// ---------------------------------------------------------------------------
// Small-matrix part of the MEVP (the residual test of Algorithm 1 and the
// coefficients of the update; the invert-Krylov section): with
// M = h H_m^{-1} and E = exp([[M, e_1], [0, 0]]),
//   y = E[:m, 0] = e^M e_1,  f = E[:m, m] = phi_1(M) e_1,
//   d = -M f = (I - e^M) e_1  (no cancellation against e_1),
//   rho = beta h_{m+1,m} |(H_m^{-1} y)_{m-1}| = beta h_{m+1,m} |(M y)_{m-1}| / h.
// Matrices are NP x NP (NP = 16 ceil((m+1)/16), zero padded, row-major with
// leading dimension NP + 1 so that a column read spreads over the LDS banks),
// in the LDS dense area for NP <= 32 and in global scratch beyond.
//  * H_m^{-1}: Hessenberg elimination with partial pivoting by one wave
//    (lanes own columns of [H | h I], the row being eliminated is carried in
//    registers), then back substitution with groups of G lanes per
//    right-hand-side column that sum their share of each row's products on
//    the DPP network.
//  * exp: Taylor polynomial of degree 18 with scaling and squaring.  With
//    2^-s ||A||_1 <= 1 the truncated tail is below e/19! ~ 2e-17 relative.
//    The polynomial is evaluated in Paterson-Stockmeyer form (blocks of three
//    in A^3): seven matrix products and no linear solve, each product on FP64
//    MFMA 16x16x4 tiles, one output tile per wave.
// ---------------------------------------------------------------------------



// 1 / k!, folded at compile time
template <int K>
struct InvFact {
  static constexpr double v = InvFact<K - 1>::v / K;
};
template <>
struct InvFact<0> {
  static constexpr double v = 1.0;
};

// C = A B (+ c0 I + c1 P1 + c2 P2 when add), all NP x NP with leading
// dimension ld.  Wave w computes output tiles w, w + NW, ...  MFMA f64
// 16x16x4 lane layout: operand A lane i + 16 k holds A[i][k]; operand B lane
// j + 16 k holds B[k][j]; result element v of lane j + 16 q is C[q + 4 v][j].
// With Dout (and add false) the tile also gives
// Dout = ((d0 I + d1 P1) + d2 P2) + d3 C.
template <int BS, int NP, class PT>
__device__ __forceinline__ void mm_mfma(PT A, PT B, PT C, int ld, bool add, double c0, double c1, double c2,
                                        PT P1, PT P2, PT Dout = nullptr, double d0 = 0.0, double d1 = 0.0,
                                        double d2 = 0.0, double d3 = 0.0) {
  constexpr int T = NP / 16, NW = BS / 64;
  const int lane = tid() & 63, wave = tid() >> 6;
  const int r = lane & 15, q = lane >> 4;
  for (int tile = wave; tile < T * T; tile += NW) {
    const int i0 = (tile / T) * 16, j0 = (tile % T) * 16;
    dbl4 acc;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + q + 4 * v, j = j0 + r;
      acc[v] = add ? ((i == j ? c0 : 0.0) + c1 * P1[i * ld + j]) + c2 * P2[i * ld + j] : 0.0;
    }
#pragma unroll 4
    for (int k = 0; k < NP; k += 4) {
      const double a = A[(i0 + r) * ld + k + q];
      const double b = B[(k + q) * ld + j0 + r];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) C[(i0 + q + 4 * v) * ld + j0 + r] = acc[v];
    if (Dout) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + q + 4 * v, j = j0 + r, o = i * ld + j;
        Dout[o] = (((i == j ? d0 : 0.0) + d1 * P1[o]) + d2 * P2[o]) + d3 * acc[v];
      }
    }
  }
  __syncthreads();
}

// entry (r, c) of [H | h I] (m x 2m; zero beyond), H read from the global
// copy (column-major, leading dimension kHLd) or, when IN_LDS, from the
// row-major staged copy Hs (leading dimension ld, zeros below the subdiagonal)
template <bool IN_LDS, class PT>
__device__ __forceinline__ double hess_aug(const GMEM double *H, PT Hs, int ld, int m, double h, int r, int c) {
  if (c >= 2 * m) return 0.0;
  if (c >= m) return c - m == r ? h : 0.0;
  if (IN_LDS) return Hs[r * ld + c];
  return r <= c + 1 ? H[r + c * kHLd] : 0.0;
}

// X = h H^{-1} for the m x m upper Hessenberg H (column-major, leading
// dimension kHLd, entries r <= c + 1 stored); U receives the triangular
// factor and rinv the reciprocals of its diagonal.  U and X are m x m with
// leading dimension ld.  With IN_LDS, H is first staged into Hs (m x m,
// leading dimension ld) so that the elimination's row reads are LDS reads,
// each issued one elimination step ahead.
template <int BS, int NP, bool IN_LDS, class PT>
__device__ __forceinline__ void hess_inverse(const GMEM double *H, PT Hs, int m, double h, PT U, PT X, PT rinv,
                                             int ld) {
  const int t = tid();
  if (IN_LDS) {
    for (int idx = t; idx < m * m; idx += BS) {
      const int r = idx % m, c = idx / m;
      Hs[r * ld + c] = r <= c + 1 ? H[r + c * kHLd] : 0.0;
    }
    __syncthreads();
  }
  if (t < 64) {
    // lane t owns columns t and t + 64 of [H | h I] (2 m <= 126)
    double R0 = hess_aug<IN_LDS>(H, Hs, ld, m, h, 0, t);  // the carried row
    double R1 = hess_aug<IN_LDS>(H, Hs, ld, m, h, 0, t + 64);
    double N0 = m > 1 ? hess_aug<IN_LDS>(H, Hs, ld, m, h, 1, t) : 0.0;  // row k + 1
    double N1 = m > 1 ? hess_aug<IN_LDS>(H, Hs, ld, m, h, 1, t + 64) : 0.0;
    for (int k = 0; k + 1 < m; ++k) {
      const double F0 = N0, F1 = N1;
      if (k + 2 < m) {
        N0 = hess_aug<IN_LDS>(H, Hs, ld, m, h, k + 2, t);
        N1 = hess_aug<IN_LDS>(H, Hs, ld, m, h, k + 2, t + 64);
      }
      const double Rk = readlane_d(R0, k), Fk = readlane_d(F0, k);
      const bool sw = fabs(Fk) > fabs(Rk);
      const double P0 = sw ? F0 : R0, P1 = sw ? F1 : R1;
      double O0 = sw ? R0 : F0, O1 = sw ? R1 : F1;
      const double l = (sw ? Rk : Fk) / (sw ? Fk : Rk);
      if (t > k) O0 -= l * P0;
      else O0 = 0.0;
      O1 -= l * P1;  // columns >= 64 are right-hand-side columns (m <= 63)
      if (t < m) U[k * ld + t] = P0;
      else if (t < 2 * m) X[k * ld + t - m] = P0;
      if (t + 64 < 2 * m) X[k * ld + t + 64 - m] = P1;
      R0 = O0;
      R1 = O1;
    }
    if (t < m) U[(m - 1) * ld + t] = R0;
    else if (t < 2 * m) X[(m - 1) * ld + t - m] = R0;
    if (t + 64 < 2 * m) X[(m - 1) * ld + t + 64 - m] = R1;
    // lane t wrote the diagonal entry u_tt itself
    if (t < m) rinv[t] = 1.0 / U[t * ld + t];
  }
  __syncthreads();
  if (IN_LDS && NP <= 32) {
    // back substitution U X = Y (Y in X), right-looking: column c by the 8
    // lanes of group c, lane p keeping rows p, p + 8, ... of the column in
    // registers.  At row r (descending) the owner scales its entry by
    // 1 / u_rr, the group reads it from the owner, and every lane subtracts
    // u_ir x_r from its rows i < r.
    constexpr int RPL = NP / 8;
    const int c = t >> 3, p = t & 7;
    const bool own = c < m;
    double y[RPL];
#pragma unroll
    for (int q = 0; q < RPL; ++q) y[q] = (own && p + 8 * q < m) ? X[(p + 8 * q) * ld + c] : 0.0;
#pragma unroll
    for (int r = NP - 1; r >= 0; --r) {
      if (r < m) {
        const int qr = r >> 3, pr = r & 7;
        if (p == pr) y[qr] *= rinv[r];
        const double xr = __shfl(y[qr], (t & ~7) | pr, 64);
#pragma unroll
        for (int q = 0; q < RPL; ++q)
          if (p + 8 * q < r) y[q] -= U[(p + 8 * q) * ld + r] * xr;
      }
    }
#pragma unroll
    for (int q = 0; q < RPL; ++q)
      if (own && p + 8 * q < m) X[(p + 8 * q) * ld + c] = y[q];
    __syncthreads();
    return;
  }
  // back substitution U X = Y, Y in X: column c by the G lanes of group c
  const int G = 8 * m <= BS ? 8 : 4;
  const int c = t / G, p = t % G;
  const bool own = c < m;
  for (int r = m - 1; r >= 0; --r) {
    double s = 0.0;
    if (own)
      for (int j = r + 1 + p; j < m; j += G) s += U[r * ld + j] * X[j * ld + c];
    s = group_sum(s, G);
    if (own && p == 0) X[r * ld + c] = (X[r * ld + c] - s) * rinv[r];
    if (IN_LDS) wfence();  // the group's lanes share one wave; LDS is in order
    else __syncthreads();
  }
  __syncthreads();
}

template <int BS, int NP, bool IN_LDS, class PT>
__device__ __forceinline__ double hess_phi_np(Lds<BS> &L, PT base, const GMEM double *H, int m, double h,
                                              double beta, double h_next, double *dout, double *dout2) {
  constexpr int ld = NP + 1;
  PT P1 = base, P2 = base + NP * ld, P3 = base + 2 * NP * ld, Ta = base + 3 * NP * ld, Tb = base + 4 * NP * ld;
  // ---- M = h H^{-1} into P3 (P2 holds the triangular factor) ----
  hess_inverse<BS, NP, IN_LDS>(H, P1, m, h, P2, P3, Ta, ld);
  // ---- A = [[M, e_1], [0, 0]] padded to NP x NP; with the phi_2 column it
  // is [[M, e_1, 0], [0, 0, 1], [0, 0, 0]].  ||A||_1 from M's column sums
  // (a non-finite entry of M, H_m singular, makes it non-finite: not
  // converged), then A scaled by 2^-s into P1 ----
  const bool two = dout2 != nullptr;
  double cs = 0.0;
  if (tid() < NP) {
    const int c = tid();
    if (c < m) {
      for (int r = 0; r < m; ++r) cs += fabs(P3[r * ld + c]);
    } else if (c == m || (two && c == m + 1)) {
      cs = 1.0;
    }
    if (!isfinite(cs)) cs = INFINITY;
  }
  const double nrm = wg_max(L, cs);
  if (!isfinite(nrm)) return INFINITY;
  // 2^-s ||A||_1 <= 1; beyond 2^64 every entry of exp(A) under- or overflows
  // anyway
  int s = 0;
  if (nrm > 1.0) {
    int e;
    const double f = frexp(nrm, &e);
    s = e > 64 ? 64 : (f == 0.5 ? e - 1 : e);
  }
  const double sc = ldexp(1.0, -s);
  for (int i = tid(); i < NP * NP; i += BS) {
    const int r = i / NP, c = i % NP;
    double v = (r < m && c < m) ? P3[r * ld + c] : (r == 0 && c == m ? 1.0 : 0.0);
    if (two && r == m && c == m + 1) v = 1.0;
    P1[r * ld + c] = v * sc;
  }
  __syncthreads();
  // ---- Taylor degree 18, Paterson-Stockmeyer with A^3 (the A^3 product
  // also gives the first term 1/15! I + A/16! + A^2/17! + A^3/18!) ----
  mm_mfma<BS, NP>(P1, P1, P2, ld, false, 0.0, 0.0, 0.0, P1, P1);
  mm_mfma<BS, NP>(P2, P1, P3, ld, false, 0.0, 0.0, 0.0, P1, P1, Ta, InvFact<15>::v, InvFact<16>::v,
                  InvFact<17>::v, InvFact<18>::v);
  mm_mfma<BS, NP>(Ta, P3, Tb, ld, true, InvFact<12>::v, InvFact<13>::v, InvFact<14>::v, P1, P2);
  mm_mfma<BS, NP>(Tb, P3, Ta, ld, true, InvFact<9>::v, InvFact<10>::v, InvFact<11>::v, P1, P2);
  mm_mfma<BS, NP>(Ta, P3, Tb, ld, true, InvFact<6>::v, InvFact<7>::v, InvFact<8>::v, P1, P2);
  mm_mfma<BS, NP>(Tb, P3, Ta, ld, true, InvFact<3>::v, InvFact<4>::v, InvFact<5>::v, P1, P2);
  mm_mfma<BS, NP>(Ta, P3, Tb, ld, true, InvFact<0>::v, InvFact<1>::v, InvFact<2>::v, P1, P2);
  // ---- squaring ----
  PT E = Tb, Y = Ta;
  for (int k = 0; k < s; ++k) {
    mm_mfma<BS, NP>(E, E, Y, ld, false, 0.0, 0.0, 0.0, P1, P1);
    PT tmp = E;
    E = Y;
    Y = tmp;
  }
  // ---- d = -M f and (M y)_{m-1};  M = 2^s A[:m, :m] exactly; with the
  // phi_2 column also d2 = -M phi_2(M) e_1.  m < 64: the first wave does it
  // and broadcasts rho ----
  double rho = 0.0;
  if (tid() < 64) {
    const int r = tid();
    double bad = 0.0, part = 0.0;
    if (r < m) {
      double acc = 0.0, acc2 = 0.0;
      for (int c = 0; c < m; ++c) {
        const double mrc = ldexp(P1[r * ld + c], s);
        acc += mrc * E[c * ld + m];
        if (two) acc2 += mrc * E[c * ld + m + 1];
      }
      dout[r] = -acc;
      if (two) dout2[r] = -acc2;
      if (!isfinite(acc) || !isfinite(acc2)) bad = 1.0;
      part = ldexp(P1[(m - 1) * ld + r], s) * E[r * ld];
    }
    const double my = wave_sum(part);
    const double anybad = wave_max(bad);
    rho = beta * h_next * fabs(my / h);
    if (anybad != 0.0 || !isfinite(rho)) rho = INFINITY;
  }
  return wg_bcast0(L, rho);
}

// d -> dout (LDS, m doubles), and -M phi_2(M) e_1 -> dout2 when it is not
// null; returns rho (inf if anything is not finite)
template <int BS>
__device__ __forceinline__ double hess_phi(const InstDesc &D, Lds<BS> &L, const double *H, int m, double h,
                                           double beta, double h_next, double *dout, double *dout2 = nullptr) {
  const int n1 = m + (dout2 ? 2 : 1);
  if (n1 <= 16 && 5 * 16 * 17 <= L.RD)
    return hess_phi_np<BS, 16, true>(L, L.dense, gbl(H), m, h, beta, h_next, dout, dout2);
  if (n1 <= 32 && 5 * 32 * 33 <= L.RD)
    return hess_phi_np<BS, 32, true>(L, L.dense, gbl(H), m, h, beta, h_next, dout, dout2);
  return hess_phi_np<BS, 64, false>(L, gbl(D.mat), gbl(H), m, h, beta, h_next, dout, dout2);
}

// ---------------------------------------------------------------------------
// Arnoldi (Algorithm 1)
// ---------------------------------------------------------------------------

struct Basis {
  int m;
  int exact;
  double beta;
  double hscale;
};

struct Work {  // exact work counters of one launch
  int64_t mgs, comb;
  int trials;
};

// One Arnoldi step j = B.m (Algorithm 1): w = -G^{-1} C v_j, modified
// Gram-Schmidt against v_0..v_j in increasing order, h_{j+1,j} = ||w||_2,
// v_{j+1} = w / h_{j+1,j}.  v_j is in the LDS vector area on entry and
// v_{j+1} on exit.  Thread t owns rows t + e BS (e < E): C v_j is gathered
// from LDS with the ELL loads of all E rows issued together, w stays in
// registers through the Gram-Schmidt sweep, and v_{i+1} is loaded while the
// inner product with v_i is reduced.  The basis and C's ELL columns are
// padded with zeros to E BS rows, so these loads need no bound test (a
// branch around them would make the compiler wait for every load in flight
// before the next inner product); rows past n keep w = 0.
template <int BS, int E>
__device__ __forceinline__ void arnoldi_step_e(const InstDesc &D, Lds<BS> &L, double *V, double *H, Basis &B,
                               double breakdown, Prof &pf) {
  const int n = D.n, j = B.m, t0 = tid();
  const int64_t ldv = D.ldv;
  double *xs = L.region;
  double *hcol = L.hcol;  // this step's Hessenberg column, stored to H once at the end
  GMEM double *Vg = gbl(V);
  GMEM double *Hg = gbl(H);
  // ---- q = C v_j: one ELL column at a time, its loads for all E rows together ----
  double w[E];
#pragma unroll
  for (int e = 0; e < E; ++e) w[e] = 0.0;
  const int K = D.c_ell_k;
  for (int k = 0; k < K; ++k) {
    const GMEM int *__restrict__ ccol = gbl(D.c_ell_col) + (int64_t)k * D.c_ell_ld + t0;
    const GMEM double *__restrict__ cval = gbl(D.c_ell_val) + (int64_t)k * D.c_ell_ld + t0;
    int cc[E];
    double cv[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      cc[e] = ccol[e * BS];
      cv[e] = cval[e * BS];
    }
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (cc[e] >= 0) w[e] += cv[e] * xs[cc[e]];
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < E; ++e)
    if (t0 + e * BS < n) xs[t0 + e * BS] = -w[e];
  __syncthreads();
  solve_lds<BS>(D, xs);
  pf.mark(2);
  // ---- modified Gram-Schmidt ----
#pragma unroll
  for (int e = 0; e < E; ++e) w[e] = t0 + e * BS < n ? xs[t0 + e * BS] : 0.0;
  double cur[E], nxt[E];
#pragma unroll
  for (int e = 0; e < E; ++e) cur[e] = Vg[t0 + e * BS];
  for (int i = 0; i <= j; ++i) {
    double part = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) part += w[e] * cur[e];
    {
      // v_{i+1} (v_j again after the last product: no branch around the loads)
      const GMEM double *vn = Vg + (int64_t)(i < j ? i + 1 : j) * ldv + t0;
#pragma unroll
      for (int e = 0; e < E; ++e) nxt[e] = vn[e * BS];
    }
    const double hij = wg_sum(L, part);
#pragma unroll
    for (int e = 0; e < E; ++e) w[e] -= hij * cur[e];
    if (t0 == 0) hcol[i] = hij;
    B.hscale = nmax(B.hscale, fabs(hij));
#pragma unroll
    for (int e = 0; e < E; ++e) cur[e] = nxt[e];
  }
  double part = 0.0;
#pragma unroll
  for (int e = 0; e < E; ++e) part += w[e] * w[e];
  const double hn = sqrt(wg_sum(L, part));
  B.hscale = nmax(B.hscale, hn);
  B.m = j + 1;
  const bool brk = hn <= breakdown * B.hscale;
  if (brk) B.exact = 1;
  if (!brk) {
    GMEM double *vn = Vg + (int64_t)(j + 1) * ldv;
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (t0 + e * BS < n) {
        const double v = w[e] / hn;
        vn[t0 + e * BS] = v;
        xs[t0 + e * BS] = v;
      }
  }
  for (int i = t0; i <= j; i += BS) Hg[i + j * kHLd] = hcol[i];
  if (t0 == 0) Hg[j + 1 + j * kHLd] = brk ? 0.0 : hn;
  __syncthreads();
  pf.mark(3);
}

// Basis combinations of the trial (thread t owns rows t + e BS, e < E; the
// zero rows past n are loaded and not stored).  The columns run outermost, so
// each thread keeps E loads of a column in flight; each row's sum still runs
// over j in increasing order.
//  main:  x_{k+1} = (x_k + h p) + beta V_m d; returns 1 if an entry is not finite
template <int BS, int E>
__device__ __forceinline__ double combine_main(const InstDesc &D, const double *d, int m, double beta, double h) {
  const int n = D.n, t0 = tid();
  const GMEM double *Vg = gbl(D.V) + t0, *xk = gbl(D.xk), *pp = gbl(D.p);
  GMEM double *x1 = gbl(D.x1);
  double acc[E];
#pragma unroll
  for (int e = 0; e < E; ++e) acc[e] = 0.0;
#pragma unroll 2
  for (int j = 0; j < m; ++j) {
    const double dj = d[j];
    const GMEM double *col = Vg + (int64_t)j * D.ldv;
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] += col[e * BS] * dj;
  }
  double bad = 0.0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int i = t0 + e * BS;
    if (i < n) {
      const double v = (xk[i] + h * pp[i]) + beta * acc[e];
      x1[i] = v;
      if (!isfinite(v)) bad = 1.0;
    }
  }
  return bad;
}

//  error: max_i |beta_e (V_e d_e)_i|; with ER-C also x_{k+1} -= gamma beta_e V_e d2
template <int BS, int E>
__device__ __forceinline__ double combine_err(const InstDesc &D, const double *de, const double *d2, int m,
                                              double beta, double gamma, bool erc) {
  const int n = D.n, t0 = tid();
  const GMEM double *Vg = gbl(D.Ve) + t0;
  GMEM double *x1 = gbl(D.x1);
  double acc[E], acc2[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    acc[e] = 0.0;
    acc2[e] = 0.0;
  }
#pragma unroll 2
  for (int j = 0; j < m; ++j) {
    const double dj = de[j], d2j = erc ? d2[j] : 0.0;
    const GMEM double *col = Vg + (int64_t)j * D.ldv;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const double vji = col[e * BS];
      acc[e] += vji * dj;
      if (erc) acc2[e] += vji * d2j;
    }
  }
  double emax = 0.0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int i = t0 + e * BS;
    if (i < n) {
      emax = nmax(emax, fabs(beta * acc[e]));
      if (erc) x1[i] -= gamma * (beta * acc2[e]);
    }
  }
  return emax;
}

// rows per thread: rows_per_thread(n, BS) = 4, 6, 9, 12 or 18; set-up keeps
// n <= EM BS for the kernel's bound EM (12 and 18 only at 512 threads)
template <int BS, int EM = max_rows_per_thread(BS)>
__device__ __forceinline__ void arnoldi_step(const InstDesc &D, Lds<BS> &L, double *V, double *H, Basis &B,
                             double breakdown, Prof &pf) {
  const int e = rows_per_thread(D.n, BS);
  if (e == 4) arnoldi_step_e<BS, 4>(D, L, V, H, B, breakdown, pf);
  else if (e == 6) arnoldi_step_e<BS, 6>(D, L, V, H, B, breakdown, pf);
  else if (EM <= 9 || e == 9) arnoldi_step_e<BS, 9>(D, L, V, H, B, breakdown, pf);
  else if (e == 12) arnoldi_step_e<BS, (EM > 9 ? 12 : 9)>(D, L, V, H, B, breakdown, pf);
  else arnoldi_step_e<BS, (EM > 9 ? 18 : 9)>(D, L, V, H, B, breakdown, pf);
}

// Start a basis from the vector v (global or the LDS vector area):
// beta = ||v||_2, v_0 = v / beta, written to V and to the LDS vector area.
template <int BS>
__device__ __forceinline__ void basis_start(const InstDesc &D, Lds<BS> &L, const double *v, double *V, Basis &B) {
  double part = 0.0;
  for (int t = tid(); t < D.n; t += BS) part += v[t] * v[t];
  B.beta = sqrt(wg_sum(L, part));
  B.m = 0;
  B.exact = B.beta == 0.0;
  B.hscale = 0.0;
  if (B.beta > 0.0)
    for (int t = tid(); t < D.n; t += BS) {
      const double u = v[t] / B.beta;
      gbl(V)[t] = u;
      L.region[t] = u;
    }
  __syncthreads();
}

// grow the basis until rho_m(h) <= eps; d -> dout.  Returns a status code.
template <int BS, int EM = max_rows_per_thread(BS)>
__device__ __forceinline__ int mevp_converge(const InstDesc &D, Lds<BS> &L, const Opts &o, double *V, double *H,
                             Basis &B, double h, double eps, double *dout, double &rho,
                             int &iters, Prof &pf, Work &wk, int m_first = 1, double *dout2 = nullptr) {
  if (B.beta == 0.0) {
    rho = 0.0;
    return kOK;
  }
  // one call site each for the residual test and the Arnoldi step (the code
  // is inlined: a second copy would only cost instruction cache).  The
  // residual is tested from m_first on (every j when m_first = 1, as in
  // Algorithm 1), and always once the basis is complete.
  for (int it = 0;; ++it) {
    if (B.m > 0 && (B.m >= m_first || B.exact)) {
      rho = hess_phi<BS>(D, L, H, B.m, h, B.beta, B.exact ? 0.0 : gbl(H)[B.m + (B.m - 1) * kHLd], dout, dout2);
      pf.mark(4);
      if (rho <= eps) return kOK;
      if (B.exact) return kEKRYLOV;
    }
    if (it == 0 && B.m > 0) {
      // a reused basis continues from v_m; the LDS vector area has been reused
      const GMEM double *vm = gbl(V) + (int64_t)B.m * D.ldv;
      for (int t = tid(); t < D.n; t += BS) L.region[t] = vm[t];
      __syncthreads();
    }
    if (B.m >= o.m_max) return kEKRYLOV;
    arnoldi_step<BS, EM>(D, L, V, H, B, o.breakdown, pf);
    ++iters;
    wk.mgs += B.m;
  }
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

template <int BS>
__device__ Lds<BS> lds_setup(int R, int NX) {
  extern __shared__ double smem[];
  Lds<BS> L;
  L.region = smem;
  L.dense = smem + NX;
  L.slots = smem + R;
  L.dmain = L.slots + 2 * (BS / 64);
  L.derr = L.dmain + kHLd;
  L.prof = reinterpret_cast<long long *>(L.derr + kHLd + 4);
  L.hcol = L.derr + kHLd + 4 + kPhases;
  L.derr2 = L.hcol + kHLd;
  L.R = R;
  L.RD = R - NX;
  L.par = 0;
  return L;
}

// Load the caller's state x (caller numbering) into x_k and reset the run state.
__global__ void k_begin(const InstDesc *descs, const double *const *xin, double t0, double h0) {
  const InstDesc &D = descs[blockIdx.x];
  const double *x = xin[blockIdx.x];
  for (int i = tid(); i < D.n; i += blockDim.x) gbl(D.xk)[i] = x[gbl(D.perm)[i]];
  if (tid() == 0) {
    InstState &S = *D.state;
    S.t = t0;
    S.h_prop = fmin(h0, D.h_max);
    S.steps = 0;
    S.status = kOK;
    S.done = 0;
    S.lu_count = 0;
    S.rejects = 0;
    S.arnoldi = 0;
    S.lu_valid = 0;
    S.trials = 0;
    S.mgs_terms = 0;
    S.comb_terms = 0;
    for (int i = 0; i < kPhases; ++i) S.ph[i] = 0.0;
    S.h_prev = S.h_prop;
    S.rho_prev = 0.0;
    S.err_prev = 0.0;
    S.m_prev = 0;
    S.rej_prev = 0;
    S.m_err_prev = 0;
    int b = 0;
    while (b < D.n_bp - 1 && gbl(D.bp)[b] <= t0) ++b;
    S.bp_idx = b;
  }
}

// Workspace entries that the kernels read but never write: the padding rows
// n .. ldv - 1 of every column of V and V_e (0), the solve slots without an
// entry (0) and the U row slots without a row (pivot 1).
__global__ void k_init_workspace(const InstDesc *descs) {
  const InstDesc &D = descs[blockIdx.x];
  const int pad = (int)D.ldv - D.n;
  for (int idx = tid(); idx < pad * D.vcols; idx += blockDim.x) {
    const int64_t o = (int64_t)(idx / pad) * D.ldv + D.n + idx % pad;
    gbl(D.V)[o] = 0.0;
    gbl(D.Ve)[o] = 0.0;
  }
  for (int k = tid(); k < D.n_slots; k += blockDim.x) gbl(D.sval)[k] = 0.0;
  for (int r = tid(); r < D.n_srows; r += blockDim.x) gbl(D.rdv)[r] = 1.0;
}

// Write x_k back in the caller's numbering.
__global__ void k_end(const InstDesc *descs, double *const *xout) {
  const InstDesc &D = descs[blockIdx.x];
  double *x = xout[blockIdx.x];
  for (int i = tid(); i < D.n; i += blockDim.x) x[gbl(D.perm)[i]] = gbl(D.xk)[i];
}

// The ER transient (Algorithm 2) of one instance, resumable: runs at most
// max_steps accepted steps unless the instance is done.  replay != 0: the
// step ends are taken from gbl(D.bp) (the given grid) and every first trial
// is accepted.
template <int BS, int EM>
__device__ __forceinline__ void run_instance(const InstDesc &D, Lds<BS> &L, const Opts &o, int max_steps,
                                             int replay) {
  InstState &S = *D.state;
  if (S.done) return;
  double *xs = L.region;
  const int n = D.n;
  double t = S.t, h_prop = S.h_prop;
  int bp_idx = S.bp_idx, steps = S.steps, status = kOK;
  int lu_count = S.lu_count, rej_total = S.rejects, iters = S.arnoldi;
  int lu_valid = S.lu_valid;
  double h_prev = S.h_prev, rho_prev = S.rho_prev, err_prev = S.err_prev;
  int m_prev = S.m_prev, rej_prev = S.rej_prev, m_err_prev = S.m_err_prev;
  const bool learned = o.controller && !replay;
  const int steps0 = steps;
  const int rec = kRecFixed + D.n_probe;
  Prof pf;
  pf.start(L.prof);
  Work wk{0, 0, 0};
  __syncthreads();

  for (int it = 0; it < max_steps; ++it) {
    if (replay ? (steps >= D.n_bp) : !(t < D.T)) {
      S.done = 1;
      break;
    }
    if (steps - steps0 >= D.trace_cap) break;
    // ---- step size: clip to the next source corner / T ----
    double h_try, t_land;
    bool land;
    double h_unc;  // the first trial before clipping to a source corner or T
    if (replay) {
      t_land = gbl(D.bp)[steps];
      h_try = h_unc = t_land - t;
      land = true;
    } else {
      t_land = gbl(D.bp)[bp_idx];
      h_try = h_unc = fmin(h_prop, D.h_max);
      land = false;
      if (t + h_try * (1.0 + 1e-3) >= t_land) {
        h_try = t_land - t;
        land = true;
      }
    }
    // ---- stamp and factor G_k at x_k (without devices G_k = G_lin is
    // constant and its factors are kept after the first step) ----
    if (D.has_dev || !lu_valid) {
      stamp_devices<BS>(D, D.xk, D.devI, D.devD);
      __syncthreads();
      assemble<BS>(D, false);
      __syncthreads();
      if (!refactor<BS>(D, L, o.piv_tol)) { status = kESINGULAR; break; }
      ++lu_count;
      lu_valid = 1;
    }
    pf.mark(0);
    // ---- the three right-hand sides, one solve each (one loop, one copy of
    // the solve code):  w = G^{-1} r with r = B u(t) - G_lin x_k - I_dev(x_k);
    // p = G^{-1} B s;  z = G^{-1} C p, leaving v = w - z in tmp ----
    // step features (used by the learned controller, recorded in every mode)
    double feat[kFeat];
    double rmax = 0.0, fkmax = 0.0;
    int m_first = 1;  // first Krylov size at which the residual is tested
#pragma nounroll
    for (int rhs = 0; rhs < 3; ++rhs) {
      if (rhs == 1) {
        // source slopes inside the current PWL segment
        const double ts = t + 0.5 * (learned ? gbl(D.bp)[bp_idx] - t : h_try);
        double smax = 0.0;
        for (int q = tid(); q < D.n_src; q += BS) smax = nmax(smax, fabs(pwl_slope(D, q, ts)));
        const double r_inf = wg_max(L, rmax), f_inf = wg_max(L, fkmax), s_inf = wg_max(L, smax);
        feat[0] = log10(fmax(r_inf, 1e-30));
        feat[1] = m_prev / 60.0;
        feat[2] = log10(h_prev);
        feat[3] = log10(fmax(rho_prev, 1e-30));
        feat[4] = log10(1.0 + s_inf * 1e-9);
        feat[5] = log10(fmax(f_inf, 1e-30));
        feat[6] = log10(fmax(err_prev / o.E_rr, 1e-30));
        feat[7] = rej_prev;
        if (learned) {
          // the network proposes (m, log10 h); the step stays within a
          // factor alpha..beta of the previous accepted one and the error
          // test below still judges it (rejections halve as before)
          if (tid() < 64) {
            float ff[kFeat], out[2];
#pragma unroll
            for (int i = 0; i < kFeat; ++i) ff[i] = (float)feat[i];
            mlp_infer_wave(o.ctrl_w, o.ctrl_norm, ff, out);
            if (tid() == 0) {
              L.hcol[0] = out[0];
              L.hcol[1] = out[1];
            }
          }
          __syncthreads();
          const double m_hat = L.hcol[0], lh = L.hcol[1];
          __syncthreads();
          m_first = (int)fmin(fmax(rint(m_hat) - 1.0, 1.0), (double)o.m_max);
          double hl = o.ctrl_safety * exp10(lh);
          if (!(hl == hl)) hl = h_prev;
          hl = fmin(fmax(hl, o.alpha * h_prev), o.beta * h_prev);
          // corners: stretch by up to 25 % to land on one, and split a gap
          // shorter than two steps into two equal halves, so that no tiny
          // remainder step is left (the invert-Krylov basis needed at small
          // h grows, up to the m_max limit)
          t_land = gbl(D.bp)[bp_idx];
          h_try = h_unc = fmin(hl, D.h_max);
          land = false;
          if (t + h_try * 1.25 >= t_land) {
            h_try = t_land - t;
            land = true;
          } else if (t + 2.0 * h_try > t_land) {
            h_try = 0.5 * (t_land - t);
          }
        }
      }
      const double tm = t + 0.5 * h_try;
      for (int i = tid(); i < n; i += BS) {
        double b = 0.0;
        if (rhs == 0) {
          for (int e = gbl(D.b_rowptr)[i]; e < gbl(D.b_rowptr)[i + 1]; ++e) b += gbl(D.b_val)[e] * pwl_value(D, gbl(D.b_col)[e], t);
          b = (b - csr_row_dot(D.g_rowptr, D.g_col, D.g_val, D.xk, i)) - gbl(D.Ik)[i];
          rmax = nmax(rmax, fabs(b));
          // F_k(x_k) = J_dev(x_k) x_k - I_dev(x_k) at node i
          double lin = 0.0;
          for (int c = gbl(D.node_ptr)[i]; c < gbl(D.node_ptr)[i + 1]; ++c) {
            const int code = gbl(D.node_code)[c], k = code >> 1;
            double dv = 0.0;
            for (int v = 0; v < 3; ++v) {
              const int nd = gbl(D.dev_node)[3 * k + v];
              if (nd >= 0) dv += gbl(D.devD)[3 * k + v] * gbl(D.xk)[nd];
            }
            lin += (code & 1) ? -dv : dv;
          }
          fkmax = nmax(fkmax, fabs(lin - gbl(D.Ik)[i]));
        } else if (rhs == 1) {
          for (int e = gbl(D.b_rowptr)[i]; e < gbl(D.b_rowptr)[i + 1]; ++e) b += gbl(D.b_val)[e] * pwl_slope(D, gbl(D.b_col)[e], tm);
        } else {
          b = c_row(D, D.p, i);
        }
        xs[i] = b;
      }
      __syncthreads();
      solve_lds<BS>(D, xs);
      GMEM double *dst = rhs == 0 ? gbl(D.w) : rhs == 1 ? gbl(D.p) : gbl(D.tmp);
      for (int i = tid(); i < n; i += BS) dst[i] = rhs == 2 ? gbl(D.w)[i] - xs[i] : xs[i];
      __syncthreads();
    }
    Basis Bm;
    basis_start<BS>(D, L, D.tmp, D.V, Bm);
    pf.mark(1);
    // ---- trial loop ----
    double h = h_try, rho = 0.0, err = 0.0;
    int rej = 0, m_err = 0;
    bool fell_back = false;
    for (;;) {
      ++wk.trials;
      status = mevp_converge<BS, EM>(D, L, o, D.V, D.H, Bm, h, o.eps_K, L.dmain, rho, iters, pf, wk,
                                 rej == 0 ? m_first : 1);
      // a learned proposal whose MEVP does not converge within m_max (the
      // invert-Krylov residual grows as h shrinks, so halving would not help)
      // falls back to the paper's proposal for this step; the basis is kept
      if (status == kEKRYLOV && learned && !fell_back) {
        fell_back = true;
        double hp = fmin(h_prop, D.h_max);
        h_unc = hp;
        t_land = gbl(D.bp)[bp_idx];
        land = false;
        if (t + hp * (1.0 + 1e-3) >= t_land) {
          hp = t_land - t;
          land = true;
        }
        h = h_try = hp;
        rej = 0;
        status = kOK;
        continue;
      }
      if (status != kOK) break;
      wk.comb += Bm.m;
      // x_{k+1} = x_k + h p + beta V_m d
      const int rpt = rows_per_thread(n, BS);
      constexpr int E12 = EM > 9 ? 12 : 9, E18 = EM > 9 ? 18 : 9;
      const double bad = rpt == 4    ? combine_main<BS, 4>(D, L.dmain, Bm.m, Bm.beta, h)
                         : rpt == 6  ? combine_main<BS, 6>(D, L.dmain, Bm.m, Bm.beta, h)
                         : rpt == 9  ? combine_main<BS, 9>(D, L.dmain, Bm.m, Bm.beta, h)
                         : rpt == 12 ? combine_main<BS, E12>(D, L.dmain, Bm.m, Bm.beta, h)
                                     : combine_main<BS, E18>(D, L.dmain, Bm.m, Bm.beta, h);
      if (wg_max(L, bad) != 0.0) { status = kENONFINITE; break; }
      err = 0.0;
      m_err = 0;
      if (D.has_dev) {
        stamp_devices<BS>(D, D.x1, D.devI1, nullptr);
        __syncthreads();
        // dF = J_dev(x_k)(x_{k+1} - x_k) - (I_dev(x_{k+1}) - I_dev(x_k))
        for (int i = tid(); i < n; i += BS) {
          double s = 0.0;
          for (int c = gbl(D.node_ptr)[i]; c < gbl(D.node_ptr)[i + 1]; ++c) {
            const int code = gbl(D.node_code)[c], k = code >> 1;
            double lin = 0.0;
            for (int v = 0; v < 3; ++v) {
              const int nd = gbl(D.dev_node)[3 * k + v];
              if (nd >= 0) lin += gbl(D.devD)[3 * k + v] * (D.x1[nd] - gbl(D.xk)[nd]);
            }
            const double df = lin - (D.devI1[k] - gbl(D.devI)[k]);
            s += (code & 1) ? -df : df;
          }
          xs[i] = s;
        }
        __syncthreads();
        solve_lds<BS>(D, xs);
        Basis Be;
        basis_start<BS>(D, L, xs, D.Ve, Be);
        pf.mark(5);
        double rho_e;
        // under the learned controller the residual tests of the error MEVP
        // start two sizes below the previous step's (every size otherwise)
        status = mevp_converge<BS, EM>(D, L, o, D.Ve, D.He, Be, h, o.eps_K, L.derr, rho_e, iters, pf, wk,
                                   learned ? max(1, m_err_prev - 2) : 1, o.erc ? L.derr2 : nullptr);
        if (status == kEKRYLOV && learned && !fell_back) {
          fell_back = true;
          double hp = fmin(h_prop, D.h_max);
          h_unc = hp;
          t_land = gbl(D.bp)[bp_idx];
          land = false;
          if (t + hp * (1.0 + 1e-3) >= t_land) {
            hp = t_land - t;
            land = true;
          }
          h = h_try = hp;
          rej = 0;
          status = kOK;
          continue;
        }
        if (status != kOK) break;
        m_err = Be.m;
        wk.comb += Be.m;
        // ER-C: x_{k+1} -= gamma h phi_2(hJ) C^{-1} dF = gamma beta_e V_e d2
        const int rpe = rows_per_thread(n, BS);
        constexpr int F12 = EM > 9 ? 12 : 9, F18 = EM > 9 ? 18 : 9;
        const double emax =
            rpe == 4    ? combine_err<BS, 4>(D, L.derr, L.derr2, Be.m, Be.beta, o.gamma, o.erc != 0)
            : rpe == 6  ? combine_err<BS, 6>(D, L.derr, L.derr2, Be.m, Be.beta, o.gamma, o.erc != 0)
            : rpe == 9  ? combine_err<BS, 9>(D, L.derr, L.derr2, Be.m, Be.beta, o.gamma, o.erc != 0)
            : rpe == 12 ? combine_err<BS, F12>(D, L.derr, L.derr2, Be.m, Be.beta, o.gamma, o.erc != 0)
                        : combine_err<BS, F18>(D, L.derr, L.derr2, Be.m, Be.beta, o.gamma, o.erc != 0);
        if (o.erc) wk.comb += Be.m;
        err = wg_max(L, emax);
      }
      pf.mark(5);
      if (replay || err <= o.E_rr) break;
      ++rej;
      h *= o.alpha;
      if (h < o.h_min) { status = kESTEPMIN; break; }
    }
    if (status != kOK) break;
    // ---- accept ----
    const double t_new = (land && rej == 0) ? t_land : t + h;
    for (int i = tid(); i < n; i += BS) gbl(D.xk)[i] = gbl(D.x1)[i];
    GMEM double *r = gbl(D.trace) + (int64_t)(steps - steps0) * rec;
    if (tid() == 0) {
      r[0] = t_new; r[1] = h; r[2] = h_unc; r[3] = Bm.m;
      r[4] = m_err; r[5] = rej; r[6] = err; r[7] = rho;
#pragma unroll
      for (int i = 0; i < kFeat; ++i) r[8 + i] = feat[i];
    }
    for (int q = tid(); q < D.n_probe; q += BS) r[kRecFixed + q] = gbl(D.x1)[gbl(D.probe)[q]];
    __syncthreads();
    const double grow = rej < o.grow_if_rejects_lt ? o.beta : 1.0;
    h_prop = fmin(D.h_max, grow * (rej == 0 ? h_prop : h));
    t = t_new;
    if (!replay)
      while (bp_idx < D.n_bp - 1 && gbl(D.bp)[bp_idx] <= t) ++bp_idx;
    rej_total += rej;
    ++steps;
    // the nominal size of this step: a first-try step clipped to a corner
    // counts with its unclipped size (as the paper's h_prop does)
    h_prev = (land && rej == 0) ? h_unc : h;
    rho_prev = rho;
    err_prev = err;
    m_prev = Bm.m;
    rej_prev = rej;
    m_err_prev = m_err;
  }
  if (tid() == 0) {
    S.t = t;
    S.h_prop = h_prop;
    S.bp_idx = bp_idx;
    S.steps = steps;
    S.lu_count = lu_count;
    S.rejects = rej_total;
    S.arnoldi = iters;
    S.lu_valid = lu_valid;
    S.h_prev = h_prev;
    S.rho_prev = rho_prev;
    S.err_prev = err_prev;
    S.m_prev = m_prev;
    S.rej_prev = rej_prev;
    S.m_err_prev = m_err_prev;
    S.trials += wk.trials;
    S.mgs_terms += wk.mgs;
    S.comb_terms += wk.comb;
#pragma unroll
    for (int i = 0; i < kPhases; ++i) S.ph[i] += (double)L.prof[i];
    if (status != kOK) {
      S.status = status;
      S.done = 1;
    }
  }
}

// The transient of one launch class: a grid of at most one workgroup per
// compute unit left to the class, each taking the next instance of the class's
// slice of the launch order (largest first) from the counter *next until the
// slice is exhausted, so that the classes launched together never wait for
// one another's compute units.  *next starts at 0; every workgroup leaves once
// the counter passes count.
// EM bounds the rows per thread (9, or 18 at 512 threads).  With EM = 9 the
// kernel is held to the registers of two workgroups per compute unit (two
// waves per SIMD at 256 threads, four at 512), so that a batch with more
// such instances than free compute units runs in one round; at 512 threads
// and EM = 18 it keeps one workgroup per compute unit.
template <int BS, int EM>
__global__ void __launch_bounds__(BS, BS == 256 ? 2 : (BS == 512 && EM > 9) ? 2 : 4) k_run(const InstDesc *descs, const int *order, int count, int *next,
                                            Opts o, int max_steps, int replay, int R, int NX) {
  Lds<BS> L = lds_setup<BS>(R, NX);
  for (;;) {
    // thread 0 takes a ticket; the workgroup maximum broadcasts it, and
    // readfirstlane tells the compiler it is uniform, so that the descriptor
    // is addressed (and its fields loaded) through scalar registers
    const double got = wg_max(L, tid() == 0 ? (double)atomicAdd(next, 1) : -1.0);
    const int idx = __builtin_amdgcn_readfirstlane((int)got);
    if (idx >= count) break;
    const int inst = __builtin_amdgcn_readfirstlane(order[idx]);
    run_instance<BS, EM>(descs[inst], L, o, max_steps, replay);
    __syncthreads();
  }
}

// next[i] = 0 for the launch classes' instance counters
__global__ void k_zero_counters(int *next, int n) {
  if ((int)threadIdx.x < n) next[threadIdx.x] = 0;
}

// DC operating point: Newton with the derivative couplings between DC blocks
// dropped (block Jacobi; the blocks form a DAG so it converges in at most
// #levels sweeps), updates clipped per node to vclip, until max|dx| <= 1e-9 V;
// then full Newton (uniformly damped to vclip) until max|dx| <= 1e-12 V.
template <int BS>
__global__ void __launch_bounds__(BS) k_dc(const InstDesc *descs, const int *order, Opts o, double t0,
                                           int max_it, int R, int NX) {
  const InstDesc &D = descs[order[blockIdx.x]];
  InstState &S = *D.state;
  Lds<BS> L = lds_setup<BS>(R, NX);
  double *xs = L.region;
  const int n = D.n;
  const double vclip = 0.3;
  int status = kOK;
  int its = 0;
  for (int phase = 0; phase < 2; ++phase) {
    const bool block = phase == 0;
    const double tol = block ? 1e-9 : 1e-12;
    bool conv = false;
    for (int it = 0; it < max_it; ++it, ++its) {
      stamp_devices<BS>(D, D.xk, D.devI, D.devD);
      __syncthreads();
      assemble<BS>(D, block);
      __syncthreads();
      if (!refactor<BS>(D, L, o.piv_tol)) { status = kESINGULAR; break; }
      for (int i = tid(); i < n; i += BS) {
        double bu = 0.0;
        for (int e = gbl(D.b_rowptr)[i]; e < gbl(D.b_rowptr)[i + 1]; ++e) bu += gbl(D.b_val)[e] * pwl_value(D, gbl(D.b_col)[e], t0);
        xs[i] = (bu - csr_row_dot(D.g_rowptr, D.g_col, D.g_val, D.xk, i)) - gbl(D.Ik)[i];
      }
      __syncthreads();
      solve_lds<BS>(D, xs);
      double big = 0.0;
      for (int i = tid(); i < n; i += BS) big = nmax(big, fabs(xs[i]));
      big = wg_max(L, big);
      if (!isfinite(big)) { status = kENONFINITE; break; }
      const double sc = (!block && big > vclip) ? vclip / big : 1.0;
      for (int i = tid(); i < n; i += BS) {
        const double dx = xs[i];
        gbl(D.xk)[i] += block ? fmin(fmax(dx, -vclip), vclip) : sc * dx;
      }
      __syncthreads();
      if (big <= tol) { conv = true; break; }
    }
    if (status != kOK) break;
    if (!conv) {
      status = kENOCONV;
      break;
    }
  }
  if (tid() == 0) {
    S.status = status;
    S.steps = its;
  }
}

// Test hooks ----------------------------------------------------------------

// stamp + assemble + refactor at x_k
template <int BS>
__global__ void __launch_bounds__(BS) k_factor(const InstDesc *descs, const int *order, Opts o, int R,
                                               int NX) {
  const InstDesc &D = descs[order[blockIdx.x]];
  Lds<BS> L = lds_setup<BS>(R, NX);
  stamp_devices<BS>(D, D.xk, D.devI, D.devD);
  __syncthreads();
  assemble<BS>(D, false);
  __syncthreads();
  const bool ok = refactor<BS>(D, L, o.piv_tol);
  if (tid() == 0) D.state->status = ok ? kOK : kESINGULAR;
}

// y = G_k^{-1} b with the current factors (caller numbering in and out)
template <int BS>
__global__ void __launch_bounds__(BS) k_solve(const InstDesc *descs, const int *order, const double *const *bin,
                                              double *const *yout, int R, int NX) {
  const int k = order[blockIdx.x];
  const InstDesc &D = descs[k];
  Lds<BS> L = lds_setup<BS>(R, NX);
  double *xs = L.region;
  for (int i = tid(); i < D.n; i += BS) xs[i] = bin[k][gbl(D.perm)[i]];
  __syncthreads();
  solve_lds<BS>(D, xs);
  for (int i = tid(); i < D.n; i += BS) yout[k][gbl(D.perm)[i]] = xs[i];
}

// out = (I - e^{hJ}) v by MEVP_IKS with the current factors; reports m, rho
template <int BS>
__global__ void __launch_bounds__(BS) k_mevp(const InstDesc *descs, const int *order, Opts o,
                                             const double *const *vin, double *const *out, double h, double eps,
                                             int R, int NX) {
  const int k = order[blockIdx.x];
  const InstDesc &D = descs[k];
  Lds<BS> L = lds_setup<BS>(R, NX);
  for (int i = tid(); i < D.n; i += BS) gbl(D.tmp)[i] = vin[k][gbl(D.perm)[i]];
  __syncthreads();
  Basis B;
  basis_start<BS>(D, L, D.tmp, D.V, B);
  double rho = 0.0;
  int iters = 0;
  Prof pf;
  pf.start(L.prof);
  Work wk{0, 0, 0};
  __syncthreads();
  const int st = mevp_converge<BS>(D, L, o, D.V, D.H, B, h, eps, L.dmain, rho, iters, pf, wk);
  for (int i = tid(); i < D.n; i += BS) {
    double acc = 0.0;
    for (int j = 0; j < B.m; ++j) acc += gbl(D.V)[(int64_t)j * D.ldv + i] * L.dmain[j];
    out[k][gbl(D.perm)[i]] = B.beta * acc;
  }
  if (tid() == 0) {
    D.state->status = st;
    D.state->arnoldi = B.m;
    D.state->t = rho;
    for (int i = 0; i < kPhases; ++i) D.state->ph[i] = (double)L.prof[i];
  }
}

// ---------------------------------------------------------------------------
// host-side launchers (internal C++ API used by the C-ABI layer)
// ---------------------------------------------------------------------------

// The small-matrix part of Algorithm 1 for an engine that keeps its
// Hessenberg matrix in global memory (the multifrontal engine of one large
// circuit): one workgroup evaluates hess_phi on H (column-major, leading
// dimension kHLd, with h_{m+1,m} stored below column m - 1, zero at a happy
// breakdown) at step size h and basis norm beta[0].  out[0..m) = d,
// out[kHLd..kHLd + m) = the phi_2 coefficients when want2, out[2 kHLd] = rho.
// mat: global scratch of 5 x 64 x 65 doubles for m + 2 > 32.
constexpr int kHessRD = 5 * 32 * 33;
__global__ void __launch_bounds__(256) k_hess_phi1(const double *H, int m, double h, const double *beta,
                                                   int want2, double *mat, double *out) {
  Lds<256> L = lds_setup<256>(kHessRD, 0);
  InstDesc D{};
  D.mat = mat;
  const double rho = hess_phi<256>(D, L, H, m, h, beta[0], H[m + (m - 1) * kHLd], L.dmain, want2 ? L.derr2 : nullptr);
  for (int i = tid(); i < m; i += 256) {
    gbl(out)[i] = L.dmain[i];
    if (want2) gbl(out)[kHLd + i] = L.derr2[i];
  }
  if (tid() == 0) gbl(out)[2 * kHLd] = rho;
}

#define EXPRI_DISPATCH(BS_, CALL)                 \
  switch (BS_) {                                  \
    case 256: { constexpr int BS = 256; CALL; } break; \
    case 512: { constexpr int BS = 512; CALL; } break; \
    default:  { constexpr int BS = 1024; CALL; } break; \
  }

size_t lds_bytes(int bs, int R) {
  // region, reduction slots, dmain, derr, 4 doubles (unused), kPhases
  // profile counters, hcol, derr2
  return sizeof(double) * ((size_t)R + 2 * (bs / 64) + 4 * kHLd + 4 + kPhases);
}

hipError_t set_lds_limits(size_t bytes) {
  hipError_t e = hipSuccess;
#define SETA(K) \
  if (e == hipSuccess) e = hipFuncSetAttribute(reinterpret_cast<const void *>(K), hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  SETA((k_run<256, 9>)) SETA((k_run<512, 9>)) SETA((k_run<512, 18>)) SETA((k_run<1024, 9>))
  SETA(k_dc<256>) SETA(k_dc<512>) SETA(k_dc<1024>)
  SETA(k_factor<256>) SETA(k_factor<512>) SETA(k_factor<1024>)
  SETA(k_solve<256>) SETA(k_solve<512>) SETA(k_solve<1024>)
  SETA(k_mevp<256>) SETA(k_mevp<512>) SETA(k_mevp<1024>)
#undef SETA
  return e;
}


// Diagnostic: times `reps` repetitions of one primitive on instance 0's data
// (what: 0 full solve, 1 L solve, 2 U solve, 3 C SpMV, 4 workgroup sum,
// 5 level loop with barriers only, 6 MGS step against 9 basis vectors).
// Writes wall-clock ticks to out[0].
template <int BS>
__global__ void __launch_bounds__(BS) k_diag(const InstDesc *descs, int what, int reps, int arg,
                                             long long *out, int R, int NX) {
  const InstDesc &D = descs[0];
  Lds<BS> L = lds_setup<BS>(R, NX);
  double *xs = L.region;
  const int n = D.n;
  // finite data in the vector area, the first arg + 2 basis columns and a
  // synthetic Hessenberg (diagonally dominant, entries of the size a circuit
  // gives: time constants of 0.1 ps and up)
  for (int i = tid(); i < n; i += BS) xs[i] = 1.0 / (1.0 + i);
  for (int c = 0; c < arg + 2 && c <= kMaxKrylov; ++c)
    for (int i = tid(); i < n; i += BS) gbl(D.V)[(int64_t)c * D.ldv + i] = (((i * 7 + c * 3) % 11) - 5) * 0.01;
  for (int idx = tid(); idx < kHLd * kMaxKrylov; idx += BS) {
    const int r = idx % kHLd, c = idx / kHLd;
    double v = 0.0;
    if (r == c) v = -1e-13 * (1.0 + 0.5 * r);
    else if (r == c + 1) v = 3e-14;
    else if (r < c) v = 1e-14 / (1 + c - r);
    gbl(D.He)[idx] = v;
  }
  __syncthreads();
  Prof pf;
  pf.start(L.prof);
  double acc = 0.0;
  const long long t0 = wall_clock64();
  for (int r = 0; r < reps; ++r) {
    if (what <= 2) {
      solve_lds<BS>(D, xs, what != 2, what != 1);
    } else if (what == 3) {
      Basis B{arg, 0, 1.0, 0.0};
      arnoldi_step<BS>(D, L, D.V, D.H, B, 0.0, pf);
    } else if (what == 4) {
      acc += wg_sum(L, acc + 1.0);
    } else if (what == 5) {
      for (int l = 0; l < D.n_lpass + D.n_upass; ++l) __syncthreads();
    } else if (what == 6) {
      acc += hess_phi<BS>(D, L, D.He, arg, 2e-12, 1.0, 1e-14, L.derr);
    } else if (what == 7) {
      assemble<BS>(D, false);
      __syncthreads();
      acc += refactor<BS>(D, L, 0.0) ? 1.0 : 0.0;
    } else if (what == 8) {
      assemble<BS>(D, false);
      __syncthreads();
    } else if (what == 9) {
      pack_slots<BS>(D);
    } else if (what == 10) {
      stamp_devices<BS>(D, D.xk, D.devI, D.devD);
      __syncthreads();
    } else if (what == 11) {
      acc += refactor<BS>(D, L, 0.0, arg) ? 1.0 : 0.0;  // the first arg levels, then the repacking
    }
  }
  const long long t1 = wall_clock64();
  if (tid() == 0) { out[0] = t1 - t0; out[1] = (long long)acc; }
}

hipError_t launch_diag(const InstDesc *d, int what, int reps, int arg, long long *out, int bs, int R, int NX,
                       hipStream_t s) {
  const size_t sh = lds_bytes(bs, R);
  EXPRI_DISPATCH(bs, {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_diag<BS>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_diag<BS>, dim3(1), dim3(BS), sh, s, d, what, reps, arg, out, R, NX);
  });
  return hipGetLastError();
}

hipError_t launch_begin(const InstDesc *d, int n_inst, const double *const *xin, double t0, double h0,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_begin, dim3(n_inst), dim3(256), 0, s, d, xin, t0, h0);
  return hipGetLastError();
}

hipError_t launch_init_workspace(const InstDesc *d, int n_inst, hipStream_t s) {
  hipLaunchKernelGGL(k_init_workspace, dim3(n_inst), dim3(256), 0, s, d);
  return hipGetLastError();
}

hipError_t launch_hess_phi1(const double *H, int m, double h, const double *beta, int want2, double *mat,
                            double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_hess_phi1, dim3(1), dim3(256), lds_bytes(256, kHessRD), s, H, m, h, beta, want2, mat, out);
  return hipGetLastError();
}

hipError_t launch_end(const InstDesc *d, int n_inst, double *const *xout, hipStream_t s) {
  hipLaunchKernelGGL(k_end, dim3(n_inst), dim3(256), 0, s, d, xout);
  return hipGetLastError();
}

hipError_t launch_run(const InstDesc *d, const int *order, int n_inst, int grid, int *next, const Opts &o,
                      int max_steps, int replay, int bs, int em, int R, int NX, hipStream_t s) {
  const size_t sh = lds_bytes(bs, R);
  if (bs == 512 && em > 9)
    hipLaunchKernelGGL((k_run<512, 18>), dim3(grid), dim3(512), sh, s, d, order, n_inst, next, o, max_steps, replay,
                       R, NX);
  else
    EXPRI_DISPATCH(bs, hipLaunchKernelGGL((k_run<BS, 9>), dim3(grid), dim3(BS), sh, s, d, order, n_inst, next, o,
                                          max_steps, replay, R, NX));
  return hipGetLastError();
}

hipError_t launch_zero_counters(int *next, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, s, next, n);
  return hipGetLastError();
}

hipError_t launch_dc(const InstDesc *d, const int *order, int n_inst, const Opts &o, double t0, int max_it,
                     int bs, int R, int NX, hipStream_t s) {
  const size_t sh = lds_bytes(bs, R);
  EXPRI_DISPATCH(bs, hipLaunchKernelGGL(k_dc<BS>, dim3(n_inst), dim3(BS), sh, s, d, order, o, t0, max_it, R, NX));
  return hipGetLastError();
}

hipError_t launch_factor(const InstDesc *d, const int *order, int n_inst, const Opts &o, int bs, int R, int NX,
                         hipStream_t s) {
  const size_t sh = lds_bytes(bs, R);
  EXPRI_DISPATCH(bs, hipLaunchKernelGGL(k_factor<BS>, dim3(n_inst), dim3(BS), sh, s, d, order, o, R, NX));
  return hipGetLastError();
}

hipError_t launch_solve(const InstDesc *d, const int *order, int n_inst, const double *const *b,
                        double *const *y, int bs, int R, int NX, hipStream_t s) {
  const size_t sh = lds_bytes(bs, R);
  EXPRI_DISPATCH(bs, hipLaunchKernelGGL(k_solve<BS>, dim3(n_inst), dim3(BS), sh, s, d, order, b, y, R, NX));
  return hipGetLastError();
}

hipError_t launch_mevp(const InstDesc *d, const int *order, int n_inst, const Opts &o, const double *const *v,
                       double *const *out, double h, double eps, int bs, int R, int NX, hipStream_t s) {
  const size_t sh = lds_bytes(bs, R);
  EXPRI_DISPATCH(bs, hipLaunchKernelGGL(k_mevp<BS>, dim3(n_inst), dim3(BS), sh, s, d, order, o, v, out, h, eps,
                                        R, NX));
  return hipGetLastError();
}

}  // namespace expri
