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

#include "layout.hpp"

namespace expri {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

// Wave-wide reductions on the DPP network: a butterfly inside each 16-lane
// row (pairs of lanes 1 and 2 apart, then the 8- and 16-lane mirrors), then
// the four row results read out in a fixed order.  Every lane ends with the
// bit-identical value.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141; // lane i <-> 7 - i in each 8 lanes
constexpr int kDppMirror = 0x140;     // lane i <-> 15 - i in each 16 lanes

__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_d<kDppXor1>(v);
  v += dpp_d<kDppXor2>(v);
  v += dpp_d<kDppHalfMirror>(v);
  v += dpp_d<kDppMirror>(v);
  return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

// max that propagates NaN
__device__ __forceinline__ double nmax(double a, double b) {
  return (isnan(a) || a > b) ? a : b;
}

__device__ __forceinline__ double wave_max(double v) {
  v = nmax(v, dpp_d<kDppXor1>(v));
  v = nmax(v, dpp_d<kDppXor2>(v));
  v = nmax(v, dpp_d<kDppHalfMirror>(v));
  v = nmax(v, dpp_d<kDppMirror>(v));
  return nmax(nmax(readlane_d(v, 0), readlane_d(v, 16)), nmax(readlane_d(v, 32), readlane_d(v, 48)));
}

// sum over aligned groups of G lanes (G a power of two <= 64); the group's
// lanes end with the same value
__device__ __forceinline__ double group_sum(double v, int G) {
  if (G >= 2) v += dpp_d<kDppXor1>(v);
  if (G >= 4) v += dpp_d<kDppXor2>(v);
  if (G >= 8) v += dpp_d<kDppHalfMirror>(v);
  if (G >= 16) v += dpp_d<kDppMirror>(v);
  if (G >= 32) v += __shfl_xor(v, 16, 64);
  if (G >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}

// LDS scratch layout (dynamic shared memory):
//   region : R doubles  -- solve vector, or small dense matrices
//   slots  : 2 * NW doubles -- reduction exchange (double buffered)
//   dmain, derr : kHLd doubles each -- small vectors d of the two MEVPs
//   ipiv   : 8 ints
template <int BS>
struct Lds {
  double *region;
  double *slots;
  double *dmain;
  double *derr;
  int *ipiv;   // 4 ints of pivot exchange
  double *bc;  // 1 double of broadcast from wave 0
  double *hcol; // kHLd doubles: current Hessenberg column
  long long *prof;  // kPhases phase counters
  int R;
  int par;
};

template <int BS>
__device__ __forceinline__ double wg_sum(Lds<BS> &L, double v) {
  v = wave_sum(v);
  double *s = L.slots + L.par * (BS / 64);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
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
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = s[0];
#pragma unroll
  for (int i = 1; i < BS / 64; ++i) r = nmax(r, s[i]);
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
  __device__ void start(long long *lds) {
    acc = lds;
    if (threadIdx.x < kPhases) acc[threadIdx.x] = 0;
    last = wall_clock64();
  }
  __device__ __forceinline__ void mark(int p) {
    const long long now = wall_clock64();
    if (threadIdx.x == 0) acc[p] += now - last;
    last = now;
  }
};

// ---------------------------------------------------------------------------
// level-1 MOSFET (Shichman-Hodges with channel-length modulation)
// I is the current into the drain terminal; derivatives w.r.t. V_d, V_g, V_s.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void mos_forward(double va, double vg, double vb, double K, double vth,
                                            double lam, double &f, double &fa, double &fg,
                                            double &fb) {
  const double vov = vg - vb - vth;
  const double vds = va - vb;
  f = 0.0; fa = 0.0; fg = 0.0; fb = 0.0;
  if (vov > 0.0) {
    const double q = 1.0 + lam * vds;
    double f_ov, f_ds;
    if (vds < vov) {
      const double P = vov * vds - 0.5 * vds * vds;
      f = K * P * q;
      f_ov = K * vds * q;
      f_ds = K * ((vov - vds) * q + P * lam);
    } else {
      f = 0.5 * K * vov * vov * q;
      f_ov = K * vov * q;
      f_ds = 0.5 * K * vov * vov * lam;
    }
    fa = f_ds;
    fg = f_ov;
    fb = -f_ov - f_ds;
  }
}

__device__ __forceinline__ void mos_eval(double type, double vd, double vg, double vs, double K,
                                         double vth, double lam, double &I, double &dd,
                                         double &dg, double &ds) {
  const double sg = type > 0.0 ? 1.0 : -1.0;   // PMOS = mirror image of NMOS
  vd *= sg; vg *= sg; vs *= sg;
  double f, fa, fg, fb;
  if (vd >= vs) {
    mos_forward(vd, vg, vs, K, vth, lam, f, fa, fg, fb);
    I = f; dd = fa; dg = fg; ds = fb;
  } else {
    mos_forward(vs, vg, vd, K, vth, lam, f, fa, fg, fb);
    I = -f; dd = -fb; dg = -fg; ds = -fa;
  }
  I *= sg;
}

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
  const int lo = D.src_ptr[src], hi = D.src_ptr[src + 1] - 1;
  if (t <= D.src_t[lo]) return D.src_v[lo];
  if (t >= D.src_t[hi]) return D.src_v[hi];
  const int i = pwl_seg(D.src_t, lo, hi, t);
  const double slope = (D.src_v[i + 1] - D.src_v[i]) / (D.src_t[i + 1] - D.src_t[i]);
  return D.src_v[i] + (t - D.src_t[i]) * slope;
}

__device__ __forceinline__ double pwl_slope(const InstDesc &D, int src, double tm) {
  const int lo = D.src_ptr[src], hi = D.src_ptr[src + 1] - 1;
  if (hi <= lo || tm < D.src_t[lo] || tm >= D.src_t[hi]) return 0.0;
  const int i = pwl_seg(D.src_t, lo, hi, tm);
  return (D.src_v[i + 1] - D.src_v[i]) / (D.src_t[i + 1] - D.src_t[i]);
}

// ---------------------------------------------------------------------------
// device stamp and G_k assembly
// ---------------------------------------------------------------------------

template <int BS>
__device__ void stamp_devices(const InstDesc &D, const double *x, double *devI, double *devD) {
  for (int k = threadIdx.x; k < D.n_dev; k += BS) {
    const int nd = D.dev_node[3 * k], ng = D.dev_node[3 * k + 1], ns = D.dev_node[3 * k + 2];
    const double *par = D.dev_par + 4 * k;
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
// dc_block is set) ;  Ik <- I_dev(x) per node
template <int BS>
__device__ void assemble(const InstDesc &D, bool dc_block) {
  for (int p = threadIdx.x; p < D.nnz_lu; p += BS) {
    const int gi = D.lu_gidx[p];
    double v = gi >= 0 ? D.g_val[gi] : 0.0;
    for (int c = D.jac_ptr[p]; c < D.jac_ptr[p + 1]; ++c) {
      const int code = D.jac_code[c];
      if (dc_block && ((code >> 3) & 1)) continue;
      const double dv = D.devD[3 * (code >> 4) + (code & 3)];
      v += ((code >> 2) & 1) ? -dv : dv;
    }
    D.lu[p] = v;
  }
  for (int i = threadIdx.x; i < D.n; i += BS) {
    double s = 0.0;
    for (int c = D.node_ptr[i]; c < D.node_ptr[i + 1]; ++c) {
      const int code = D.node_code[c];
      const double Iv = D.devI[code >> 1];
      s += (code & 1) ? -Iv : Iv;
    }
    D.Ik[i] = s;
  }
}

// numeric refactor of the L\U storage (row-wise Doolittle, static pivots).
// Returns false when a pivot is small: |u_ii| <= piv_tol * max_j |G_k(i, j)|.
template <int BS>
__device__ bool refactor(const InstDesc &D, Lds<BS> &L, double piv_tol) {
  double *a = D.lu;
  int bad = 0;
  for (int lv = 0; lv < D.n_lev; ++lv) {
    for (int q = D.lev_ptr[lv] + threadIdx.x; q < D.lev_ptr[lv + 1]; q += BS) {
      const int i = D.lev_rows[q];
      double rmax = 0.0;
      for (int p = D.lu_rowptr[i]; p < D.lu_rowptr[i + 1]; ++p) rmax = fmax(rmax, fabs(a[p]));
      for (int g = D.row_grp[i]; g < D.row_grp[i + 1]; ++g) {
        const int pik = D.grp_pos[g];
        const double l = a[pik] / a[D.grp_diag[g]];
        a[pik] = l;
        for (int u = D.grp_ptr[g]; u < D.grp_ptr[g + 1]; ++u) a[D.pair_dst[u]] -= l * a[D.pair_src[u]];
      }
      const double dii = a[D.lu_diag[i]];
      if (!(fabs(dii) > piv_tol * rmax)) bad = 1;
    }
    __syncthreads();
  }
  return wg_max(L, (double)bad) == 0.0;
}

// row-wise (CSR) level-scheduled solve: one thread per row
template <int BS>
__device__ void solve_lds_rows(const InstDesc &D, double *xs) {
  const double *a = D.lu;
  for (int lv = 0; lv < D.n_lev; ++lv) {
    for (int q = D.lev_ptr[lv] + threadIdx.x; q < D.lev_ptr[lv + 1]; q += BS) {
      const int i = D.lev_rows[q];
      double s = xs[i];
      for (int p = D.lu_rowptr[i]; p < D.lu_diag[i]; ++p) s -= a[p] * xs[D.lu_col[p]];
      xs[i] = s;
    }
    __syncthreads();
  }
  for (int lv = 0; lv < D.n_ulev; ++lv) {
    for (int q = D.ulev_ptr[lv] + threadIdx.x; q < D.ulev_ptr[lv + 1]; q += BS) {
      const int i = D.ulev_rows[q];
      double s = xs[i];
      const int dg = D.lu_diag[i];
      for (int p = dg + 1; p < D.lu_rowptr[i + 1]; ++p) s -= a[p] * xs[D.lu_col[p]];
      xs[i] = s / a[dg];
    }
    __syncthreads();
  }
}

// in-place solve G_k y = b with b (and then y) in LDS vector xs, following
// the flattened level schedules: on every level the rows are handled by
// groups of G lanes, lane t of the block reading slots (q P + j) BS + t of the
// level (coalesced index and position arrays; the L\U values are gathered);
// group partial sums meet in a butterfly over the group's lanes.
// one pass of one level: lane t multiplies its (at most kSlots) entries;
// every load is issued before the first product is formed
constexpr int kSlots = 8;
template <int BS>
__device__ __forceinline__ double level_pass(const double *__restrict__ a, const int *__restrict__ spos,
                                             const int *__restrict__ scol, const double *xs, int base,
                                             int P) {
  int pos[kSlots], col[kSlots];
#pragma unroll
  for (int j = 0; j < kSlots; ++j) {
    pos[j] = j < P ? spos[base + j * BS] : -1;
    col[j] = j < P ? scol[base + j * BS] : 0;
  }
  double av[kSlots], xv[kSlots];
#pragma unroll
  for (int j = 0; j < kSlots; ++j) {
    av[j] = pos[j] >= 0 ? a[pos[j]] : 0.0;
    xv[j] = pos[j] >= 0 ? xs[col[j]] : 0.0;
  }
  double acc = 0.0;
#pragma unroll
  for (int j = 0; j < kSlots; ++j) acc += av[j] * xv[j];
  return acc;
}

template <int BS>
__device__ void solve_lds(const InstDesc &D, double *xs, int variant = 0) {
  if (variant & 4) {
    solve_lds_rows<BS>(D, xs);
    return;
  }
  // descriptor fields in registers (a barrier would otherwise make the
  // compiler reload them from memory on every level)
  const double *__restrict__ a = D.lu;
  const SolveLevel *__restrict__ ls = D.lsched;
  const SolveLevel *__restrict__ us = D.usched;
  const int *__restrict__ spos = D.slot_pos;
  const int *__restrict__ scol = D.slot_col;
  const int *__restrict__ rowof = D.row_of;
  const int *__restrict__ diag = D.lu_diag;
  const int nl = D.n_lsched, nu = D.n_usched;
  const int t = threadIdx.x;
  for (int l = 0; l < nl; ++l) {
    const SolveLevel S = ls[l];
    for (int q = 0; q < S.passes; ++q) {
      double acc = level_pass<BS>(a, spos, scol, xs, S.slot_base + q * S.P * BS + t, S.P);
      acc = group_sum(acc, S.G);
      if ((t & (S.G - 1)) == 0) {
        const int r = rowof[S.row_base + q * (BS / S.G) + t / S.G];
        if (r >= 0) xs[r] -= acc;
      }
    }
    __syncthreads();
  }
  for (int l = 0; l < nu; ++l) {
    const SolveLevel S = us[l];
    for (int q = 0; q < S.passes; ++q) {
      const int ridx = S.row_base + q * (BS / S.G) + t / S.G;
      const int r = rowof[ridx];
      const double dv = r >= 0 ? a[diag[r]] : 1.0;
      double acc = level_pass<BS>(a, spos, scol, xs, S.slot_base + q * S.P * BS + t, S.P);
      acc = group_sum(acc, S.G);
      if ((t & (S.G - 1)) == 0 && r >= 0) xs[r] = (xs[r] - acc) / dv;
    }
    __syncthreads();
  }
}

// (C v)_i from the ELL copy of C (entries in the CSR order of the row)
__device__ __forceinline__ double c_row(const InstDesc &D, const double *v, int i) {
  double s = 0.0;
  for (int k = 0; k < D.c_ell_k; ++k) {
    const int c = D.c_ell_col[(int64_t)k * D.n + i];
    if (c >= 0) s += D.c_ell_val[(int64_t)k * D.n + i] * v[c];
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
// The same small-matrix algebra executed by one wave (wave 0) for
// n <= 32: lanes own matrix columns, matrices live in LDS, and a wavefront
// fence orders the LDS traffic between phases (a wave's LDS operations
// complete in order).  No workgroup barrier is needed inside.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void wfence() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

// Solve P X = Q (n x n, nrhs columns; LDS) by Gaussian elimination with
// partial pivoting (largest magnitude, first on ties); Q <- X.  Lane c owns
// the columns c, c + 64, ... of [P | Q].
__device__ void w_lu_solve(double *P, double *Q, int n, int nrhs, int lane) {
  const int ncol = n + nrhs;
  for (int k = 0; k < n; ++k) {
    wfence();
    int pr = k;
    double best = fabs(P[k * n + k]);
    for (int r = k + 1; r < n; ++r) {
      const double v = fabs(P[r * n + k]);
      if (v > best) { best = v; pr = r; }
    }
    if (pr != k)
      for (int c = lane; c < ncol; c += 64) {
        double *A = c < n ? P : Q;
        const int cc = c < n ? c : c - n, ld = c < n ? n : nrhs;
        const double t = A[k * ld + cc];
        A[k * ld + cc] = A[pr * ld + cc];
        A[pr * ld + cc] = t;
      }
    wfence();
    const double piv = P[k * n + k];
    for (int r = k + 1; r < n; ++r) {
      const double l = P[r * n + k] / piv;
      for (int c = lane; c < ncol; c += 64) {
        if (c < n) {
          if (c > k) P[r * n + c] -= l * P[k * n + c];
        } else {
          Q[r * nrhs + (c - n)] -= l * Q[k * nrhs + (c - n)];
        }
      }
    }
  }
  wfence();
  for (int c = lane; c < nrhs; c += 64)
    for (int r = n - 1; r >= 0; --r) {
      double sacc = Q[r * nrhs + c];
      for (int j = r + 1; j < n; ++j) sacc -= P[r * n + j] * Q[j * nrhs + c];
      Q[r * nrhs + c] = sacc / P[r * n + r];
    }
  wfence();
}

// Solve P X = Q for upper Hessenberg P (n x n, LDS): partial pivoting only
// ever compares rows k and k+1, so each elimination step touches one row.
__device__ void w_hess_solve(double *P, double *Q, int n, int nrhs, int lane) {
  const int ncol = n + nrhs;
  for (int k = 0; k + 1 < n; ++k) {
    wfence();
    const bool sw = fabs(P[(k + 1) * n + k]) > fabs(P[k * n + k]);
    if (sw)
      for (int c = lane; c < ncol; c += 64) {
        double *A = c < n ? P : Q;
        const int cc = c < n ? c : c - n, ld = c < n ? n : nrhs;
        const double t = A[k * ld + cc];
        A[k * ld + cc] = A[(k + 1) * ld + cc];
        A[(k + 1) * ld + cc] = t;
      }
    wfence();
    const double l = P[(k + 1) * n + k] / P[k * n + k];
    for (int c = lane; c < ncol; c += 64) {
      if (c < n) {
        if (c > k) P[(k + 1) * n + c] -= l * P[k * n + c];
      } else {
        Q[(k + 1) * nrhs + (c - n)] -= l * Q[k * nrhs + (c - n)];
      }
    }
  }
  wfence();
  for (int c = lane; c < nrhs; c += 64)
    for (int r = n - 1; r >= 0; --r) {
      double sacc = Q[r * nrhs + c];
      for (int j = r + 1; j < n; ++j) sacc -= P[r * n + j] * Q[j * nrhs + c];
      Q[r * nrhs + c] = sacc / P[r * n + r];
    }
  wfence();
}

// C = A B (n x n, n <= 32): lane -> column (lane & 31), half of the rows.
__device__ __forceinline__ void w_mat_mul(const double *A, const double *B, double *C, int n, int lane) {
  wfence();
  const int c = lane & 31, half = (n + 1) >> 1;
  const int r0 = (lane >> 5) ? half : 0, r1 = (lane >> 5) ? n : half;
  if (c < n)
    for (int r = r0; r < r1; ++r) {
      double sacc = 0.0;
      for (int k = 0; k < n; ++k) sacc += A[r * n + k] * B[k * n + c];
      C[r * n + c] = sacc;
    }
  wfence();
}

__device__ __forceinline__ double w_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = nmax(v, __shfl_xor(v, o, 64));
  return v;
}

// exp(A) by scaling and squaring with the degree-13 Pade approximant in one
// wave; buf holds 5 n x n matrices; returns the matrix holding exp(A).
__device__ double *w_expm_pade13(double *A, double *buf, int n, int lane) {
  const double b[14] = {64764752532480000.0, 32382376266240000.0, 7771770303897600.0,
                        1187353796428800.0,  129060195264000.0,   10559470521600.0,
                        670442572800.0,      33522128640.0,       1323241920.0,
                        40840800.0,          960960.0,            16380.0,
                        182.0,               1.0};
  const double theta13 = 5.371920351148152;
  const int nn = n * n;
  double *A2 = buf, *A4 = buf + nn, *A6 = buf + 2 * nn, *T1 = buf + 3 * nn, *T2 = buf + 4 * nn;
  wfence();
  double cs = 0.0;
  if (lane < n)
    for (int r = 0; r < n; ++r) cs += fabs(A[r * n + lane]);
  const double nrm = w_max(cs);
  int s = 0;
  if (nrm > theta13) s = (nrm < theta13 * 0x1p64) ? (int)ceil(log2(nrm / theta13)) : 64;
  if (s > 0) {
    const double sc = ldexp(1.0, -s);
    for (int i = lane; i < nn; i += 64) A[i] *= sc;
  }
  w_mat_mul(A, A, A2, n, lane);
  w_mat_mul(A2, A2, A4, n, lane);
  w_mat_mul(A4, A2, A6, n, lane);
  for (int i = lane; i < nn; i += 64) T1[i] = b[13] * A6[i] + b[11] * A4[i] + b[9] * A2[i];
  w_mat_mul(A6, T1, T2, n, lane);
  for (int i = lane; i < nn; i += 64) {
    const int r = i / n, c = i - r * n;
    T2[i] += b[7] * A6[i] + b[5] * A4[i] + b[3] * A2[i] + (r == c ? b[1] : 0.0);
  }
  w_mat_mul(A, T2, T1, n, lane);  // T1 = U
  for (int i = lane; i < nn; i += 64) T2[i] = b[12] * A6[i] + b[10] * A4[i] + b[8] * A2[i];
  w_mat_mul(A6, T2, A, n, lane);
  for (int i = lane; i < nn; i += 64) {
    const int r = i / n, c = i - r * n;
    const double V = A[i] + b[6] * A6[i] + b[4] * A4[i] + b[2] * A2[i] + (r == c ? b[0] : 0.0);
    A2[i] = V - T1[i];
    A4[i] = V + T1[i];
  }
  w_lu_solve(A2, A4, n, n, lane);
  double *X = A4, *Y = A6;
  for (int k = 0; k < s; ++k) {
    w_mat_mul(X, X, Y, n, lane);
    double *t = X; X = Y; Y = t;
  }
  return X;
}

// One-wave version of hess_phi for m + 1 <= 32 (R holds 7 (m+1)^2 doubles in
// LDS).  Wave 0 computes; the result is broadcast through LDS.
template <int BS>
__device__ double hess_phi_wave(Lds<BS> &L, const double *H, int m, double h, double beta,
                                double h_next, double *dout) {
  const int n1 = m + 1;
  double *M = L.region, *Aug = L.region + n1 * n1, *buf = L.region + 2 * n1 * n1;
  double *bcast = L.bc;
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    double *P = Aug;
    if (lane < m)
      for (int r = 0; r < m; ++r) {
        P[r * m + lane] = (r <= lane + 1) ? H[r + lane * kHLd] : 0.0;
        M[r * m + lane] = (r == lane) ? h : 0.0;
      }
    w_lu_solve(P, M, m, m, lane);  // M = h H^{-1}
    double bad = 0.0;
    for (int i = lane; i < m * m; i += 64)
      if (!isfinite(M[i])) bad = 1.0;
    double rho = INFINITY;
    if (w_max(bad) == 0.0) {
      for (int i = lane; i < n1 * n1; i += 64) {
        const int r = i / n1, c = i - r * n1;
        double v = 0.0;
        if (r < m && c < m) v = M[r * m + c];
        else if (r == 0 && c == m) v = 1.0;
        Aug[i] = v;
      }
      const double *E = w_expm_pade13(Aug, buf, n1, lane);
      double part = 0.0;
      bad = 0.0;
      if (lane < m) {
        double sacc = 0.0;
        for (int c = 0; c < m; ++c) sacc += M[lane * m + c] * E[c * n1 + m];
        dout[lane] = -sacc;
        if (!isfinite(sacc)) bad = 1.0;
        part = M[(m - 1) * m + lane] * E[lane * n1];
      }
      const double my = wave_sum(part);
      rho = beta * h_next * fabs(my / h);
      if (w_max(bad) != 0.0 || !isfinite(rho)) rho = INFINITY;
    }
    if (lane == 0) bcast[0] = rho;
  }
  __syncthreads();
  const double rho = bcast[0];
  __syncthreads();
  return rho;
}

// ---------------------------------------------------------------------------
// small dense linear algebra for the Hessenberg exponential (row-major, ld n)
// ---------------------------------------------------------------------------

template <int BS>
__device__ void mat_mul(const double *A, const double *B, double *C, int n) {
  for (int idx = threadIdx.x; idx < n * n; idx += BS) {
    const int r = idx / n, c = idx - r * n;
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += A[r * n + k] * B[k * n + c];
    C[idx] = s;
  }
  __syncthreads();
}

// solve P X = Q (n x n, nrhs columns) by LU with partial pivoting (largest
// magnitude, first on ties); Q is overwritten by X, P is destroyed.
template <int BS>
__device__ void lu_solve(Lds<BS> &L, double *P, double *Q, int n, int nrhs) {
  for (int k = 0; k < n; ++k) {
    if (threadIdx.x < 64) {
      const int r = k + (int)threadIdx.x;
      double v = r < n ? fabs(P[r * n + k]) : -1.0;
      int id = r < n ? r : 0x7fffffff;
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        const double ov = __shfl_xor(v, o, 64);
        const int oid = __shfl_xor(id, o, 64);
        if (ov > v || (ov == v && oid < id)) { v = ov; id = oid; }
      }
      if (threadIdx.x == 0) L.ipiv[0] = (id < n) ? id : k;
    }
    __syncthreads();
    const int pr = L.ipiv[0];
    if (pr != k) {
      for (int c = threadIdx.x; c < n + nrhs; c += BS) {
        double *A = c < n ? P : Q;
        const int cc = c < n ? c : c - n, ld = c < n ? n : nrhs;
        const double t0 = A[k * ld + cc];
        A[k * ld + cc] = A[pr * ld + cc];
        A[pr * ld + cc] = t0;
      }
      __syncthreads();
    }
    const double piv = P[k * n + k];
    const int w = (n - k - 1) + nrhs;
    const int rows = n - k - 1;
    for (int idx = threadIdx.x; idx < rows * w; idx += BS) {
      const int r = k + 1 + idx / w, c = idx % w;
      const double l = P[r * n + k] / piv;
      if (c < n - k - 1) P[r * n + (k + 1 + c)] -= l * P[k * n + (k + 1 + c)];
      else Q[r * nrhs + (c - (n - k - 1))] -= l * Q[k * nrhs + (c - (n - k - 1))];
    }
    __syncthreads();
  }
  for (int c = threadIdx.x; c < nrhs; c += BS) {
    for (int r = n - 1; r >= 0; --r) {
      double s = Q[r * nrhs + c];
      for (int j = r + 1; j < n; ++j) s -= P[r * n + j] * Q[j * nrhs + c];
      Q[r * nrhs + c] = s / P[r * n + r];
    }
  }
  __syncthreads();
}

// E = exp(A) by scaling and squaring with the degree-13 Pade approximant
// (Higham, SIAM J. Matrix Anal. Appl. 26(4), 2005).  buf holds 6 n x n
// matrices; A is destroyed; returns the matrix holding exp(A).
template <int BS>
__device__ double *expm_pade13(Lds<BS> &L, double *A, double *buf, int n, bool in_lds) {
  const double b[14] = {64764752532480000.0, 32382376266240000.0, 7771770303897600.0,
                        1187353796428800.0,  129060195264000.0,   10559470521600.0,
                        670442572800.0,      33522128640.0,       1323241920.0,
                        40840800.0,          960960.0,            16380.0,
                        182.0,               1.0};
  const double theta13 = 5.371920351148152;
  const int nn = n * n;
  double *A2 = buf, *A4 = buf + nn, *A6 = buf + 2 * nn, *T1 = buf + 3 * nn, *T2 = buf + 4 * nn;
  // 1-norm
  double cs = 0.0;
  for (int c = threadIdx.x; c < n; c += BS) {
    double s = 0.0;
    for (int r = 0; r < n; ++r) s += fabs(A[r * n + c]);
    cs = nmax(cs, s);
  }
  const double nrm = wg_max(L, cs);
  // 2^64 theta13 ~ 1e20: beyond that every entry of exp(A) under- or
  // overflows anyway, and a non-finite norm is caught by the caller
  int s = 0;
  if (nrm > theta13) s = (nrm < theta13 * 0x1p64) ? (int)ceil(log2(nrm / theta13)) : 64;
  if (s > 0) {
    const double sc = ldexp(1.0, -s);
    for (int i = threadIdx.x; i < nn; i += BS) A[i] *= sc;
    __syncthreads();
  }
  mat_mul<BS>(A, A, A2, n);
  mat_mul<BS>(A2, A2, A4, n);
  mat_mul<BS>(A4, A2, A6, n);
  for (int i = threadIdx.x; i < nn; i += BS) T1[i] = b[13] * A6[i] + b[11] * A4[i] + b[9] * A2[i];
  __syncthreads();
  mat_mul<BS>(A6, T1, T2, n);
  for (int i = threadIdx.x; i < nn; i += BS) {
    const int r = i / n, c = i - r * n;
    T2[i] += b[7] * A6[i] + b[5] * A4[i] + b[3] * A2[i] + (r == c ? b[1] : 0.0);
  }
  __syncthreads();
  mat_mul<BS>(A, T2, T1, n);  // T1 = U
  for (int i = threadIdx.x; i < nn; i += BS) T2[i] = b[12] * A6[i] + b[10] * A4[i] + b[8] * A2[i];
  __syncthreads();
  mat_mul<BS>(A6, T2, A, n);  // A = A6 * (...)
  for (int i = threadIdx.x; i < nn; i += BS) {
    const int r = i / n, c = i - r * n;
    const double V = A[i] + b[6] * A6[i] + b[4] * A4[i] + b[2] * A2[i] + (r == c ? b[0] : 0.0);
    A2[i] = V - T1[i];  // P = V - U
    A4[i] = V + T1[i];  // Q = V + U
  }
  __syncthreads();
  if (in_lds) {  // one wave eliminates: no barrier per pivot step
    if (threadIdx.x < 64) w_lu_solve(A2, A4, n, n, threadIdx.x);
    __syncthreads();
  } else {
    lu_solve<BS>(L, A2, A4, n, n);
  }
  double *X = A4, *Y = A6;
  for (int k = 0; k < s; ++k) {
    mat_mul<BS>(X, X, Y, n);
    double *t = X; X = Y; Y = t;
  }
  return X;
}

// Small-matrix part of the MEVP at step h (see hessenberg_phi in the design
// notes): M = h H_m^{-1}; E = exp([[M, e1], [0, 0]]); y = E[:m, 0],
// f = E[:m, m]; d = -M f = (I - e^M) e1; rho = beta h_{m+1,m} |(H_m^{-1} y)_m|.
// d goes to dout (LDS, m doubles).  Returns rho (inf if anything is not finite).
template <int BS>
__device__ double hess_phi(const InstDesc &D, Lds<BS> &L, const double *H, int m, double h,
                           double beta, double h_next, double *dout) {
  const int n1 = m + 1;
  if ((D.variant & 1) && n1 <= 32 && 7 * n1 * n1 <= L.R)
    return hess_phi_wave<BS>(L, H, m, h, beta, h_next, dout);
  // 7 matrices of n1 x n1: M, Aug, and 5 work matrices (A2, A4, A6, T1, T2)
  const bool in_lds = 7 * n1 * n1 <= L.R;
  double *R = in_lds ? L.region : D.mat;
  double *M = R, *Aug = R + n1 * n1, *buf = R + 2 * n1 * n1;
  double *P = Aug;  // H_m copy (m x m) for the inverse, before Aug is built
  for (int i = threadIdx.x; i < m * m; i += BS) {
    const int r = i / m, c = i - r * m;
    P[i] = (r <= c + 1) ? H[r + c * kHLd] : 0.0;  // upper Hessenberg: only these are stored
    M[i] = (r == c) ? h : 0.0;
  }
  __syncthreads();
  if (in_lds) {  // M = h H^{-1}, one wave, Hessenberg elimination
    if (threadIdx.x < 64) w_hess_solve(P, M, m, m, threadIdx.x);
    __syncthreads();
  } else {
    lu_solve<BS>(L, P, M, m, m);
  }
  double mbad = 0.0;
  for (int i = threadIdx.x; i < m * m; i += BS)
    if (!isfinite(M[i])) mbad = 1.0;
  if (wg_max(L, mbad) != 0.0) return INFINITY;  // H_m singular: not converged
  for (int i = threadIdx.x; i < n1 * n1; i += BS) {
    const int r = i / n1, c = i - r * n1;
    double v = 0.0;
    if (r < m && c < m) v = M[r * m + c];
    else if (r == 0 && c == m) v = 1.0;
    Aug[i] = v;
  }
  __syncthreads();
  const double *E = expm_pade13<BS>(L, Aug, buf, n1, in_lds);
  // d = -M f  with f = E[:m, m]
  for (int r = threadIdx.x; r < m; r += BS) {
    double s = 0.0;
    for (int c = 0; c < m; ++c) s += M[r * m + c] * E[c * n1 + m];
    dout[r] = -s;
  }
  // (M y)_{m-1} with y = E[:m, 0]
  double part = 0.0, bad = 0.0;
  for (int c = threadIdx.x; c < m; c += BS) part += M[(m - 1) * m + c] * E[c * n1];
  for (int r = threadIdx.x; r < m; r += BS)
    if (!isfinite(dout[r])) bad = 1.0;
  const double my = wg_sum(L, part);
  const double anybad = wg_max(L, bad);
  double rho = beta * h_next * fabs(my / h);
  if (anybad != 0.0 || !isfinite(rho)) rho = INFINITY;
  return rho;
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

// one Arnoldi step j = B.m: solve -G w = C v_j, MGS against v_0..v_j,
// h_{j+1,j} = ||w||, v_{j+1} = w / h_{j+1,j}
template <int BS>
__device__ void arnoldi_step(const InstDesc &D, Lds<BS> &L, double *V, double *H, Basis &B,
                             double breakdown, Prof &pf) {
  const int n = D.n, j = B.m;
  const int64_t ldv = D.ldv;
  double *xs = L.region;
  double *hcol = L.hcol;  // this step's Hessenberg column, stored to H once at the end
  const double *vj = V + (int64_t)j * ldv;
  for (int i = threadIdx.x; i < n; i += BS) xs[i] = -c_row(D, vj, i);
  __syncthreads();
  solve_lds<BS>(D, xs, D.variant);
  pf.mark(2);
  constexpr int E = (4608 + BS - 1) / BS;  // elements per thread in registers (n <= E * BS)
  const int t0 = threadIdx.x;
  if (!(D.variant & 2) && n <= E * BS) {
    // modified Gram-Schmidt with v_i held in registers for its inner
    // product and its update, and v_{i+1} loaded before the reduction
    double cur[E], nxt[E];
#pragma unroll
    for (int e = 0; e < E; ++e) cur[e] = (t0 + e * BS < n) ? V[t0 + e * BS] : 0.0;
    for (int i = 0; i <= j; ++i) {
      double part = 0.0;
#pragma unroll
      for (int e = 0; e < E; ++e)
        if (t0 + e * BS < n) part += xs[t0 + e * BS] * cur[e];
      if (i < j) {
        const double *vn = V + (int64_t)(i + 1) * ldv;
#pragma unroll
        for (int e = 0; e < E; ++e) nxt[e] = (t0 + e * BS < n) ? vn[t0 + e * BS] : 0.0;
      }
      const double hij = wg_sum(L, part);
#pragma unroll
      for (int e = 0; e < E; ++e)
        if (t0 + e * BS < n) xs[t0 + e * BS] -= hij * cur[e];
      if (t0 == 0) hcol[i] = hij;
      B.hscale = nmax(B.hscale, fabs(hij));
#pragma unroll
      for (int e = 0; e < E; ++e) cur[e] = nxt[e];
    }
  } else {
    for (int i = 0; i <= j; ++i) {
      const double *vi = V + (int64_t)i * ldv;
      double part = 0.0;
      for (int t = t0; t < n; t += BS) part += xs[t] * vi[t];
      const double hij = wg_sum(L, part);
      for (int t = t0; t < n; t += BS) xs[t] -= hij * vi[t];
      if (t0 == 0) hcol[i] = hij;
      B.hscale = nmax(B.hscale, fabs(hij));
    }
  }
  double part = 0.0;
  for (int t = t0; t < n; t += BS) part += xs[t] * xs[t];
  const double hn = sqrt(wg_sum(L, part));
  B.hscale = nmax(B.hscale, hn);
  B.m = j + 1;
  const bool brk = hn <= breakdown * B.hscale;
  if (brk) B.exact = 1;
  if (!brk) {
    double *vn = V + (int64_t)(j + 1) * ldv;
    for (int t = t0; t < n; t += BS) vn[t] = xs[t] / hn;
  }
  for (int i = t0; i <= j; i += BS) H[i + j * kHLd] = hcol[i];
  if (t0 == 0) H[j + 1 + j * kHLd] = brk ? 0.0 : hn;
  __syncthreads();
  pf.mark(3);
}

// Start a basis from the vector in LDS xs: beta = ||v||, v_0 = v / beta.
template <int BS>
__device__ void basis_start(const InstDesc &D, Lds<BS> &L, const double *v, double *V, Basis &B) {
  double part = 0.0;
  for (int t = threadIdx.x; t < D.n; t += BS) part += v[t] * v[t];
  B.beta = sqrt(wg_sum(L, part));
  B.m = 0;
  B.exact = B.beta == 0.0;
  B.hscale = 0.0;
  if (B.beta > 0.0)
    for (int t = threadIdx.x; t < D.n; t += BS) V[t] = v[t] / B.beta;
  __syncthreads();
}

// grow the basis until rho_m(h) <= eps; d -> dout.  Returns a status code.
template <int BS>
__device__ int mevp_converge(const InstDesc &D, Lds<BS> &L, const Opts &o, double *V, double *H,
                             Basis &B, double h, double eps, double *dout, double &rho,
                             int &iters, Prof &pf, Work &wk) {
  if (B.beta == 0.0) {
    rho = 0.0;
    return kOK;
  }
  if (B.m > 0) {
    rho = hess_phi<BS>(D, L, H, B.m, h, B.beta, B.exact ? 0.0 : H[B.m + (B.m - 1) * kHLd], dout);
    pf.mark(4);
    if (rho <= eps) return kOK;
    if (B.exact) return kEKRYLOV;
  }
  for (;;) {
    if (B.m >= o.m_max) return kEKRYLOV;
    arnoldi_step<BS>(D, L, V, H, B, o.breakdown, pf);
    ++iters;
    wk.mgs += B.m;
    rho = hess_phi<BS>(D, L, H, B.m, h, B.beta, B.exact ? 0.0 : H[B.m + (B.m - 1) * kHLd], dout);
    pf.mark(4);
    if (rho <= eps) return kOK;
    if (B.exact) return kEKRYLOV;
  }
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

template <int BS>
__device__ Lds<BS> lds_setup(int R) {
  extern __shared__ double smem[];
  Lds<BS> L;
  L.region = smem;
  L.slots = smem + R;
  L.dmain = L.slots + 2 * (BS / 64);
  L.derr = L.dmain + kHLd;
  L.ipiv = reinterpret_cast<int *>(L.derr + kHLd);
  L.bc = L.derr + kHLd + 2;
  L.prof = reinterpret_cast<long long *>(L.derr + kHLd + 4);
  L.hcol = L.derr + kHLd + 4 + kPhases;
  L.R = R;
  L.par = 0;
  return L;
}

// Load the caller's state x (caller numbering) into x_k and reset the run state.
__global__ void k_begin(const InstDesc *descs, const double *const *xin, double t0, double h0) {
  const InstDesc &D = descs[blockIdx.x];
  const double *x = xin[blockIdx.x];
  for (int i = threadIdx.x; i < D.n; i += blockDim.x) D.xk[i] = x[D.perm[i]];
  if (threadIdx.x == 0) {
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
    int b = 0;
    while (b < D.n_bp - 1 && D.bp[b] <= t0) ++b;
    S.bp_idx = b;
  }
}

// Write x_k back in the caller's numbering.
__global__ void k_end(const InstDesc *descs, double *const *xout) {
  const InstDesc &D = descs[blockIdx.x];
  double *x = xout[blockIdx.x];
  for (int i = threadIdx.x; i < D.n; i += blockDim.x) x[D.perm[i]] = D.xk[i];
}

// The ER transient (Algorithm 2), resumable: runs at most max_steps accepted
// steps of every unfinished instance.  replay != 0: the step ends are taken
// from D.bp (the given grid) and every first trial is accepted.
template <int BS>
__global__ void __launch_bounds__(BS) k_run(const InstDesc *descs, const int *order, Opts o,
                                            int max_steps, int replay, int R) {
  // workgroups start in blockIdx order: order[] lists the largest instances first
  const InstDesc &D = descs[order[blockIdx.x]];
  InstState &S = *D.state;
  if (S.done) return;
  Lds<BS> L = lds_setup<BS>(R);
  double *xs = L.region;
  const int n = D.n;
  double t = S.t, h_prop = S.h_prop;
  int bp_idx = S.bp_idx, steps = S.steps, status = kOK;
  int lu_count = S.lu_count, rej_total = S.rejects, iters = S.arnoldi;
  int lu_valid = S.lu_valid;
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
    if (replay) {
      t_land = D.bp[steps];
      h_try = t_land - t;
      land = true;
    } else {
      t_land = D.bp[bp_idx];
      h_try = fmin(h_prop, D.h_max);
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
    // ---- w = G^{-1} r,  r = B u(t) - G_lin x_k - I_dev(x_k) ----
    for (int i = threadIdx.x; i < n; i += BS) {
      double bu = 0.0;
      for (int e = D.b_rowptr[i]; e < D.b_rowptr[i + 1]; ++e) bu += D.b_val[e] * pwl_value(D, D.b_col[e], t);
      xs[i] = (bu - csr_row_dot(D.g_rowptr, D.g_col, D.g_val, D.xk, i)) - D.Ik[i];
    }
    __syncthreads();
    solve_lds<BS>(D, xs);
    for (int i = threadIdx.x; i < n; i += BS) D.w[i] = xs[i];
    // ---- p = G^{-1} B s ----
    const double tm = t + 0.5 * h_try;
    for (int i = threadIdx.x; i < n; i += BS) {
      double bs = 0.0;
      for (int e = D.b_rowptr[i]; e < D.b_rowptr[i + 1]; ++e) bs += D.b_val[e] * pwl_slope(D, D.b_col[e], tm);
      xs[i] = bs;
    }
    __syncthreads();
    solve_lds<BS>(D, xs);
    for (int i = threadIdx.x; i < n; i += BS) D.p[i] = xs[i];
    __syncthreads();
    // ---- z = G^{-1} C p ;  v = w - z ----
    for (int i = threadIdx.x; i < n; i += BS) xs[i] = c_row(D, D.p, i);
    __syncthreads();
    solve_lds<BS>(D, xs);
    for (int i = threadIdx.x; i < n; i += BS) D.tmp[i] = D.w[i] - xs[i];
    __syncthreads();
    Basis Bm;
    basis_start<BS>(D, L, D.tmp, D.V, Bm);
    pf.mark(1);
    // ---- trial loop ----
    double h = h_try, rho = 0.0, err = 0.0;
    int rej = 0, m_err = 0;
    for (;;) {
      ++wk.trials;
      status = mevp_converge<BS>(D, L, o, D.V, D.H, Bm, h, o.eps_K, L.dmain, rho, iters, pf, wk);
      if (status != kOK) break;
      wk.comb += Bm.m;
      // x_{k+1} = x_k + h p + beta V_m d
      double bad = 0.0;
      for (int i = threadIdx.x; i < n; i += BS) {
        double acc = 0.0;
        for (int j = 0; j < Bm.m; ++j) acc += D.V[(int64_t)j * D.ldv + i] * L.dmain[j];
        const double v = (D.xk[i] + h * D.p[i]) + Bm.beta * acc;
        D.x1[i] = v;
        if (!isfinite(v)) bad = 1.0;
      }
      if (wg_max(L, bad) != 0.0) { status = kENONFINITE; break; }
      err = 0.0;
      m_err = 0;
      if (D.has_dev) {
        stamp_devices<BS>(D, D.x1, D.devI1, nullptr);
        __syncthreads();
        // dF = J_dev(x_k)(x_{k+1} - x_k) - (I_dev(x_{k+1}) - I_dev(x_k))
        for (int i = threadIdx.x; i < n; i += BS) {
          double s = 0.0;
          for (int c = D.node_ptr[i]; c < D.node_ptr[i + 1]; ++c) {
            const int code = D.node_code[c], k = code >> 1;
            double lin = 0.0;
            for (int v = 0; v < 3; ++v) {
              const int nd = D.dev_node[3 * k + v];
              if (nd >= 0) lin += D.devD[3 * k + v] * (D.x1[nd] - D.xk[nd]);
            }
            const double df = lin - (D.devI1[k] - D.devI[k]);
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
        status = mevp_converge<BS>(D, L, o, D.Ve, D.He, Be, h, o.eps_K, L.derr, rho_e, iters, pf, wk);
        if (status != kOK) break;
        m_err = Be.m;
        wk.comb += Be.m;
        double emax = 0.0;
        for (int i = threadIdx.x; i < n; i += BS) {
          double acc = 0.0;
          for (int j = 0; j < Be.m; ++j) acc += D.Ve[(int64_t)j * D.ldv + i] * L.derr[j];
          emax = nmax(emax, fabs(Be.beta * acc));
        }
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
    for (int i = threadIdx.x; i < n; i += BS) D.xk[i] = D.x1[i];
    double *r = D.trace + (int64_t)(steps - steps0) * rec;
    if (threadIdx.x == 0) {
      r[0] = t_new; r[1] = h; r[2] = h_try; r[3] = Bm.m;
      r[4] = m_err; r[5] = rej; r[6] = err; r[7] = rho;
    }
    for (int q = threadIdx.x; q < D.n_probe; q += BS) r[kRecFixed + q] = D.x1[D.probe[q]];
    __syncthreads();
    const double grow = rej < o.grow_if_rejects_lt ? o.beta : 1.0;
    h_prop = fmin(D.h_max, grow * (rej == 0 ? h_prop : h));
    t = t_new;
    if (!replay)
      while (bp_idx < D.n_bp - 1 && D.bp[bp_idx] <= t) ++bp_idx;
    rej_total += rej;
    ++steps;
  }
  if (threadIdx.x == 0) {
    S.t = t;
    S.h_prop = h_prop;
    S.bp_idx = bp_idx;
    S.steps = steps;
    S.lu_count = lu_count;
    S.rejects = rej_total;
    S.arnoldi = iters;
    S.lu_valid = lu_valid;
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

// DC operating point: Newton with the derivative couplings between DC blocks
// dropped (block Jacobi; the blocks form a DAG so it converges in at most
// #levels sweeps), updates clipped per node to vclip, until max|dx| <= 1e-9 V;
// then full Newton (uniformly damped to vclip) until max|dx| <= 1e-12 V.
template <int BS>
__global__ void __launch_bounds__(BS) k_dc(const InstDesc *descs, Opts o, double t0, int max_it,
                                           int R) {
  const InstDesc &D = descs[blockIdx.x];
  InstState &S = *D.state;
  Lds<BS> L = lds_setup<BS>(R);
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
      for (int i = threadIdx.x; i < n; i += BS) {
        double bu = 0.0;
        for (int e = D.b_rowptr[i]; e < D.b_rowptr[i + 1]; ++e) bu += D.b_val[e] * pwl_value(D, D.b_col[e], t0);
        xs[i] = (bu - csr_row_dot(D.g_rowptr, D.g_col, D.g_val, D.xk, i)) - D.Ik[i];
      }
      __syncthreads();
      solve_lds<BS>(D, xs);
      double big = 0.0;
      for (int i = threadIdx.x; i < n; i += BS) big = nmax(big, fabs(xs[i]));
      big = wg_max(L, big);
      if (!isfinite(big)) { status = kENONFINITE; break; }
      const double sc = (!block && big > vclip) ? vclip / big : 1.0;
      for (int i = threadIdx.x; i < n; i += BS) {
        const double dx = xs[i];
        D.xk[i] += block ? fmin(fmax(dx, -vclip), vclip) : sc * dx;
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
  if (threadIdx.x == 0) {
    S.status = status;
    S.steps = its;
  }
}

// Test hooks ----------------------------------------------------------------

// stamp + assemble + refactor at x_k
template <int BS>
__global__ void __launch_bounds__(BS) k_factor(const InstDesc *descs, Opts o, int R) {
  const InstDesc &D = descs[blockIdx.x];
  Lds<BS> L = lds_setup<BS>(R);
  stamp_devices<BS>(D, D.xk, D.devI, D.devD);
  __syncthreads();
  assemble<BS>(D, false);
  __syncthreads();
  const bool ok = refactor<BS>(D, L, o.piv_tol);
  if (threadIdx.x == 0) D.state->status = ok ? kOK : kESINGULAR;
}

// y = G_k^{-1} b with the current factors (caller numbering in and out)
template <int BS>
__global__ void __launch_bounds__(BS) k_solve(const InstDesc *descs, const double *const *bin,
                                              double *const *yout, int R) {
  const InstDesc &D = descs[blockIdx.x];
  Lds<BS> L = lds_setup<BS>(R);
  double *xs = L.region;
  for (int i = threadIdx.x; i < D.n; i += BS) xs[i] = bin[blockIdx.x][D.perm[i]];
  __syncthreads();
  solve_lds<BS>(D, xs);
  for (int i = threadIdx.x; i < D.n; i += BS) yout[blockIdx.x][D.perm[i]] = xs[i];
}

// out = (I - e^{hJ}) v by MEVP_IKS with the current factors; reports m, rho
template <int BS>
__global__ void __launch_bounds__(BS) k_mevp(const InstDesc *descs, Opts o, const double *const *vin,
                                             double *const *out, double h, double eps, int R) {
  const InstDesc &D = descs[blockIdx.x];
  Lds<BS> L = lds_setup<BS>(R);
  for (int i = threadIdx.x; i < D.n; i += BS) D.tmp[i] = vin[blockIdx.x][D.perm[i]];
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
  for (int i = threadIdx.x; i < D.n; i += BS) {
    double acc = 0.0;
    for (int j = 0; j < B.m; ++j) acc += D.V[(int64_t)j * D.ldv + i] * L.dmain[j];
    out[blockIdx.x][D.perm[i]] = B.beta * acc;
  }
  if (threadIdx.x == 0) {
    D.state->status = st;
    D.state->arnoldi = B.m;
    D.state->t = rho;
    for (int i = 0; i < kPhases; ++i) D.state->ph[i] = (double)L.prof[i];
  }
}

// ---------------------------------------------------------------------------
// host-side launchers (internal C++ API used by the C-ABI layer)
// ---------------------------------------------------------------------------

#define EXPRI_DISPATCH(BS_, CALL)                 \
  switch (BS_) {                                  \
    case 256: { constexpr int BS = 256; CALL; } break; \
    case 512: { constexpr int BS = 512; CALL; } break; \
    default:  { constexpr int BS = 1024; CALL; } break; \
  }

size_t lds_bytes(int bs, int R) {
  // region, reduction slots, dmain, derr, then 4 doubles (pivot ints,
  // broadcast) and kPhases profile counters
  return sizeof(double) * ((size_t)R + 2 * (bs / 64) + 3 * kHLd + 4 + kPhases);
}

hipError_t set_lds_limits(size_t bytes) {
  hipError_t e = hipSuccess;
#define SETA(K) \
  if (e == hipSuccess) e = hipFuncSetAttribute(reinterpret_cast<const void *>(K), hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  SETA(k_run<256>) SETA(k_run<512>) SETA(k_run<1024>)
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
__global__ void __launch_bounds__(BS) k_diag(const InstDesc *descs, int what, int reps, long long *out,
                                             int R) {
  const InstDesc &D = descs[0];
  Lds<BS> L = lds_setup<BS>(R);
  double *xs = L.region;
  const int n = D.n;
  for (int i = threadIdx.x; i < n; i += BS) xs[i] = D.p[i];
  __syncthreads();
  double acc = 0.0;
  const long long t0 = wall_clock64();
  for (int r = 0; r < reps; ++r) {
    if (what == 0) {
      solve_lds<BS>(D, xs);
    } else if (what == 1 || what == 2) {
      InstDesc E = D;
      if (what == 1) E.n_usched = 0; else E.n_lsched = 0;
      solve_lds<BS>(E, xs);
    } else if (what == 3) {
      for (int i = threadIdx.x; i < n; i += BS) xs[i] = c_row(D, D.p, i);
      __syncthreads();
    } else if (what == 4) {
      acc += wg_sum(L, acc + 1.0);
    } else if (what == 5) {
      for (int l = 0; l < D.n_lsched + D.n_usched; ++l) __syncthreads();
    } else if (what == 6) {
      for (int i = 0; i < 9; ++i) {
        const double *vi = D.V + (int64_t)i * D.ldv;
        double part = 0.0;
        for (int t = threadIdx.x; t < n; t += BS) part += xs[t] * vi[t];
        const double hij = wg_sum(L, part) * 1e-300;
        for (int t = threadIdx.x; t < n; t += BS) xs[t] -= hij * vi[t];
      }
    } else if (what == 7 || what == 8 || what == 9) {
      // 7: register MGS as in arnoldi_step; 8: its loads and dots without the
      // reduction; 9: its reductions without loads
      constexpr int E = (4608 + BS - 1) / BS;
      const int t0 = threadIdx.x;
      const double *V = D.V;
      const int64_t ldv = D.ldv;
      double cur[E], nxt[E];
#pragma unroll
      for (int e = 0; e < E; ++e) cur[e] = (what != 9 && t0 + e * BS < n) ? V[t0 + e * BS] : 0.0;
      for (int i = 0; i < 9; ++i) {
        double part = 0.0;
#pragma unroll
        for (int e = 0; e < E; ++e)
          if (t0 + e * BS < n) part += xs[t0 + e * BS] * cur[e];
        if (what != 9 && i < 8) {
          const double *vn = V + (int64_t)(i + 1) * ldv;
#pragma unroll
          for (int e = 0; e < E; ++e) nxt[e] = (t0 + e * BS < n) ? vn[t0 + e * BS] : 0.0;
        }
        const double hij = (what != 8 ? wg_sum(L, part) : part) * 1e-300;
#pragma unroll
        for (int e = 0; e < E; ++e)
          if (t0 + e * BS < n) xs[t0 + e * BS] -= hij * cur[e];
        if (what != 9)
#pragma unroll
          for (int e = 0; e < E; ++e) cur[e] = nxt[e];
      }
    }
  }
  const long long t1 = wall_clock64();
  if (threadIdx.x == 0) { out[0] = t1 - t0; out[1] = (long long)acc; }
}

hipError_t launch_diag(const InstDesc *d, int what, int reps, long long *out, int bs, int R, hipStream_t s) {
  const size_t sh = lds_bytes(bs, R);
  EXPRI_DISPATCH(bs, {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_diag<BS>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_diag<BS>, dim3(1), dim3(BS), sh, s, d, what, reps, out, R);
  });
  return hipGetLastError();
}

hipError_t launch_begin(const InstDesc *d, int n_inst, const double *const *xin, double t0, double h0,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_begin, dim3(n_inst), dim3(256), 0, s, d, xin, t0, h0);
  return hipGetLastError();
}

hipError_t launch_end(const InstDesc *d, int n_inst, double *const *xout, hipStream_t s) {
  hipLaunchKernelGGL(k_end, dim3(n_inst), dim3(256), 0, s, d, xout);
  return hipGetLastError();
}

hipError_t launch_run(const InstDesc *d, const int *order, int n_inst, const Opts &o, int max_steps,
                      int replay, int bs, int R, hipStream_t s) {
  const size_t sh = lds_bytes(bs, R);
  EXPRI_DISPATCH(bs, hipLaunchKernelGGL(k_run<BS>, dim3(n_inst), dim3(BS), sh, s, d, order, o, max_steps,
                                        replay, R));
  return hipGetLastError();
}

hipError_t launch_dc(const InstDesc *d, int n_inst, const Opts &o, double t0, int max_it, int bs, int R,
                     hipStream_t s) {
  const size_t sh = lds_bytes(bs, R);
  EXPRI_DISPATCH(bs, hipLaunchKernelGGL(k_dc<BS>, dim3(n_inst), dim3(BS), sh, s, d, o, t0, max_it, R));
  return hipGetLastError();
}

hipError_t launch_factor(const InstDesc *d, int n_inst, const Opts &o, int bs, int R, hipStream_t s) {
  const size_t sh = lds_bytes(bs, R);
  EXPRI_DISPATCH(bs, hipLaunchKernelGGL(k_factor<BS>, dim3(n_inst), dim3(BS), sh, s, d, o, R));
  return hipGetLastError();
}

hipError_t launch_solve(const InstDesc *d, int n_inst, const double *const *b, double *const *y, int bs,
                        int R, hipStream_t s) {
  const size_t sh = lds_bytes(bs, R);
  EXPRI_DISPATCH(bs, hipLaunchKernelGGL(k_solve<BS>, dim3(n_inst), dim3(BS), sh, s, d, b, y, R));
  return hipGetLastError();
}

hipError_t launch_mevp(const InstDesc *d, int n_inst, const Opts &o, const double *const *v,
                       double *const *out, double h, double eps, int bs, int R, hipStream_t s) {
  const size_t sh = lds_bytes(bs, R);
  EXPRI_DISPATCH(bs, hipLaunchKernelGGL(k_mevp<BS>, dim3(n_inst), dim3(BS), sh, s, d, o, v, out, h, eps, R));
  return hipGetLastError();
}

}  // namespace expri
