// gfx950 kernels of the multifrontal engine: the exponential Rosenbrock-Euler
// step (Algorithm 2, Algorithm 1 inside) for one circuit too large for one
// workgroup, with the whole GPU working on it.
//
//   * LU_decompose(G_k) is a multifrontal factorisation over the separator
//     tree of frontal.hpp, one tree height at a time (the fronts of a height
//     are independent): assembly of G_k into zeroed dense fronts, extend-add of
//     the children's Schur complements, then a blocked right-looking partial
//     LU of every front (32-wide pivot blocks: one workgroup factorises the
//     diagonal block and both panels, and the trailing update runs as 64 x 64
//     FP64 MFMA tiles over all fronts of the height).  No pivoting (static
//     order); a pivot below piv_tol times its row's largest |G_k| entry is
//     reported as singular.
//   * The solves G_k y = b walk the same tree: forward (L, bottom-up), each
//     front gathering its children's update vectors, solving its unit-lower
//     pivot block in 32-wide blocks (a wave solves the block triangle, the
//     workgroup updates the rows below) and passing its own update vector up;
//     backward (U, top-down), each front gathering the solution on its row
//     structure.
//   * Vector work (C SpMV, Gram-Schmidt products, norms, combinations) is
//     element-strided over the grid; reductions are two-pass with a fixed
//     summation order, so results do not depend on scheduling.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "devcommon.hpp"
#include "layout.hpp"
#include "mlp.hpp"
#include "mosfet.hpp"

namespace expri {

namespace {

constexpr int kNB = 32;   // pivot block of the partial factorisation
constexpr int kGT = 64;   // output tile of the trailing update
constexpr int kET = 32;   // tile of the extend-add
constexpr int kRB = 512;  // blocks of the two-pass reductions

__device__ __forceinline__ double node_volt(const double *x, int v, double vdd) {
  return v >= 0 ? x[v] : (v == -2 ? vdd : 0.0);
}

}  // namespace

// p[0..n) = v
__global__ void k_g_fill(double *p, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// y[i] = x[map[i]] (gather; map = perm takes the caller's order to the new one)
__global__ void k_g_gather(int n, const int *map, const double *x, double *y) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) y[i] = x[map[i]];
}

// y[map[i]] = x[i] (scatter back to the caller's order)
__global__ void k_g_scatter(int n, const int *map, const double *x, double *y) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) y[map[i]] = x[i];
}

// device currents I_k (into the drain) and dI_k/dV_{d,g,s} at x
__global__ void k_g_stamp(int n_dev, const int *dev_node, const double *par, const double *x, double vdd,
                          double *devI, double *devD) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n_dev; k += gridDim.x * blockDim.x) {
    const double *q = par + 4 * k;
    double I, dd, dg, ds;
    mos_eval(q[0], node_volt(x, dev_node[3 * k], vdd), node_volt(x, dev_node[3 * k + 1], vdd),
             node_volt(x, dev_node[3 * k + 2], vdd), q[1], q[2], q[3], I, dd, dg, ds);
    devI[k] = I;
    devD[3 * k] = dd;
    devD[3 * k + 1] = dg;
    devD[3 * k + 2] = ds;
  }
}

// G_k = G_lin + J_dev at its front positions (the fronts are zero); rowmax
// receives max_j |G_k(i, j)| per row as the bit pattern of a non-negative
// double (ordered like unsigned integers)
__global__ void k_g_assemble(int n_ent, const int64_t *ent_pos, const int *ent_row, const int *ent_g,
                             const int *ent_jptr, const int *ent_jcode, const double *g_val, const double *devD,
                             double *F, unsigned long long *rowmax) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n_ent; e += gridDim.x * blockDim.x) {
    double v = ent_g[e] >= 0 ? g_val[ent_g[e]] : 0.0;
    for (int q = ent_jptr[e]; q < ent_jptr[e + 1]; ++q) {
      const int code = ent_jcode[q], k = code >> 3, eq = (code >> 2) & 1, var = code & 3;
      const double d = devD[3 * k + var];
      v += eq ? -d : d;
    }
    F[ent_pos[e]] = v;
    atomicMax(rowmax + ent_row[e], (unsigned long long)__double_as_longlong(fabs(v)));
  }
}

// One pass of the extend-add: item = (child c, tile (ti, tj)); adds the
// child's Schur complement S_c (rows / columns nc_c.. of its front) into its
// parent's front at the relative indices rel.  A pass holds at most one child
// per parent, so no two items of a pass write the same entry.
__global__ void __launch_bounds__(256) k_g_extend(const int *items, const int *nc, const int *fsz,
                                                  const int *parent, const int64_t *f_off, const int *r_ptr,
                                                  const int *rel, double *F) {
  const int c = items[2 * blockIdx.x], tile = items[2 * blockIdx.x + 1];
  const int ti = tile & 0xFFFF, tj = tile >> 16;
  const int p = parent[c];
  const int fc = fsz[c], ncc = nc[c], r = fc - ncc, fp = fsz[p];
  const double *S = F + f_off[c] + (int64_t)ncc * fc + ncc;
  double *P = F + f_off[p];
  const int *rl = rel + r_ptr[c];
  const int a = ti * kET + (threadIdx.x & 31);
  if (a >= r) return;
  const int ra = rl[a];
#pragma unroll
  for (int q = 0; q < kET / 8; ++q) {
    const int b = tj * kET + (threadIdx.x >> 5) + 8 * q;
    if (b < r) P[ra + (int64_t)rl[b] * fp] += S[a + (int64_t)b * fc];
  }
}

// The extend-add of the small children (update matrices of at most 32 x 32):
// one workgroup per parent adds its small children's Schur complements in
// order, with a barrier between children (two children may reach the same
// parent entry).  The larger children go through k_g_extend passes.
__global__ void __launch_bounds__(256) k_g_extend_small(const int *parents, const int *nc, const int *fsz,
                                                        const int64_t *f_off, const int *ch_ptr, const int *ch,
                                                        const int *r_ptr, const int *rel, double *F) {
  const int p = parents[blockIdx.x];
  const int fp = fsz[p];
  double *P = F + f_off[p];
  const int t = threadIdx.x;
  for (int q = ch_ptr[p]; q < ch_ptr[p + 1]; ++q) {
    const int c = ch[q];
    const int fc = fsz[c], ncc = nc[c], r = fc - ncc;
    if (r > kET) continue;
    const double *S = F + f_off[c] + (int64_t)ncc * fc + ncc;
    const int *rl = rel + r_ptr[c];
    for (int e = t; e < r * r; e += 256) {
      const int a = e % r, b = e / r;
      P[rl[a] + (int64_t)rl[b] * fp] += S[a + (int64_t)b * fc];
    }
    __syncthreads();
  }
}

// LU without pivoting of the kb x kb block in Dm (entries outside the block
// zero), by one wave: on return Dm holds the unit-lower L below the diagonal
// and U on and above it.  Lane t keeps row t in registers; at step p lane p
// publishes its (final) row through LDS and the lanes below eliminate with
// it.  A wave's LDS operations complete in order, so no barrier is needed.
// Pivot test (static pivoting): |u_tt| must exceed piv_tol times rm, lane t's
// row maximum; the first failing row of the block is kept in *bad as
// 1 + row0 + t.
__device__ __forceinline__ void lu_block_wave(double (*Dm)[kNB + 1], int kb, double rm, double piv_tol, int row0,
                                              int *bad) {
  const int t = threadIdx.x & 63;
  double rw[kNB];
#pragma unroll
  for (int j = 0; j < kNB; ++j) rw[j] = Dm[min(t, kNB - 1)][j];
#pragma unroll
  for (int p = 0; p < kNB; ++p) {
    if (p < kb) {
      if (t == p) {
#pragma unroll
        for (int j = 0; j < kNB; ++j) Dm[p][j] = rw[j];
      }
      wfence();
      const double piv = Dm[p][p];
      if (t > p && t < kb) {
        const double l = rw[p] / piv;
        rw[p] = l;
#pragma unroll
        for (int j = p + 1; j < kNB; ++j) rw[j] -= l * Dm[p][j];
      }
    }
  }
  wfence();
  if (t < kb) {
#pragma unroll
    for (int j = 0; j < kNB; ++j) Dm[t][j] = rw[j];
  }
  wfence();
  const unsigned long long weak = __ballot(t < kb && !(fabs(Dm[t][t]) > piv_tol * rm));
  if (weak != 0ull && t == __ffsll((long long)weak) - 1) atomicCAS(bad, 0, 1 + row0 + t);
}

// Whole partial factorisation of the small fronts of a height (f <= FW,
// FW = 32 or 64), one wave per front and four fronts per workgroup, with no
// workgroup barrier: lane l keeps row l of the front in registers (zeros past
// f); for each pivot p < nc lane p publishes its (final) row through the
// wave's LDS slice and every lane below eliminates with it, pivot rows and
// update rows alike (l_lp = a_lp / u_pp, a_lj -= l_lp u_pj for j > p).  The
// rows go back in place: L and U in the pivot rows and columns, the Schur
// complement in the trailing block.  Pivot test as in lu_block_wave.
template <int FW>
__global__ void __launch_bounds__(256) k_g_small_lu(const int *fronts, int count, const int *c0, const int *nc,
                                                    const int *fsz, const int64_t *f_off,
                                                    const unsigned long long *rowmax, double piv_tol, double *F,
                                                    int *bad) {
  __shared__ double prow[4][FW];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int idx = blockIdx.x * 4 + w;
  if (idx >= count) return;  // the whole wave
  const int s = fronts[idx];
  const int f = fsz[s], np = nc[s];
  double *A = F + f_off[s];
  const double rm = l < np ? __longlong_as_double((long long)rowmax[c0[s] + l]) : 0.0;
  const int lr = min(l, f - 1);
  double row[FW];
#pragma unroll
  for (int j = 0; j < FW; ++j) row[j] = (l < f && j < f) ? A[lr + (int64_t)j * f] : 0.0;
  double *pr = prow[w];
  double diag = 1.0;
#pragma unroll
  for (int p = 0; p < FW; ++p) {
    if (p < np) {
      if (l == p) {
        diag = row[p];
#pragma unroll
        for (int j = 0; j < FW; ++j) pr[j] = row[j];
      }
      wfence();
      const double piv = pr[p];
      if (l > p) {
        const double m = row[p] / piv;
        row[p] = m;
#pragma unroll
        for (int j = p + 1; j < FW; ++j) row[j] -= m * pr[j];
      }
      wfence();
    }
  }
  const unsigned long long weak = __ballot(l < np && !(fabs(diag) > piv_tol * rm));
  if (weak != 0ull && l == __ffsll((long long)weak) - 1) atomicCAS(bad, 0, 1 + c0[s] + l);
  if (l < f) {
#pragma unroll
    for (int j = 0; j < FW; ++j)
      if (j < f) A[l + (int64_t)j * f] = row[j];
  }
}

// Step k0 of the partial factorisation, part 1, one wave per front: LU of the
// 32 x 32 diagonal block at (k0, k0).  Only a level's first step and the
// fronts whose previous step's trailing update ran inside the panel kernel
// need it; otherwise the previous step's update tile (0, 0) has factored the
// block (k_g_update).
__global__ void __launch_bounds__(64) k_g_diag(const int *fronts, int k0, const int *c0, const int *nc,
                                               const int *fsz, const int64_t *f_off, const unsigned long long *rowmax,
                                               double piv_tol, double *F, int *bad) {
  __shared__ double Dm[kNB][kNB + 1];
  const int s = fronts[blockIdx.x];
  const int f = fsz[s], kb = min(kNB, nc[s] - k0);
  double *A = F + f_off[s];
  const int t = threadIdx.x;
  // the row maxima of the block's rows, for the pivot test
  const double rm = t < kb ? __longlong_as_double((long long)rowmax[c0[s] + k0 + t]) : 0.0;
  for (int e = t; e < kNB * kNB; e += 64) {
    const int i = e % kNB, j = e / kNB;
    Dm[i][j] = (i < kb && j < kb) ? A[(k0 + i) + (int64_t)(k0 + j) * f] : 0.0;
  }
  wfence();
  lu_block_wave(Dm, kb, rm, piv_tol, c0[s] + k0, bad);
  for (int e = t; e < kb * kb; e += 64) {
    const int i = e % kb, j = e / kb;
    A[(k0 + i) + (int64_t)(k0 + j) * f] = Dm[i][j];
  }
}

// Part 2, item = (front s, chunk c): with the factored diagonal block, C rows
// of the panel L21 = F[o.., k0..] U_D^{-1} and C columns of
// U12 = L_D^{-1} F[k0.., o..], o = k0 + kb + c C.  When the whole trailing
// block fits in one chunk and has at most fuse rows, the same workgroup also
// applies the trailing update S -= L21 U12.  Dynamic LDS: 2 C (kNB + 1)
// doubles (C <= 128).
__global__ void __launch_bounds__(256) k_g_panel(const int *items, int k0, int C, int fuse, const int *nc,
                                                 const int *fsz, const int64_t *f_off, double *F) {
  __shared__ double Dm[kNB][kNB + 1];
  extern __shared__ double pn[];
  double (*Pn)[kNB + 1] = reinterpret_cast<double (*)[kNB + 1]>(pn);
  const int s = items[2 * blockIdx.x], chunk = items[2 * blockIdx.x + 1];
  const int f = fsz[s], kb = min(kNB, nc[s] - k0);
  double *A = F + f_off[s];
  const int t = threadIdx.x;
  const int rem = f - k0 - kb;
  const int o = k0 + kb + chunk * C;
  const int cnt = min(C, f - o);
  if (cnt <= 0) return;  // the whole workgroup
  // the factored diagonal block, padded to kNB x kNB with the identity so
  // that the solves below run over all kNB columns with fixed bounds (the
  // padding columns of the panels are zero and stay zero)
  for (int e = t; e < kNB * kNB; e += 256) {
    const int i = e % kNB, j = e / kNB;
    Dm[i][j] = (i < kb && j < kb) ? A[(k0 + i) + (int64_t)(k0 + j) * f] : (i == j ? 1.0 : 0.0);
  }
  // C rows of L21 in Pn[0..C), C columns of U12 in Pn[C..2C)
  for (int e = t; e < C * kNB; e += 256) {
    const int i = e % C, j = e / C;
    Pn[i][j] = (i < cnt && j < kb) ? A[(o + i) + (int64_t)(k0 + j) * f] : 0.0;
    const int jj = e % kNB, c = e / kNB;
    Pn[C + c][jj] = (c < cnt && jj < kb) ? A[(k0 + jj) + (int64_t)(o + c) * f] : 0.0;
  }
  __syncthreads();
  // each row of L21 (l U_D = a) and column of U12 (L_D u = a) is solved by
  // one thread in registers, right-looking: once entry j is final the later
  // entries are updated with it; the block's entries are LDS broadcasts
  if (t < cnt || (t >= C && t - C < cnt)) {
    const bool row = t < C;
    double r[kNB];
#pragma unroll
    for (int j = 0; j < kNB; ++j) r[j] = Pn[t][j];
    if (row) {
#pragma unroll
      for (int j = 0; j < kNB; ++j) {
        r[j] /= Dm[j][j];
#pragma unroll
        for (int jj = j + 1; jj < kNB; ++jj) r[jj] -= r[j] * Dm[j][jj];
      }
    } else {
#pragma unroll
      for (int j = 0; j < kNB - 1; ++j)
#pragma unroll
        for (int jj = j + 1; jj < kNB; ++jj) r[jj] -= Dm[jj][j] * r[j];
    }
#pragma unroll
    for (int j = 0; j < kNB; ++j) Pn[t][j] = r[j];
  }
  __syncthreads();
  for (int e = t; e < C * kNB; e += 256) {
    const int i = e % C, j = e / C;
    if (i < cnt && j < kb) A[(o + i) + (int64_t)(k0 + j) * f] = Pn[i][j];
    const int jj = e % kNB, c = e / kNB;
    if (c < cnt && jj < kb) A[(k0 + jj) + (int64_t)(o + c) * f] = Pn[C + c][jj];
  }
  if (rem <= C && rem <= fuse) {  // the trailing update of a small front, in place
    for (int e = t; e < rem * rem; e += 256) {
      const int i = e % rem, j = e / rem;
      double acc = A[(o + i) + (int64_t)(o + j) * f];
      for (int k = 0; k < kb; ++k) acc -= Pn[i][k] * Pn[C + j][k];
      A[(o + i) + (int64_t)(o + j) * f] = acc;
    }
  }
}

// Trailing update of step k0: item = (front s, tile (ti, tj)); the 64 x 64
// tile of F[o.., o..] (o = k0 + kb) gets -= L21 U12 over the kb pivot
// columns, on FP64 MFMA 16x16x4 (four waves, a 32 x 32 quadrant each).
// MFMA lane layout: operand A lane i + 16 k holds A[i][k]; operand B lane
// j + 16 k holds B[k][j]; result element v of lane j + 16 q is C[q + 4 v][j].
// Tile (0, 0)'s first quadrant is the next step's diagonal block: when the
// front has pivots left, its wave factors that block (lu_block_wave) before
// storing it, so the next step needs no k_g_diag launch for this front.
__global__ void __launch_bounds__(256) k_g_update(const int *items, int k0, const int *c0, const int *nc,
                                                  const int *fsz, const int64_t *f_off,
                                                  const unsigned long long *rowmax, double piv_tol, double *F,
                                                  int *bad) {
  __shared__ double As[kGT][kNB + 1];
  __shared__ double Bs[kNB][kGT + 1];
  const int s = items[2 * blockIdx.x], tile = items[2 * blockIdx.x + 1];
  const int f = fsz[s], kb = min(kNB, nc[s] - k0), o = k0 + kb;
  const int i0 = o + (tile & 0xFFFF) * kGT, j0 = o + (tile >> 16) * kGT;
  double *A = F + f_off[s];
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int r = lane & 15, q = lane >> 4;
  const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
  // the next step's pivot block: rows / columns o .. o + kb2 (uniform per workgroup)
  const int kb2 = tile == 0 ? min(kNB, nc[s] - o) : 0;
  const double rm = (kb2 > 0 && wave == 0 && lane < kb2)
                        ? __longlong_as_double((long long)rowmax[c0[s] + o + lane]) : 0.0;
  // the tile's loads are issued first, so that their latency overlaps the
  // staging of the panels
  dbl4 acc[2][2];
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + wi + 16 * mi + q + 4 * v, j = j0 + wj + 16 * ni + r;
        acc[mi][ni][v] = (i < f && j < f) ? A[i + (int64_t)j * f] : 0.0;
      }
  for (int e = t; e < kGT * kNB; e += 256) {
    const int i = e % kGT, k = e / kGT;
    As[i][k] = (i0 + i < f && k < kb) ? A[(i0 + i) + (int64_t)(k0 + k) * f] : 0.0;
  }
  for (int e = t; e < kNB * kGT; e += 256) {
    const int k = e % kNB, j = e / kNB;
    Bs[k][j] = (j0 + j < f && k < kb) ? A[(k0 + k) + (int64_t)(j0 + j) * f] : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kNB; k += 4) {
    double a[2], b[2];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi) a[mi] = -As[wi + 16 * mi + r][k + q];
#pragma unroll
    for (int ni = 0; ni < 2; ++ni) b[ni] = Bs[k + q][wj + 16 * ni + r];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int ni = 0; ni < 2; ++ni) acc[mi][ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[mi], b[ni], acc[mi][ni], 0, 0, 0);
  }
  if (kb2 > 0) __syncthreads();  // As is free: it becomes the pivot block (uniform branch)
  double (*Dm)[kNB + 1] = As;
  const bool lu = kb2 > 0 && wave == 0;
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int li = wi + 16 * mi + q + 4 * v, lj = wj + 16 * ni + r;
        const int i = i0 + li, j = j0 + lj;
        const bool pivot = lu && li < kb2 && lj < kb2;
        if (lu) Dm[li][lj] = pivot ? acc[mi][ni][v] : 0.0;
        if (!pivot && i < f && j < f) A[i + (int64_t)j * f] = acc[mi][ni][v];
      }
  if (lu) {
    wfence();
    lu_block_wave(Dm, kb2, rm, piv_tol, c0[s] + o, bad);
    for (int e = lane; e < kb2 * kb2; e += 64) {
      const int i = e % kb2, j = e / kb2;
      A[(o + i) + (int64_t)(o + j) * f] = Dm[i][j];
    }
  }
}

// The triangular solves with the factors of G_k, for NR right-hand sides at
// once (NR = 1 or 2): vector r of x starts at x + r ldx and its update
// vectors at upd + r ldu.  The factor entries are loaded once for all NR.

// Row t of the kNB-wide diagonal block of a pivot block that starts at b0
// (bw rows), in registers; indices are clamped into the block so every load
// is in bounds.  The triangular solves below load the next block this way
// right after solving the current one, so its latency overlaps the update.
__device__ __forceinline__ void tri_block_row(double (&col)[kNB], const double *A, int f, int b0, int bw, int t) {
  const int rt = b0 + min(t, bw - 1);
#pragma unroll
  for (int j = 0; j < kNB; ++j) col[j] = A[rt + (int64_t)(b0 + min(j, bw - 1)) * f];
}

// Forward solve of one tree height (L y = b, unit lower), part 1, one
// workgroup of BS threads per front: v = [x(cols s); 0] + the children's
// update vectors at their relative indices; the unit-lower pivot block L11 is
// solved in 32-wide blocks (a wave solves the block triangle, the workgroup
// updates the pivot rows below it); y goes to x, the rest of v (the
// children's contributions to the update vector) to upd.  Part 2
// (k_g_fwd_gemv) subtracts L21 y.  Dynamic LDS: NR f doubles.
template <int NR, int BS>
__global__ void __launch_bounds__(BS) k_g_fwd_tri(const int *fronts, const int *c0, const int *nc, const int *fsz,
                                                  const int64_t *f_off, const int *ch_ptr, const int *ch,
                                                  const int *r_ptr, const int *rel, const int *u_off,
                                                  const double *F, double *x, int64_t ldx, double *upd,
                                                  int64_t ldu, const int64_t *inv_off, double *tmp) {
  extern __shared__ double v[];
  const int s = fronts[blockIdx.x];
  // a front with an inverted pivot block leaves the triangle to k_g_trmv:
  // its assembled v goes to tmp instead
  const bool inv = inv_off[s] >= 0;
  const int f = fsz[s], p = inv ? 0 : nc[s], pv = nc[s], b = c0[s];
  double *xo = inv ? tmp : x;
  const double *A = F + f_off[s];
  const int t = threadIdx.x;
  double col[kNB];  // wave 0: row t of the current diagonal block
  if (t < 64 && p > 0) tri_block_row(col, A, f, 0, min(kNB, p), t);
#pragma unroll
  for (int r = 0; r < NR; ++r)
    for (int i = t; i < f; i += BS) v[r * f + i] = i < pv ? x[r * ldx + b + i] : 0.0;
  __syncthreads();
  for (int q = ch_ptr[s]; q < ch_ptr[s + 1]; ++q) {
    const int c = ch[q], rc = fsz[c] - nc[c];
    const int *rl = rel + r_ptr[c];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const double *uc = upd + r * ldu + u_off[c];
      for (int a = t; a < rc; a += BS) v[r * f + rl[a]] += uc[a];
    }
    __syncthreads();
  }
  for (int b0 = 0; b0 < p; b0 += kNB) {
    const int bw = min(kNB, p - b0);
    // this thread's first row below the block: its kNB entries are loaded
    // before the block triangle is solved (a row past p loads row p - 1)
    const int i0 = b0 + bw + t;
    double pa[kNB];
    {
      const int ri = min(i0, p - 1);
#pragma unroll
      for (int j = 0; j < kNB; ++j) pa[j] = A[ri + (int64_t)(b0 + min(j, bw - 1)) * f];
    }
    if (t < 64) {
      double vl[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) vl[r] = t < bw ? v[r * f + b0 + t] : 0.0;
#pragma unroll
      for (int j = 0; j < kNB; ++j) {
        if (j < bw) {
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            const double z = readlane_d(vl[r], j);
            if (t > j) vl[r] -= col[j] * z;
          }
        }
      }
      if (t < bw) {
#pragma unroll
        for (int r = 0; r < NR; ++r) v[r * f + b0 + t] = vl[r];
      }
      const int b1 = b0 + kNB;
      if (b1 < p) tri_block_row(col, A, f, b1, min(kNB, p - b1), t);
    }
    __syncthreads();
    if (i0 < p) {
      double acc[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) acc[r] = v[r * f + i0];
#pragma unroll
      for (int j = 0; j < kNB; ++j) {
#pragma unroll
        for (int r = 0; r < NR; ++r) acc[r] -= pa[j] * (j < bw ? v[r * f + b0 + j] : 0.0);
      }
#pragma unroll
      for (int r = 0; r < NR; ++r) v[r * f + i0] = acc[r];
    }
    for (int i = i0 + BS; i < p; i += BS) {
      double acc[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) acc[r] = v[r * f + i];
#pragma unroll
      for (int j = 0; j < kNB; ++j) {
        const double a = A[i + (int64_t)(b0 + min(j, bw - 1)) * f];
#pragma unroll
        for (int r = 0; r < NR; ++r) acc[r] -= a * (j < bw ? v[r * f + b0 + j] : 0.0);
      }
#pragma unroll
      for (int r = 0; r < NR; ++r) v[r * f + i] = acc[r];
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < NR; ++r)
    for (int i = t; i < f; i += BS) {
      if (i < pv) xo[r * ldx + b + i] = v[r * f + i];
      else upd[r * ldu + u_off[s] + i - pv] = v[r * f + i];
    }
}

// Forward solve, part 2: item = (front s, chunk of 64 update rows):
// upd_s[a] -= L21[a, :] y_s.  Each wave sums a quarter of the pivot columns
// for the chunk's 64 rows (one row per lane); the quarters are added in order.
// Dynamic LDS: NR nc doubles.
template <int NR>
__global__ void __launch_bounds__(256) k_g_fwd_gemv(const int *items, const int *c0, const int *nc, const int *fsz,
                                                    const int64_t *f_off, const int *u_off, const double *F,
                                                    const double *x, int64_t ldx, double *upd, int64_t ldu) {
  extern __shared__ double ys[];
  __shared__ double red[NR][4][64];
  const int s = items[2 * blockIdx.x], chunk = items[2 * blockIdx.x + 1];
  const int f = fsz[s], p = nc[s], r_ = f - p;
  const double *A = F + f_off[s];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
#pragma unroll
  for (int r = 0; r < NR; ++r)
    for (int j = t; j < p; j += 256) ys[r * p + j] = x[r * ldx + c0[s] + j];
  __syncthreads();
  const int a = chunk * 64 + lane;
  const int ra = p + min(a, r_ - 1);
  const int q = (p + 3) / 4, j0 = w * q, j1 = min(p, j0 + q);
  double acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = 0.0;
#pragma unroll 16
  for (int j = j0; j < j1; ++j) {
    const double l = A[ra + (int64_t)j * f];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] += l * ys[r * p + j];
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) red[r][w][lane] = acc[r];
  __syncthreads();
  if (w == 0 && a < r_) {
#pragma unroll
    for (int r = 0; r < NR; ++r)
      upd[r * ldu + u_off[s] + a] -= (red[r][0][lane] + red[r][1][lane]) + (red[r][2][lane] + red[r][3][lane]);
  }
}

// Forward solve of the small fronts of a height (f <= 64), one wave per
// front and four fronts per workgroup, with no workgroup barrier: lane l
// holds v[l]; the children's update vectors are added through the wave's own
// LDS slice; then for each pivot column j the lanes below j subtract
// L[l, j] y_j (pivot rows and update rows alike).
template <int NR>
__global__ void __launch_bounds__(256) k_g_fwd_small(const int *fronts, int count, const int *c0, const int *nc,
                                                     const int *fsz, const int64_t *f_off, const int *ch_ptr,
                                                     const int *ch, const int *r_ptr, const int *rel,
                                                     const int *u_off, const double *F, double *x, int64_t ldx,
                                                     double *upd, int64_t ldu) {
  __shared__ double sv[NR][4][64];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int idx = blockIdx.x * 4 + w;
  if (idx >= count) return;  // the whole wave
  const int s = fronts[idx];
  const int f = fsz[s], p = nc[s], b = c0[s];
  const double *A = F + f_off[s];
#pragma unroll
  for (int r = 0; r < NR; ++r) sv[r][w][l] = l < p ? x[r * ldx + b + l] : 0.0;
  wfence();
  for (int q = ch_ptr[s]; q < ch_ptr[s + 1]; ++q) {
    const int c = ch[q], rc = fsz[c] - nc[c];  // rc <= f <= 64
    if (l < rc) {
      const int dst = rel[r_ptr[c] + l];
#pragma unroll
      for (int r = 0; r < NR; ++r) sv[r][w][dst] += upd[r * ldu + u_off[c] + l];
    }
    wfence();
  }
  double v[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) v[r] = sv[r][w][l];
  const int lr = min(l, f - 1);
  double a_next = A[lr];
  for (int j = 0; j < p; ++j) {
    const double a = a_next;
    a_next = A[lr + (int64_t)min(j + 1, p - 1) * f];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const double z = readlane_d(v[r], j);
      if (l > j && l < f) v[r] -= a * z;
    }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (l < p) x[r * ldx + b + l] = v[r];
    else if (l < f) upd[r * ldu + u_off[s] + l - p] = v[r];
  }
}

// Backward solve of the small fronts (f <= 64), one wave per front: lane l
// holds y[l] (pivot rows) or x(R_s) (update rows); U12 x(R_s) is subtracted
// column by column, then the upper pivot block is solved from the last row.
template <int NR>
__global__ void __launch_bounds__(256) k_g_bwd_small(const int *fronts, int count, const int *c0, const int *nc,
                                                     const int *fsz, const int64_t *f_off, const int *r_ptr,
                                                     const int *r_idx, const double *F, double *x, int64_t ldx) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int idx = blockIdx.x * 4 + w;
  if (idx >= count) return;
  const int s = fronts[idx];
  const int f = fsz[s], p = nc[s], b = c0[s], r_ = f - p;
  const double *A = F + f_off[s];
  double v[NR];
  const int src = l < p ? b + l : (l < f ? r_idx[r_ptr[s] + l - p] : -1);
#pragma unroll
  for (int r = 0; r < NR; ++r) v[r] = src >= 0 ? x[r * ldx + src] : 0.0;
  const int lr = min(l, p - 1);
  for (int a = 0; a < r_; ++a) {
    const double u = A[lr + (int64_t)(p + a) * f];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const double z = readlane_d(v[r], p + a);
      if (l < p) v[r] -= u * z;
    }
  }
  for (int j = p - 1; j >= 0; --j) {
    const double u = A[lr + (int64_t)j * f];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if (l == j) v[r] = v[r] / u;
      const double z = readlane_d(v[r], j);
      if (l < j) v[r] -= u * z;
    }
  }
  if (l < p) {
#pragma unroll
    for (int r = 0; r < NR; ++r) x[r * ldx + b + l] = v[r];
  }
}

// Backward solve (U x = y), part 1: item = (front s, chunk of 64 pivot rows):
// x(cols s)[i] = y[i] - U12[i, :] x(R_s), x(R_s) being final (the ancestors
// are done).  Waves split R_s in quarters, added in order.  Dynamic LDS:
// NR (f - nc) doubles.
template <int NR>
__global__ void __launch_bounds__(256) k_g_bwd_gemv(const int *items, const int *c0, const int *nc, const int *fsz,
                                                    const int64_t *f_off, const int *r_ptr, const int *r_idx,
                                                    const double *F, double *x, int64_t ldx) {
  extern __shared__ double xr[];
  __shared__ double red[NR][4][64];
  const int s = items[2 * blockIdx.x], chunk = items[2 * blockIdx.x + 1];
  const int f = fsz[s], p = nc[s], r_ = f - p;
  const double *A = F + f_off[s];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  for (int k = t; k < r_; k += 256) {
    const int g = r_idx[r_ptr[s] + k];
#pragma unroll
    for (int r = 0; r < NR; ++r) xr[r * r_ + k] = x[r * ldx + g];
  }
  __syncthreads();
  const int i = chunk * 64 + lane;
  const int ri = min(i, p - 1);
  const int q = (r_ + 3) / 4, k0 = w * q, k1 = min(r_, k0 + q);
  double acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = 0.0;
#pragma unroll 16
  for (int k = k0; k < k1; ++k) {
    const double u = A[ri + (int64_t)(p + k) * f];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] += u * xr[r * r_ + k];
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) red[r][w][lane] = acc[r];
  __syncthreads();
  if (w == 0 && i < p) {
#pragma unroll
    for (int r = 0; r < NR; ++r)
      x[r * ldx + c0[s] + i] -= (red[r][0][lane] + red[r][1][lane]) + (red[r][2][lane] + red[r][3][lane]);
  }
}

// Backward solve, part 2, one workgroup of BS threads per front: the upper
// pivot block U11 in 32-wide blocks from the last, each block updating the
// pivot rows above.
// Dynamic LDS: NR nc doubles.
template <int NR, int BS>
__global__ void __launch_bounds__(BS) k_g_bwd_tri(const int *fronts, const int *c0, const int *nc, const int *fsz,
                                                  const int64_t *f_off, const double *F, double *x, int64_t ldx,
                                                  const int64_t *inv_off) {
  extern __shared__ double v[];
  const int s = fronts[blockIdx.x];
  if (inv_off[s] >= 0) return;  // the inverted pivot block is applied by k_g_trmv
  const int f = fsz[s], p = nc[s], b = c0[s];
  const double *A = F + f_off[s];
  const int t = threadIdx.x;
  const int last = p > 0 ? ((p - 1) / kNB) * kNB : 0;
  double col[kNB];  // wave 0: row t of the current diagonal block of U
  if (t < 64 && p > 0) tri_block_row(col, A, f, last, min(kNB, p - last), t);
#pragma unroll
  for (int r = 0; r < NR; ++r)
    for (int i = t; i < p; i += BS) v[r * p + i] = x[r * ldx + b + i];
  __syncthreads();
  for (int b0 = p > 0 ? last : -1; b0 >= 0; b0 -= kNB) {
    const int bw = min(kNB, p - b0);
    // this thread's first row above the block: its kNB entries are loaded
    // before the block triangle is solved (with no row above, row 0)
    double pa[kNB];
    {
      const int ri = min(t, max(b0 - 1, 0));
#pragma unroll
      for (int j = 0; j < kNB; ++j) pa[j] = A[ri + (int64_t)(b0 + min(j, bw - 1)) * f];
    }
    if (t < 64) {
      double vl[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) vl[r] = t < bw ? v[r * p + b0 + t] : 0.0;
#pragma unroll
      for (int j = kNB - 1; j >= 0; --j) {
        if (j < bw) {
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            if (t == j) vl[r] = vl[r] / col[j];
            const double z = readlane_d(vl[r], j);
            if (t < j) vl[r] -= col[j] * z;
          }
        }
      }
      if (t < bw) {
#pragma unroll
        for (int r = 0; r < NR; ++r) v[r * p + b0 + t] = vl[r];
      }
      if (b0 > 0) tri_block_row(col, A, f, b0 - kNB, kNB, t);
    }
    __syncthreads();
    if (t < b0) {
      double acc[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) acc[r] = v[r * p + t];
#pragma unroll
      for (int j = 0; j < kNB; ++j) {
#pragma unroll
        for (int r = 0; r < NR; ++r) acc[r] -= pa[j] * (j < bw ? v[r * p + b0 + j] : 0.0);
      }
#pragma unroll
      for (int r = 0; r < NR; ++r) v[r * p + t] = acc[r];
    }
    for (int i = t + BS; i < b0; i += BS) {
      double acc[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) acc[r] = v[r * p + i];
#pragma unroll
      for (int j = 0; j < kNB; ++j) {
        const double a = A[i + (int64_t)(b0 + min(j, bw - 1)) * f];
#pragma unroll
        for (int r = 0; r < NR; ++r) acc[r] -= a * (j < bw ? v[r * p + b0 + j] : 0.0);
      }
#pragma unroll
      for (int r = 0; r < NR; ++r) v[r * p + i] = acc[r];
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < NR; ++r)
    for (int i = t; i < p; i += BS) x[r * ldx + b + i] = v[r * p + i];
}

// Inverses of the pivot blocks of the fronts with many pivots, once per
// factorisation.  Item (s, 2 cb + u): column block cb (32 columns) of
// L11^{-1} (u = 0; unit lower, its strictly lower part stored) or of U11^{-1}
// (u = 1; upper, stored with the diagonal), into Finv + inv_off[s] (p x p,
// column-major; the two inverses share the array as L and U share the
// front).  Left-looking over 32-row blocks r in the order the recurrence
// needs them: X_r = A_rr^{-1} (delta_r,cb I - sum_k A_rk X_k), k running over
// the finished blocks between cb and r, two blocks per step on FP64 MFMA;
// the next pair of tiles is loaded while the current one is multiplied.
__global__ void __launch_bounds__(256) k_g_inv(const int *items, const int *nc, const int *fsz,
                                               const int64_t *f_off, const int64_t *inv_off, const double *F,
                                               double *Finv) {
  __shared__ double As[32][65], Xs[64][33];
  const int s = items[2 * blockIdx.x], code = items[2 * blockIdx.x + 1];
  const int cb = code >> 1;
  const bool upper = (code & 1) != 0;
  const int f = fsz[s], p = nc[s], R = (p + 31) / 32, j0 = cb * 32;
  const double *A = F + f_off[s];
  double *X = Finv + inv_off[s];
  const int t = threadIdx.x;
  // the 32 x 32 block T is four 16 x 16 FP64 MFMA quadrants, one per wave
  // (lane layout as in k_g_update)
  const int lane = t & 63, wave = t >> 6, lr = lane & 15, lq = lane >> 4;
  const int wi = (wave >> 1) * 16, wj = (wave & 1) * 16;
  // tiles A(r-block, columns k*32 .. k*32 + 63) and X(rows k*32 .. k*32 + 63,
  // cb-block), columns / rows past block kmax zero
  auto load = [&](int r, int k, int kmax, double (&an)[8], double (&xn)[8]) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = t + 256 * q;
      {
        const int a = e & 31, c = e >> 5;
        const int ra = r * 32 + a, ca = k * 32 + c;
        const double av = A[min(ra, p - 1) + (int64_t)min(ca, p - 1) * f];
        an[q] = (ra < p && ca < p && ca < (kmax + 1) * 32) ? av : 0.0;
      }
      {
        const int a = e & 63, c = e >> 6;
        const int rx = k * 32 + a, cx = j0 + c;
        const double xv = X[min(rx, p - 1) + (int64_t)min(cx, p - 1) * p];
        // entries outside this inverse's triangle are its known zeros (and
        // the unit diagonal of L^{-1}); the array holds the other inverse there
        const bool mine = upper ? rx <= cx : rx > cx;
        xn[q] = (rx < p && cx < p && rx < (kmax + 1) * 32) ? (mine ? xv : (!upper && rx == cx ? 1.0 : 0.0)) : 0.0;
      }
    }
  };
  for (int st = 0; st < R; ++st) {
    const int r = upper ? cb - st : cb + st;
    if (r < 0 || r >= R) break;
    dbl4 acc;
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] = (r == cb && wi + lq + 4 * v == wj + lr) ? 1.0 : 0.0;
    const int k_lo = upper ? r + 1 : cb, k_hi = upper ? cb : r - 1;
    double an[8], xn[8];
    if (k_lo <= k_hi) load(r, k_lo, k_hi, an, xn);
    for (int k = k_lo; k <= k_hi; k += 2) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int e = t + 256 * q;
        As[e & 31][e >> 5] = an[q];
        Xs[e & 63][e >> 6] = xn[q];
      }
      __syncthreads();
      if (k + 2 <= k_hi) load(r, k + 2, k_hi, an, xn);
#pragma unroll
      for (int l = 0; l < 64; l += 4)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-As[wi + lr][l + lq], Xs[l + lq][wj + lr], acc, 0, 0, 0);
      __syncthreads();
    }
    // X_r = A_rr^{-1} T: T through Xs, A_rr (identity past p) through As;
    // thread j < 32 substitutes column j
#pragma unroll
    for (int v = 0; v < 4; ++v) Xs[wi + lq + 4 * v][wj + lr] = acc[v];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = t + 256 * q, a = e & 31, c = e >> 5;
      const int ra = r * 32 + a, ca = r * 32 + c;
      const double av = A[min(ra, p - 1) + (int64_t)min(ca, p - 1) * f];
      As[a][c] = (ra < p && ca < p) ? av : (a == c ? 1.0 : 0.0);
    }
    __syncthreads();
    {
      // eight groups of 32 lanes, each substituting columns cg, cg + 8, ...:
      // lane a of a group holds row a of A_rr and x_a; x_l reaches the other
      // lanes of its half-wave by readlane
      const int a = lane & 31, cg = t >> 5, hb = lane & 32;
      double arow[32];
#pragma unroll
      for (int l = 0; l < 32; ++l) arow[l] = As[a][l];
#pragma unroll 1
      for (int jj = 0; jj < 4; ++jj) {
        const int j = cg + 8 * jj;
        double xv = Xs[a][j];
        if (!upper) {
#pragma unroll
          for (int l = 0; l < 32; ++l) {
            const double z0 = readlane_d(xv, l), z1 = readlane_d(xv, 32 + l);
            if (a > l) xv -= arow[l] * (hb ? z1 : z0);
          }
        } else {
#pragma unroll
          for (int l = 31; l >= 0; --l) {
            if (a == l) xv = xv / arow[l];
            const double z0 = readlane_d(xv, l), z1 = readlane_d(xv, 32 + l);
            if (a < l) xv -= arow[l] * (hb ? z1 : z0);
          }
        }
        const int row = r * 32 + a, col = j0 + j;
        if (row < p && col < p && (upper ? row <= col : row > col)) X[row + (int64_t)col * p] = xv;
      }
    }
    __syncthreads();  // this block's X is read by the later row blocks
  }
}

// y = X v on the pivot rows of a front with an inverted pivot block: item
// (s, chunk of 64 rows); X = L11^{-1} (UPPER false: unit lower, y = v + the
// strictly lower part times v) or U11^{-1} (UPPER true).  v is read from `in`
// (vector r at + r ldx), the chunk's rows written to `out`.  Each of the eight
// waves sums an eighth of the columns that reach the chunk (many loads in
// flight per compute unit); the eighths are added in order.  Dynamic LDS:
// NR p doubles.
template <int NR, bool UPPER>
__global__ void __launch_bounds__(512) k_g_trmv(const int *items, const int *c0, const int *nc,
                                                const int64_t *inv_off, const double *Finv, const double *in,
                                                double *out, int64_t ldx) {
  extern __shared__ double vs[];
  __shared__ double red[NR][8][64];
  const int s = items[2 * blockIdx.x], chunk = items[2 * blockIdx.x + 1];
  const int p = nc[s], b = c0[s];
  const double *X = Finv + inv_off[s];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
#pragma unroll
  for (int r = 0; r < NR; ++r)
    for (int j = t; j < p; j += 512) vs[r * p + j] = in[r * ldx + b + j];
  __syncthreads();
  const int i = chunk * 64 + lane, ri = min(i, p - 1);
  const int jlo = UPPER ? chunk * 64 : 0, jhi = UPPER ? p : min(p, chunk * 64 + 64);
  const int q = (jhi - jlo + 7) / 8, j0 = jlo + w * q, j1 = min(jhi, j0 + q);
  double acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = 0.0;
#pragma unroll 16
  for (int j = j0; j < j1; ++j) {
    const double xv = X[ri + (int64_t)j * p];
    const bool nz = UPPER ? j >= ri : j < ri;
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] += nz ? xv * vs[r * p + j] : 0.0;
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) red[r][w][lane] = acc[r];
  __syncthreads();
  if (w == 0 && i < p) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      double y = ((red[r][0][lane] + red[r][1][lane]) + (red[r][2][lane] + red[r][3][lane])) +
                 ((red[r][4][lane] + red[r][5][lane]) + (red[r][6][lane] + red[r][7][lane]));
      if (!UPPER) y += vs[r * p + i];
      out[r * ldx + b + i] = y;
    }
  }
}

// the pivot rows of the fronts with inverted pivot blocks, src -> dst (the
// k_g_trmv items; vector r at + r ldx)
template <int NR>
__global__ void __launch_bounds__(256) k_g_copy_rows(const int *items, const int *c0, const int *nc,
                                                     const double *src, double *dst, int64_t ldx) {
  const int s = items[2 * blockIdx.x], chunk = items[2 * blockIdx.x + 1];
  const int i = chunk * 64 + (threadIdx.x & 63), r = threadIdx.x >> 6;
  if (r < NR && i < nc[s]) dst[r * ldx + c0[s] + i] = src[r * ldx + c0[s] + i];
}

// PWL sources: u(t) and the slope on the piece holding tm
__global__ void k_g_sources(int n_src, const int *src_ptr, const double *src_t, const double *src_v, double t,
                            double tm, double *u, double *slope) {
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n_src; q += gridDim.x * blockDim.x) {
    const int lo = src_ptr[q], hi = src_ptr[q + 1] - 1;
    double val, sl = 0.0;
    if (t <= src_t[lo]) val = src_v[lo];
    else if (t >= src_t[hi]) val = src_v[hi];
    else {
      int a = lo, b = hi;
      while (b - a > 1) {
        const int mid = (a + b) >> 1;
        if (src_t[mid] <= t) a = mid; else b = mid;
      }
      val = src_v[a] + (t - src_t[a]) * ((src_v[a + 1] - src_v[a]) / (src_t[a + 1] - src_t[a]));
    }
    if (hi > lo && tm >= src_t[lo] && tm < src_t[hi]) {
      int a = lo, b = hi;
      while (b - a > 1) {
        const int mid = (a + b) >> 1;
        if (src_t[mid] <= tm) a = mid; else b = mid;
      }
      sl = (src_v[a + 1] - src_v[a]) / (src_t[a + 1] - src_t[a]);
    }
    u[q] = val;
    slope[q] = sl;
  }
}

// r = B u - G_lin x - I_dev(x) and bs = B s (the right-hand sides of w and p)
__global__ void k_g_rhs(int n, const int *g_rowptr, const int *g_col, const double *g_val, const int *b_rowptr,
                        const int *b_col, const double *b_val, const int *node_ptr, const int *node_code,
                        const double *devI, const double *x, const double *u, const double *sl, double *r,
                        double *bs) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    double bu = 0.0, bsl = 0.0;
    for (int e = b_rowptr[i]; e < b_rowptr[i + 1]; ++e) {
      bu += b_val[e] * u[b_col[e]];
      bsl += b_val[e] * sl[b_col[e]];
    }
    double gx = 0.0;
    for (int e = g_rowptr[i]; e < g_rowptr[i + 1]; ++e) gx += g_val[e] * x[g_col[e]];
    double id = 0.0;
    for (int c = node_ptr[i]; c < node_ptr[i + 1]; ++c) {
      const int code = node_code[c];
      id += (code & 1) ? -devI[code >> 1] : devI[code >> 1];
    }
    r[i] = (bu - gx) - id;
    bs[i] = bsl;
  }
}

// y = alpha C x
__global__ void k_g_spmv(int n, const int *rp, const int *ci, const double *val, const double *x, double alpha,
                         double *y) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int e = rp[i]; e < rp[i + 1]; ++e) acc += val[e] * x[ci[e]];
    y[i] = alpha * acc;
  }
}

// partial[blk * ncol + c] = sum over the block's rows of V[:, c] . w (first
// pass of V^T w over kRB blocks; the second pass adds the blocks in order)
__global__ void __launch_bounds__(256) k_g_dots(int n, const double *V, int64_t ldv, int ncol, const double *w,
                                                double *partial) {
  __shared__ double red[4][64];
  const int t = threadIdx.x;
  for (int c0 = 0; c0 < ncol; c0 += 64) {
    const int cw = min(64, ncol - c0);
    for (int cc = 0; cc < cw; ++cc) {
      double acc = 0.0;
      const double *col = V + (int64_t)(c0 + cc) * ldv;
      for (int i = blockIdx.x * 256 + t; i < n; i += gridDim.x * 256) acc += col[i] * w[i];
      acc = wave_sum(acc);
      if ((t & 63) == 0) red[t >> 6][cc] = acc;
    }
    __syncthreads();
    if (t < cw) partial[(int64_t)blockIdx.x * ncol + c0 + t] = (red[0][t] + red[1][t]) + (red[2][t] + red[3][t]);
    __syncthreads();
  }
}

// out[c] = sum over blocks b (in order) of partial[b * ncol + c]
__global__ void k_g_reduce(const double *partial, int nblk, int ncol, double *out) {
  for (int c = threadIdx.x; c < ncol; c += blockDim.x) {
    double acc = 0.0;
    for (int b = 0; b < nblk; ++b) acc += partial[(int64_t)b * ncol + c];
    out[c] = acc;
  }
}

// partial[blk] = max over the block's rows of |x[i]| (NaN propagates)
__global__ void __launch_bounds__(256) k_g_absmax(int n, const double *x, double *partial) {
  __shared__ double red[4];
  double m = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) m = nmax(m, fabs(x[i]));
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = nmax(nmax(red[0], red[1]), nmax(red[2], red[3]));
}

__global__ void k_g_maxreduce(const double *partial, int nblk, double *out) {
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int b = 0; b < nblk; ++b) m = nmax(m, partial[b]);
    out[0] = m;
  }
}

// w -= V[:, 0..ncol) hcoef
__global__ void k_g_gemv_sub(int n, const double *V, int64_t ldv, int ncol, const double *hcoef, double *w) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    double acc = w[i];
    for (int c = 0; c < ncol; ++c) acc -= V[i + (int64_t)c * ldv] * hcoef[c];
    w[i] = acc;
  }
}

// Hessenberg column j after two Gram-Schmidt passes: H[0..j, j] = h1 + h2,
// H[j+1, j] = ||w|| (sc[1] holds ||w||^2); sc[2] = 1 when the new vector is
// a happy breakdown (||w|| <= breakdown max |H[0..j+1, 0..j]|), else sc[3] =
// 1 / ||w|| (the scale of v_{j+1})
__global__ void k_g_hcol(int j, const double *h1, const double *h2, double *H, double breakdown, double *sc) {
  if (threadIdx.x != 0) return;
  double hmax = 0.0;
  for (int i = 0; i <= j; ++i) {
    const double v = h1[i] + h2[i];
    H[i + j * kHLd] = v;
  }
  const double nrm = sqrt(sc[1]);
  H[j + 1 + j * kHLd] = nrm;
  for (int c = 0; c <= j; ++c)
    for (int i = 0; i <= c + 1; ++i) hmax = nmax(hmax, fabs(H[i + c * kHLd]));
  if (!(nrm > breakdown * hmax)) {
    sc[2] = 1.0;
    H[j + 1 + j * kHLd] = 0.0;
  } else {
    sc[2] = 0.0;
    sc[3] = 1.0 / nrm;
  }
}

// out = x * sc[idx]
__global__ void k_g_scale(int n, const double *x, const double *sc, int idx, double *out) {
  const double a = sc[idx];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) out[i] = x[i] * a;
}

// sc[0] = ||v||_2 = sqrt(sc[1]); v_1 = v / sc[0] (zero vector: sc[0] = 0)
__global__ void k_g_start(int n, const double *v, double *sc, double *v1) {
  const double beta = sqrt(sc[1]);
  if (blockIdx.x == 0 && threadIdx.x == 0) sc[0] = beta;
  const double a = beta > 0.0 ? 1.0 / beta : 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) v1[i] = v[i] * a;
}

// out = base + h p + beta V[:, 0..m) d   (p may be null: no h p term)
__global__ void k_g_combine(int n, const double *base, const double *p, double h, const double *V, int64_t ldv,
                            int m, const double *beta, const double *d, double *out) {
  const double bt = beta[0];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int c = 0; c < m; ++c) acc += V[i + (int64_t)c * ldv] * d[c];
    double v = base ? base[i] : 0.0;
    if (p) v += h * p[i];
    out[i] = v + bt * acc;
  }
}

// y += a x
__global__ void k_g_axpy(int n, double a, const double *x, double *y) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) y[i] += a * x[i];
}

// out = a - b
__global__ void k_g_sub(int n, const double *a, const double *b, double *out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) out[i] = a[i] - b[i];
}

// dF = J_dev(x_k)(x1 - x_k) - (I_dev(x1) - I_dev(x_k)) per node
__global__ void k_g_dF(int n, const int *node_ptr, const int *node_code, const int *dev_node, const double *devD,
                       const double *devI0, const double *devI1, const double *xk, const double *x1, double *out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int c = node_ptr[i]; c < node_ptr[i + 1]; ++c) {
      const int code = node_code[c], k = code >> 1;
      double lin = 0.0;
      for (int v = 0; v < 3; ++v) {
        const int nd = dev_node[3 * k + v];
        if (nd >= 0) lin += devD[3 * k + v] * (x1[nd] - xk[nd]);
      }
      const double term = lin - (devI1[k] - devI0[k]);
      acc += (code & 1) ? -term : term;
    }
    out[i] = acc;
  }
}

// F_k(x_k) at every node: J_dev(x_k) x_k - I_dev(x_k), the part of the
// device currents that the linearisation at x_k leaves (a step feature of the
// learned controller)
__global__ void k_g_fk(int n, const int *node_ptr, const int *node_code, const int *dev_node, const double *devD,
                       const double *devI, const double *x, double *out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int c = node_ptr[i]; c < node_ptr[i + 1]; ++c) {
      const int code = node_code[c], k = code >> 1;
      double lin = 0.0;
      for (int v = 0; v < 3; ++v) {
        const int nd = dev_node[3 * k + v];
        if (nd >= 0) lin += devD[3 * k + v] * x[nd];
      }
      const double term = lin - devI[k];
      acc += (code & 1) ? -term : term;
    }
    out[i] = acc;
  }
}

// The learned step controller on one feature vector (one wave): the
// bfloat16 network of the transient kernel, out = (m, log10 h)
__global__ void __launch_bounds__(64) k_g_ctrl(const uint16_t *w, const float *norm, const float *feat, float *out) {
  float f[kMlpIn], o[kMlpOut];
#pragma unroll
  for (int i = 0; i < kMlpIn; ++i) f[i] = feat[i];
  mlp_infer_wave(w, norm, f, o);
  if (threadIdx.x == 0) {
    out[0] = o[0];
    out[1] = o[1];
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

namespace {
constexpr int kTB = 256;
int blocks_for(int64_t n) { return (int)std::min<int64_t>(std::max<int64_t>((n + kTB - 1) / kTB, 1), 4096); }
}  // namespace

hipError_t g_fill(double *p, int64_t n, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_g_fill, dim3(blocks_for(n)), dim3(kTB), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t g_gather(int n, const int *map, const double *x, double *y, hipStream_t s) {
  hipLaunchKernelGGL(k_g_gather, dim3(blocks_for(n)), dim3(kTB), 0, s, n, map, x, y);
  return hipGetLastError();
}
hipError_t g_scatter(int n, const int *map, const double *x, double *y, hipStream_t s) {
  hipLaunchKernelGGL(k_g_scatter, dim3(blocks_for(n)), dim3(kTB), 0, s, n, map, x, y);
  return hipGetLastError();
}
hipError_t g_stamp(int n_dev, const int *dev_node, const double *par, const double *x, double vdd, double *devI,
                   double *devD, hipStream_t s) {
  if (n_dev == 0) return hipSuccess;
  hipLaunchKernelGGL(k_g_stamp, dim3(blocks_for(n_dev)), dim3(kTB), 0, s, n_dev, dev_node, par, x, vdd, devI, devD);
  return hipGetLastError();
}
hipError_t g_assemble(int n_ent, const int64_t *ent_pos, const int *ent_row, const int *ent_g, const int *ent_jptr,
                      const int *ent_jcode, const double *g_val, const double *devD, double *F,
                      unsigned long long *rowmax, hipStream_t s) {
  hipLaunchKernelGGL(k_g_assemble, dim3(blocks_for(n_ent)), dim3(kTB), 0, s, n_ent, ent_pos, ent_row, ent_g,
                     ent_jptr, ent_jcode, g_val, devD, F, rowmax);
  return hipGetLastError();
}
hipError_t g_extend(int n_items, const int *items, const int *nc, const int *fsz, const int *parent,
                    const int64_t *f_off, const int *r_ptr, const int *rel, double *F, hipStream_t s) {
  if (n_items == 0) return hipSuccess;
  hipLaunchKernelGGL(k_g_extend, dim3(n_items), dim3(256), 0, s, items, nc, fsz, parent, f_off, r_ptr, rel, F);
  return hipGetLastError();
}
hipError_t g_extend_small(int n_parents, const int *parents, const int *nc, const int *fsz, const int64_t *f_off,
                          const int *ch_ptr, const int *ch, const int *r_ptr, const int *rel, double *F, hipStream_t s) {
  if (n_parents == 0) return hipSuccess;
  hipLaunchKernelGGL(k_g_extend_small, dim3(n_parents), dim3(256), 0, s, parents, nc, fsz, f_off, ch_ptr, ch, r_ptr,
                     rel, F);
  return hipGetLastError();
}
hipError_t g_panel(int n_fronts, const int *fronts, int n_items, const int *items, int k0, int C, int fuse,
                   const int *c0, const int *nc, const int *fsz, const int64_t *f_off,
                   const unsigned long long *rowmax, double piv_tol, double *F, int *bad, hipStream_t s) {
  if (n_fronts > 0)
    hipLaunchKernelGGL(k_g_diag, dim3(n_fronts), dim3(64), 0, s, fronts, k0, c0, nc, fsz, f_off, rowmax, piv_tol, F,
                       bad);
  if (n_items > 0)
    hipLaunchKernelGGL(k_g_panel, dim3(n_items), dim3(256), sizeof(double) * 2 * (size_t)C * (kNB + 1), s, items,
                       k0, C, fuse, nc, fsz, f_off, F);
  return hipGetLastError();
}
hipError_t g_small_lu(int n32, const int *f32, int n64, const int *f64, const int *c0, const int *nc, const int *fsz,
                      const int64_t *f_off, const unsigned long long *rowmax, double piv_tol, double *F, int *bad,
                      hipStream_t s) {
  if (n32 > 0)
    hipLaunchKernelGGL(k_g_small_lu<32>, dim3((n32 + 3) / 4), dim3(256), 0, s, f32, n32, c0, nc, fsz, f_off, rowmax,
                       piv_tol, F, bad);
  if (n64 > 0)
    hipLaunchKernelGGL(k_g_small_lu<64>, dim3((n64 + 3) / 4), dim3(256), 0, s, f64, n64, c0, nc, fsz, f_off, rowmax,
                       piv_tol, F, bad);
  return hipGetLastError();
}
hipError_t g_set_limits() {
  return hipFuncSetAttribute(reinterpret_cast<const void *>(k_g_panel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)(sizeof(double) * 2 * 128 * (kNB + 1)));
}
hipError_t g_update(int n_items, const int *items, int k0, const int *c0, const int *nc, const int *fsz,
                    const int64_t *f_off, const unsigned long long *rowmax, double piv_tol, double *F, int *bad,
                    hipStream_t s) {
  if (n_items == 0) return hipSuccess;
  hipLaunchKernelGGL(k_g_update, dim3(n_items), dim3(256), 0, s, items, k0, c0, nc, fsz, f_off, rowmax, piv_tol, F,
                     bad);
  return hipGetLastError();
}
// tri_bs: workgroup size of the pivot-block kernels with one right-hand side
// (256 or 512); two right-hand sides always take 256 threads, whose register
// budget holds both vectors' accumulators without spilling.
hipError_t g_fwd(int n_small, const int *small, int n_big, const int *big, int n_items, const int *items,
                 int max_f, int max_nc, const int *c0, const int *nc, const int *fsz, const int64_t *f_off,
                 const int *ch_ptr, const int *ch, const int *r_ptr, const int *rel, const int *u_off, const double *F,
                 double *x, int nr, int64_t ldx, double *upd, int64_t ldu, int tri_bs, int n_trmv,
                 const int *trmv, int max_p_inv, const int64_t *inv_off, const double *Finv, double *tmp,
                 hipStream_t s) {
#define G_FWD_TRI(NR, BS)                                                                                           \
  hipLaunchKernelGGL((k_g_fwd_tri<NR, BS>), dim3(n_big), dim3(BS), sizeof(double) * NR * (size_t)max_f, s, big, c0,  \
                     nc, fsz, f_off, ch_ptr, ch, r_ptr, rel, u_off, F, x, ldx, upd, ldu, inv_off, tmp);
#define G_FWD(NR)                                                                                                   \
  if (n_small > 0)                                                                                                  \
    hipLaunchKernelGGL(k_g_fwd_small<NR>, dim3((n_small + 3) / 4), dim3(256), 0, s, small, n_small, c0, nc, fsz,    \
                       f_off, ch_ptr, ch, r_ptr, rel, u_off, F, x, ldx, upd, ldu);                                  \
  if (n_big > 0) {                                                                                                  \
    if (tri_bs == 512 && NR == 1) {                                                                                 \
      G_FWD_TRI(NR, 512)                                                                                            \
    } else {                                                                                                        \
      G_FWD_TRI(NR, 256)                                                                                            \
    }                                                                                                               \
  }                                                                                                                 \
  if (n_trmv > 0)                                                                                                   \
    hipLaunchKernelGGL((k_g_trmv<NR, false>), dim3(n_trmv), dim3(512), sizeof(double) * NR * (size_t)max_p_inv, s,  \
                       trmv, c0, nc, inv_off, Finv, tmp, x, ldx);                                                   \
  if (n_items > 0)                                                                                                  \
    hipLaunchKernelGGL(k_g_fwd_gemv<NR>, dim3(n_items), dim3(256), sizeof(double) * NR * (size_t)max_nc, s, items,  \
                       c0, nc, fsz, f_off, u_off, F, x, ldx, upd, ldu);
  if (nr == 2) {
    G_FWD(2)
  } else {
    G_FWD(1)
  }
#undef G_FWD
#undef G_FWD_TRI
  return hipGetLastError();
}
hipError_t g_bwd(int n_small, const int *small, int n_big, const int *big, int n_items, const int *items,
                 int max_f, int max_nc, const int *c0, const int *nc, const int *fsz, const int64_t *f_off,
                 const int *r_ptr, const int *r_idx, const double *F, double *x, int nr, int64_t ldx, int tri_bs,
                 int n_trmv, const int *trmv, int max_p_inv, const int64_t *inv_off, const double *Finv,
                 double *tmp, hipStream_t s) {
#define G_BWD_TRI(NR, BS)                                                                                           \
  hipLaunchKernelGGL((k_g_bwd_tri<NR, BS>), dim3(n_big), dim3(BS), sizeof(double) * NR * (size_t)max_nc, s, big, c0, \
                     nc, fsz, f_off, F, x, ldx, inv_off);
#define G_BWD(NR)                                                                                                   \
  if (n_small > 0)                                                                                                  \
    hipLaunchKernelGGL(k_g_bwd_small<NR>, dim3((n_small + 3) / 4), dim3(256), 0, s, small, n_small, c0, nc, fsz,    \
                       f_off, r_ptr, r_idx, F, x, ldx);                                                             \
  if (n_items > 0)                                                                                                  \
    hipLaunchKernelGGL(k_g_bwd_gemv<NR>, dim3(n_items), dim3(256), sizeof(double) * NR * (size_t)max_f, s, items,   \
                       c0, nc, fsz, f_off, r_ptr, r_idx, F, x, ldx);                                                \
  if (n_big > 0) {                                                                                                  \
    if (tri_bs == 512 && NR == 1) {                                                                                 \
      G_BWD_TRI(NR, 512)                                                                                            \
    } else {                                                                                                        \
      G_BWD_TRI(NR, 256)                                                                                            \
    }                                                                                                               \
  }                                                                                                                 \
  if (n_trmv > 0) {                                                                                                 \
    hipLaunchKernelGGL((k_g_trmv<NR, true>), dim3(n_trmv), dim3(512), sizeof(double) * NR * (size_t)max_p_inv, s,   \
                       trmv, c0, nc, inv_off, Finv, x, tmp, ldx);                                                   \
    hipLaunchKernelGGL(k_g_copy_rows<NR>, dim3(n_trmv), dim3(256), 0, s, trmv, c0, nc, tmp, x, ldx);               \
  }
  if (nr == 2) {
    G_BWD(2)
  } else {
    G_BWD(1)
  }
#undef G_BWD
#undef G_BWD_TRI
  return hipGetLastError();
}
hipError_t g_inv(int n_items, const int *items, const int *nc, const int *fsz, const int64_t *f_off,
                 const int64_t *inv_off, const double *F, double *Finv, hipStream_t s) {
  if (n_items == 0) return hipSuccess;
  hipLaunchKernelGGL(k_g_inv, dim3(n_items), dim3(256), 0, s, items, nc, fsz, f_off, inv_off, F, Finv);
  return hipGetLastError();
}
hipError_t g_sources(int n_src, const int *src_ptr, const double *src_t, const double *src_v, double t, double tm,
                     double *u, double *slope, hipStream_t s) {
  if (n_src == 0) return hipSuccess;
  hipLaunchKernelGGL(k_g_sources, dim3(blocks_for(n_src)), dim3(kTB), 0, s, n_src, src_ptr, src_t, src_v, t, tm, u,
                     slope);
  return hipGetLastError();
}
hipError_t g_rhs(int n, const int *g_rowptr, const int *g_col, const double *g_val, const int *b_rowptr,
                 const int *b_col, const double *b_val, const int *node_ptr, const int *node_code, const double *devI,
                 const double *x, const double *u, const double *sl, double *r, double *bs, hipStream_t s) {
  hipLaunchKernelGGL(k_g_rhs, dim3(blocks_for(n)), dim3(kTB), 0, s, n, g_rowptr, g_col, g_val, b_rowptr, b_col,
                     b_val, node_ptr, node_code, devI, x, u, sl, r, bs);
  return hipGetLastError();
}
hipError_t g_spmv(int n, const int *rp, const int *ci, const double *val, const double *x, double alpha, double *y,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_g_spmv, dim3(blocks_for(n)), dim3(kTB), 0, s, n, rp, ci, val, x, alpha, y);
  return hipGetLastError();
}
// out[0..ncol) = V[:, 0..ncol)^T w, fixed summation order; partial: kRB * ncol doubles
hipError_t g_dots(int n, const double *V, int64_t ldv, int ncol, const double *w, double *partial, double *out,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_g_dots, dim3(kRB), dim3(256), 0, s, n, V, ldv, ncol, w, partial);
  hipLaunchKernelGGL(k_g_reduce, dim3(1), dim3(64), 0, s, partial, kRB, ncol, out);
  return hipGetLastError();
}
hipError_t g_absmax(int n, const double *x, double *partial, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_g_absmax, dim3(kRB), dim3(256), 0, s, n, x, partial);
  hipLaunchKernelGGL(k_g_maxreduce, dim3(1), dim3(64), 0, s, partial, kRB, out);
  return hipGetLastError();
}
hipError_t g_gemv_sub(int n, const double *V, int64_t ldv, int ncol, const double *hcoef, double *w, hipStream_t s) {
  hipLaunchKernelGGL(k_g_gemv_sub, dim3(blocks_for(n)), dim3(kTB), 0, s, n, V, ldv, ncol, hcoef, w);
  return hipGetLastError();
}
hipError_t g_hcol(int j, const double *h1, const double *h2, double *H, double breakdown, double *sc, hipStream_t s) {
  hipLaunchKernelGGL(k_g_hcol, dim3(1), dim3(64), 0, s, j, h1, h2, H, breakdown, sc);
  return hipGetLastError();
}
hipError_t g_scale(int n, const double *x, const double *sc, int idx, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_g_scale, dim3(blocks_for(n)), dim3(kTB), 0, s, n, x, sc, idx, out);
  return hipGetLastError();
}
hipError_t g_start(int n, const double *v, double *sc, double *v1, hipStream_t s) {
  hipLaunchKernelGGL(k_g_start, dim3(blocks_for(n)), dim3(kTB), 0, s, n, v, sc, v1);
  return hipGetLastError();
}
hipError_t g_combine(int n, const double *base, const double *p, double h, const double *V, int64_t ldv, int m,
                     const double *beta, const double *d, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_g_combine, dim3(blocks_for(n)), dim3(kTB), 0, s, n, base, p, h, V, ldv, m, beta, d, out);
  return hipGetLastError();
}
hipError_t g_axpy(int n, double a, const double *x, double *y, hipStream_t s) {
  hipLaunchKernelGGL(k_g_axpy, dim3(blocks_for(n)), dim3(kTB), 0, s, n, a, x, y);
  return hipGetLastError();
}
hipError_t g_sub(int n, const double *a, const double *b, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_g_sub, dim3(blocks_for(n)), dim3(kTB), 0, s, n, a, b, out);
  return hipGetLastError();
}
hipError_t g_fk(int n, const int *node_ptr, const int *node_code, const int *dev_node, const double *devD,
                const double *devI, const double *x, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_g_fk, dim3(blocks_for(n)), dim3(kTB), 0, s, n, node_ptr, node_code, dev_node, devD, devI, x,
                     out);
  return hipGetLastError();
}
hipError_t g_ctrl(const uint16_t *w, const float *norm, const float *feat, float *out, hipStream_t s) {
  hipLaunchKernelGGL(k_g_ctrl, dim3(1), dim3(64), 0, s, w, norm, feat, out);
  return hipGetLastError();
}
hipError_t g_dF(int n, const int *node_ptr, const int *node_code, const int *dev_node, const double *devD,
                const double *devI0, const double *devI1, const double *xk, const double *x1, double *out,
                hipStream_t s) {
  hipLaunchKernelGGL(k_g_dF, dim3(blocks_for(n)), dim3(kTB), 0, s, n, node_ptr, node_code, dev_node, devD, devI0,
                     devI1, xk, x1, out);
  return hipGetLastError();
}

}  // namespace expri
