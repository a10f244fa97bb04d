// Training and batch inference of the learned step controller's network
// (mlp.hpp) on gfx950: float32 forward and backward passes over a minibatch
// with a deterministic reduction of the per-workgroup gradients, Adam, the
// standardisation statistics, and inference in float32 or bfloat16.  The
// C-ABI entry points are at the end (declared in include/expri.h).
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/expri.h"
#include "mlp.hpp"

namespace expri {

constexpr int kMlpBS = 256;       // threads per workgroup of the training kernels
constexpr int kMlpS = 64;         // samples per workgroup
constexpr int kPartial = kMlpParams + 1;  // per-workgroup gradient + loss

// training layout -> inference layout (W1, W2 transposed); W = float or bf16 bits
template <class W>
__global__ void k_mlp_pack(const float *p, W *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kMlpParams) return;
  int src = i;
  if (i < kMlpB1) {  // W1T[a][j] <- W1[j][a]
    const int a = i / kMlpHid, j = i % kMlpHid;
    src = kMlpW1 + j * kMlpIn + a;
  } else if (i >= kMlpW2 && i < kMlpB2) {  // W2T[a][j] <- W2[j][a]
    const int r = i - kMlpW2, a = r / kMlpHid, j = r % kMlpHid;
    src = kMlpW2 + j * kMlpHid + a;
  }
  const float v = p[src];
  if constexpr (sizeof(W) == 2) out[i] = (uint16_t)(__float_as_uint(bf16_round(v)) >> 16);
  else out[i] = v;
}

// one wave per sample
template <class W>
__global__ void __launch_bounds__(256) k_mlp_forward(const W *w, const float *norm, const float *X, float *Y, int n) {
  const int s = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (s >= n) return;
  float f[kMlpIn], y[kMlpOut];
#pragma unroll
  for (int i = 0; i < kMlpIn; ++i) f[i] = X[(int64_t)s * kMlpIn + i];
  mlp_infer_wave(w, norm, f, y);
  if ((threadIdx.x & 63) < kMlpOut) Y[(int64_t)s * kMlpOut + (threadIdx.x & 63)] = y[threadIdx.x & 63];
}

// mean and standard deviation (population) of the 8 inputs and 2 targets;
// one workgroup, double sums in a fixed order
__global__ void __launch_bounds__(256) k_mlp_norm(const float *X, const float *T, int n, float *norm) {
  constexpr int C = kMlpIn + kMlpOut;
  __shared__ double red[256][C];
  __shared__ double mean[C];
  const int t = threadIdx.x;
  for (int pass = 0; pass < 2; ++pass) {
    double acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = 0.0;
    for (int s = t; s < n; s += 256)
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const double v = c < kMlpIn ? X[(int64_t)s * kMlpIn + c] : T[(int64_t)s * kMlpOut + c - kMlpIn];
        acc[c] += pass == 0 ? v : (v - mean[c]) * (v - mean[c]);
      }
#pragma unroll
    for (int c = 0; c < C; ++c) red[t][c] = acc[c];
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
      if (t < h)
#pragma unroll
        for (int c = 0; c < C; ++c) red[t][c] += red[t + h][c];
      __syncthreads();
    }
    if (t < C) {
      if (pass == 0) {
        mean[t] = red[0][t] / n;
      } else {
        double sd = sqrt(red[0][t] / n);
        if (sd == 0.0) sd = 1.0;
        const int mo = t < kMlpIn ? t : 2 * kMlpIn + (t - kMlpIn);
        norm[mo] = (float)mean[t];
        norm[mo + (t < kMlpIn ? kMlpIn : kMlpOut)] = (float)sd;
      }
    }
    __syncthreads();
  }
}

// forward + backward of kMlpS samples; writes this workgroup's gradient sum
// and loss sum (already divided by n) to partial[blockIdx.x]
__global__ void __launch_bounds__(kMlpBS) k_mlp_grad(const float *p, const float *norm, const float *X,
                                                     const float *T, int n, float *partial) {
  extern __shared__ float sm[];
  float *P = sm;                              // kMlpParams
  float *Xs = P + kMlpParams;                 // S x 8
  float *Ts = Xs + kMlpS * kMlpIn;            // S x 2
  float *A1 = Ts + kMlpS * kMlpOut;           // S x 64
  float *A2 = A1 + kMlpS * kMlpHid;           // S x 64
  float *D2 = A2 + kMlpS * kMlpHid;           // S x 64
  float *D1 = D2 + kMlpS * kMlpHid;           // S x 64
  float *DY = D1 + kMlpS * kMlpHid;           // S x 2
  float *red = DY + kMlpS * kMlpOut;          // kMlpBS
  const int t = threadIdx.x;
  const int s0 = blockIdx.x * kMlpS;
  for (int i = t; i < kMlpParams; i += kMlpBS) P[i] = p[i];
  for (int i = t; i < kMlpS * kMlpIn; i += kMlpBS) {
    const int s = s0 + i / kMlpIn, c = i % kMlpIn;
    Xs[i] = s < n ? (X[(int64_t)s * kMlpIn + c] - norm[c]) / norm[kMlpIn + c] : 0.0f;
  }
  for (int i = t; i < kMlpS * kMlpOut; i += kMlpBS) {
    const int s = s0 + i / kMlpOut, o = i % kMlpOut;
    Ts[i] = s < n ? (T[(int64_t)s * kMlpOut + o] - norm[2 * kMlpIn + o]) / norm[2 * kMlpIn + kMlpOut + o] : 0.0f;
  }
  __syncthreads();
  for (int i = t; i < kMlpS * kMlpHid; i += kMlpBS) {
    const int s = i / kMlpHid, j = i % kMlpHid;
    float z = P[kMlpB1 + j];
    for (int a = 0; a < kMlpIn; ++a) z = fmaf(P[kMlpW1 + j * kMlpIn + a], Xs[s * kMlpIn + a], z);
    A1[i] = fmaxf(z, 0.0f);
  }
  __syncthreads();
  for (int i = t; i < kMlpS * kMlpHid; i += kMlpBS) {
    const int s = i / kMlpHid, j = i % kMlpHid;
    float z = P[kMlpB2 + j];
    for (int a = 0; a < kMlpHid; ++a) z = fmaf(P[kMlpW2 + j * kMlpHid + a], A1[s * kMlpHid + a], z);
    A2[i] = fmaxf(z, 0.0f);
  }
  __syncthreads();
  float lp = 0.0f;
  for (int i = t; i < kMlpS * kMlpOut; i += kMlpBS) {
    const int s = i / kMlpOut, o = i % kMlpOut;
    float y = P[kMlpB3 + o];
    for (int a = 0; a < kMlpHid; ++a) y = fmaf(P[kMlpW3 + o * kMlpHid + a], A2[s * kMlpHid + a], y);
    const float r = s0 + s < n ? y - Ts[i] : 0.0f;
    DY[i] = r / n;
    lp += 0.5f * r * r / n;
  }
  __syncthreads();
  for (int i = t; i < kMlpS * kMlpHid; i += kMlpBS) {
    const int s = i / kMlpHid, j = i % kMlpHid;
    float d = 0.0f;
    for (int o = 0; o < kMlpOut; ++o) d = fmaf(P[kMlpW3 + o * kMlpHid + j], DY[s * kMlpOut + o], d);
    D2[i] = A2[i] > 0.0f ? d : 0.0f;
  }
  __syncthreads();
  for (int i = t; i < kMlpS * kMlpHid; i += kMlpBS) {
    const int s = i / kMlpHid, a = i % kMlpHid;
    float d = 0.0f;
    for (int j = 0; j < kMlpHid; ++j) d = fmaf(P[kMlpW2 + j * kMlpHid + a], D2[s * kMlpHid + j], d);
    D1[i] = A1[i] > 0.0f ? d : 0.0f;
  }
  __syncthreads();
  float *out = partial + (int64_t)blockIdx.x * kPartial;
  for (int q = t; q < kMlpParams; q += kMlpBS) {
    float g = 0.0f;
    if (q < kMlpB1) {
      const int j = q / kMlpIn, a = q % kMlpIn;
      for (int s = 0; s < kMlpS; ++s) g = fmaf(D1[s * kMlpHid + j], Xs[s * kMlpIn + a], g);
    } else if (q < kMlpW2) {
      const int j = q - kMlpB1;
      for (int s = 0; s < kMlpS; ++s) g += D1[s * kMlpHid + j];
    } else if (q < kMlpB2) {
      const int j = (q - kMlpW2) / kMlpHid, a = (q - kMlpW2) % kMlpHid;
      for (int s = 0; s < kMlpS; ++s) g = fmaf(D2[s * kMlpHid + j], A1[s * kMlpHid + a], g);
    } else if (q < kMlpW3) {
      const int j = q - kMlpB2;
      for (int s = 0; s < kMlpS; ++s) g += D2[s * kMlpHid + j];
    } else if (q < kMlpB3) {
      const int o = (q - kMlpW3) / kMlpHid, a = (q - kMlpW3) % kMlpHid;
      for (int s = 0; s < kMlpS; ++s) g = fmaf(DY[s * kMlpOut + o], A2[s * kMlpHid + a], g);
    } else {
      const int o = q - kMlpB3;
      for (int s = 0; s < kMlpS; ++s) g += DY[s * kMlpOut + o];
    }
    out[q] = g;
  }
  red[t] = lp;
  __syncthreads();
  for (int h = kMlpBS / 2; h >= 1; h >>= 1) {
    if (t < h) red[t] += red[t + h];
    __syncthreads();
  }
  if (t == 0) out[kMlpParams] = red[0];
}

// sum of the per-workgroup partials in workgroup order; optionally one Adam
// step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on the parameters
__global__ void __launch_bounds__(256) k_mlp_reduce(const float *partial, int n_wg, float *grad, float *loss,
                                                    int adam, float *p, float *m, float *v, float lr, int step) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q > kMlpParams) return;
  float g = 0.0f;
  for (int w = 0; w < n_wg; ++w) g += partial[(int64_t)w * kPartial + q];
  if (q == kMlpParams) {
    *loss = g;
    return;
  }
  grad[q] = g;
  if (adam) {
    const float b1 = 0.9f, b2 = 0.999f;
    const float mq = b1 * m[q] + (1.0f - b1) * g;
    const float vq = b2 * v[q] + (1.0f - b2) * g * g;
    m[q] = mq;
    v[q] = vq;
    const float mh = mq / (1.0f - powf(b1, (float)step));
    const float vh = vq / (1.0f - powf(b2, (float)step));
    p[q] -= lr * mh / (sqrtf(vh) + 1e-8f);
  }
}

size_t mlp_grad_lds() {
  return sizeof(float) * (kMlpParams + kMlpS * (kMlpIn + kMlpOut) + 4 * kMlpS * kMlpHid + kMlpS * kMlpOut + kMlpBS);
}

hipError_t launch_mlp_pack(const float *p, void *out, bool bf16, hipStream_t s) {
  const int g = (kMlpParams + 255) / 256;
  if (bf16) hipLaunchKernelGGL(k_mlp_pack<uint16_t>, dim3(g), dim3(256), 0, s, p, static_cast<uint16_t *>(out));
  else hipLaunchKernelGGL(k_mlp_pack<float>, dim3(g), dim3(256), 0, s, p, static_cast<float *>(out));
  return hipGetLastError();
}

}  // namespace expri

using namespace expri;

struct expri_mlp {
  hipStream_t stream = nullptr;
  float *p = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr, *norm = nullptr, *loss = nullptr;
  float *partial = nullptr;
  void *infer = nullptr;       // packed inference weights (float or bf16)
  int partial_cap = 0;         // workgroups the partial buffer holds
  int step = 0;
  std::string err;
};

namespace {

expri_status mlp_fail(expri_mlp *m, hipError_t e, const char *what) {
  if (m) m->err = std::string(what) + ": " + hipGetErrorString(e);
  return EXPRI_EHIP;
}

#define MCHK(M, X)                                  \
  do {                                              \
    hipError_t e_ = (X);                            \
    if (e_ != hipSuccess) return mlp_fail(M, e_, #X); \
  } while (0)

expri_status ensure_partial(expri_mlp *m, int n_wg) {
  if (n_wg <= m->partial_cap) return EXPRI_OK;
  if (m->partial) (void)hipFree(m->partial);
  m->partial = nullptr;
  MCHK(m, hipMalloc(reinterpret_cast<void **>(&m->partial), sizeof(float) * (size_t)n_wg * kPartial));
  m->partial_cap = n_wg;
  return EXPRI_OK;
}

expri_status run_grad(expri_mlp *m, const float *X, const float *T, int32_t n, bool adam, float lr) {
  if (n < 1 || !X || !T) return EXPRI_EINVAL;
  const int n_wg = (n + kMlpS - 1) / kMlpS;
  expri_status st = ensure_partial(m, n_wg);
  if (st != EXPRI_OK) return st;
  hipLaunchKernelGGL(k_mlp_grad, dim3(n_wg), dim3(kMlpBS), mlp_grad_lds(), m->stream, m->p, m->norm, X, T, n,
                     m->partial);
  MCHK(m, hipGetLastError());
  if (adam) ++m->step;
  hipLaunchKernelGGL(k_mlp_reduce, dim3((kMlpParams + 1 + 255) / 256), dim3(256), 0, m->stream, m->partial, n_wg,
                     m->grad, m->loss, adam ? 1 : 0, m->p, m->m, m->v, lr, m->step);
  MCHK(m, hipGetLastError());
  return EXPRI_OK;
}

}  // namespace

extern "C" {

expri_status expri_mlp_create(expri_mlp **out, const float *params, void *hip_stream) {
  if (!out || !params) return EXPRI_EINVAL;
  *out = nullptr;
  expri_mlp *m = new (std::nothrow) expri_mlp();
  if (!m) return EXPRI_ENOMEM;
  m->stream = static_cast<hipStream_t>(hip_stream);
  const size_t pb = sizeof(float) * kMlpParams;
  hipError_t e = hipMalloc(reinterpret_cast<void **>(&m->p), pb);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&m->m), pb);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&m->v), pb);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&m->grad), pb);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&m->norm), sizeof(float) * kMlpNorm);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&m->loss), sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&m->infer, pb);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_mlp_grad), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)mlp_grad_lds());
  if (e == hipSuccess) e = hipMemcpy(m->p, params, pb, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(m->m, 0, pb);
  if (e == hipSuccess) e = hipMemset(m->v, 0, pb);
  if (e == hipSuccess) {
    float unit[kMlpNorm];
    for (int i = 0; i < kMlpNorm; ++i) unit[i] = 0.0f;
    for (int i = 0; i < kMlpIn; ++i) unit[kMlpIn + i] = 1.0f;
    for (int o = 0; o < kMlpOut; ++o) unit[2 * kMlpIn + kMlpOut + o] = 1.0f;
    e = hipMemcpy(m->norm, unit, sizeof(unit), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    expri_mlp_destroy(m);
    return EXPRI_EHIP;
  }
  *out = m;
  return EXPRI_OK;
}

expri_status expri_mlp_set_norm(expri_mlp *m, const float *norm) {
  if (!m || !norm) return EXPRI_EINVAL;
  for (int i = 0; i < kMlpIn; ++i)
    if (!(norm[kMlpIn + i] > 0.0f)) return EXPRI_EINVAL;
  for (int o = 0; o < kMlpOut; ++o)
    if (!(norm[2 * kMlpIn + kMlpOut + o] > 0.0f)) return EXPRI_EINVAL;
  MCHK(m, hipMemcpyAsync(m->norm, norm, sizeof(float) * kMlpNorm, hipMemcpyHostToDevice, m->stream));
  MCHK(m, hipStreamSynchronize(m->stream));
  return EXPRI_OK;
}

expri_status expri_mlp_fit_norm(expri_mlp *m, const float *X, const float *T, int32_t n) {
  if (!m || !X || !T || n < 1) return EXPRI_EINVAL;
  hipLaunchKernelGGL(k_mlp_norm, dim3(1), dim3(256), 0, m->stream, X, T, n, m->norm);
  MCHK(m, hipGetLastError());
  MCHK(m, hipStreamSynchronize(m->stream));
  return EXPRI_OK;
}

expri_status expri_mlp_get(const expri_mlp *m, float *params, float *norm) {
  if (!m || (!params && !norm)) return EXPRI_EINVAL;
  expri_mlp *mm = const_cast<expri_mlp *>(m);
  MCHK(mm, hipStreamSynchronize(m->stream));
  if (params) MCHK(mm, hipMemcpy(params, m->p, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost));
  if (norm) MCHK(mm, hipMemcpy(norm, m->norm, sizeof(float) * kMlpNorm, hipMemcpyDeviceToHost));
  return EXPRI_OK;
}

expri_status expri_mlp_grad(expri_mlp *m, const float *X, const float *T, int32_t n, float *loss, float *grad) {
  if (!m) return EXPRI_EINVAL;
  expri_status st = run_grad(m, X, T, n, false, 0.0f);
  if (st != EXPRI_OK) return st;
  MCHK(m, hipStreamSynchronize(m->stream));
  if (loss) MCHK(m, hipMemcpy(loss, m->loss, sizeof(float), hipMemcpyDeviceToHost));
  if (grad) MCHK(m, hipMemcpy(grad, m->grad, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost));
  return EXPRI_OK;
}

expri_status expri_mlp_adam_step(expri_mlp *m, const float *X, const float *T, int32_t n, float lr, float *loss) {
  if (!m || !(lr > 0.0f)) return EXPRI_EINVAL;
  expri_status st = run_grad(m, X, T, n, true, lr);
  if (st != EXPRI_OK) return st;
  if (loss) {
    MCHK(m, hipMemcpyAsync(loss, m->loss, sizeof(float), hipMemcpyDeviceToHost, m->stream));
    MCHK(m, hipStreamSynchronize(m->stream));
  }
  return EXPRI_OK;
}

expri_status expri_mlp_forward(expri_mlp *m, const float *X, float *Y, int32_t n, int32_t bf16) {
  if (!m || !X || !Y || n < 1) return EXPRI_EINVAL;
  MCHK(m, launch_mlp_pack(m->p, m->infer, bf16 != 0, m->stream));
  const int g = (n + 3) / 4;
  if (bf16)
    hipLaunchKernelGGL(k_mlp_forward<uint16_t>, dim3(g), dim3(256), 0, m->stream,
                       static_cast<const uint16_t *>(m->infer), m->norm, X, Y, n);
  else
    hipLaunchKernelGGL(k_mlp_forward<float>, dim3(g), dim3(256), 0, m->stream,
                       static_cast<const float *>(m->infer), m->norm, X, Y, n);
  MCHK(m, hipGetLastError());
  MCHK(m, hipStreamSynchronize(m->stream));
  return EXPRI_OK;
}

const char *expri_mlp_last_error(const expri_mlp *m) { return m ? m->err.c_str() : "null network"; }

void expri_mlp_destroy(expri_mlp *m) {
  if (!m) return;
  for (void *q : {static_cast<void *>(m->p), static_cast<void *>(m->m), static_cast<void *>(m->v),
                  static_cast<void *>(m->grad), static_cast<void *>(m->norm), static_cast<void *>(m->loss),
                  static_cast<void *>(m->partial), m->infer})
    if (q) (void)hipFree(q);
  delete m;
}

}  // extern "C"
