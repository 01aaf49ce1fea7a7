// Loading / window predictor for windowed beamspace MVDR (an addition to the paper's method:
// the paper fixes the loading and the window width).  Per (target, subband) pair the input is
// the 64-bin training power profile around the target's beam bin, log10(P / sigma^2); a
// multilayer perceptron 64 -> 128 -> 128 -> 2 (GELU, exact erf) predicts out0 = ln(delta /
// sigma^2) and out1 = log2(W - 1).  Weights are kept in FP32 by the caller and used rounded
// to BF16 (round to nearest even); activations and accumulation are FP32.  Training labels
// come from a sweep of the plain method scored by output SINR against the exact
// interference-plus-noise covariance of the synthetic scene.
#include <math.h>

#include <mutex>

#include "wbm_dev.h"
#include "wbm_learned.h"
#include "wbmvdr.h"

namespace wbm {

constexpr int kIn = 64, kH = 128, kOut = 2;
constexpr int oW1 = 0, oB1 = oW1 + kH * kIn, oW2 = oB1 + kH, oB2 = oW2 + kH * kH,
              oW3 = oB2 + kH, oB3 = oW3 + kOut * kH, kParams = oB3 + kOut;
static_assert(kParams == 25090, "parameter count");

constexpr int kFwdSB = 32;   // samples per workgroup, forward
constexpr int kBwdSB = 16;   // samples per workgroup, backward

__device__ __forceinline__ float bf16r(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xffff0000u);
}

__device__ __forceinline__ float gelu_f(float a) {
  return 0.5f * a * (1.0f + erff(a * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad_f(float a) {
  return 0.5f * (1.0f + erff(a * 0.70710678118654752f)) +
         a * expf(-0.5f * a * a) * 0.39894228040143268f;
}

// ------------------------------------------------------------------------------------------
// feat[t][k][j] = log10(sum_g prof[k][g][t][j] / (L sigma^2) + 1e-30)
__global__ void k_features(const float* __restrict__ prof, int T, int K, int G, int L,
                           float noise, float* __restrict__ feat) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)T * K * 64) return;
  const int j = (int)(idx & 63);
  const int64_t pk = idx >> 6;
  const int k = (int)(pk % K), t = (int)(pk / K);
  float s = 0.f;
  for (int gg = 0; gg < G; ++gg) s += prof[(((int64_t)k * G + gg) * T + t) * 64 + j];
  feat[idx] = log10f(s / ((float)L * noise) + 1e-30f);
}

// ------------------------------------------------------------------------------------------
// Forward pass of kFwdSB samples per workgroup of 128 threads (one hidden unit per thread).
__global__ __launch_bounds__(128) void k_mlp_forward(const float* __restrict__ P,
                                                     const float* __restrict__ in, int n,
                                                     float* __restrict__ out) {
  __shared__ float xs[kFwdSB][kIn];
  __shared__ float h1[kFwdSB][kH];
  __shared__ float h2[kFwdSB][kH];
  const int s0 = blockIdx.x * kFwdSB;
  const int tid = threadIdx.x;
  for (int i = tid; i < kFwdSB * kIn; i += 128) {
    const int s = i / kIn, c = i - s * kIn;
    xs[s][c] = (s0 + s < n) ? in[(int64_t)(s0 + s) * kIn + c] : 0.f;
  }
  __syncthreads();
  {
    float w[kIn];
#pragma unroll
    for (int i = 0; i < kIn; ++i) w[i] = bf16r(P[oW1 + tid * kIn + i]);
    const float b = bf16r(P[oB1 + tid]);
    for (int s = 0; s < kFwdSB; ++s) {
      float a = b;
#pragma unroll
      for (int i = 0; i < kIn; ++i) a += w[i] * xs[s][i];
      h1[s][tid] = gelu_f(a);
    }
  }
  __syncthreads();
  {
    float acc[kFwdSB];
    const float b = bf16r(P[oB2 + tid]);
#pragma unroll
    for (int s = 0; s < kFwdSB; ++s) acc[s] = b;
    for (int i0 = 0; i0 < kH; i0 += 32) {
      float w[32];
#pragma unroll
      for (int i = 0; i < 32; ++i) w[i] = bf16r(P[oW2 + tid * kH + i0 + i]);
#pragma unroll
      for (int s = 0; s < kFwdSB; ++s)
#pragma unroll
        for (int i = 0; i < 32; ++i) acc[s] += w[i] * h1[s][i0 + i];
    }
#pragma unroll
    for (int s = 0; s < kFwdSB; ++s) h2[s][tid] = gelu_f(acc[s]);
  }
  __syncthreads();
  if (tid < kFwdSB * kOut) {
    const int s = tid >> 1, o = tid & 1;
    float a = bf16r(P[oB3 + o]);
    for (int j = 0; j < kH; ++j) a += bf16r(P[oW3 + o * kH + j]) * h2[s][j];
    if (s0 + s < n) out[(int64_t)(s0 + s) * kOut + o] = a;
  }
}

// Loss and gradient partials of kBwdSB samples per workgroup: loss = mean over the n samples
// and both outputs of (out - y)^2.  part [gridDim.x][kParams], loss_part [gridDim.x].
__global__ __launch_bounds__(128) void k_mlp_backward(const float* __restrict__ P,
                                                      const float* __restrict__ in,
                                                      const float* __restrict__ tgt, int n,
                                                      float* __restrict__ part,
                                                      float* __restrict__ loss_part) {
  __shared__ float xs[kBwdSB][kIn];
  __shared__ float a1[kBwdSB][kH], h1[kBwdSB][kH], a2[kBwdSB][kH], h2[kBwdSB][kH];
  __shared__ float d2[kBwdSB][kH], d1[kBwdSB][kH];
  __shared__ float dout[kBwdSB][kOut];
  __shared__ float lred[128];
  const int s0 = blockIdx.x * kBwdSB;
  const int tid = threadIdx.x;
  float* g = part + (int64_t)blockIdx.x * kParams;
  for (int i = tid; i < kBwdSB * kIn; i += 128) {
    const int s = i / kIn, c = i - s * kIn;
    xs[s][c] = (s0 + s < n) ? in[(int64_t)(s0 + s) * kIn + c] : 0.f;
  }
  __syncthreads();
  // forward, keeping pre-activations
  {
    const float b = bf16r(P[oB1 + tid]);
    for (int s = 0; s < kBwdSB; ++s) {
      float a = b;
      for (int i = 0; i < kIn; ++i) a += bf16r(P[oW1 + tid * kIn + i]) * xs[s][i];
      a1[s][tid] = a;
      h1[s][tid] = gelu_f(a);
    }
  }
  __syncthreads();
  {
    const float b = bf16r(P[oB2 + tid]);
    for (int s = 0; s < kBwdSB; ++s) {
      float a = b;
      for (int i = 0; i < kH; ++i) a += bf16r(P[oW2 + tid * kH + i]) * h1[s][i];
      a2[s][tid] = a;
      h2[s][tid] = gelu_f(a);
    }
  }
  __syncthreads();
  float lsum = 0.f;
  if (tid < kBwdSB * kOut) {
    const int s = tid >> 1, o = tid & 1;
    float a = bf16r(P[oB3 + o]);
    for (int j = 0; j < kH; ++j) a += bf16r(P[oW3 + o * kH + j]) * h2[s][j];
    float d = 0.f;
    if (s0 + s < n) {
      const float e = a - tgt[(int64_t)(s0 + s) * kOut + o];
      lsum = e * e / (float)(n * kOut);
      d = 2.0f * e / (float)(n * kOut);
    }
    dout[s][o] = d;
  }
  lred[tid] = lsum;
  __syncthreads();
  for (int off = 64; off > 0; off >>= 1) {
    if (tid < off) lred[tid] += lred[tid + off];
    __syncthreads();
  }
  if (tid == 0) loss_part[blockIdx.x] = lred[0];
  // layer 3
  for (int o = 0; o < kOut; ++o) {
    float acc = 0.f;
    for (int s = 0; s < kBwdSB; ++s) acc += dout[s][o] * h2[s][tid];
    g[oW3 + o * kH + tid] = acc;
  }
  if (tid < kOut) {
    float acc = 0.f;
    for (int s = 0; s < kBwdSB; ++s) acc += dout[s][tid];
    g[oB3 + tid] = acc;
  }
  {
    const float w0 = bf16r(P[oW3 + tid]), w1 = bf16r(P[oW3 + kH + tid]);
    for (int s = 0; s < kBwdSB; ++s)
      d2[s][tid] = (dout[s][0] * w0 + dout[s][1] * w1) * gelu_grad_f(a2[s][tid]);
  }
  __syncthreads();
  // layer 2: row tid of dW2, bias, and d1 = (W2^T d2) * gelu'(a1) (column tid of W2)
  {
    float bsum = 0.f;
    for (int s = 0; s < kBwdSB; ++s) bsum += d2[s][tid];
    g[oB2 + tid] = bsum;
    for (int i = 0; i < kH; ++i) {
      float acc = 0.f;
      for (int s = 0; s < kBwdSB; ++s) acc += d2[s][tid] * h1[s][i];
      g[oW2 + tid * kH + i] = acc;
    }
    for (int s = 0; s < kBwdSB; ++s) {
      float acc = 0.f;
      for (int j = 0; j < kH; ++j) acc += d2[s][j] * bf16r(P[oW2 + j * kH + tid]);
      d1[s][tid] = acc * gelu_grad_f(a1[s][tid]);
    }
  }
  __syncthreads();
  {
    float bsum = 0.f;
    for (int s = 0; s < kBwdSB; ++s) bsum += d1[s][tid];
    g[oB1 + tid] = bsum;
    for (int i = 0; i < kIn; ++i) {
      float acc = 0.f;
      for (int s = 0; s < kBwdSB; ++s) acc += d1[s][tid] * xs[s][i];
      g[oW1 + tid * kIn + i] = acc;
    }
  }
}

// grad[p] = sum over workgroups of part[wg][p] (fixed order); loss = sum of loss_part.
__global__ void k_mlp_reduce(const float* __restrict__ part, const float* __restrict__ loss_part,
                             int nwg, float* __restrict__ grad, float* __restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < kParams) {
    float s = 0.f;
    for (int w = 0; w < nwg; ++w) s += part[(int64_t)w * kParams + p];
    grad[p] = s;
  }
  if (p == 0 && loss) {
    float s = 0.f;
    for (int w = 0; w < nwg; ++w) s += loss_part[w];
    *loss = s;
  }
}

// Adam (Kingma & Ba, Algorithm 1) on the FP32 master weights; c1 = 1 - beta1^t, c2 = 1 - beta2^t.
__global__ void k_adam(float* __restrict__ P, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ grad, float lr, float beta1, float beta2,
                       float eps, float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kParams) return;
  const float gr = grad[p];
  const float mm = beta1 * m[p] + (1.f - beta1) * gr;
  const float vv = beta2 * v[p] + (1.f - beta2) * gr * gr;
  m[p] = mm;
  v[p] = vv;
  P[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// ------------------------------------------------------------------------------------------
// Network outputs -> per-pair loading and window: delta = sigma^2 exp(clamp(out0)), W =
// 2^clamp(rint(out1), 2, 5) + 1; non-finite outputs fall back to the fixed method.
__global__ void k_decide(const float* __restrict__ out, int n, float noise, float fb_delta,
                         int fb_win, int* __restrict__ pw, float* __restrict__ pdelta,
                         int* __restrict__ fallback) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float o0 = out[2 * i], o1 = out[2 * i + 1];
  if (!isfinite(o0) || !isfinite(o1)) {
    pw[i] = fb_win;
    pdelta[i] = fb_delta;
    if (fallback) fallback[i] = 1;
    return;
  }
  const float ld = fminf(fmaxf(o0, -2.302585093f), 9.210340372f);   // ln 0.1 .. ln 1e4
  const float lw = fminf(fmaxf(rintf(o1), 2.f), 5.f);
  pw[i] = (1 << (int)lw) + 1;
  pdelta[i] = noise * expf(ld);
  if (fallback) fallback[i] = 0;
}

// Output SINR of every pair's weights against the exact interference-plus-noise covariance of
// jammers (sin az, INR) and white noise sigma^2, windowed: |w^H a|^2 / (sigma^2 w^H H w +
// sum_j INR_j |a_j^H w|^2), H_ii' = (1/M) sum_{e<N} e^{-j 2 pi (i - i') e / M}.
__global__ void k_sinr(WindowGeom g, const float2* __restrict__ w, int wmax,
                       const int* __restrict__ pw, const int* __restrict__ starts,
                       const double* __restrict__ jam_sin, const double* __restrict__ jam_inr,
                       int J, double noise, float* __restrict__ sinr) {
  const int64_t pair = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pair >= (int64_t)g.T * g.K) return;
  const int t = (int)(pair / g.K), k = (int)(pair % g.K);
  // the width the pair kernels solved: a per-pair width outside [1, W_t] or of the other
  // parity was rejected for the gathered window W_t; never more than the weight row holds
  int W = g.win[t];
  if (pw) {
    const int Wp = pw[pair];
    if (Wp >= 1 && Wp <= W && ((W - Wp) & 1) == 0) W = Wp;
  }
  W = W < wmax ? W : wmax;
  const int s = starts[pair];
  const float2* wp = w + pair * wmax;
  double u;
  int s0;
  window_of(g, t, k, &u, &s0);
  // signal response
  double sx = 0.0, sy = 0.0;
  for (int i = 0; i < W; ++i) {
    const double2 a = window_steering(g, u, s, i);
    const float2 c = wp[i];
    sx += c.x * a.x + c.y * a.y;   // conj(w) a
    sy += c.x * a.y - c.y * a.x;
  }
  // noise term w^H H w
  double nq = 0.0;
  for (int i = 0; i < W; ++i) {
    for (int i2 = 0; i2 < W; ++i2) {
      const int dlt = i - i2;
      double hx, hy;
      if (dlt == 0) {
        hx = (double)g.N / g.M;
        hy = 0.0;
      } else {
        const double xx = (double)dlt / g.M;
        const double mag = sinpi((double)g.N * xx) / sinpi(xx) / g.M;
        double sp, cp;
        sincospi(-(double)(g.N - 1) * xx, &sp, &cp);
        hx = mag * cp;
        hy = mag * sp;
      }
      const float2 a = wp[i], b = wp[i2];
      // conj(a) h b
      const double rx = hx * b.x - hy * b.y, ry = hx * b.y + hy * b.x;
      nq += a.x * rx + a.y * ry;
    }
  }
  double iq = 0.0;
  const int ks = (k < g.K / 2) ? k : k - g.K;
  const double ratio = 1.0 + (g.beta * ((double)ks + (g.half_bin ? 0.5 : 0.0))) / (double)g.K;
  for (int j = 0; j < J; ++j) {
    const double uj = ((double)g.M * g.dl) * jam_sin[j] * ratio;
    double rx = 0.0, ry = 0.0;
    for (int i = 0; i < W; ++i) {
      const double2 a = window_steering(g, uj, s, i);
      const float2 c = wp[i];
      rx += c.x * a.x + c.y * a.y;
      ry += c.x * a.y - c.y * a.x;
    }
    iq += jam_inr[j] * (rx * rx + ry * ry);
  }
  sinr[pair] = (float)((sx * sx + sy * sy) / (noise * nq + iq));
}

// Label of every pair from the sweep table sinr[c][pair], c = id * nW + iw over loadings
// deltas[id] and widths widths[iw]: the best SINR; ties go to the smaller width, then to the
// larger loading.  label [pair][2] = (ln(delta / sigma^2), log2(W - 1)).
__global__ void k_label(const float* __restrict__ sinr, int npairs, const float* __restrict__ deltas,
                        int nd, const int* __restrict__ widths, int nw, float noise,
                        float* __restrict__ label) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npairs) return;
  int best_d = 0, best_w = 0;
  float best = -1.f;
  for (int iw = 0; iw < nw; ++iw) {
    for (int id = nd - 1; id >= 0; --id) {
      const float v = sinr[(int64_t)(id * nw + iw) * npairs + i];
      if (v > best) {
        best = v;
        best_d = id;
        best_w = iw;
      }
    }
  }
  label[2 * i] = logf(deltas[best_d] / noise);
  label[2 * i + 1] = log2f((float)(widths[best_w] - 1));
}

// ------------------------------------------------------------------------------------------
hipError_t launch_features(const float* prof, int T, int K, int G, int L, float noise,
                           float* feat, hipStream_t s) {
  const int64_t n = (int64_t)T * K * 64;
  hipLaunchKernelGGL(k_features, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, prof, T, K, G,
                     L, noise, feat);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const float* P, const float* in, int n, float* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_forward, dim3((n + kFwdSB - 1) / kFwdSB), dim3(128), 0, s, P, in, n, out);
  return hipGetLastError();
}

int mlp_backward_workgroups(int n) { return (n + kBwdSB - 1) / kBwdSB; }
int mlp_param_count() { return kParams; }

hipError_t launch_mlp_backward(const float* P, const float* in, const float* tgt, int n,
                               float* part, float* loss_part, float* grad, float* loss,
                               hipStream_t s) {
  const int nwg = mlp_backward_workgroups(n);
  hipLaunchKernelGGL(k_mlp_backward, dim3(nwg), dim3(128), 0, s, P, in, tgt, n, part, loss_part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_reduce, dim3((kParams + 255) / 256), dim3(256), 0, s, part, loss_part,
                     nwg, grad, loss);
  return hipGetLastError();
}

// Device scratch of the allocation-free gradient entry point: the gradient and loss partials
// of up to WBM_MLP_STATIC_MAX_BATCH samples (kStaticWG workgroups of kBwdSB samples).  Every
// call on a device overwrites the rows it uses before reading them, so nothing is cleared
// between calls; calls that overlap on one device race on it.
constexpr int kStaticWG = WBM_MLP_STATIC_MAX_BATCH / kBwdSB;
static_assert(WBM_MLP_STATIC_MAX_BATCH % kBwdSB == 0, "static batch limit");
static __device__ __align__(256) float scratch[(size_t)kStaticWG * kParams + kStaticWG];

namespace {
std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
float* g_scratch_dev[kMaxDevices] = {};  // the array's device address, per device
}  // namespace

hipError_t mlp_static_scratch(float** part, float** loss_part) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    // each device holds its own copy of the array: look up its address with that device
    // current, once, and use only that address from the host
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_dev[dev] = static_cast<float*>(p);
  }
  *part = g_scratch_dev[dev];
  *loss_part = g_scratch_dev[dev] + (size_t)kStaticWG * kParams;
  return hipSuccess;
}

hipError_t launch_adam(float* P, float* m, float* v, const float* grad, float lr, float beta1,
                       float beta2, float eps, float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3((kParams + 255) / 256), dim3(256), 0, s, P, m, v, grad, lr, beta1,
                     beta2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_decide(const float* out, int n, float noise, float fb_delta, int fb_win, int* pw,
                         float* pdelta, int* fallback, hipStream_t s) {
  hipLaunchKernelGGL(k_decide, dim3((n + 255) / 256), dim3(256), 0, s, out, n, noise, fb_delta,
                     fb_win, pw, pdelta, fallback);
  return hipGetLastError();
}

hipError_t launch_sinr(const WindowGeom& g, const float2* w, int wmax, const int* pw,
                       const int* starts, const double* jam_sin, const double* jam_inr, int J,
                       double noise, float* sinr, hipStream_t s) {
  const int64_t n = (int64_t)g.T * g.K;
  hipLaunchKernelGGL(k_sinr, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, s, g, w, wmax, pw,
                     starts, jam_sin, jam_inr, J, noise, sinr);
  return hipGetLastError();
}

hipError_t launch_label(const float* sinr, int npairs, const float* deltas, int nd,
                        const int* widths, int nw, float noise, float* label, hipStream_t s) {
  hipLaunchKernelGGL(k_label, dim3((npairs + 255) / 256), dim3(256), 0, s, sinr, npairs, deltas, nd,
                     widths, nw, noise, label);
  return hipGetLastError();
}

}  // namespace wbm
