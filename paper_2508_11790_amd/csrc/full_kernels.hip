// Full-dimensional element-space MVDR per subband (Sec. II-B, Eq. 11-13), the comparison the
// windowed beamspace method is measured against.  Per subband k:
//   R = (1/L) sum_{b<L} X_b X_b^H + delta I_N      (N x N, FP64 accumulation of FP32 products)
//   R = G G^H                                        (blocked right-looking Cholesky, FP64)
//   v = G^-1 a_t, q = v^H v, c_t = G^-H v / q        (T right-hand sides)
//   out[t][k][l] = c_t^H X_{L+l}
#include <math.h>

#include "wbm_dev.h"
#include "wbm_launch.h"

namespace wbm {

constexpr int kFT = 32;        // covariance tile (rows and columns)
constexpr int kFB = 32;        // snapshots per covariance chunk
constexpr int kNBMax = 16;     // widest Cholesky panel
constexpr size_t kLdsBudget = 150 * 1024;
constexpr int kFThreads = 256;

// Lower-triangle 32x32 tiles of R for subband k0 + blockIdx.y.
__global__ __launch_bounds__(kFThreads) void k_full_cov(FullArgs a, const float2* __restrict__ X,
                                                        double2* __restrict__ R) {
  __shared__ float2 xi[kFB][kFT + 1];
  __shared__ float2 xj[kFB][kFT + 1];
  const int kk = blockIdx.y, k = a.k0 + kk;
  // tile index -> (ti, tj), tj <= ti
  const int e = blockIdx.x;
  int ti = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
  while ((ti + 1) * (ti + 2) / 2 <= e) ++ti;
  while (ti * (ti + 1) / 2 > e) --ti;
  const int tj = e - ti * (ti + 1) / 2;
  const int i0 = ti * kFT, j0 = tj * kFT;
  const int tid = threadIdx.x;
  const int r = tid >> 3, c4 = (tid & 7) * 4;     // each thread: row r, columns c4..c4+3
  double ax[4] = {0, 0, 0, 0}, ay[4] = {0, 0, 0, 0};
  const float2* Xk = X + (int64_t)k * a.B * a.N;
  for (int b0 = 0; b0 < a.L; b0 += kFB) {
    __syncthreads();
    for (int idx = tid; idx < kFB * kFT; idx += kFThreads) {
      const int bb = idx / kFT, c = idx - bb * kFT;
      const int b = b0 + bb;
      float2 vi = make_float2(0.f, 0.f), vj = vi;
      if (b < a.L) {
        if (i0 + c < a.N) vi = Xk[(int64_t)b * a.N + i0 + c];
        if (j0 + c < a.N) vj = Xk[(int64_t)b * a.N + j0 + c];
      }
      xi[bb][c] = vi;
      xj[bb][c] = vj;
    }
    __syncthreads();
    for (int bb = 0; bb < kFB; ++bb) {
      const float2 u = xi[bb][r];
      const double ux = u.x, uy = u.y;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float2 v = xj[bb][c4 + q];
        const double vx = v.x, vy = v.y;
        ax[q] += ux * vx + uy * vy;
        ay[q] += uy * vx - ux * vy;
      }
    }
  }
  const double invL = 1.0 / (double)a.L;
  double2* Rk = R + (int64_t)kk * a.N * a.N;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = i0 + r, j = j0 + c4 + q;
    if (i < a.N && j < a.N && j <= i) {
      double2 v = make_double2(ax[q] * invL, ay[q] * invL);
      if (i == j) v = make_double2(v.x + a.delta, 0.0);
      Rk[(int64_t)i * a.N + j] = v;
    }
  }
}

// Blocked right-looking Cholesky of one subband's R (lower, row-major N x N in global memory),
// one workgroup per subband.  info[k] = j + 1 on a non-positive pivot j.
__global__ __launch_bounds__(kFThreads) void k_full_chol(FullArgs a, double2* __restrict__ R,
                                                         int* __restrict__ info, int kNB) {
  extern __shared__ __align__(16) unsigned char smem[];
  double2* P = reinterpret_cast<double2*>(smem);            // panel [N][kNB]
  __shared__ int fail;
  const int kk = blockIdx.x, N = a.N;
  double2* A = R + (int64_t)kk * N * N;
  const int tid = threadIdx.x;
  if (tid == 0) fail = 0;
  __syncthreads();
  for (int c0 = 0; c0 < N; c0 += kNB) {
    if (fail) break;
    const int nb = min(kNB, N - c0);
    const int rows = N - c0;
    // load the panel (rows c0.., columns c0..c0+nb) into LDS
    for (int idx = tid; idx < rows * kNB; idx += kFThreads) {
      const int i = idx / kNB, c = idx - i * kNB;
      P[idx] = (c < nb && c <= i) ? A[(int64_t)(c0 + i) * N + c0 + c] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    // unblocked factorisation of the panel (diagonal block + rows below)
    for (int j = 0; j < nb; ++j) {
      const double d = P[j * kNB + j].x;
      if (!(d > 0.0) || !(d < INFINITY)) {
        if (tid == 0) fail = c0 + j + 1;
        break;
      }
      const double inv = 1.0 / sqrt(d);
      __syncthreads();
      for (int i = j + tid; i < rows; i += kFThreads) {
        double2 v = P[i * kNB + j];
        P[i * kNB + j] = (i == j) ? make_double2(sqrt(d), 0.0) : make_double2(v.x * inv, v.y * inv);
      }
      __syncthreads();
      // update the remaining panel columns c in (j, nb): P[i][c] -= P[i][j] conj(P[c][j]), i >= c
      for (int idx = tid; idx < rows * kNB; idx += kFThreads) {
        const int i = idx / kNB, c = idx - i * kNB;
        if (c > j && c < nb && i >= c) {
          const double2 gi = P[i * kNB + j], gc = P[c * kNB + j];
          double2 v = P[idx];
          v.x -= gi.x * gc.x + gi.y * gc.y;
          v.y -= gi.y * gc.x - gi.x * gc.y;
          P[idx] = v;
        }
      }
      __syncthreads();
    }
    __syncthreads();
    if (fail) break;
    // store the panel back
    for (int idx = tid; idx < rows * kNB; idx += kFThreads) {
      const int i = idx / kNB, c = idx - i * kNB;
      if (c < nb && c <= i) A[(int64_t)(c0 + i) * N + c0 + c] = P[idx];
    }
    // trailing update A22[i][j] -= sum_c P[i][c] conj(P[j][c]) for c0+nb <= j <= i < N
    const int m = rows - nb;
    const int64_t cnt = (int64_t)m * (m + 1) / 2;
    for (int64_t e = tid; e < cnt; e += kFThreads) {
      int ii = (int)((sqrt(8.0 * (double)e + 1.0) - 1.0) * 0.5);
      while ((int64_t)(ii + 1) * (ii + 2) / 2 <= e) ++ii;
      while ((int64_t)ii * (ii + 1) / 2 > e) --ii;
      const int jj = (int)(e - (int64_t)ii * (ii + 1) / 2);
      const double2* pi = P + (nb + ii) * kNB;
      const double2* pj = P + (nb + jj) * kNB;
      double sx = 0.0, sy = 0.0;
      for (int c = 0; c < nb; ++c) {
        const double2 u = pi[c], v = pj[c];
        sx += u.x * v.x + u.y * v.y;
        sy += u.y * v.x - u.x * v.y;
      }
      double2* dst = A + (int64_t)(c0 + nb + ii) * N + c0 + nb + jj;
      double2 w = *dst;
      *dst = make_double2(w.x - sx, w.y - sy);
    }
    __syncthreads();
  }
  if (info && tid == 0) info[a.k0 + kk] = fail;
}

// Solves for all targets of one subband: v = G^-1 a_t, q = |v|^2, c = G^-H v / q -> wtmp [nk][T][N].
__global__ __launch_bounds__(kFThreads) void k_full_solve(FullArgs a, DevDesc d,
                                                          const double2* __restrict__ R,
                                                          const int* __restrict__ info,
                                                          double2* __restrict__ wtmp, int TG) {
  extern __shared__ __align__(16) unsigned char smem[];
  double2* v = reinterpret_cast<double2*>(smem);           // [TG][N]
  __shared__ double qs[kFThreads];
  const int kk = blockIdx.x, k = a.k0 + kk, N = a.N;
  const int tbase = blockIdx.y * TG;
  const int T = min(TG, a.T - tbase);
  wtmp += (int64_t)tbase * N;    // rows of this target group inside [nk][T][N]
  const double2* G = R + (int64_t)kk * N * N;
  const int tid = threadIdx.x;
  const bool bad = info && info[k] != 0;
  const int ks = (k < a.K / 2) ? k : k - a.K;
  const double ratio = 1.0 + (a.beta * ((double)ks + (a.half_bin ? 0.5 : 0.0))) / (double)a.K;
  for (int idx = tid; idx < T * N; idx += kFThreads) {
    const int t = idx / N, e = idx - t * N;
    double sp, cp;
    sincospi(2.0 * a.dl * d.sin_az[tbase + t] * ratio * (double)e, &sp, &cp);
    v[idx] = make_double2(cp, sp);
  }
  __syncthreads();
  if (bad) {
    for (int idx = tid; idx < T * N; idx += kFThreads) wtmp[(int64_t)kk * a.T * N + idx] = make_double2(0, 0);
    return;
  }
  // forward: column j of G
  for (int j = 0; j < N; ++j) {
    const double dinv = 1.0 / G[(int64_t)j * N + j].x;
    if (tid < T) {
      double2 x = v[tid * N + j];
      v[tid * N + j] = make_double2(x.x * dinv, x.y * dinv);
    }
    __syncthreads();
    const int rem = N - j - 1;
    for (int idx = tid; idx < rem * T; idx += kFThreads) {
      const int t = idx / rem, i = j + 1 + (idx - t * rem);
      const double2 g = G[(int64_t)i * N + j], vj = v[t * N + j];
      double2 x = v[t * N + i];
      x.x -= g.x * vj.x - g.y * vj.y;
      x.y -= g.x * vj.y + g.y * vj.x;
      v[t * N + i] = x;
    }
    __syncthreads();
  }
  // q per target
  for (int t = tid; t < T; t += kFThreads) {
    double q = 0.0;
    for (int e = 0; e < N; ++e) q += v[t * N + e].x * v[t * N + e].x + v[t * N + e].y * v[t * N + e].y;
    qs[t] = q;
  }
  __syncthreads();
  // backward: G^H x = v, row j of G^H is conj of column j of G
  for (int j = N - 1; j >= 0; --j) {
    const double dinv = 1.0 / G[(int64_t)j * N + j].x;
    if (tid < T) {
      double2 x = v[tid * N + j];
      v[tid * N + j] = make_double2(x.x * dinv, x.y * dinv);
    }
    __syncthreads();
    for (int idx = tid; idx < j * T; idx += kFThreads) {
      const int t = idx / j, i = idx - t * j;
      const double2 g = G[(int64_t)j * N + i], xj = v[t * N + j];   // conj(G[j][i]) * x_j
      double2 x = v[t * N + i];
      x.x -= g.x * xj.x + g.y * xj.y;
      x.y -= g.x * xj.y - g.y * xj.x;
      v[t * N + i] = x;
    }
    __syncthreads();
  }
  for (int idx = tid; idx < T * N; idx += kFThreads) {
    const int t = idx / N;
    const double qi = 1.0 / qs[t];
    wtmp[(int64_t)kk * a.T * N + idx] = make_double2(v[idx].x * qi, v[idx].y * qi);
  }
}

// out[t][k][l] = c_t^H X_{L+l}; one workgroup per (subband, 64 test snapshots).
__global__ __launch_bounds__(kFThreads) void k_full_apply(FullArgs a, const float2* __restrict__ X,
                                                          const double2* __restrict__ wtmp,
                                                          float2* __restrict__ out,
                                                          float2* __restrict__ wout) {
  const int kk = blockIdx.y, k = a.k0 + kk, N = a.N, T = a.T;
  const int l0 = blockIdx.x * 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double2* wk = wtmp + (int64_t)kk * T * N;
  for (int l = l0 + wave; l < min(l0 + 64, a.Lt); l += kFThreads / 64) {
    const float2* xr = X + ((int64_t)k * a.B + a.L + l) * N;
    for (int t = 0; t < T; ++t) {
      double zx = 0.0, zy = 0.0;
      for (int e = lane; e < N; e += 64) {
        const float2 y = xr[e];
        const double2 w = wk[(int64_t)t * N + e];
        zx += w.x * (double)y.x + w.y * (double)y.y;
        zy += w.x * (double)y.y - w.y * (double)y.x;
      }
      for (int off = 32; off > 0; off >>= 1) {
        zx += __shfl_xor(zx, off);
        zy += __shfl_xor(zy, off);
      }
      if (lane == 0) out[((int64_t)t * a.K + k) * a.Lt + l] = make_float2((float)zx, (float)zy);
    }
  }
  if (wout && blockIdx.x == 0) {
    for (int idx = threadIdx.x; idx < T * N; idx += kFThreads) {
      const int t = idx / N, e = idx - t * N;
      wout[((int64_t)t * a.K + k) * N + e] = make_float2((float)wk[idx].x, (float)wk[idx].y);
    }
  }
}

hipError_t launch_full_mvdr(const FullArgs& a, const DevDesc& d, const float2* X, double2* R,
                            double2* wtmp, float2* out, float2* wout, int* info, hipStream_t s) {
  const int nt = (a.N + kFT - 1) / kFT;
  hipLaunchKernelGGL(k_full_cov, dim3(nt * (nt + 1) / 2, a.nk), dim3(kFThreads), 0, s, a, X, R);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int nb = kNBMax;
  while (nb > 1 && sizeof(double2) * (size_t)a.N * nb > kLdsBudget) nb >>= 1;
  const size_t shm_chol = sizeof(double2) * (size_t)a.N * nb;
  hipLaunchKernelGGL(k_full_chol, dim3(a.nk), dim3(kFThreads), shm_chol, s, a, R, info, nb);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  int TG = (int)(kLdsBudget / (sizeof(double2) * (size_t)a.N));
  if (TG > a.T) TG = a.T;
  if (TG > kFThreads) TG = kFThreads;
  if (TG < 1) return hipErrorInvalidValue;
  const size_t shm_solve = sizeof(double2) * (size_t)TG * a.N;
  hipLaunchKernelGGL(k_full_solve, dim3(a.nk, (a.T + TG - 1) / TG), dim3(kFThreads), shm_solve, s,
                     a, d, R, info, wtmp, TG);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_full_apply, dim3(a.Lt > 0 ? (a.Lt + 63) / 64 : 1, a.nk), dim3(kFThreads), 0, s, a, X, wtmp,
                     out, wout);
  return hipGetLastError();
}

hipError_t set_full_attributes() {
  // dynamic LDS of both kernels is at most kLdsBudget; their static LDS is a few KiB
  hipError_t e = hipFuncSetAttribute((const void*)k_full_chol,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBudget);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_full_solve, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)kLdsBudget);
}

}  // namespace wbm
