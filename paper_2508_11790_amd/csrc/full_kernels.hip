// Full-dimensional element-space MVDR per subband (Sec. II-B, Eq. 11-13), the comparison the
// windowed beamspace method is measured against.  Per subband k:
//   R = (1/L) sum_{b<L} X_b X_b^H + delta I_N      (N x N, FP64 accumulation of FP32 products)
//   R = G G^H                                        (blocked right-looking Cholesky, FP64)
//   v = G^-1 a_t, q = v^H v, c_t = G^-H v / q        (T right-hand sides, blocked)
//   out[t][k][l] = c_t^H X_{L+l}
#include <math.h>

#include <algorithm>

#include "wbm_dev.h"
#include "wbm_launch.h"

namespace wbm {

constexpr int kFT = 32;        // covariance tile (rows and columns)
constexpr int kFB = 32;        // snapshots per covariance chunk
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

// Blocked right-looking Cholesky R = G G^H of every subband's R (lower, row-major N x N in
// global memory), in panels of kCB columns, each panel three launches over all subbands:
//   k_full_potrf: factor the panel's diagonal tile (one workgroup per subband, in LDS);
//   k_full_trsm:  rows below it, A21 := A21 G11^-H by forward substitution (one workgroup per
//                 subband and kCB-row tile);
//   k_full_herk:  trailing update A22 -= A21 A21^H on the lower kCB x kCB tiles.
// Entries past N are read as zeros (the diagonal tile as an identity block) and not written.
// info[k] = j + 1 on a non-positive or non-finite pivot j, and every later launch then leaves
// that subband alone.
constexpr int kCB = 64;

__global__ __launch_bounds__(kFThreads) void k_full_potrf(FullArgs a, double2* __restrict__ R,
                                                          int* __restrict__ info, int c0) {
  __shared__ double2 A[kCB][kCB + 1];
  __shared__ int fail;
  const int kk = blockIdx.x, k = a.k0 + kk, N = a.N;
  if (c0 > 0 && info[k] != 0) return;
  double2* Rk = R + (int64_t)kk * N * N;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < kCB * kCB; idx += kFThreads) {
    const int i = idx / kCB, c = idx - i * kCB;
    double2 v = make_double2(i == c ? 1.0 : 0.0, 0.0);
    if (c <= i && c0 + i < N) v = Rk[(int64_t)(c0 + i) * N + c0 + c];
    A[i][c] = v;
  }
  if (tid == 0) fail = 0;
  __syncthreads();
  for (int j = 0; j < kCB; ++j) {
    const double d = A[j][j].x;
    if (!(d > 0.0) || !(d < INFINITY)) {
      if (tid == 0) fail = c0 + j + 1;
      break;
    }
    const double g = sqrt(d), inv = 1.0 / g;
    __syncthreads();                       // every thread has read the pivot
    for (int i = j + 1 + tid; i < kCB; i += kFThreads) {
      const double2 v = A[i][j];
      A[i][j] = make_double2(v.x * inv, v.y * inv);
    }
    if (tid == 0) A[j][j] = make_double2(g, 0.0);
    __syncthreads();
    // A[i][c] -= A[i][j] conj(A[c][j]) for j < c <= i
    const int m = kCB - 1 - j;
    for (int e = tid; e < m * m; e += kFThreads) {
      const int i = j + 1 + e / m, c = j + 1 + e % m;
      if (c <= i) {
        const double2 u = A[i][j], v = A[c][j];
        double2 r = A[i][c];
        r.x -= u.x * v.x + u.y * v.y;
        r.y -= u.y * v.x - u.x * v.y;
        A[i][c] = r;
      }
    }
    __syncthreads();
  }
  __syncthreads();
  if (fail) {
    if (tid == 0) info[k] = fail;
    return;
  }
  if (c0 == 0 && tid == 0) info[k] = 0;
  for (int idx = tid; idx < kCB * kCB; idx += kFThreads) {
    const int i = idx / kCB, c = idx - i * kCB;
    if (c <= i && c0 + i < N) Rk[(int64_t)(c0 + i) * N + c0 + c] = A[i][c];
  }
}

// Rows r0 .. r0 + kCB - 1 (r0 = c0 + kCB (blockIdx.x + 1)) of the panel: x G11^H = a row by row,
// G11 the factored diagonal tile.  Thread (row tid % kCB, column group tid / kCB) keeps its 16
// columns in registers; each step publishes the finished column through LDS.
__global__ __launch_bounds__(kFThreads) void k_full_trsm(FullArgs a, double2* __restrict__ R,
                                                         const int* __restrict__ info, int c0) {
  __shared__ double2 G[kCB][kCB + 1];
  __shared__ double2 xj[kCB];
  constexpr int NG = kFThreads / kCB, PER = kCB / NG;   // 4 groups of 16 columns
  const int kk = blockIdx.y, k = a.k0 + kk, N = a.N;
  if (info[k] != 0) return;
  const int r0 = c0 + kCB * (blockIdx.x + 1);
  double2* Rk = R + (int64_t)kk * N * N;
  const int tid = threadIdx.x, r = tid % kCB, grp = tid / kCB;
  for (int idx = tid; idx < kCB * kCB; idx += kFThreads) {
    const int i = idx / kCB, c = idx - i * kCB;
    G[i][c] = (c <= i && c0 + i < N) ? Rk[(int64_t)(c0 + i) * N + c0 + c]
                                     : make_double2(i == c ? 1.0 : 0.0, 0.0);
  }
  const bool row_ok = r0 + r < N;
  double2 x[PER];                 // columns grp + NG q
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int c = grp + NG * q;
    x[q] = (row_ok && c0 + c < N) ? Rk[(int64_t)(r0 + r) * N + c0 + c] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  for (int j = 0; j < kCB; ++j) {
    const double inv = 1.0 / G[j][j].x;
#pragma unroll
    for (int q = 0; q < PER; ++q) {        // the owner of column j finishes it
      if (grp + NG * q == j) {
        x[q] = make_double2(x[q].x * inv, x[q].y * inv);
        xj[r] = x[q];
      }
    }
    __syncthreads();
    const double2 u = xj[r];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int c = grp + NG * q;
      if (c > j) {                // x_c -= x_j conj(G[c][j])
        const double2 v = G[c][j];
        x[q].x -= u.x * v.x + u.y * v.y;
        x[q].y -= u.y * v.x - u.x * v.y;
      }
    }
    __syncthreads();
  }
  if (row_ok) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int c = grp + NG * q;
      if (c0 + c < N) Rk[(int64_t)(r0 + r) * N + c0 + c] = x[q];
    }
  }
}

// Trailing update of the lower tiles (ti >= tj) below the panel: C -= A_i A_j^H with A_i, A_j the
// panel rows of tiles ti and tj.  Thread (tr, tc) owns rows tr + 16 u and columns tc + 16 v of
// the tile; the panel columns are staged through LDS 16 at a time, rows padded to 17 entries so
// that the 16 distinct rows a wave reads fall in distinct banks.
__global__ __launch_bounds__(kFThreads) void k_full_herk(FullArgs a, double2* __restrict__ R,
                                                         const int* __restrict__ info, int c0) {
  constexpr int KC = 16;
  __shared__ double2 Ai[kCB][KC + 1];
  __shared__ double2 Aj[kCB][KC + 1];
  const int kk = blockIdx.y, k = a.k0 + kk, N = a.N;
  if (info[k] != 0) return;
  int ti = (int)((sqrt(8.0 * (double)blockIdx.x + 1.0) - 1.0) * 0.5);
  while ((ti + 1) * (ti + 2) / 2 <= (int)blockIdx.x) ++ti;
  while (ti * (ti + 1) / 2 > (int)blockIdx.x) --ti;
  const int tj = (int)blockIdx.x - ti * (ti + 1) / 2;
  const int i0 = c0 + kCB * (ti + 1), j0 = c0 + kCB * (tj + 1);
  double2* Rk = R + (int64_t)kk * N * N;
  const int tid = threadIdx.x, tr = tid / 16, tc = tid % 16;
  double ax[4][4], ay[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) ax[u][v] = ay[u][v] = 0.0;
  for (int q0 = 0; q0 < kCB; q0 += KC) {
    __syncthreads();
    for (int idx = tid; idx < kCB * KC; idx += kFThreads) {
      const int rr = idx / KC, q = idx - rr * KC, col = c0 + q0 + q;
      const bool cok = col < N;
      Ai[rr][q] = (cok && i0 + rr < N) ? Rk[(int64_t)(i0 + rr) * N + col] : make_double2(0.0, 0.0);
      Aj[rr][q] = (cok && j0 + rr < N) ? Rk[(int64_t)(j0 + rr) * N + col] : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll 4
    for (int q = 0; q < KC; ++q) {
      double2 p[4], c[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        p[u] = Ai[tr + 16 * u][q];
        c[u] = Aj[tc + 16 * u][q];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {   // p_u conj(c_v)
          ax[u][v] = fma(p[u].x, c[v].x, ax[u][v]);
          ax[u][v] = fma(p[u].y, c[v].y, ax[u][v]);
          ay[u][v] = fma(p[u].y, c[v].x, ay[u][v]);
          ay[u][v] = fma(-p[u].x, c[v].y, ay[u][v]);
        }
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + tr + 16 * u, j = j0 + tc + 16 * v;
      if (i < N && j <= i) {
        double2* dst = Rk + (int64_t)i * N + j;
        const double2 w = *dst;
        *dst = make_double2(w.x - ax[u][v], w.y - ay[u][v]);
      }
    }
}

// Solves for all targets, blocked like the factorisation: V [nk][N][T] (node-major so that a
// panel's rows are contiguous) starts as the steering vectors a_t, the forward sweep leaves
// v = G^-1 a (diagonal tile by substitution, then V_R -= G_RP V_P on the tiles below), q = v^H v,
// the backward sweep leaves x = G^-H v (diagonal tile, then V_R -= G_PR^H V_P on the tiles
// above), and c_t = x / q is written to wtmp [nk][T][N].  Targets go kTC per workgroup.
constexpr int kTC = 32;

__global__ __launch_bounds__(kFThreads) void k_full_steer(FullArgs a, DevDesc d,
                                                          double2* __restrict__ V) {
  const int kk = blockIdx.y, k = a.k0 + kk;
  const int ks = (k < a.K / 2) ? k : k - a.K;
  const double ratio = 1.0 + (a.beta * ((double)ks + (a.half_bin ? 0.5 : 0.0))) / (double)a.K;
  const int64_t n = (int64_t)a.N * a.T;
  double2* Vk = V + (int64_t)kk * n;
  for (int64_t idx = (int64_t)blockIdx.x * kFThreads + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * kFThreads) {
    const int e = (int)(idx / a.T), t = (int)(idx - (int64_t)e * a.T);
    double sp, cp;
    sincospi(2.0 * a.dl * d.sin_az[t] * ratio * (double)e, &sp, &cp);
    Vk[idx] = make_double2(cp, sp);
  }
}

// Diagonal tile of panel c0 (FORWARD: G_PP y = v, else G_PP^H y = v), targets t0 .. t0 + kTC - 1.
template <bool FORWARD>
__global__ __launch_bounds__(kFThreads) void k_full_tsolve(FullArgs a, const double2* __restrict__ R,
                                                           const int* __restrict__ info,
                                                           double2* __restrict__ V, int c0) {
  __shared__ double2 G[kCB][kCB + 1];
  __shared__ double2 Y[kCB][kTC + 1];
  const int kk = blockIdx.x, k = a.k0 + kk, N = a.N, T = a.T, t0 = blockIdx.y * kTC;
  if (info[k] != 0) return;
  const double2* Rk = R + (int64_t)kk * N * N;
  double2* Vk = V + (int64_t)kk * N * T;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < kCB * kCB; idx += kFThreads) {
    const int i = idx / kCB, c = idx - i * kCB;
    G[i][c] = (c <= i && c0 + i < N) ? Rk[(int64_t)(c0 + i) * N + c0 + c]
                                     : make_double2(i == c ? 1.0 : 0.0, 0.0);
  }
  for (int idx = tid; idx < kCB * kTC; idx += kFThreads) {
    const int i = idx / kTC, t = idx - i * kTC;
    Y[i][t] = (c0 + i < N && t0 + t < T) ? Vk[(int64_t)(c0 + i) * T + t0 + t]
                                         : make_double2(0.0, 0.0);
  }
  __syncthreads();
  for (int s = 0; s < kCB; ++s) {
    const int j = FORWARD ? s : kCB - 1 - s;
    if (tid < kTC) {
      const double inv = 1.0 / G[j][j].x;
      Y[j][tid] = make_double2(Y[j][tid].x * inv, Y[j][tid].y * inv);
    }
    __syncthreads();
    const int m = FORWARD ? kCB - 1 - j : j;     // rows still to update
    for (int e = tid; e < m * kTC; e += kFThreads) {
      const int i = (FORWARD ? j + 1 : 0) + e / kTC, t = e % kTC;
      const double2 y = Y[j][t];
      double2 r = Y[i][t];
      if (FORWARD) {                     // y_i -= G[i][j] y_j
        const double2 g = G[i][j];
        r.x -= g.x * y.x - g.y * y.y;
        r.y -= g.x * y.y + g.y * y.x;
      } else {                           // y_i -= conj(G[j][i]) y_j
        const double2 g = G[j][i];
        r.x -= g.x * y.x + g.y * y.y;
        r.y -= g.x * y.y - g.y * y.x;
      }
      Y[i][t] = r;
    }
    __syncthreads();
  }
  for (int idx = tid; idx < kCB * kTC; idx += kFThreads) {
    const int i = idx / kTC, t = idx - i * kTC;
    if (c0 + i < N && t0 + t < T) Vk[(int64_t)(c0 + i) * T + t0 + t] = Y[i][t];
  }
}

// Off-diagonal tiles of panel c0: FORWARD, the tiles below it (R = c0 + kCB (blockIdx.x + 1)):
// V_R -= G_RP V_P; else the tiles above it (R = kCB blockIdx.x): V_R -= G_PR^H V_P.  Thread
// (row tid / 4, target group tid % 4) accumulates 8 targets of one row.
template <bool FORWARD>
__global__ __launch_bounds__(kFThreads) void k_full_tupdate(FullArgs a,
                                                            const double2* __restrict__ R,
                                                            const int* __restrict__ info,
                                                            double2* __restrict__ V, int c0) {
  __shared__ double2 G[kCB][kCB + 1];      // FORWARD: G[r][p] = G_RP, else G[p][r] = G_PR
  __shared__ double2 Y[kCB][kTC + 1];
  const int kk = blockIdx.y, k = a.k0 + kk, N = a.N, T = a.T, t0 = blockIdx.z * kTC;
  if (info[k] != 0) return;
  const int r0 = FORWARD ? c0 + kCB * (blockIdx.x + 1) : kCB * blockIdx.x;
  const double2* Rk = R + (int64_t)kk * N * N;
  double2* Vk = V + (int64_t)kk * N * T;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < kCB * kCB; idx += kFThreads) {
    const int i = idx / kCB, c = idx - i * kCB;
    // FORWARD: row r0 + i, column c0 + c; else row c0 + i, column r0 + c
    const int row = FORWARD ? r0 + i : c0 + i, col = FORWARD ? c0 + c : r0 + c;
    G[i][c] = (row < N && col < N) ? Rk[(int64_t)row * N + col] : make_double2(0.0, 0.0);
  }
  for (int idx = tid; idx < kCB * kTC; idx += kFThreads) {
    const int i = idx / kTC, t = idx - i * kTC;
    Y[i][t] = (c0 + i < N && t0 + t < T) ? Vk[(int64_t)(c0 + i) * T + t0 + t]
                                         : make_double2(0.0, 0.0);
  }
  __syncthreads();
  const int r = tid >> 2, tg = (tid & 3) * 8;
  double ax[8], ay[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) ax[u] = ay[u] = 0.0;
  for (int q = 0; q < kCB; ++q) {
    const double2 g = FORWARD ? G[r][q] : G[q][r];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double2 y = Y[q][tg + u];
      if (FORWARD) {                     // G[r][q] y_q
        ax[u] = fma(g.x, y.x, fma(-g.y, y.y, ax[u]));
        ay[u] = fma(g.x, y.y, fma(g.y, y.x, ay[u]));
      } else {                           // conj(G[q][r]) y_q
        ax[u] = fma(g.x, y.x, fma(g.y, y.y, ax[u]));
        ay[u] = fma(g.x, y.y, fma(-g.y, y.x, ay[u]));
      }
    }
  }
  if (r0 + r < N) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (t0 + tg + u < T) {
        double2* dst = Vk + (int64_t)(r0 + r) * T + t0 + tg + u;
        const double2 w = *dst;
        *dst = make_double2(w.x - ax[u], w.y - ay[u]);
      }
    }
  }
}

// q[kk][t] = sum_e |V[kk][e][t]|^2 (eight partial sums per target, added in a fixed order).
__global__ __launch_bounds__(kFThreads) void k_full_q(FullArgs a, const int* __restrict__ info,
                                                      const double2* __restrict__ V,
                                                      double* __restrict__ q) {
  __shared__ double part[8][kTC];
  const int kk = blockIdx.x, k = a.k0 + kk, N = a.N, T = a.T, t0 = blockIdx.y * kTC;
  const int tid = threadIdx.x, t = tid % kTC, g = tid / kTC;
  const double2* Vk = V + (int64_t)kk * N * T;
  double sum = 0.0;
  if (info[k] == 0 && t0 + t < T)
    for (int e = g; e < N; e += 8) {
      const double2 v = Vk[(int64_t)e * T + t0 + t];
      sum += v.x * v.x + v.y * v.y;
    }
  part[g][t] = sum;
  __syncthreads();
  if (tid < kTC && t0 + tid < T) {
    double s = 0.0;
    for (int j = 0; j < 8; ++j) s += part[j][tid];
    q[(int64_t)kk * T + t0 + tid] = s;
  }
}

// wtmp[kk][t][e] = V[kk][e][t] / q[kk][t], zero for a subband whose factorisation failed.
__global__ __launch_bounds__(kFThreads) void k_full_scale(FullArgs a, const int* __restrict__ info,
                                                          const double2* __restrict__ V,
                                                          const double* __restrict__ q,
                                                          double2* __restrict__ wtmp) {
  const int kk = blockIdx.y, k = a.k0 + kk, N = a.N, T = a.T;
  const bool bad = info[k] != 0;
  const int64_t n = (int64_t)N * T;
  for (int64_t idx = (int64_t)blockIdx.x * kFThreads + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * kFThreads) {
    const int t = (int)(idx / N), e = (int)(idx - (int64_t)t * N);
    double2 w = make_double2(0.0, 0.0);
    if (!bad) {
      const double qi = 1.0 / q[(int64_t)kk * T + t];
      const double2 v = V[(int64_t)kk * n + (int64_t)e * T + t];
      w = make_double2(v.x * qi, v.y * qi);
    }
    wtmp[(int64_t)kk * n + idx] = w;
  }
}

// out[t][k][l] = c_t^H X_{L+l}: one workgroup per (subband, kAS test snapshots), every target
// kTC at a time; the snapshots' elements and the weights are staged through LDS kAE elements
// at a time.  Thread (snapshot tid % kAS, target group tid / kAS) sums two targets.
constexpr int kAS = 16, kAE = 64;

__global__ __launch_bounds__(kFThreads) void k_full_apply(FullArgs a, const float2* __restrict__ X,
                                                          const double2* __restrict__ wtmp,
                                                          float2* __restrict__ out,
                                                          float2* __restrict__ wout) {
  __shared__ float2 xs[kAS][kAE + 1];
  __shared__ double2 ws[kTC][kAE + 1];
  const int kk = blockIdx.y, k = a.k0 + kk, N = a.N, T = a.T;
  const int l0 = blockIdx.x * kAS;
  const int tid = threadIdx.x, sn = tid % kAS, tg = tid / kAS;   // tg in [0, 16)
  const double2* wk = wtmp + (int64_t)kk * T * N;
  const float2* Xk = X + ((int64_t)k * a.B + a.L) * N;
  for (int tc0 = 0; tc0 < T; tc0 += kTC) {
    double ax[2] = {0.0, 0.0}, ay[2] = {0.0, 0.0};
    for (int e0 = 0; e0 < N; e0 += kAE) {
      __syncthreads();
      for (int idx = tid; idx < kAS * kAE; idx += kFThreads) {
        const int ss = idx / kAE, ee = idx - ss * kAE;
        xs[ss][ee] = (l0 + ss < a.Lt && e0 + ee < N) ? Xk[(int64_t)(l0 + ss) * N + e0 + ee]
                                                       : make_float2(0.f, 0.f);
      }
      for (int idx = tid; idx < kTC * kAE; idx += kFThreads) {
        const int tt = idx / kAE, ee = idx - tt * kAE;
        ws[tt][ee] = (tc0 + tt < T && e0 + ee < N) ? wk[(int64_t)(tc0 + tt) * N + e0 + ee]
                                                     : make_double2(0.0, 0.0);
      }
      __syncthreads();
#pragma unroll 8
      for (int ee = 0; ee < kAE; ++ee) {
        const float2 xv = xs[sn][ee];
        const double x_re = xv.x, x_im = xv.y;
#pragma unroll
        for (int u = 0; u < 2; ++u) {            // conj(w) x
          const double2 w = ws[tg + 16 * u][ee];
          ax[u] = fma(w.x, x_re, fma(w.y, x_im, ax[u]));
          ay[u] = fma(w.x, x_im, fma(-w.y, x_re, ay[u]));
        }
      }
    }
    if (l0 + sn < a.Lt) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int t = tc0 + tg + 16 * u;
        if (t < T) out[((int64_t)t * a.K + k) * a.Lt + l0 + sn] = make_float2((float)ax[u], (float)ay[u]);
      }
    }
  }
  if (wout && blockIdx.x == 0) {
    for (int idx = tid; idx < T * N; idx += kFThreads) {
      const int t = idx / N, e = idx - t * N;
      wout[((int64_t)t * a.K + k) * N + e] = make_float2((float)wk[idx].x, (float)wk[idx].y);
    }
  }
}

hipError_t launch_full_mvdr(const FullArgs& a, const DevDesc& d, const float2* X, double2* R,
                            double2* V, double* q, double2* wtmp, float2* out, float2* wout,
                            int* info, hipStream_t s) {
  const int nt = (a.N + kFT - 1) / kFT;
  hipLaunchKernelGGL(k_full_cov, dim3(nt * (nt + 1) / 2, a.nk), dim3(kFThreads), 0, s, a, X, R);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int np = (a.N + kCB - 1) / kCB;      // panels
  for (int p = 0; p < np; ++p) {
    const int c0 = p * kCB, m = np - 1 - p;   // tiles below the panel
    hipLaunchKernelGGL(k_full_potrf, dim3(a.nk), dim3(kFThreads), 0, s, a, R, info, c0);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (m == 0) break;
    hipLaunchKernelGGL(k_full_trsm, dim3(m, a.nk), dim3(kFThreads), 0, s, a, R, info, c0);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_full_herk, dim3(m * (m + 1) / 2, a.nk), dim3(kFThreads), 0, s, a, R,
                       info, c0);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int tc = (a.T + kTC - 1) / kTC;
  const int64_t nv = (int64_t)a.N * a.T;
  const int gs = (int)std::min<int64_t>((nv + kFThreads - 1) / kFThreads, 1024);
  hipLaunchKernelGGL(k_full_steer, dim3(gs, a.nk), dim3(kFThreads), 0, s, a, d, V);
  for (int p = 0; p < np; ++p) {              // forward sweep: v = G^-1 a
    const int c0 = p * kCB, m = np - 1 - p;
    hipLaunchKernelGGL(k_full_tsolve<true>, dim3(a.nk, tc), dim3(kFThreads), 0, s, a, R, info, V, c0);
    if (m > 0)
      hipLaunchKernelGGL(k_full_tupdate<true>, dim3(m, a.nk, tc), dim3(kFThreads), 0, s, a, R,
                         info, V, c0);
  }
  hipLaunchKernelGGL(k_full_q, dim3(a.nk, tc), dim3(kFThreads), 0, s, a, info, V, q);
  for (int p = np - 1; p >= 0; --p) {         // backward sweep: x = G^-H v
    const int c0 = p * kCB;
    hipLaunchKernelGGL(k_full_tsolve<false>, dim3(a.nk, tc), dim3(kFThreads), 0, s, a, R, info, V, c0);
    if (p > 0)
      hipLaunchKernelGGL(k_full_tupdate<false>, dim3(p, a.nk, tc), dim3(kFThreads), 0, s, a, R,
                         info, V, c0);
  }
  hipLaunchKernelGGL(k_full_scale, dim3(gs, a.nk), dim3(kFThreads), 0, s, a, info, V, q, wtmp);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_full_apply, dim3(a.Lt > 0 ? (a.Lt + kAS - 1) / kAS : 1, a.nk),
                     dim3(kFThreads), 0, s, a, X, wtmp, out, wout);
  return hipGetLastError();
}

hipError_t set_full_attributes() { return hipSuccess; }   // every kernel uses static LDS

}  // namespace wbm
