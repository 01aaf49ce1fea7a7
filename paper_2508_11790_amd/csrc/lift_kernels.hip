// Lifted correlators (Eq. 21) and their use in element space: c^ = D^H S^T c~ maps a pair's
// windowed beamspace weights back to the N array elements; applying c^ to the channelized
// element snapshots gives the same beam outputs without the spatial transform or the window
// gather (the remark after Eq. 21).
#include "wbm_dev.h"
#include "wbm_launch.h"

namespace wbm {

// c_hat[pair][n] = M^-1/2 sum_{i < wmax} w[pair][i] exp(+j 2 pi n m_i / M), m_i = (s + i) mod M
// (s = the pair's window start; weights past the pair's width are zero).  The phase index
// (n m_i) mod M is exact in integers and reads the M-entry table tw[q] = exp(-j 2 pi q / M);
// products summed in FP64.  Grid: (ceil(N / 256), pairs).
__global__ __launch_bounds__(256) void k_lift(const float2* __restrict__ w,
                                              const int* __restrict__ starts, int wmax, int N,
                                              int M, const float2* __restrict__ tw,
                                              float2* __restrict__ c_hat) {
  const int64_t pair = blockIdx.y;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const int s = starts[pair];
  const float2* wp = w + pair * wmax;
  double ax = 0.0, ay = 0.0;
  for (int i = 0; i < wmax; ++i) {
    const int m = (s + i) & (M - 1);   // M is a power of two; two's complement wraps s < 0
    const float2 e = tw[(int)(((int64_t)n * m) & (M - 1))];   // exp(-j 2 pi n m / M)
    const float2 c = wp[i];
    ax += (double)c.x * e.x + (double)c.y * e.y;   // c conj(e)
    ay += (double)c.y * e.x - (double)c.x * e.y;
  }
  const double r = 1.0 / sqrt((double)M);
  c_hat[pair * N + n] = make_float2((float)(ax * r), (float)(ay * r));
}

// out[t][k][l] = sum_n conj(c_hat[t][k][n]) X[k][L + l][n]: per subband a (T x N) by (N x Lt)
// product, HBM-bound at these shapes (one pass over the test snapshots per 8 targets).
// Workgroup = (64 test snapshots, 8 targets, subband k); N in chunks of 64 staged in LDS
// (snapshot rows padded by one), each thread sums two targets for one snapshot in FP32.
constexpr int kLaTL = 64, kLaTT = 8, kLaNC = 64;

__global__ __launch_bounds__(256) void k_lift_apply(const float2* __restrict__ X,
                                                    const float2* __restrict__ c_hat,
                                                    float2* __restrict__ out, int N, int K,
                                                    int B, int L, int Lt, int T) {
  __shared__ float2 xs[kLaTL][kLaNC + 1];
  __shared__ float2 cs[kLaTT][kLaNC];
  const int tid = threadIdx.x, li = tid & (kLaTL - 1), tg = tid / kLaTL;   // tg in 0..3
  const int l0 = blockIdx.x * kLaTL, t0 = blockIdx.y * kLaTT, k = blockIdx.z;
  float ax0 = 0.f, ay0 = 0.f, ax1 = 0.f, ay1 = 0.f;
  for (int n0 = 0; n0 < N; n0 += kLaNC) {
    for (int e = tid; e < kLaTL * kLaNC; e += 256) {
      const int r = e / kLaNC, c = e % kLaNC, l = l0 + r;
      float2 v = make_float2(0.f, 0.f);
      if (l < Lt && n0 + c < N) v = X[((int64_t)k * B + L + l) * N + n0 + c];
      xs[r][c] = v;
    }
    for (int e = tid; e < kLaTT * kLaNC; e += 256) {
      const int tt = e / kLaNC, c = e % kLaNC, t = t0 + tt;
      float2 v = make_float2(0.f, 0.f);
      if (t < T && n0 + c < N) v = c_hat[((int64_t)t * K + k) * N + n0 + c];
      cs[tt][c] = v;
    }
    __syncthreads();
#pragma unroll 8
    for (int c = 0; c < kLaNC; ++c) {
      const float2 x = xs[li][c], c0 = cs[tg][c], c1 = cs[tg + 4][c];
      ax0 = fmaf(c0.x, x.x, fmaf(c0.y, x.y, ax0));   // conj(c) x
      ay0 = fmaf(c0.x, x.y, fmaf(-c0.y, x.x, ay0));
      ax1 = fmaf(c1.x, x.x, fmaf(c1.y, x.y, ax1));
      ay1 = fmaf(c1.x, x.y, fmaf(-c1.y, x.x, ay1));
    }
    __syncthreads();
  }
  const int l = l0 + li;
  if (l < Lt) {
    if (t0 + tg < T) out[((int64_t)(t0 + tg) * K + k) * Lt + l] = make_float2(ax0, ay0);
    if (t0 + tg + 4 < T) out[((int64_t)(t0 + tg + 4) * K + k) * Lt + l] = make_float2(ax1, ay1);
  }
}

// The same product on the FP32 matrix cores, for many targets (T > 8): per complex element n,
// with A = [Re c, Im c] (targets x 2) and B = [Re x; Im x] or [Im x; -Re x] (2 x snapshots),
// Re out += A B1 and Im out += A B2 are two v_mfma_f32_32x32x2f32 steps (conj(c) x =
// (cr xr + ci xi) + j (cr xi - ci xr)).  Workgroup = 32 targets x 128 test snapshots of one
// subband, four waves of 32 snapshots each; N in chunks of 32 staged in LDS (rows padded by
// one).  Lane l supplies A[l % 32][l / 32] and B[l / 32][l % 32]; accumulator register r of
// lane l is target 8 (r / 4) + 4 (l / 32) + r % 4, snapshot l % 32.
typedef float f32x16_t __attribute__((ext_vector_type(16)));
constexpr int kLmTT = 32, kLmTL = 128, kLmNC = 32;

__global__ __launch_bounds__(256) void k_lift_apply_mfma(const float2* __restrict__ X,
                                                         const float2* __restrict__ c_hat,
                                                         float2* __restrict__ out, int N, int K,
                                                         int B, int L, int Lt, int T) {
  __shared__ float2 xs[kLmTL][kLmNC + 1];
  __shared__ float2 cs[kLmTT][kLmNC + 1];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l0 = blockIdx.x * kLmTL, t0 = blockIdx.y * kLmTT, k = blockIdx.z;
  const bool hi = lane >= 32;
  const int lr = lane & 31;
  f32x16_t accr = {}, acci = {};
  for (int n0 = 0; n0 < N; n0 += kLmNC) {
    for (int e = tid; e < kLmTL * kLmNC; e += 256) {
      const int r = e / kLmNC, c = e % kLmNC, l = l0 + r;
      float2 v = make_float2(0.f, 0.f);
      if (l < Lt && n0 + c < N) v = X[((int64_t)k * B + L + l) * N + n0 + c];
      xs[r][c] = v;
    }
    for (int e = tid; e < kLmTT * kLmNC; e += 256) {
      const int r = e / kLmNC, c = e % kLmNC, t = t0 + r;
      float2 v = make_float2(0.f, 0.f);
      if (t < T && n0 + c < N) v = c_hat[((int64_t)t * K + k) * N + n0 + c];
      cs[r][c] = v;
    }
    __syncthreads();
#pragma unroll 8
    for (int c = 0; c < kLmNC; ++c) {
      const float2 cv = cs[lr][c], xv = xs[wave * 32 + lr][c];
      const float a = hi ? cv.y : cv.x;
      const float b1 = hi ? xv.y : xv.x;
      const float b2 = hi ? -xv.x : xv.y;
      accr = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b1, accr, 0, 0, 0);
      acci = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b2, acci, 0, 0, 0);
    }
    __syncthreads();
  }
  const int l = l0 + wave * 32 + lr;
  if (l < Lt) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int t = t0 + 8 * (r / 4) + 4 * (lane / 32) + (r % 4);
      if (t < T) out[((int64_t)t * K + k) * Lt + l] = make_float2(accr[r], acci[r]);
    }
  }
}

// Beam pattern of a correlator (Eq. 22): cosine similarity |<c, a(Omega)>| / (||c|| ||a||),
// a(Omega)_e = exp(j Omega e), ||a|| = sqrt(N).  Workgroup = one correlator (staged in LDS
// with its FP64 norm); each thread sweeps angles q = tid, tid + 256, ...: the sum
// sum_e conj(c_e) exp(j Omega e) in FP64, the phase advanced by one FP64 complex product per
// element from exp(j Omega).  Grid: (pairs).
constexpr int kBpMaxN = 4096;

__global__ __launch_bounds__(256) void k_beam_pattern(const float2* __restrict__ c, int N,
                                                      const double* __restrict__ omega, int Q,
                                                      float* __restrict__ pattern) {
  __shared__ float2 cs[kBpMaxN];
  __shared__ double red[256];
  const int64_t p = blockIdx.x;
  const int tid = threadIdx.x;
  double nn = 0.0;
  for (int e = tid; e < N; e += 256) {
    const float2 v = c[p * N + e];
    cs[e] = v;
    nn += (double)v.x * v.x + (double)v.y * v.y;
  }
  red[tid] = nn;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  const double scale = 1.0 / (sqrt(red[0]) * sqrt((double)N));
  for (int q = tid; q < Q; q += 256) {
    double sx, cx;
    sincos(omega[q], &sx, &cx);
    double zr = 1.0, zi = 0.0, ar = 0.0, ai = 0.0;
    for (int e = 0; e < N; ++e) {
      const float2 v = cs[e];
      ar += (double)v.x * zr + (double)v.y * zi;   // conj(c_e) z
      ai += (double)v.x * zi - (double)v.y * zr;
      const double t = zr * cx - zi * sx;
      zi = zr * sx + zi * cx;
      zr = t;
    }
    pattern[p * Q + q] = (float)(sqrt(ar * ar + ai * ai) * scale);
  }
}

// Planar array (Eq. 21 with D = D_h^T kron D_v): c_hat[pair][ix Nz + iz] =
// M^-1/2 sum_i w[pair][i] exp(+j 2 pi (mz_i iz / Mz + mx_i ix / Mx)), window cell
// i = ix_w Wz + iz_w at beam (mz_i, mx_i) = ((s_z + iz_w) mod Mz, (s_x + ix_w) mod Mx), M = Mz Mx.
// The phase index (mz iz Mx + mx ix Mz) mod M is exact in integers and reads the M-entry table;
// weights past the pair's window are zero.  Grid: (ceil(N / 256), pairs = T K).
__global__ __launch_bounds__(256) void k_lift_upa(const float2* __restrict__ w,
                                                  const int* __restrict__ starts,
                                                  const int* __restrict__ wz, int K, int wmax,
                                                  int Nz, int Nx, int Mz, int Mx,
                                                  const float2* __restrict__ tw,
                                                  float2* __restrict__ c_hat) {
  const int64_t pair = blockIdx.y;
  const int N = Nz * Nx, M = Mz * Mx;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const int ix = n / Nz, iz = n - ix * Nz;
  const int sz = starts[2 * pair], sx = starts[2 * pair + 1];
  const int Wz = wz[pair / K];
  const float2* wp = w + pair * wmax;
  double ax = 0.0, ay = 0.0;
  for (int i = 0; i < wmax; ++i) {
    const int ixw = i / Wz, izw = i - ixw * Wz;
    const int mz = (sz + izw) & (Mz - 1), mx = (sx + ixw) & (Mx - 1);
    const int q = (int)(((int64_t)mz * iz * Mx + (int64_t)mx * ix * Mz) & (M - 1));
    const float2 e = tw[q];                      // exp(-j 2 pi q / M)
    const float2 c = wp[i];
    ax += (double)c.x * e.x + (double)c.y * e.y;   // c conj(e)
    ay += (double)c.y * e.x - (double)c.x * e.y;
  }
  const double r = 1.0 / sqrt((double)M);
  c_hat[pair * N + n] = make_float2((float)(ax * r), (float)(ay * r));
}

// Planar beam patterns (Eq. 22 with a = a_x kron a_z): pattern[p][q] =
// |sum_{ix, iz} conj(c[ix Nz + iz]) e^{j (Omega_z iz + Omega_x ix)}| / (||c|| sqrt(N)) at
// omega[q] = (Omega_z, Omega_x), FP64 with the phase recurrences along z inside x.  One
// workgroup per correlator (staged in LDS), one thread per angle.
__global__ __launch_bounds__(256) void k_beam_pattern_upa(const float2* __restrict__ c, int Nz,
                                                          int Nx, const double* __restrict__ omega,
                                                          int Q, float* __restrict__ pattern) {
  __shared__ float2 cs[kBpMaxN];
  __shared__ double red[256];
  const int N = Nz * Nx;
  const int64_t p = blockIdx.x;
  const int tid = threadIdx.x;
  double nn = 0.0;
  for (int e = tid; e < N; e += 256) {
    const float2 v = c[p * N + e];
    cs[e] = v;
    nn += (double)v.x * v.x + (double)v.y * v.y;
  }
  red[tid] = nn;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  const double scale = 1.0 / (sqrt(red[0]) * sqrt((double)N));
  for (int q = tid; q < Q; q += 256) {
    double szs, szc, sxs, sxc;
    sincos(omega[2 * q], &szs, &szc);
    sincos(omega[2 * q + 1], &sxs, &sxc);
    double xr = 1.0, xi = 0.0, ar = 0.0, ai = 0.0;
    for (int ix = 0; ix < Nx; ++ix) {
      double zr = 1.0, zi = 0.0, br = 0.0, bi = 0.0;
      for (int iz = 0; iz < Nz; ++iz) {
        const float2 v = cs[ix * Nz + iz];
        br += (double)v.x * zr + (double)v.y * zi;   // conj(c) e^{j Omega_z iz}
        bi += (double)v.x * zi - (double)v.y * zr;
        const double t = zr * szc - zi * szs;
        zi = zr * szs + zi * szc;
        zr = t;
      }
      ar += br * xr - bi * xi;                       // times e^{j Omega_x ix}
      ai += br * xi + bi * xr;
      const double t = xr * sxc - xi * sxs;
      xi = xr * sxs + xi * sxc;
      xr = t;
    }
    pattern[p * Q + q] = (float)(sqrt(ar * ar + ai * ai) * scale);
  }
}

hipError_t launch_lift_upa(const float2* w, const int* starts, const int* wz, int T, int K,
                           int wmax, int Nz, int Nx, int Mz, int Mx, const float2* twM,
                           float2* c_hat, hipStream_t s) {
  const int pairs = T * K;
  if (pairs < 1) return hipSuccess;
  if (pairs > 65535 || (Mz & (Mz - 1)) != 0 || (Mx & (Mx - 1)) != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_lift_upa, dim3((Nz * Nx + 255) / 256, pairs), dim3(256), 0, s, w, starts,
                     wz, K, wmax, Nz, Nx, Mz, Mx, twM, c_hat);
  return hipGetLastError();
}

hipError_t launch_beam_pattern_upa(const float2* c, int pairs, int Nz, int Nx,
                                   const double* omega, int Q, float* pattern, hipStream_t s) {
  if (pairs < 1 || Q < 1) return hipSuccess;
  if (Nz < 1 || Nx < 1 || Nz * Nx > kBpMaxN) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_beam_pattern_upa, dim3(pairs), dim3(256), 0, s, c, Nz, Nx, omega, Q,
                     pattern);
  return hipGetLastError();
}

hipError_t launch_beam_pattern(const float2* c, int pairs, int N, const double* omega, int Q,
                               float* pattern, hipStream_t s) {
  if (pairs < 1 || Q < 1) return hipSuccess;
  if (N < 1 || N > kBpMaxN) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_beam_pattern, dim3(pairs), dim3(256), 0, s, c, N, omega, Q, pattern);
  return hipGetLastError();
}

hipError_t launch_lift(const float2* w, const int* starts, int pairs, int wmax, int N, int M,
                       const float2* twM, float2* c_hat, hipStream_t s) {
  if (pairs < 1) return hipSuccess;
  if (pairs > 65535 || (M & (M - 1)) != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_lift, dim3((N + 255) / 256, pairs), dim3(256), 0, s, w, starts, wmax, N, M,
                     twM, c_hat);
  return hipGetLastError();
}

hipError_t launch_lift_apply(const float2* X, const float2* c_hat, float2* out, int N, int K,
                             int B, int L, int Lt, int T, hipStream_t s) {
  if (Lt < 1 || T < 1) return hipSuccess;
  if (K > 65535) return hipErrorInvalidValue;
  if (T > kLaTT) {
    hipLaunchKernelGGL(k_lift_apply_mfma,
                       dim3((Lt + kLmTL - 1) / kLmTL, (T + kLmTT - 1) / kLmTT, K), dim3(256), 0,
                       s, X, c_hat, out, N, K, B, L, Lt, T);
  } else {
    hipLaunchKernelGGL(k_lift_apply, dim3((Lt + kLaTL - 1) / kLaTL, (T + kLaTT - 1) / kLaTT, K),
                       dim3(256), 0, s, X, c_hat, out, N, K, B, L, Lt, T);
  }
  return hipGetLastError();
}

}  // namespace wbm
