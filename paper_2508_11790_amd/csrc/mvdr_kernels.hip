// Window placement / windowed steering, and the per-(target, subband) reduced-dimension MVDR
// kernels for gfx950: loaded W x W sample covariance (Eq. 11), Cholesky factorisation, the
// two triangular solves giving c = R^-1 a / (a^H R^-1 a) (Eq. 13 / Eq. 20) and the beam
// output c^H y on the test snapshots.
//
// Fused form: one workgroup per pair runs everything, placing its window and evaluating its
// steering vector itself; the covariance accumulates exact FP32 x FP32 products in FP64 and
// the Cholesky / solves run in FP64 (window covariances next to strong interferers reach
// condition numbers ~1e6, where FP32 accumulation loses the weights).  Windows up to 40 bins
// run one wave64 per pair; wider windows run four waves per pair.
// Plain form: the same steps as three FP32 launches with R and c in HBM, gathering the window
// rows from the full beamspace.
#include <math.h>

#include "wbm_dev.h"
#include "wbm_launch.h"

namespace wbm {

template <typename T>
struct C2 {
  T x, y;
};
template <typename T>
__device__ __forceinline__ C2<T> c2(T a, T b) {
  C2<T> r;
  r.x = a;
  r.y = b;
  return r;
}

constexpr int kCH = 64;        // snapshots per LDS chunk of the covariance
constexpr int kCHS = kCH + 1;  // LDS row stride of a staged chunk: rows two banks apart
constexpr int kWaveWMax = 40;  // widest window of the one-wave kernel

// ------------------------------------------------------------------------------------------
// One thread per (t, k, i < wmax): start s of the pair and its windowed steering vector.
__global__ void k_steer(WindowGeom g, int wmax, int* __restrict__ starts,
                        double2* __restrict__ abar) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)g.T * g.K * wmax;
  if (idx >= total) return;
  const int i = (int)(idx % wmax);
  const int64_t pk = idx / wmax;
  const int k = (int)(pk % g.K), t = (int)(pk / g.K);
  double u;
  int s;
  window_of(g, t, k, &u, &s);
  if (i == 0) starts[t * g.K + k] = s;
  abar[idx] = (i < g.win[t]) ? window_steering(g, u, s, i) : make_double2(0.0, 0.0);
}

hipError_t launch_steer(const WindowGeom& g, int wmax, int* starts, double2* abar,
                        hipStream_t s) {
  const int64_t total = (int64_t)g.T * g.K * wmax;
  const int bs = 256;
  hipLaunchKernelGGL(k_steer, dim3((unsigned)((total + bs - 1) / bs)), dim3(bs), 0, s, g, wmax,
                     starts, abar);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Row e of the packed lower triangle -> (i, j), j <= i.
__device__ __forceinline__ void tri_index(int e, int& i, int& j) {
  int ii = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
  while ((ii + 1) * (ii + 2) / 2 <= e) ++ii;
  while (ii * (ii + 1) / 2 > e) --ii;
  i = ii;
  j = e - ii * (ii + 1) / 2;
}

// Snapshot b of window row i of pair (t, k).
template <bool WINDOWED>
__device__ __forceinline__ float2 load_y(const float2* __restrict__ src, const PairArgs& a, int k,
                                         int woff, int s, int i, int b) {
  if constexpr (WINDOWED) {
    const int TB = 1 << a.logTB;
    return src[(((int64_t)k * a.nbt + (b >> a.logTB)) * a.sumW + woff + i) * TB + (b & (TB - 1))];
  } else {
    return src[((int64_t)k * a.M + ((s + i) & (a.M - 1))) * a.B + b];
  }
}

// Stage window rows i < W, snapshots b0 .. b0 + kCH - 1 (zero at b >= limit) into
// ys[i * kCHS + bb].  The thread-to-element order follows the source layout so that
// consecutive threads read consecutive addresses: snapshot-fastest runs for the full beamspace
// and for window tiles of at least kCH snapshots, otherwise one contiguous [W][TB] tile block
// after another.
template <bool WINDOWED, int THREADS>
__device__ __forceinline__ void stage_rows(const float2* __restrict__ src, const PairArgs& a,
                                           int k, int woff, int s, int W, int b0, int limit,
                                           float2* ys) {
  const int tid = threadIdx.x;
  if (!WINDOWED || a.logTB >= 6) {
    for (int idx = tid; idx < W * kCH; idx += THREADS) {
      const int i = idx / kCH, bb = idx - i * kCH;
      const int b = b0 + bb;
      ys[i * kCHS + bb] =
          (b < limit) ? load_y<WINDOWED>(src, a, k, woff, s, i, b) : make_float2(0.f, 0.f);
    }
  } else {
    const int per = W << a.logTB;
    const int tbm = (1 << a.logTB) - 1;
    for (int idx = tid; idx < W * kCH; idx += THREADS) {
      const int q = idx / per, r = idx - q * per;
      const int i = r >> a.logTB, bb = (q << a.logTB) + (r & tbm);
      const int b = b0 + bb;
      ys[i * kCHS + bb] =
          (b < limit) ? load_y<WINDOWED>(src, a, k, woff, s, i, b) : make_float2(0.f, 0.f);
    }
  }
}

// R (LDS, row stride RS, lower triangle) = (1/L) sum_{b<L} y_b y_b^H + delta I, accumulated
// in ACC by THREADS threads, up to EPT lower-triangle entries per thread (W(W+1)/2 <=
// EPT * THREADS).  ys is an LDS scratch of W x kCHS float2 that may alias R.
template <typename ACC, bool WINDOWED, int THREADS, int EPT>
__device__ void pair_covariance(const float2* __restrict__ src, const PairArgs& a, int k, int W,
                                int woff, int s, float2* ys, C2<ACC>* R, int RS, double delta) {
  const int tid = threadIdx.x;
  const int nE = W * (W + 1) / 2;
  int S = 1;
  if (nE < THREADS) {
    S = THREADS / nE;
    S = 1 << (31 - __clz(S));
    if (S > 64) S = 64;
  }
  const int groups = THREADS / S;
  const int g = tid / S, sl = tid & (S - 1);
  C2<ACC> acc[EPT];
  int ei[EPT], ej[EPT];
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    acc[q] = c2<ACC>(0, 0);
    const int e = g + q * groups;
    ei[q] = -1;
    ej[q] = 0;
    if (e < nE) tri_index(e, ei[q], ej[q]);
  }
  for (int c0 = 0; c0 < a.L; c0 += kCH) {
    __syncthreads();
    stage_rows<WINDOWED, THREADS>(src, a, k, woff, s, W, c0, a.L, ys);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      if (ei[q] >= 0) {
        const float2* yi = ys + ei[q] * kCHS;
        const float2* yj = ys + ej[q] * kCHS;
        ACC ax = acc[q].x, ay = acc[q].y;
        for (int bb = sl; bb < kCH; bb += S) {
          const float2 u = yi[bb], v = yj[bb];
          const ACC ux = u.x, uy = u.y, vx = v.x, vy = v.y;
          ax += ux * vx + uy * vy;   // y_i conj(y_j)
          ay += uy * vx - ux * vy;
        }
        acc[q] = c2<ACC>(ax, ay);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    for (int off = S >> 1; off > 0; off >>= 1) {
      acc[q].x += __shfl_xor(acc[q].x, off);
      acc[q].y += __shfl_xor(acc[q].y, off);
    }
  }
  __syncthreads();   // ys (may alias R) no longer read
  const ACC invL = (ACC)1 / (ACC)a.L;
  if (sl == 0) {
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      if (ei[q] >= 0) {
        C2<ACC> r = c2<ACC>(acc[q].x * invL, acc[q].y * invL);
        if (ei[q] == ej[q]) {
          r.x += (ACC)delta;
          r.y = 0;
        }
        R[ei[q] * RS + ej[q]] = r;
      }
    }
  }
  __syncthreads();
}

// In-LDS right-looking Cholesky R = G G^H (lower), G's diagonal in diag[], strictly lower part
// overwriting R.  Returns 0, or j + 1 when pivot j is not positive and finite (uniform).
template <typename T, int THREADS>
__device__ int chol_lds(C2<T>* R, int RS, T* diag, int W) {
  const int tid = threadIdx.x;
  for (int j = 0; j < W; ++j) {
    const T d = R[j * RS + j].x;
    if (!(d > (T)0) || !(d < (T)INFINITY)) return j + 1;
    const T dj = sqrt(d);
    const T inv = (T)1 / dj;
    if (tid == 0) diag[j] = dj;
    for (int i = j + 1 + tid; i < W; i += THREADS) {
      C2<T> v = R[i * RS + j];
      R[i * RS + j] = c2<T>(v.x * inv, v.y * inv);
    }
    __syncthreads();
    const int nT = W - j - 1;
    const int cnt = nT * (nT + 1) / 2;
    for (int e = tid; e < cnt; e += THREADS) {
      int ii, cc;
      tri_index(e, ii, cc);
      const int i = j + 1 + ii, c = j + 1 + cc;
      const C2<T> gi = R[i * RS + j], gc = R[c * RS + j];
      C2<T> r = R[i * RS + c];
      r.x -= gi.x * gc.x + gi.y * gc.y;   // g_i conj(g_c)
      r.y -= gi.y * gc.x - gi.x * gc.y;
      R[i * RS + c] = r;
    }
    __syncthreads();
  }
  return 0;
}

// Wave 0 solves G v = a, q = v^H v, G^H x = v, w = x / q (one lane per row, W <= 64) and
// stores w in wv[] (LDS).  Caller syncs afterwards.
template <typename T>
__device__ void solve_lds(const C2<T>* R, int RS, const T* diag, int W, const double2* av,
                          C2<T>* wv) {
  if (threadIdx.x >= 64) return;
  const int lane = threadIdx.x;
  C2<T> v = c2<T>(0, 0);
  if (lane < W) v = c2<T>((T)av[lane].x, (T)av[lane].y);
  for (int j = 0; j < W; ++j) {
    const T dinv = (T)1 / diag[j];
    const T vx = __shfl(v.x, j) * dinv, vy = __shfl(v.y, j) * dinv;
    if (lane == j) {
      v = c2<T>(vx, vy);
    } else if (lane > j && lane < W) {
      const C2<T> g = R[lane * RS + j];
      v.x -= g.x * vx - g.y * vy;
      v.y -= g.x * vy + g.y * vx;
    }
  }
  T q = v.x * v.x + v.y * v.y;
  for (int off = 32; off > 0; off >>= 1) q += __shfl_xor(q, off);
  C2<T> x = v;
  for (int j = W - 1; j >= 0; --j) {
    const T dinv = (T)1 / diag[j];
    const T xx = __shfl(x.x, j) * dinv, xy = __shfl(x.y, j) * dinv;
    if (lane == j) {
      x = c2<T>(xx, xy);
    } else if (lane < j) {
      const C2<T> g = R[j * RS + lane];   // (G^H)[lane][j] = conj(G[j][lane])
      x.x -= g.x * xx + g.y * xy;
      x.y -= g.x * xy - g.y * xx;
    }
  }
  const T qinv = (T)1 / q;
  if (lane < W) wv[lane] = c2<T>(x.x * qinv, x.y * qinv);
}

// out[l] = w^H y_{L + l} for the Lt test snapshots, staged through LDS (ys, which may alias
// the factorised R: it is no longer read).  Zero outputs when fail.
template <int THREADS>
__device__ void apply_staged(const float2* __restrict__ Yw, const PairArgs& a, int k, int woff,
                             int s, int W, int fail, const C2<double>* wv, float2* ys,
                             float2* __restrict__ out) {
  constexpr int SPL = THREADS / kCH;    // threads per snapshot
  const int tid = threadIdx.x;
  const int l0 = tid / SPL, part = tid - l0 * SPL;
  for (int c0 = 0; c0 < a.Lt; c0 += kCH) {
    __syncthreads();
    stage_rows<true, THREADS>(Yw, a, k, woff, s, W, a.L + c0, a.L + a.Lt, ys);
    __syncthreads();
    double zx = 0.0, zy = 0.0;
    if (!fail) {
      for (int i = part; i < W; i += SPL) {
        const float2 y = ys[i * kCHS + l0];
        const C2<double> w = wv[i];
        zx += w.x * (double)y.x + w.y * (double)y.y;    // conj(w) y
        zy += w.x * (double)y.y - w.y * (double)y.x;
      }
    }
    for (int off = SPL >> 1; off > 0; off >>= 1) {
      zx += __shfl_xor(zx, off);
      zy += __shfl_xor(zy, off);
    }
    if (part == 0 && c0 + l0 < a.Lt) out[c0 + l0] = make_float2((float)zx, (float)zy);
  }
}

struct PairLds {
  int RS;
  size_t r_off, diag_off, wv_off, av_off, total;
};

template <typename T>
__host__ __device__ inline PairLds pair_lds_layout(int wmax) {
  PairLds p;
  p.RS = wmax + 1;
  size_t rbytes = sizeof(C2<T>) * (size_t)wmax * p.RS;
  size_t ybytes = sizeof(float2) * (size_t)wmax * kCHS;
  size_t big = rbytes > ybytes ? rbytes : ybytes;
  big = (big + 15) & ~(size_t)15;
  p.r_off = 0;
  p.diag_off = big;
  p.wv_off = big + ((sizeof(T) * 64 + 15) & ~(size_t)15);
  p.av_off = p.wv_off + sizeof(C2<T>) * 64;
  p.total = p.av_off + sizeof(double2) * 64;
  return p;
}

// ------------------------------------------------------------------------------------------
// Fused form: one workgroup of THREADS per pair p = k * T + t.
template <int THREADS, int EPT>
__global__ __launch_bounds__(THREADS) void k_mvdr_fused(PairArgs a, WindowGeom g, DevDesc d,
                                                        const float2* __restrict__ Yw,
                                                        float2* __restrict__ out,
                                                        float2* __restrict__ wout,
                                                        int* __restrict__ starts_out,
                                                        int* __restrict__ info) {
  extern __shared__ __align__(16) unsigned char smem[];
  const PairLds lay = pair_lds_layout<double>(a.wmax);
  C2<double>* R = reinterpret_cast<C2<double>*>(smem + lay.r_off);
  float2* ys = reinterpret_cast<float2*>(smem + lay.r_off);
  double* diag = reinterpret_cast<double*>(smem + lay.diag_off);
  C2<double>* wv = reinterpret_cast<C2<double>*>(smem + lay.wv_off);
  double2* av = reinterpret_cast<double2*>(smem + lay.av_off);

  const int p = blockIdx.x;
  const int k = p / a.T, t = p - k * a.T;
  int W = d.win[t], woff = d.woff[t];
  const int64_t pair = (int64_t)t * a.K + k;
  double u;
  int s;
  window_of(g, t, k, &u, &s);
  if (a.pw) {
    // centred sub-window: for widths of equal parity the start moves by the half difference
    const int Wp = a.pw[pair];
    if (Wp >= 1 && Wp <= W && ((W - Wp) & 1) == 0) {
      const int off = (W - Wp) >> 1;
      woff += off;
      s += off;
      W = Wp;
    }
  }
  const double delta = a.pdelta ? (double)a.pdelta[pair] : a.delta;
  if (threadIdx.x < W) av[threadIdx.x] = window_steering(g, u, s, threadIdx.x);
  if (starts_out && threadIdx.x == 0) starts_out[pair] = s;

  pair_covariance<double, true, THREADS, EPT>(Yw, a, k, W, woff, s, ys, R, lay.RS, delta);
  const int fail = chol_lds<double, THREADS>(R, lay.RS, diag, W);
  if (!fail) solve_lds<double>(R, lay.RS, diag, W, av, wv);
  apply_staged<THREADS>(Yw, a, k, woff, s, W, fail, wv, ys, out + pair * a.Lt);
  if (wout) {
    for (int i = threadIdx.x; i < a.wmax; i += THREADS) {
      float2 v = make_float2(0.f, 0.f);
      if (!fail && i < W) v = make_float2((float)wv[i].x, (float)wv[i].y);
      wout[pair * a.wmax + i] = v;
    }
  }
  if (info && threadIdx.x == 0) info[pair] = fail;
}

template <int THREADS, int EPT>
static hipError_t fused_launch(const PairArgs& a, const WindowGeom& g, const DevDesc& d,
                               const float2* Yw, float2* out, float2* wout, int* starts,
                               int* info, hipStream_t s) {
  const PairLds lay = pair_lds_layout<double>(a.wmax);
  hipLaunchKernelGGL((k_mvdr_fused<THREADS, EPT>), dim3(a.T * a.K), dim3(THREADS), lay.total, s,
                     a, g, d, Yw, out, wout, starts, info);
  return hipGetLastError();
}

bool mvdr_wave_supported(int wmax) { return wmax <= kWaveWMax; }

hipError_t launch_mvdr_fused(const PairArgs& a, const WindowGeom& g, const DevDesc& d,
                             const float2* Yw, float2* out, float2* wout, int* starts, int* info,
                             int threads, hipStream_t s) {
  const int nE = a.wmax * (a.wmax + 1) / 2;
  if (threads == 64 && a.wmax <= kWaveWMax) {
    // one wave64 per pair; entries per lane = ceil(nE / 64)
    const int ept = (nE + 63) / 64;
    if (ept <= 1) return fused_launch<64, 1>(a, g, d, Yw, out, wout, starts, info, s);
    if (ept <= 2) return fused_launch<64, 2>(a, g, d, Yw, out, wout, starts, info, s);
    if (ept <= 3) return fused_launch<64, 3>(a, g, d, Yw, out, wout, starts, info, s);
    if (ept <= 5) return fused_launch<64, 5>(a, g, d, Yw, out, wout, starts, info, s);
    if (ept <= 9) return fused_launch<64, 9>(a, g, d, Yw, out, wout, starts, info, s);
    return fused_launch<64, 13>(a, g, d, Yw, out, wout, starts, info, s);
  }
  return fused_launch<256, 9>(a, g, d, Yw, out, wout, starts, info, s);
}

// ------------------------------------------------------------------------------------------
// Plain form, FP32 throughout, three launches.
constexpr int kPlainThreads = 256;

__global__ __launch_bounds__(kPlainThreads) void k_plain_cov(PairArgs a, DevDesc d,
                                                             const float2* __restrict__ Y,
                                                             const int* __restrict__ starts,
                                                             float2* __restrict__ R32) {
  extern __shared__ __align__(16) unsigned char smem[];
  const PairLds lay = pair_lds_layout<float>(a.wmax);
  C2<float>* R = reinterpret_cast<C2<float>*>(smem + lay.r_off);
  float2* ys = reinterpret_cast<float2*>(smem + lay.r_off);
  const int p = blockIdx.x;
  const int k = p / a.T, t = p - k * a.T;
  const int W = d.win[t];
  const int s = starts[t * a.K + k];
  const int64_t pair = (int64_t)t * a.K + k;
  pair_covariance<float, false, kPlainThreads, 9>(Y, a, k, W, 0, s, ys, R, lay.RS, a.delta);
  float2* dst = R32 + pair * a.wmax * a.wmax;
  for (int e = threadIdx.x; e < W * W; e += kPlainThreads) {
    const int i = e / W, j = e - i * W;
    if (j <= i) dst[i * a.wmax + j] = make_float2(R[i * lay.RS + j].x, R[i * lay.RS + j].y);
  }
}

__global__ __launch_bounds__(kPlainThreads) void k_plain_solve(PairArgs a, DevDesc d,
                                                               const float2* __restrict__ R32,
                                                               const double2* __restrict__ abar,
                                                               float2* __restrict__ w32,
                                                               int* __restrict__ info) {
  extern __shared__ __align__(16) unsigned char smem[];
  const PairLds lay = pair_lds_layout<float>(a.wmax);
  C2<float>* R = reinterpret_cast<C2<float>*>(smem + lay.r_off);
  float* diag = reinterpret_cast<float*>(smem + lay.diag_off);
  C2<float>* wv = reinterpret_cast<C2<float>*>(smem + lay.wv_off);
  const int p = blockIdx.x;
  const int k = p / a.T, t = p - k * a.T;
  const int W = d.win[t];
  const int64_t pair = (int64_t)t * a.K + k;
  const float2* src = R32 + pair * a.wmax * a.wmax;
  for (int e = threadIdx.x; e < W * W; e += kPlainThreads) {
    const int i = e / W, j = e - i * W;
    if (j <= i) R[i * lay.RS + j] = c2<float>(src[i * a.wmax + j].x, src[i * a.wmax + j].y);
  }
  __syncthreads();
  const int fail = chol_lds<float, kPlainThreads>(R, lay.RS, diag, W);
  if (!fail) solve_lds<float>(R, lay.RS, diag, W, abar + pair * a.wmax, wv);
  __syncthreads();
  for (int i = threadIdx.x; i < a.wmax; i += kPlainThreads) {
    float2 v = make_float2(0.f, 0.f);
    if (!fail && i < W) v = make_float2(wv[i].x, wv[i].y);
    w32[pair * a.wmax + i] = v;
  }
  if (info && threadIdx.x == 0) info[pair] = fail;
}

__global__ __launch_bounds__(kPlainThreads) void k_plain_apply(PairArgs a, DevDesc d,
                                                               const float2* __restrict__ Y,
                                                               const int* __restrict__ starts,
                                                               const float2* __restrict__ w32,
                                                               float2* __restrict__ out,
                                                               float2* __restrict__ wout) {
  __shared__ float2 wv[64];
  const int p = blockIdx.x;
  const int k = p / a.T, t = p - k * a.T;
  const int W = d.win[t];
  const int s = starts[t * a.K + k];
  const int64_t pair = (int64_t)t * a.K + k;
  if (threadIdx.x < a.wmax) {
    wv[threadIdx.x] = w32[pair * a.wmax + threadIdx.x];
    if (wout) wout[pair * a.wmax + threadIdx.x] = w32[pair * a.wmax + threadIdx.x];
  }
  __syncthreads();
  for (int l = threadIdx.x; l < a.Lt; l += kPlainThreads) {
    float zx = 0.f, zy = 0.f;
    for (int i = 0; i < W; ++i) {
      const float2 y = load_y<false>(Y, a, k, 0, s, i, a.L + l);
      const float2 w = wv[i];
      zx += w.x * y.x + w.y * y.y;
      zy += w.x * y.y - w.y * y.x;
    }
    out[pair * a.Lt + l] = make_float2(zx, zy);
  }
}

hipError_t launch_mvdr_plain(const PairArgs& a, const DevDesc& d, const float2* Y,
                             const int* starts, const double2* abar, float2* R32, float2* w32,
                             float2* out, float2* wout, int* info, hipStream_t s) {
  const PairLds lay = pair_lds_layout<float>(a.wmax);
  const dim3 grid(a.T * a.K), blk(kPlainThreads);
  hipLaunchKernelGGL(k_plain_cov, grid, blk, lay.total, s, a, d, Y, starts, R32);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_plain_solve, grid, blk, lay.total, s, a, d, R32, abar, w32, info);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_plain_apply, grid, blk, 0, s, a, d, Y, starts, w32, out, wout);
  return hipGetLastError();
}

hipError_t set_pair_attributes() {
  hipError_t e = hipFuncSetAttribute((const void*)k_mvdr_fused<256, 9>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_mvdr_fused<64, 13>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, 64 * 1024);
}

}  // namespace wbm

// ==========================================================================================
// Mixed-precision form.  The W x W covariance is the one dense contraction of the path: with
// Z = [Re Y; Im Y] (2W x L real) the Gram G = Z Z^T gives Re R = G11 + G22 and
// Im R = G21 - G12.  G runs on MFMA (v_mfma_f32_32x32x16_bf16, FP32 accumulation) over 32 x 32
// tiles of the lower triangle, either with the BF16-rounded snapshots (one product per tile and
// step) or with each FP32 snapshot split into BF16 hi + lo parts (hi*hi + hi*lo + lo*hi, three
// products).  The Cholesky and both triangular solves run in FP32; the residual of one
// iterative-refinement step and the normalisation a^H R^-1 a run in FP64.  A window whose
// Cholesky pivots span more than kRouteKappa (condition-number estimate) is routed to the exact
// path instead: FP64 accumulation of the FP32 snapshots and FP64 Cholesky; its info entry then
// carries bit 30.
namespace wbm {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

constexpr int kMixThreads = 256;
constexpr int kMixCH = 64;                 // snapshots per LDS chunk (4 MFMA k-steps)
constexpr int kMixRS = kMixCH + 8;         // bf16 row stride (144 B: off the bank period)
constexpr int kMaxTiles = 10;              // lower-triangle 32x32 tiles of 2W <= 128
constexpr double kRouteKappa = 1.0e4;
constexpr int kInfoRouted = 1 << 30;

__device__ __forceinline__ __bf16 to_bf16(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  const unsigned short h = (unsigned short)(u >> 16);
  return __builtin_bit_cast(__bf16, h);
}
__device__ __forceinline__ float from_bf16(__bf16 b) {
  const unsigned short h = __builtin_bit_cast(unsigned short, b);
  return __uint_as_float(((unsigned)h) << 16);
}

struct MixLds {
  size_t zhi, zlo, g, r, diag, wv, av, total;
  int RS;
};

__host__ __device__ inline MixLds mix_lds_layout(int wmax) {
  MixLds p;
  const int rows = 2 * wmax;
  const int pad = (rows + 31) / 32 * 32;
  size_t o = 0;
  p.zhi = o;
  o += sizeof(__bf16) * (size_t)pad * kMixRS;
  p.zlo = o;
  o += sizeof(__bf16) * (size_t)pad * kMixRS;
  o = (o + 15) & ~(size_t)15;
  // G (FP32, pad x pad) aliases the staging area after the last chunk
  const size_t gbytes = sizeof(float) * (size_t)pad * pad;
  const size_t ybytes = sizeof(float2) * (size_t)wmax * kCHS;  // FP64-route / apply staging
  p.g = 0;
  if (gbytes > o) o = (gbytes + 15) & ~(size_t)15;
  if (ybytes > o) o = (ybytes + 15) & ~(size_t)15;
  p.RS = wmax + 1;
  p.r = o;                                               // complex R, FP64 (routing needs it)
  o += sizeof(C2<double>) * (size_t)wmax * p.RS;
  p.diag = o;
  o += sizeof(double) * 64;
  p.wv = o;
  o += sizeof(C2<double>) * 64;
  p.av = o;
  o += sizeof(double2) * 64;
  p.total = o;
  return p;
}

template <bool SPLIT>
__global__ __launch_bounds__(kMixThreads) void k_mvdr_mixed(PairArgs a, WindowGeom g, DevDesc d,
                                                            const float2* __restrict__ Yw,
                                                            float2* __restrict__ out,
                                                            float2* __restrict__ wout,
                                                            int* __restrict__ starts_out,
                                                            int* __restrict__ info) {
  extern __shared__ __align__(16) unsigned char smem[];
  const MixLds lay = mix_lds_layout(a.wmax);
  __bf16* zhi = reinterpret_cast<__bf16*>(smem + lay.zhi);
  __bf16* zlo = reinterpret_cast<__bf16*>(smem + lay.zlo);
  float* G = reinterpret_cast<float*>(smem + lay.g);
  C2<double>* R = reinterpret_cast<C2<double>*>(smem + lay.r);
  double* diag = reinterpret_cast<double*>(smem + lay.diag);
  C2<double>* wv = reinterpret_cast<C2<double>*>(smem + lay.wv);
  double2* av = reinterpret_cast<double2*>(smem + lay.av);
  float* R32 = reinterpret_cast<float*>(smem + lay.r);   // FP32 view used by the FP32 Cholesky
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  const int p = blockIdx.x;
  const int k = p / a.T, t = p - k * a.T;
  const int W = d.win[t], woff = d.woff[t];
  const int64_t pair = (int64_t)t * a.K + k;
  double u;
  int s;
  window_of(g, t, k, &u, &s);
  if (tid < W) av[tid] = window_steering(g, u, s, tid);
  if (starts_out && tid == 0) starts_out[pair] = s;

  const int rows = 2 * W;
  const int nt = (rows + 31) / 32;
  const int ntiles = nt * (nt + 1) / 2;
  f32x16_t acc[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) acc[q] = f32x16_t{};
  // this wave's tiles: q-th tile = wave + 4 q
  for (int c0 = 0; c0 < a.L; c0 += kMixCH) {
    __syncthreads();
    // complex snapshots in the source order (as stage_rows), real parts to rows i, imaginary
    // parts to rows W + i; padding rows stay zero
    for (int idx = tid; idx < (nt * 32 - rows) * kMixCH; idx += kMixThreads) {
      const int r = rows + idx / kMixCH, bb = idx % kMixCH;
      zhi[r * kMixRS + bb] = to_bf16(0.f);
      if (SPLIT) zlo[r * kMixRS + bb] = to_bf16(0.f);
    }
    const bool runs = a.logTB >= 6;
    const int per = W << a.logTB, tbm = (1 << a.logTB) - 1;
    for (int idx = tid; idx < W * kMixCH; idx += kMixThreads) {
      int i, bb;
      if (runs) {
        i = idx / kMixCH;
        bb = idx - i * kMixCH;
      } else {
        const int q = idx / per, r = idx - q * per;
        i = r >> a.logTB;
        bb = (q << a.logTB) + (r & tbm);
      }
      const int b = c0 + bb;
      const float2 y = (b < a.L) ? load_y<true>(Yw, a, k, woff, s, i, b) : make_float2(0.f, 0.f);
      const __bf16 hr = to_bf16(y.x), hi = to_bf16(y.y);
      zhi[i * kMixRS + bb] = hr;
      zhi[(W + i) * kMixRS + bb] = hi;
      if (SPLIT) {
        zlo[i * kMixRS + bb] = to_bf16(y.x - from_bf16(hr));
        zlo[(W + i) * kMixRS + bb] = to_bf16(y.y - from_bf16(hi));
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int tile = wave + 4 * q;
      if (tile < ntiles) {
        int ti, tj;
        tri_index(tile, ti, tj);
        const int ra = ti * 32 + (lane & 31), rb = tj * 32 + (lane & 31);
        const int kofs = (lane >> 5) * 8;
#pragma unroll
        for (int ks = 0; ks < kMixCH; ks += 16) {
          const bf16x8_t ah = *reinterpret_cast<const bf16x8_t*>(zhi + ra * kMixRS + ks + kofs);
          const bf16x8_t bh = *reinterpret_cast<const bf16x8_t*>(zhi + rb * kMixRS + ks + kofs);
          acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc[q], 0, 0, 0);
          if (SPLIT) {
            const bf16x8_t al = *reinterpret_cast<const bf16x8_t*>(zlo + ra * kMixRS + ks + kofs);
            const bf16x8_t bl = *reinterpret_cast<const bf16x8_t*>(zlo + rb * kMixRS + ks + kofs);
            acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc[q], 0, 0, 0);
            acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc[q], 0, 0, 0);
          }
        }
      }
    }
  }
  __syncthreads();   // staging no longer read; G aliases it
  const int pad = nt * 32;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const int tile = wave + 4 * q;
    if (tile < ntiles) {
      int ti, tj;
      tri_index(tile, ti, tj);
      const int col = tj * 32 + (lane & 31);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = ti * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        G[row * pad + col] = acc[q][r];
      }
    }
  }
  __syncthreads();
  // complex R (lower) from the real Gram, scaled and loaded; FP32 copy for the FP32 Cholesky
  const int RS = lay.RS;
  const float invL = 1.0f / (float)a.L;
  for (int e = tid; e < W * W; e += kMixThreads) {
    const int i = e / W, j = e - i * W;
    if (j <= i) {
      const float g11 = G[i * pad + j], g22 = G[(W + i) * pad + (W + j)];
      const float g21 = G[(W + i) * pad + j], g12t = G[(W + j) * pad + i];   // G12[i][j] = G[W+j][i]
      float re = (g11 + g22) * invL, im = (g21 - g12t) * invL;
      if (i == j) {
        re += (float)a.delta;
        im = 0.f;
      }
      R32[2 * (i * RS + j)] = re;       // FP32 complex in the first half of R's storage
      R32[2 * (i * RS + j) + 1] = im;
    }
  }
  __syncthreads();
  C2<float>* Rf = reinterpret_cast<C2<float>*>(R32);
  float* diagf = reinterpret_cast<float*>(diag);
  int fail = chol_lds<float, kMixThreads>(Rf, RS, diagf, W);
  // condition estimate from the pivots: (max / min)^2
  bool route = fail != 0;
  if (!fail) {
    float dmax = 0.f, dmin = 3.0e38f;
    for (int j = 0; j < W; ++j) {
      dmax = fmaxf(dmax, diagf[j]);
      dmin = fminf(dmin, diagf[j]);
    }
    route = (double)dmax * dmax > kRouteKappa * (double)dmin * dmin;
  }
  __syncthreads();
  if (!route) {
    // FP32 solves of R x = a, one FP64-residual refinement, FP64 normalisation (wave 0)
    if (tid < 64) {
      C2<double> x = c2<double>(0, 0);
      C2<double> b = c2<double>(0, 0);
      if (lane < W) b = c2<double>(av[lane].x, av[lane].y);
      for (int it = 0; it < 2; ++it) {
        // rhs = b - R x in FP64 with R the MFMA-formed matrix, read back from the Gram G
        // (lower tiles): R_ij = (G[i][j] + G[W+i][W+j] + i (G[W+i][j] - G[W+j][i])) / L for
        // i >= j, R_ij = conj(R_ji) above the diagonal, + delta on it.
        C2<float> v = c2<float>(0.f, 0.f);
        {
          double rx = 0.0, ry = 0.0;
          for (int j = 0; j < W; ++j) {
            const double xj_x = __shfl(x.x, j), xj_y = __shfl(x.y, j);
            if (lane < W) {
              const int hi = lane >= j ? lane : j, lo = lane >= j ? j : lane;
              double re = ((double)G[hi * pad + lo] + (double)G[(W + hi) * pad + (W + lo)]) / a.L;
              double im = ((double)G[(W + hi) * pad + lo] - (double)G[(W + lo) * pad + hi]) / a.L;
              if (lane < j) im = -im;
              if (lane == j) {
                re += a.delta;
                im = 0.0;
              }
              rx += re * xj_x - im * xj_y;
              ry += re * xj_y + im * xj_x;
            }
          }
          if (lane < W) v = c2<float>((float)(b.x - rx), (float)(b.y - ry));
        }
        // dx = R^-1 rhs in FP32: forward then backward substitution with the factor
        for (int j = 0; j < W; ++j) {
          const float dinv = 1.0f / diagf[j];
          const float vx = __shfl(v.x, j) * dinv, vy = __shfl(v.y, j) * dinv;
          if (lane == j) {
            v = c2<float>(vx, vy);
          } else if (lane > j && lane < W) {
            const C2<float> gg = Rf[lane * RS + j];
            v.x -= gg.x * vx - gg.y * vy;
            v.y -= gg.x * vy + gg.y * vx;
          }
        }
        for (int j = W - 1; j >= 0; --j) {
          const float dinv = 1.0f / diagf[j];
          const float xx = __shfl(v.x, j) * dinv, xy = __shfl(v.y, j) * dinv;
          if (lane == j) {
            v = c2<float>(xx, xy);
          } else if (lane < j) {
            const C2<float> gg = Rf[j * RS + lane];
            v.x -= gg.x * xx + gg.y * xy;
            v.y -= gg.x * xy - gg.y * xx;
          }
        }
        x.x += (double)v.x;
        x.y += (double)v.y;
      }
      // q = a^H x in FP64 (real for Hermitian positive definite R)
      double qq = (lane < W) ? b.x * x.x + b.y * x.y : 0.0;
      for (int off = 32; off > 0; off >>= 1) qq += __shfl_xor(qq, off);
      if (lane < W) wv[lane] = c2<double>(x.x / qq, x.y / qq);
    }
  } else {
    // exact route: FP64 accumulation of the FP32 snapshots and FP64 Cholesky
    float2* ys = reinterpret_cast<float2*>(smem);
    pair_covariance<double, true, kMixThreads, 9>(Yw, a, k, W, woff, s, ys, R, RS, a.delta);
    fail = chol_lds<double, kMixThreads>(R, RS, diag, W);
    if (!fail) solve_lds<double>(R, RS, diag, W, av, wv);
  }
  apply_staged<kMixThreads>(Yw, a, k, woff, s, W, fail, wv, reinterpret_cast<float2*>(smem),
                            out + pair * a.Lt);
  if (wout) {
    for (int i = tid; i < a.wmax; i += kMixThreads) {
      float2 v = make_float2(0.f, 0.f);
      if (!fail && i < W) v = make_float2((float)wv[i].x, (float)wv[i].y);
      wout[pair * a.wmax + i] = v;
    }
  }
  if (info && tid == 0) info[pair] = fail | (route ? kInfoRouted : 0);
}

hipError_t launch_mvdr_mixed(const PairArgs& a, const WindowGeom& g, const DevDesc& d,
                             const float2* Yw, float2* out, float2* wout, int* starts, int* info,
                             bool split, hipStream_t s) {
  if (a.wmax > 64) return hipErrorInvalidValue;
  MixLds lay = mix_lds_layout(a.wmax);
  const unsigned grid = (unsigned)(a.T * a.K);
  if (split) {
    hipError_t e = hipFuncSetAttribute((const void*)k_mvdr_mixed<true>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lay.total);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mvdr_mixed<true>, dim3(grid), dim3(kMixThreads), lay.total, s, a, g, d, Yw,
                       out, wout, starts, info);
  } else {
    hipError_t e = hipFuncSetAttribute((const void*)k_mvdr_mixed<false>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lay.total);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mvdr_mixed<false>, dim3(grid), dim3(kMixThreads), lay.total, s, a, g, d,
                       Yw, out, wout, starts, info);
  }
  return hipGetLastError();
}

}  // namespace wbm
