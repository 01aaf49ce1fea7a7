// Window placement / windowed steering, and the per-(target, subband) reduced-dimension MVDR
// kernels for gfx950: loaded W x W sample covariance (Eq. 11), its factorisation, the two
// triangular solves giving c = R^-1 a / (a^H R^-1 a) (Eq. 13 / Eq. 20) and the beam output
// c^H y on the test snapshots.
//
// Fused forms: one workgroup per pair runs everything, placing its window and evaluating its
// steering vector itself; the covariance accumulates exact FP32 x FP32 products in FP64 and the
// LDL^H factorisation and solves run in FP64 (window covariances next to strong interferers
// reach condition numbers ~1e6, where FP32 accumulation loses the weights).  Variants: four
// waves or one wave per pair on the vector units, four waves on the FP64 matrix cores.
// Plain form: the same steps as three FP32 launches with R and c in HBM, gathering the window
// rows from the full beamspace.
// Mixed form (end of file): BF16 matrix-core covariance, FP32 LDL^H, FP64 refinement.
#include <math.h>

#include "wbm_dev.h"
#include "wbm_launch.h"

#include <type_traits>

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

// Planar array: one thread per (t, k, i < wmax): window starts (s_z, s_x) of the pair and its
// windowed steering a~ = S D a, cell i = ix_w Wz + iz_w the product of the two axes' Dirichlet
// sums (D a of Eq. 6 factors over the Kronecker product); optionally the beam index of every
// window cell (the plain form's row table).
__global__ void k_steer_upa(UpaGeom g, int wmax, int* __restrict__ starts,
                            double2* __restrict__ abar, int* __restrict__ rows) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)g.T * g.K * wmax;
  if (idx >= total) return;
  const int i = (int)(idx % wmax);
  const int64_t pk = idx / wmax;
  const int k = (int)(pk % g.K), t = (int)(pk / g.K);
  double uz, ux;
  int sz, sx;
  upa_window_of(g, t, k, &uz, &sz, &ux, &sx);
  if (starts && i == 0) {
    starts[2 * pk] = sz;
    starts[2 * pk + 1] = sx;
  }
  double2 a = make_double2(0.0, 0.0);
  int m = 0;
  if (i < g.win[t]) {
    const int Wz = g.wz[t], ixw = i / Wz, izw = i - ixw * Wz;
    a = dmul(axis_steering(g.Nx, g.Mx, ux, sx + ixw), axis_steering(g.Nz, g.Mz, uz, sz + izw));
    m = ((sx + ixw) & (g.Mx - 1)) * g.Mz + ((sz + izw) & (g.Mz - 1));
  }
  abar[idx] = a;
  if (rows) rows[idx] = m;
}

hipError_t launch_steer_upa(const UpaGeom& g, int wmax, int* starts, double2* abar,
                            hipStream_t s, int* rows) {
  const int64_t total = (int64_t)g.T * g.K * wmax;
  const int bs = 256;
  hipLaunchKernelGGL(k_steer_upa, dim3((unsigned)((total + bs - 1) / bs)), dim3(bs), 0, s, g,
                     wmax, starts, abar, rows);
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

// Workgroup -> (target, subband) of the pair kernels over subbands k0 .. k0 + kc - 1: targets
// widest window first (d.torder), subbands fastest, so that workgroups, handed out in index
// order, start every costly pair before any cheaper one (longest-processing-time order over
// the whole grid; grouping the targets of a subband per XCD instead left the widest pairs of
// late subbands to the tail).
__device__ __forceinline__ void pair_of_block(const PairArgs& a, const DevDesc& d, int& t, int& k) {
  const int p = blockIdx.x;
  const int kc = a.kc > 0 ? a.kc : a.K;
  t = d.torder[p / kc];
  k = a.k0 + p % kc;
}

// Snapshot b of window row i of pair (t, k).  From the full beamspace the row is bin
// (s + i) mod M, or with a row table (a.rows, the planar windows) beam a.rows[s wmax + i],
// s then being the pair index.
template <bool WINDOWED>
__device__ __forceinline__ float2 load_y(const float2* __restrict__ src, const PairArgs& a, int k,
                                         int woff, int s, int i, int b) {
  if constexpr (WINDOWED) {
    const int TB = 1 << a.logTB;
    return src[(((int64_t)k * a.nbt + (b >> a.logTB)) * a.sumW + woff + i) * TB + (b & (TB - 1))];
  } else {
    const int m = a.rows ? a.rows[(int64_t)s * a.wmax + i] : ((s + i) & (a.M - 1));
    return src[((int64_t)k * a.M + m) * a.B + b];
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

bool mvdr_wave_supported(int wmax) { return wmax <= kWaveWMax; }

hipError_t launch_mvdr_mfma(const PairArgs& a, const WindowGeom& g, const DevDesc& d,
                            const float2* Yw, float2* out, float2* wout, int* starts, int* info,
                            hipStream_t s);
hipError_t launch_mvdr_vector(const PairArgs& a, const WindowGeom& g, const DevDesc& d,
                              const float2* Yw, float2* out, float2* wout, int* starts, int* info,
                              int threads, hipStream_t s);
hipError_t launch_mvdr_resident(const PairArgs& a, const WindowGeom& g, const DevDesc& d,
                                const float2* Yw, float2* out, float2* wout, int* starts,
                                int* info, hipStream_t s);

hipError_t launch_mvdr_fused(const PairArgs& a, const WindowGeom& g, const DevDesc& d,
                             const float2* Yw, float2* out, float2* wout, int* starts, int* info,
                             int threads, hipStream_t s) {
  if (a.ywl && threads != 256 && threads != 64) return hipErrorInvalidValue;
  if (threads == kPairMfma) return launch_mvdr_mfma(a, g, d, Yw, out, wout, starts, info, s);
  if (threads == kPairResident)
    return launch_mvdr_resident(a, g, d, Yw, out, wout, starts, info, s);
  if (threads == 256 || (threads == 64 && a.wmax <= kWaveWMax))
    return launch_mvdr_vector(a, g, d, Yw, out, wout, starts, info, threads, s);
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------------------------------------
// Fused pair kernels, second generation.  One workgroup of TH threads per (target, subband)
// pair, in chunks of CH training snapshots staged through LDS, the next chunk already
// in flight in registers (after the last training chunk, the first test chunk), each thread's
// chunk elements mapped once per pair:
//   - vector form (TH = 256: four waves per pair; TH = 64: one wave per pair, more pairs per
//     CU): the loaded covariance on the FP64 vector units, a thread owning a BS x BS block of
//     the lower triangle and an interleaved slice of the chunk's snapshots;
//   - matrix-core form (TH = 256): with Z = [Re Y; Im Y] (2W x L) the real Gram G = Z Z^T
//     carries the covariance, Re R_ij = G_ij + G_{W+i,W+j}, Im R_ij = G_{W+i,j} - G_{W+j,i};
//     G's lower 16 x 16 tiles accumulate on v_mfma_f64_16x16x4f64, the four waves splitting
//     tiles (TG groups) and snapshot steps (4 / TG slices, summed in slice order).
// Either way the FP32 snapshots' products are exact in FP64 and every sum is FP64; results
// are deterministic.  Then an LDL^H factorisation (one barrier per column), the solves of
// Eq. 13 / Eq. 20 in FP64 on one wave, and the beam outputs on the test snapshots.
typedef double f64x4_t __attribute__((ext_vector_type(4)));

constexpr int kXRSP = 64 + 4;   // float row stride of the matrix-core form's staged planes:
                                // an operand's 16 rows x 4 steps hit distinct banks

// Register budgets for windows up to WCAP bins and TH threads: Gram tiles per wave (matrix
// cores), staged elements per thread and chunk, covariance entries per thread (matrix cores).
template <int WCAP, int TH, int CHUNK>
struct XCap {
  static constexpr int CH = CHUNK;
  static constexpr int kMaxT = WCAP <= 40 ? 4 : 9;
  static constexpr int kPre = (WCAP * CH + TH - 1) / TH;
  static constexpr int kEnt = (WCAP * (WCAP + 1) / 2 + TH - 1) / TH;
};

struct XLds {
  size_t region, diag, wv, av, red, total;
  int RS;
};

// LDS of the pair kernels: one region reused by the staged chunks, the Gram tiles (matrix
// cores) and the complex R, then the pivots, weights, steering vector and the apply's partial
// sums.
template <bool MF, int TH, int CH>
__host__ __device__ inline XLds x_lds_layout(int wmax, bool ext = false) {
  constexpr int NG = TH / CH > 0 ? TH / CH : 1;   // row groups of the apply
  XLds p;
  p.RS = wmax + 1;
  const size_t r = sizeof(C2<double>) * (size_t)wmax * p.RS;          // complex R (lower)
  size_t big = r;
  if (MF) {
    const int pad = (2 * wmax + 15) / 16 * 16;
    const int nt = pad / 16;
    const size_t z = sizeof(float) * (size_t)pad * kXRSP;              // staged chunk planes
    const size_t gram = sizeof(double) * 256 * (size_t)(nt * (nt + 1) / 2);
    if (z > big) big = z;
    if (gram > big) big = gram;
  } else {
    // staged chunk rows: FP32 complex, or FP64 complex (hi + lo joined) in extended precision
    const size_t zf = (ext ? sizeof(double2) : sizeof(float2)) * (size_t)((wmax + 3) / 4 * 4) *
                      (CH + 1);
    if (zf > big) big = zf;
  }
  p.region = 0;
  p.diag = (big + 15) & ~(size_t)15;
  p.wv = p.diag + sizeof(double) * 64;
  p.av = p.wv + sizeof(C2<double>) * 64;
  p.red = p.av + sizeof(double2) * 64;
  p.total = p.red + sizeof(double2) * NG * CH;
  return p;
}

// Tile groups for ntiles lower tiles: the fewest MFMAs on the busiest wave, ties to more
// groups (fewer slices to sum), at most maxt tiles per wave.
__device__ __forceinline__ int mfma_tile_groups(int ntiles, int maxt) {
  int best = 4;
  float cost = 1e30f;
  for (int tg = 1; tg <= 4; tg <<= 1) {
    const int per = (ntiles + tg - 1) / tg;
    if (per > maxt) continue;
    const float c = (float)per * (float)tg * 0.25f;   // per / (4 / tg)
    if (c <= cost) {
      cost = c;
      best = tg;
    }
  }
  return best;
}

// Element e of a chunk of W rows x CH snapshots in source order -> (row, snapshot): snapshot
// runs when a window tile block holds at least CH snapshots, else one contiguous [W][TB] block
// after another.
template <int CH>
__device__ __forceinline__ void chunk_elem(const PairArgs& a, int W, int e, int& i, int& bb) {
  if ((1 << a.logTB) >= CH) {
    i = e / CH;
    bb = e - i * CH;
  } else {
    const int per = W << a.logTB;
    const int q = e / per, r = e - q * per;
    i = r >> a.logTB;
    bb = (q << a.logTB) + (r & ((1 << a.logTB) - 1));
  }
}

// Storage order of a pair's window rows in the window layout, relative to the first row of the
// window its target gathered: natural (row i at i), or, after the split-half spatial DFT
// (a.split_rows), the rows whose bin is even first in ascending order, then the odd ones --
// slot(i) = ((s + i) odd ? ne : 0) + i / 2 for row i of the gathered window (start s, ne
// even-bin rows).  so: offset of the pair's (sub-)window inside the gathered one.
struct RowOrder {
  int split = 0, so = 0, s = 0, ne = 0;
};
__device__ __forceinline__ int row_slot(const RowOrder& ro, int i) {
  if (!ro.split) return i;
  const int ii = i + ro.so;
  return (((ro.s + ii) & 1) ? ro.ne : 0) + (ii >> 1);
}

// This thread's elements of a chunk, packed as (row << 8) | snapshot, -1 past the end, and
// their offsets from the chunk's first element in the window layout (valid when chunks start
// at multiples of CH: then a chunk never splits a tile block differently).  The mapping is the
// same for every chunk.  Offsets count from the first row of the gathered window when rows
// are in split order (ro.split), else from the pair's own first row.
template <int PRE, int TH, int CH>
__device__ __forceinline__ void chunk_map(const PairArgs& a, int W, int* map, int* off,
                                          const RowOrder& ro = RowOrder()) {
  const int TB = 1 << a.logTB;
#pragma unroll
  for (int m = 0; m < PRE; ++m) {
    const int e = threadIdx.x + m * TH;
    map[m] = -1;
    off[m] = 0;
    if (e < W * CH) {
      int i, bb;
      chunk_elem<CH>(a, W, e, i, bb);
      map[m] = (i << 8) | bb;
      off[m] = ((bb >> a.logTB) * a.sumW + row_slot(ro, i)) * TB + (bb & (TB - 1));
    }
  }
}

// Snapshots c0 + (mapped snapshot) of the window rows (zero at b >= lim) into registers.  With
// aligned chunks (c0 a multiple of CH) one add per element; otherwise the full address.  EXT:
// also the BF16 remainders of the extended-precision windows (a.ywl, same layout) into prel.
template <int PRE, bool EXT = false>
__device__ __forceinline__ void fetch_chunk(const float2* __restrict__ Yw, const PairArgs& a,
                                            int k, int woff, const int* map, const int* off,
                                            bool aligned, int c0, int lim, float2* pre,
                                            uint32_t* prel = nullptr,
                                            const RowOrder& ro = RowOrder()) {
  const int TB = 1 << a.logTB;
  const int64_t ebase = (int64_t)k * a.nbt * a.sumW * TB + (int64_t)woff * TB;
  const float2* base = Yw + ebase;
  if (aligned) {
    // the chunk base is uniform; each element adds a 32-bit byte offset, kept opaque (empty
    // register constraint) so that the compiler does not hoist PRE 64-bit addresses out of
    // the chunk loops, where they would be spilled to scratch.  The 64-bin builds (PRE = 16)
    // derive each offset from an opaque copy of the element's packed position instead of
    // keeping PRE offsets live through the Gram: registers their Gram needs.
    constexpr bool kDerive = PRE >= 16;
    const int64_t cofs = (int64_t)(c0 >> a.logTB) * a.sumW * TB + (c0 & (TB - 1));
    const char* cb = reinterpret_cast<const char*>(base + cofs);
    const char* cl = EXT ? reinterpret_cast<const char*>(a.ywl + ebase + cofs) : nullptr;
    const int rem = lim - c0;
#pragma unroll
    for (int m = 0; m < PRE; ++m) {
      pre[m] = make_float2(0.f, 0.f);
      if constexpr (EXT) prel[m] = 0u;
      int mm = map[m];
      uint32_t o = 0;
      if constexpr (kDerive) {
        asm volatile("" : "+v"(mm));
        const int i = mm >> 8, bb = mm & 255;
        o = (uint32_t)(((bb >> a.logTB) * a.sumW + row_slot(ro, i)) * TB + (bb & (TB - 1))) << 3;
      } else {
        o = (uint32_t)off[m] << 3;
        asm volatile("" : "+v"(o));
      }
      if (mm >= 0 && (mm & 255) < rem) {
        pre[m] = *reinterpret_cast<const float2*>(cb + o);
        if constexpr (EXT) prel[m] = *reinterpret_cast<const uint32_t*>(cl + (o >> 1));
      }
    }
  } else {
#pragma unroll
    for (int m = 0; m < PRE; ++m) {
      pre[m] = make_float2(0.f, 0.f);
      int mm = map[m];
      asm volatile("" : "+v"(mm));   // as above: no hoisted per-element addresses
      const int i = mm >> 8, b = c0 + (mm & 255);
      if constexpr (EXT) prel[m] = 0u;
      if (mm >= 0 && b < lim) {
        const int64_t o =
            ((int64_t)(b >> a.logTB) * a.sumW + row_slot(ro, i)) * TB + (b & (TB - 1));
        pre[m] = base[o];
        if constexpr (EXT) prel[m] = a.ywl[ebase + o];
      }
    }
  }
}

// Registers -> LDS planes (matrix cores): real parts in rows i, imaginary parts in rows W + i.
template <int PRE>
__device__ __forceinline__ void store_planes(int W, const int* map, const float2* pre, float* z) {
#pragma unroll
  for (int m = 0; m < PRE; ++m) {
    if (map[m] >= 0) {
      const int o = (map[m] >> 8) * kXRSP + (map[m] & 255);
      z[o] = pre[m].x;
      z[o + W * kXRSP] = pre[m].y;
    }
  }
}

// Registers -> LDS complex rows, zf[i * RSF + snapshot]: FP32 complex, or with EXT the FP64
// complex hi + lo.
template <int PRE, int RSF, bool EXT = false>
__device__ __forceinline__ void store_rows(const int* map, const float2* pre, void* zf,
                                           const uint32_t* prel = nullptr) {
#pragma unroll
  for (int m = 0; m < PRE; ++m) {
    if (map[m] >= 0) {
      const int o = (map[m] >> 8) * RSF + (map[m] & 255);
      if constexpr (EXT)
        static_cast<double2*>(zf)[o] = ext_join(pre[m], prel[m]);
      else
        static_cast<float2*>(zf)[o] = pre[m];
    }
  }
}

// Staged snapshot element -> FP64 complex.
__device__ __forceinline__ double2 staged_c64(const float2* zf, int o) {
  const float2 v = zf[o];
  return make_double2((double)v.x, (double)v.y);
}
__device__ __forceinline__ double2 staged_c64(const double2* zf, int o) { return zf[o]; }

struct GramArgs {
  int W, woff, k, ntiles, TG, tg, kq, lane;
  bool aligned;
  RowOrder ro;
};

// Matrix-core Gram (TH = 256, CH = 64) into the tile-packed P[tile][16][16] (FP64): NT tiles
// per wave (tile tg + q TG; past ntiles a stand-in tile whose sum is dropped), snapshot steps
// split over KS = 4 / TG slices.  NT is a compile-time count so that no MFMA sits under a
// branch.
template <int NT, int PRE>
__device__ __forceinline__ void gram_mfma(const float2* __restrict__ Yw, const PairArgs& a,
                                          const GramArgs& ga, const int* map, const int* off,
                                          float2* pre, float* z, double* P) {
  constexpr int CH = 64;
  const int KS = 4 / ga.TG;
  int ra[NT], rb[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) {
    int tile = ga.tg + q * ga.TG, ti, tj;
    if (tile >= ga.ntiles) tile = 0;
    tri_index(tile, ti, tj);
    // lane's snapshots in a chunk: 16 consecutive ones from (lane >> 4) * 16, step s using
    // the s-th (A and B agree, so the sum over the chunk is the same)
    ra[q] = (ti * 16 + (ga.lane & 15)) * kXRSP + ((ga.lane >> 4) << 4);
    rb[q] = (tj * 16 + (ga.lane & 15)) * kXRSP + ((ga.lane >> 4) << 4);
  }
  f64x4_t acc[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) acc[q] = f64x4_t{0.0, 0.0, 0.0, 0.0};
  for (int c0 = 0; c0 < a.L; c0 += CH) {
    __syncthreads();   // previous chunk consumed
    store_planes<PRE>(ga.W, map, pre, z);
    __syncthreads();
    // the next training chunk, or after the last one the first test chunk: one call site,
    // so that the loads stay in flight through this chunk's Gram (two calls made the
    // compiler merge their results with copies that wait for the loads)
    if (c0 + CH < a.L || a.Lt > 0) {
      const bool more = c0 + CH < a.L;
      const int from = more ? c0 + CH : a.L, to = more ? a.L : a.L + a.Lt;
      fetch_chunk<PRE>(Yw, a, ga.k, ga.woff, map, off, ga.aligned, from, to, pre);
    }
    for (int sb = ga.kq; sb < CH / 16; sb += KS) {
      float4 A[NT], Bv[NT];
#pragma unroll
      for (int q = 0; q < NT; ++q) {
        A[q] = *reinterpret_cast<const float4*>(z + ra[q] + 4 * sb);
        Bv[q] = *reinterpret_cast<const float4*>(z + rb[q] + 4 * sb);
      }
#pragma unroll
      for (int q = 0; q < NT; ++q) {
        acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)A[q].x, (double)Bv[q].x, acc[q], 0, 0, 0);
        acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)A[q].y, (double)Bv[q].y, acc[q], 0, 0, 0);
        acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)A[q].z, (double)Bv[q].z, acc[q], 0, 0, 0);
        acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)A[q].w, (double)Bv[q].w, acc[q], 0, 0, 0);
      }
    }
  }
  for (int sl = 0; sl < KS; ++sl) {
    __syncthreads();
    if (ga.kq == sl) {
#pragma unroll
      for (int q = 0; q < NT; ++q) {
        const int tile = ga.tg + q * ga.TG;
        if (tile < ga.ntiles) {
          double* dst = P + (size_t)tile * 256 + ga.lane;
#pragma unroll
          for (int r = 0; r < 4; ++r) dst[r * 64] = (sl == 0 ? 0.0 : dst[r * 64]) + acc[q][r];
        }
      }
    }
  }
}

// Vector Gram: R_ij = (1/L) sum_b y_ib conj(y_jb) (+ delta on the diagonal), i >= j, into R
// (LDS, row stride RS).  A thread owns a BS x BS block of the lower triangle and a slice of S
// interleaved snapshots (S a power of two; the S slices of a block on consecutive lanes,
// summed by shuffles in a fixed order).  Requires nblk <= TH.
template <int BS, int PRE, int TH, int CH, bool EXT = false>
__device__ __forceinline__ void gram_vec(const float2* __restrict__ Yw, const PairArgs& a,
                                         const GramArgs& ga, const int* map, const int* off,
                                         float2* pre, void* zfv, C2<double>* R, int RS,
                                         double delta, uint32_t* prel = nullptr) {
  constexpr int RSF = CH + 1;
  using SV = typename std::conditional<EXT, double2, float2>::type;
  SV* zf = static_cast<SV*>(zfv);
  const int W = ga.W;
  const int nb = (W + BS - 1) / BS, nblk = nb * (nb + 1) / 2;
  int S = 1;
  while (2 * S * nblk <= TH && S < CH) S *= 2;
  const int tid = threadIdx.x;
  const int blk = tid / S, sg = tid & (S - 1);
  const bool act = blk < nblk;
  int bi = 0, bj = 0;
  if (act) tri_index(blk, bi, bj);
  const SV* yr0 = zf + bi * BS * RSF;
  const SV* yc0 = zf + bj * BS * RSF;
  double ax[BS][BS], ay[BS][BS];
#pragma unroll
  for (int u = 0; u < BS; ++u)
#pragma unroll
    for (int v = 0; v < BS; ++v) ax[u][v] = ay[u][v] = 0.0;
  for (int c0 = 0; c0 < a.L; c0 += CH) {
    __syncthreads();   // previous chunk consumed
    store_rows<PRE, RSF, EXT>(map, pre, zf, prel);
    __syncthreads();
    // the next training chunk, or after the last one the first test chunk: one call site,
    // so that the loads stay in flight through this chunk's Gram (two calls made the
    // compiler merge their results with copies that wait for the loads)
    if (c0 + CH < a.L || a.Lt > 0) {
      const bool more = c0 + CH < a.L;
      const int from = more ? c0 + CH : a.L, to = more ? a.L : a.L + a.Lt;
      fetch_chunk<PRE, EXT>(Yw, a, ga.k, ga.woff, map, off, ga.aligned, from, to, pre, prel, ga.ro);
    }
    if (act) {
      for (int bb = sg; bb < CH; bb += S) {
        double rx[BS], ry[BS], cx[BS], cy[BS];
#pragma unroll
        for (int u = 0; u < BS; ++u) {
          const double2 yr = staged_c64(yr0, u * RSF + bb), yc = staged_c64(yc0, u * RSF + bb);
          rx[u] = yr.x;
          ry[u] = yr.y;
          cx[u] = yc.x;
          cy[u] = yc.y;
        }
#pragma unroll
        for (int u = 0; u < BS; ++u)
#pragma unroll
          for (int v = 0; v < BS; ++v) {   // y_i conj(y_j), two FMAs per part
            ax[u][v] = fma(rx[u], cx[v], ax[u][v]);
            ax[u][v] = fma(ry[u], cy[v], ax[u][v]);
            ay[u][v] = fma(ry[u], cx[v], ay[u][v]);
            ay[u][v] = fma(-rx[u], cy[v], ay[u][v]);
          }
      }
    }
  }
#pragma unroll
  for (int u = 0; u < BS; ++u)
#pragma unroll
    for (int v = 0; v < BS; ++v)
      for (int off = S >> 1; off > 0; off >>= 1) {
        ax[u][v] += __shfl_xor(ax[u][v], off);
        ay[u][v] += __shfl_xor(ay[u][v], off);
      }
  __syncthreads();   // staging no longer read: R aliases it
  const double invL = 1.0 / (double)a.L;
  if (act && sg == 0) {
#pragma unroll
    for (int u = 0; u < BS; ++u)
#pragma unroll
      for (int v = 0; v < BS; ++v) {
        const int i = bi * BS + u, j = bj * BS + v;
        if (i < W && j <= i) {
          C2<double> r = c2<double>(ax[u][v] * invL, ay[u][v] * invL);
          if (i == j) {
            r.x += delta;
            r.y = 0.0;
          }
          R[i * RS + j] = r;
        }
      }
  }
  __syncthreads();
}

// Vector Gram for 61..64 bins (16 block rows of 4) on 256 threads.  Its 4 x 4 blocks of the
// lower triangle number 136, so gram_vec<4> gives each one thread and leaves 120 idle; here the
// 120 blocks below the diagonal take two snapshot slices each (threads 0..239, the slices on
// adjacent lanes, summed by one shuffle), and the 160 entries of the 16 diagonal blocks' lower
// triangles take one thread each over every snapshot (threads 0..159): about 36 instead of
// 64 FMA-instructions per snapshot and wave.  Same sums as gram_vec (FP64 accumulation of
// exact products), in another order.
template <int PRE, int TH, int CH, bool EXT = false>
__device__ __forceinline__ void gram_vec64(const float2* __restrict__ Yw, const PairArgs& a,
                                           const GramArgs& ga, const int* map,
                                           const int* off, float2* pre, void* zfv, C2<double>* R, int RS,
                                           double delta, uint32_t* prel = nullptr) {
  static_assert(TH == 256, "two slices of the 120 off-diagonal blocks fill 240 threads");
  constexpr int RSF = CH + 1, NB = 16, NOD = NB * (NB - 1) / 2;
  using SV = typename std::conditional<EXT, double2, float2>::type;
  SV* zf = static_cast<SV*>(zfv);
  const int W = ga.W;
  const int tid = threadIdx.x;
  // phase 1: block (bi, bj), bi > bj, snapshots sg, sg + 2, ...
  const int sg = tid & 1;
  const bool act1 = (tid >> 1) < NOD;
  int bi = 1, bj = 0;
  if (act1) {
    tri_index(tid >> 1, bi, bj);
    bi += 1;
  }
  // phase 2: entry (4 d + u, 4 d + v), u >= v, of diagonal block d
  const bool act2 = tid < NB * 10;
  int d = 0, u2 = 0, v2 = 0;
  if (act2) {
    d = tid / 10;
    tri_index(tid - 10 * d, u2, v2);
  }
  const int r2 = 4 * d + u2, c2r = 4 * d + v2;
  const SV* yr0 = zf + bi * 4 * RSF;
  const SV* yc0 = zf + bj * 4 * RSF;
  const SV* yd0 = zf + r2 * RSF;
  const SV* ye0 = zf + c2r * RSF;
  double ax[4][4], ay[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) ax[u][v] = ay[u][v] = 0.0;
  double px = 0.0, py = 0.0;
  for (int c0 = 0; c0 < a.L; c0 += CH) {
    __syncthreads();   // previous chunk consumed
    store_rows<PRE, RSF, EXT>(map, pre, zf, prel);
    __syncthreads();
    // the next training chunk, or after the last one the first test chunk: one call site,
    // so that the loads stay in flight through this chunk's Gram (two calls made the
    // compiler merge their results with copies that wait for the loads)
    if (c0 + CH < a.L || a.Lt > 0) {
      const bool more = c0 + CH < a.L;
      const int from = more ? c0 + CH : a.L, to = more ? a.L : a.L + a.Lt;
      fetch_chunk<PRE, EXT>(Yw, a, ga.k, ga.woff, map, off, ga.aligned, from, to, pre, prel, ga.ro);
    }
    if (act1) {
      for (int bb = sg; bb < CH; bb += 2) {
        double rx[4], ry[4], cx[4], cy[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const double2 yr = staged_c64(yr0, u * RSF + bb), yc = staged_c64(yc0, u * RSF + bb);
          rx[u] = yr.x;
          ry[u] = yr.y;
          cx[u] = yc.x;
          cy[u] = yc.y;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) {   // y_i conj(y_j), two FMAs per part
            ax[u][v] = fma(rx[u], cx[v], ax[u][v]);
            ax[u][v] = fma(ry[u], cy[v], ax[u][v]);
            ay[u][v] = fma(ry[u], cx[v], ay[u][v]);
            ay[u][v] = fma(-rx[u], cy[v], ay[u][v]);
          }
      }
    }
    if (act2) {
      for (int bb = 0; bb < CH; ++bb) {
        const double2 yr = staged_c64(yd0, bb), yc = staged_c64(ye0, bb);
        px = fma(yr.x, yc.x, px);
        px = fma(yr.y, yc.y, px);
        py = fma(yr.y, yc.x, py);
        py = fma(-yr.x, yc.y, py);
      }
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      ax[u][v] += __shfl_xor(ax[u][v], 1);
      ay[u][v] += __shfl_xor(ay[u][v], 1);
    }
  __syncthreads();   // staging no longer read: R aliases it
  const double invL = 1.0 / (double)a.L;
  if (act1 && sg == 0) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = bi * 4 + u, j = bj * 4 + v;   // j < i: below the diagonal blocks
        if (i < W) R[i * RS + j] = c2<double>(ax[u][v] * invL, ay[u][v] * invL);
      }
  }
  if (act2 && r2 < W) {
    C2<double> r = c2<double>(px * invL, py * invL);
    if (r2 == c2r) {
      r.x += delta;
      r.y = 0.0;
    }
    R[r2 * RS + c2r] = r;
  }
  __syncthreads();
}

// In-LDS LDL^H factorisation R = L D L^H (L unit lower) by TH threads on a G x G grid
// (G = 16 or 8), one barrier per column: column j keeps l_ij d_j below the diagonal, d_j on
// it.  Returns 0, or j + 1 when pivot d_j is not positive and finite (uniform).
template <int TH, typename T = double>
__device__ int ldl_lds(C2<T>* R, int RS, int W) {
  constexpr int G = TH >= 256 ? 16 : 8;
  const int tx = threadIdx.x % G, ty = threadIdx.x / G;
  for (int j = 0; j < W; ++j) {
    const T d = R[j * RS + j].x;
    if (!(d > (T)0) || !(d < (T)INFINITY)) return j + 1;
    const T inv = (T)1 / d;
    for (int i = j + 1 + ty; i < W; i += G) {
      const C2<T> gi = R[i * RS + j];
      const T lx = gi.x * inv, ly = gi.y * inv;         // l_ij
      for (int c = j + 1 + tx; c <= i; c += G) {
        const C2<T> gc = R[c * RS + j];                 // l_cj d_j
        C2<T> r = R[i * RS + c];
        r.x = fma(-lx, gc.x, fma(-ly, gc.y, r.x));      // - l_ij conj(l_cj) d_j
        r.y = fma(-ly, gc.x, fma(lx, gc.y, r.y));
        R[i * RS + c] = r;
      }
    }
    __syncthreads();
  }
  return 0;
}

// Wave 0: y = L^-1 a, q = a^H R^-1 a = sum |y_i|^2 / d_i, x = L^-H D^-1 y, w = x / q into wv[]
// (one lane per row, W <= 64).  Caller syncs afterwards.
__device__ void ldl_solve(const C2<double>* R, int RS, int W, const double2* av,
                          C2<double>* wv) {
  if (threadIdx.x >= 64) return;
  const int lane = threadIdx.x;
  const double invd = (lane < W) ? 1.0 / R[lane * RS + lane].x : 0.0;
  C2<double> y = c2<double>(0.0, 0.0);
  if (lane < W) y = c2<double>(av[lane].x, av[lane].y);
  for (int j = 0; j < W; ++j) {
    const double ivj = __shfl(invd, j);
    const double yx = __shfl(y.x, j) * ivj, yy = __shfl(y.y, j) * ivj;   // y_j / d_j
    if (lane > j && lane < W) {
      const C2<double> g = R[lane * RS + j];                              // l_ij d_j
      y.x -= g.x * yx - g.y * yy;
      y.y -= g.x * yy + g.y * yx;
    }
  }
  double q = (y.x * y.x + y.y * y.y) * invd;
  for (int off = 32; off > 0; off >>= 1) q += __shfl_xor(q, off);
  C2<double> x = c2<double>(y.x * invd, y.y * invd);
  for (int j = W - 1; j >= 0; --j) {
    const double xx = __shfl(x.x, j), xy = __shfl(x.y, j);               // x_j, final
    if (lane < j) {
      const C2<double> g = R[j * RS + lane];                              // l_ji d_i
      x.x -= (g.x * xx + g.y * xy) * invd;                                // conj(l_ji) x_j
      x.y -= (g.x * xy - g.y * xx) * invd;
    }
  }
  const double qinv = 1.0 / q;
  if (lane < W) wv[lane] = c2<double>(x.x * qinv, x.y * qinv);
}

__device__ __forceinline__ double readlane_f64(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// Wave 0, W <= WCAP: the same LDL^H factorisation and solves as ldl_lds + ldl_solve with the
// matrix in registers, no barriers.  Lane i holds row i of the full Hermitian matrix (the part
// above the diagonal as the conjugate of the lower part, updated alongside it); column j's
// entries l_cj d_j reach every lane as scalars (readlane of lane c).  The forward substitution
// y = L^-1 a runs with the elimination (column j is final at step j); the backward one,
// x = L^-H D^-1 y, reads conj(l_ci) d_i from lane i's own upper part.  The matrix is padded to
// WCAP with an identity block and zero steering, so every loop runs its compile-time count
// without branches; the padding adds and subtracts exact zeros to rows 0..W-1.  Writes
// w = x / q (q = a^H R^-1 a = sum |y_i|^2 / d_i) into wv[0..W); returns 0 or j + 1 for a pivot
// that is not positive and finite (uniform over the wave).  Caller syncs afterwards.
template <int WCAP>
__device__ __forceinline__ int ldl_reg_solve(const C2<double>* R, int RS, int W, const double2* av,
                                             C2<double>* wv) {
  const int lane = threadIdx.x & 63;
  C2<double> r[WCAP];
#pragma unroll
  for (int c = 0; c < WCAP; ++c) {
    r[c] = c2<double>(c == lane ? 1.0 : 0.0, 0.0);
    if (lane < W && c < W) {
      const bool lo = c <= lane;   // lower part: R[lane][c]; upper: conj(R[c][lane])
      const C2<double> u = R[lo ? lane * RS + c : c * RS + lane];
      r[c] = c2<double>(u.x, lo ? u.y : -u.y);
    }
  }
  C2<double> y = c2<double>(0.0, 0.0);
  if (lane < W) y = c2<double>(av[lane].x, av[lane].y);
  double invd = 0.0;   // 1 / d_lane
#pragma unroll
  for (int j = 0; j < WCAP; ++j) {
    const double dj = readlane_f64(r[j].x, j);
    if (!(dj > 0.0) || !(dj < (double)INFINITY)) return j + 1;
    const double inv = 1.0 / dj;
    if (lane == j) invd = inv;
    // l_ij on lanes i > j; zero on lanes i <= j, whose rows the updates below then leave as
    // they are (they subtract exact zeros)
    const bool below = lane > j;
    const double gjx = below ? r[j].x : 0.0, gjy = below ? r[j].y : 0.0;
    const double lx = gjx * inv, ly = gjy * inv;
    const double yx = readlane_f64(y.x, j) * inv, yy = readlane_f64(y.y, j) * inv;
    y.x -= gjx * yx - gjy * yy;
    y.y -= gjx * yy + gjy * yx;
#pragma unroll
    for (int c = j + 1; c < WCAP; ++c) {
      const double gx = readlane_f64(r[j].x, c), gy = readlane_f64(r[j].y, c);   // l_cj d_j
      r[c].x = fma(-lx, gx, fma(-ly, gy, r[c].x));   // - l_ij conj(l_cj) d_j
      r[c].y = fma(-ly, gx, fma(lx, gy, r[c].y));
    }
  }
  double q = (lane < W) ? (y.x * y.x + y.y * y.y) * invd : 0.0;
  for (int off = 32; off > 0; off >>= 1) q += __shfl_xor(q, off);
  C2<double> x = c2<double>(y.x * invd, y.y * invd);
#pragma unroll
  for (int c = WCAP - 1; c >= 0; --c) {
    const double xx = readlane_f64(x.x, c), xy = readlane_f64(x.y, c);   // x_c, final
    if (lane < c) {
      const C2<double> h = r[c];                                          // conj(l_ci) d_i
      x.x -= (h.x * xx - h.y * xy) * invd;
      x.y -= (h.x * xy + h.y * xx) * invd;
    }
  }
  const double qinv = 1.0 / q;
  if (lane < W) wv[lane] = c2<double>(x.x * qinv, x.y * qinv);
  return 0;
}

// ldl_reg_solve at the smallest of 4, 8, 12, 16 rows that holds W (W <= 16; uniform branch).
__device__ __forceinline__ int ldl_reg_solve_w(const C2<double>* R, int RS, int W,
                                               const double2* av, C2<double>* wv) {
  if (W <= 4) return ldl_reg_solve<4>(R, RS, W, av, wv);
  if (W <= 8) return ldl_reg_solve<8>(R, RS, W, av, wv);
  if (W <= 12) return ldl_reg_solve<12>(R, RS, W, av, wv);
  return ldl_reg_solve<16>(R, RS, W, av, wv);
}

// info bit of a pair whose per-pair width was rejected (the gathered window was solved)
constexpr int kInfoWidth = 1 << 29;

struct PairSetup {
  int t, k, W, woff, s;
  int wflag;        // kInfoWidth when the pair's per-pair width was rejected, else 0
  int64_t pair;
  double u, delta;
};

// The pair of this workgroup, its window (start, width, first row in the window layout; with a
// per-pair width, the centred sub-window of the gathered one: for widths of equal parity the
// start moves by half the difference) and its loading.
__device__ __forceinline__ PairSetup pair_setup(const PairArgs& a, const WindowGeom& g,
                                                const DevDesc& d) {
  PairSetup ps;
  pair_of_block(a, d, ps.t, ps.k);
  ps.W = d.win[ps.t];
  ps.woff = d.woff[ps.t];
  ps.pair = (int64_t)ps.t * a.K + ps.k;
  window_of(g, ps.t, ps.k, &ps.u, &ps.s);
  ps.wflag = 0;
  if (a.pw) {
    const int Wp = a.pw[ps.pair];
    if (Wp >= 1 && Wp <= ps.W && ((ps.W - Wp) & 1) == 0) {
      const int off = (ps.W - Wp) >> 1;
      ps.woff += off;
      ps.s += off;
      ps.W = Wp;
    } else {
      ps.wflag = kInfoWidth;
    }
  }
  ps.delta = a.pdelta ? (double)a.pdelta[ps.pair] : a.delta;
  return ps;
}

// Beam outputs on the test snapshots, CH at a time staged like the training chunks (pre holds
// the first test chunk on entry): thread (row group q = tid / CH, snapshot l = tid % CH) sums
// window rows i = q mod NG in FP64, then the NG partials are added in order.  Zero outputs
// when fail.
template <int PRE, int TH, int CH, bool PLANES, bool EXT = false>
__device__ __forceinline__ void apply_chunks(const float2* __restrict__ Yw, const PairArgs& a,
                                             int k, int woff, int W, const int* map,
                                             const int* off, bool aligned, float2* pre, float* z,
                                             void* zfv, const C2<double>* wv, double2* red,
                                             int fail, float2* __restrict__ o,
                                             uint32_t* prel = nullptr,
                                             const RowOrder& ro = RowOrder()) {
  constexpr int NG = TH / CH, RSF = CH + 1;
  using SV = typename std::conditional<EXT, double2, float2>::type;
  SV* zf = static_cast<SV*>(zfv);
  const int tid = threadIdx.x;
  const int rg = tid / CH, ls = tid % CH;
  const int nch = (a.Lt + CH - 1) / CH;
  for (int c = 0; c < nch; ++c) {
    __syncthreads();   // R / the previous chunk no longer read
    if constexpr (PLANES)
      store_planes<PRE>(W, map, pre, z);
    else
      store_rows<PRE, RSF, EXT>(map, pre, zf, prel);
    __syncthreads();
    if (c + 1 < nch)
      fetch_chunk<PRE, EXT>(Yw, a, k, woff, map, off, aligned, a.L + (c + 1) * CH, a.L + a.Lt,
                            pre, prel, ro);
    double zx = 0.0, zy = 0.0;
    if (!fail) {
      for (int i = rg; i < W; i += NG) {
        double yr, yi;
        if constexpr (PLANES) {
          yr = z[i * kXRSP + ls];
          yi = z[(W + i) * kXRSP + ls];
        } else {
          const double2 y = staged_c64(zf, i * RSF + ls);
          yr = y.x;
          yi = y.y;
        }
        const C2<double> w = wv[i];
        zx = fma(w.x, yr, fma(w.y, yi, zx));     // conj(w) y
        zy = fma(w.x, yi, fma(-w.y, yr, zy));
      }
    }
    red[rg * CH + ls] = make_double2(zx, zy);
    __syncthreads();
    const int l = c * CH + tid;
    if (tid < CH && l < a.Lt) {
      double2 acc = red[tid];
#pragma unroll
      for (int q = 1; q < NG; ++q) {
        acc.x += red[q * CH + tid].x;
        acc.y += red[q * CH + tid].y;
      }
      o[l] = make_float2((float)acc.x, (float)acc.y);
    }
  }
}

template <int WCAP, bool MF, int TH, int CHUNK, bool EXT = false>
__device__ __forceinline__ void mvdr_x_body(const PairArgs& a, const WindowGeom& g,
                                            const DevDesc& d, const float2* __restrict__ Yw,
                                            float2* __restrict__ out, float2* __restrict__ wout,
                                            int* __restrict__ starts_out, int* __restrict__ info) {
  using Cap = XCap<WCAP, TH, CHUNK>;
  constexpr int CH = Cap::CH, PRE = Cap::kPre, RSF = CH + 1;
  constexpr int NG = TH / CH;   // row groups of the apply
  static_assert(TH % CH == 0 && CH <= 256, "chunk: a divisor of the workgroup, at most 256");
  static_assert(!MF || CH == 64, "the matrix-core Gram steps through 64-snapshot chunks");
  static_assert(!(MF && EXT), "extended-precision windows use the vector Gram");
  extern __shared__ __align__(16) unsigned char smem[];
  const XLds lay = x_lds_layout<MF, TH, CH>(a.wmax, EXT);
  float* z = reinterpret_cast<float*>(smem + lay.region);
  float2* zf = reinterpret_cast<float2*>(smem + lay.region);
  double* P = reinterpret_cast<double*>(smem + lay.region);
  C2<double>* R = reinterpret_cast<C2<double>*>(smem + lay.region);
  C2<double>* wv = reinterpret_cast<C2<double>*>(smem + lay.wv);
  double2* av = reinterpret_cast<double2*>(smem + lay.av);
  double2* red = reinterpret_cast<double2*>(smem + lay.red);
  // the wave index is uniform per wave: readfirstlane lets the compiler branch on it with
  // scalar instructions
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const PairSetup ps = pair_setup(a, g, d);
  const int k = ps.k, W = ps.W;
  const int64_t pair = ps.pair;
  const double delta = ps.delta;
  if (a.route && !a.route[pair]) return;   // solved by the mixed-precision launch

  // rows in split order: address from the gathered window's first row (see row_slot)
  RowOrder ro;
  int woff = ps.woff;
  if (a.split_rows) {
    ro.split = 1;
    ro.so = ps.woff - d.woff[ps.t];
    ro.s = ps.s - ro.so;
    ro.ne = (d.win[ps.t] + ((ro.s & 1) ? 0 : 1)) >> 1;
    woff = ps.woff - ro.so;
  }
  int map[PRE], off[PRE];
  chunk_map<PRE, TH, CH>(a, W, map, off, ro);
  const bool aligned = (a.L % CH) == 0;
  float2 pre[PRE];
  uint32_t prel[EXT ? PRE : 1];
  fetch_chunk<PRE, EXT>(Yw, a, k, woff, map, off, aligned, 0, a.L, pre, prel, ro);
  for (int i = tid; i < W; i += TH)
    av[i] = a.abar ? a.abar[ps.pair * a.wmax + i] : window_steering(g, ps.u, ps.s, i);
  if (starts_out && tid == 0) starts_out[pair] = ps.s;

  if constexpr (!MF) {
    GramArgs ga{W, woff, k, 0, 0, 0, 0, lane, aligned, ro};
    if constexpr (TH >= 256) {
      // 2 x 2 blocks up to 44 bins (at most 253 blocks), 4 x 4 beyond
      if (WCAP <= 44 || W <= 44)
        gram_vec<2, PRE, TH, CH, EXT>(Yw, a, ga, map, off, pre, zf, R, lay.RS, delta, prel);
      else if constexpr (WCAP > 60) {
        // 16 block rows: gram_vec<4> would leave 120 of the 256 threads idle
        if (W > 60)
          gram_vec64<PRE, TH, CH, EXT>(Yw, a, ga, map, off, pre, zf, R, lay.RS, delta, prel);
        else
          gram_vec<4, PRE, TH, CH, EXT>(Yw, a, ga, map, off, pre, zf, R, lay.RS, delta, prel);
      } else if constexpr (WCAP > 44)
        gram_vec<4, PRE, TH, CH, EXT>(Yw, a, ga, map, off, pre, zf, R, lay.RS, delta, prel);
    } else {
      // one wave: 4 x 4 blocks (at most 55 blocks for 40 bins)
      gram_vec<4, PRE, TH, CH, EXT>(Yw, a, ga, map, off, pre, zf, R, lay.RS, delta, prel);
    }
  } else {
    static_assert(!MF || TH == 256, "the matrix-core form runs four waves");
    constexpr int kXMaxT = Cap::kMaxT, kXEnt = Cap::kEnt;
    const int rows = 2 * W;
    const int nt = (rows + 15) >> 4;
    const int ntiles = nt * (nt + 1) / 2;
    const int TG = mfma_tile_groups(ntiles, kXMaxT);
    const int NT = (ntiles + TG - 1) / TG;   // tiles per wave, the same on every wave
    // rows 2W .. 16 nt - 1 stay zero for the whole loop
    for (int e = tid; e < (nt * 16 - rows) * CH; e += TH)
      z[(rows + e / CH) * kXRSP + (e % CH)] = 0.f;
    GramArgs ga{W, woff, k, ntiles, TG, wave % TG, wave / TG, lane, aligned};
    switch (NT) {
#define WBM_GRAM_CASE(n) \
  case n:                \
    if constexpr (n <= kXMaxT) gram_mfma<n, PRE>(Yw, a, ga, map, off, pre, z, P); \
    break;
      WBM_GRAM_CASE(1) WBM_GRAM_CASE(2) WBM_GRAM_CASE(3) WBM_GRAM_CASE(4) WBM_GRAM_CASE(5)
      WBM_GRAM_CASE(6) WBM_GRAM_CASE(7) WBM_GRAM_CASE(8) WBM_GRAM_CASE(9)
#undef WBM_GRAM_CASE
    }
    __syncthreads();
    // complex R (lower), scaled and loaded; read into registers, then written over P
    const int nE = W * (W + 1) / 2;
    const double invL = 1.0 / (double)a.L;
    C2<double> rv[kXEnt];
    int ri[kXEnt], rj[kXEnt];
    auto gram = [&](int r, int c) -> double {
      const int ti = r >> 4, tj = c >> 4;
      return P[(size_t)(ti * (ti + 1) / 2 + tj) * 256 + (r & 15) * 16 + (c & 15)];
    };
#pragma unroll
    for (int q = 0; q < kXEnt; ++q) {
      const int e = tid + q * TH;
      ri[q] = -1;
      rj[q] = 0;
      rv[q] = c2<double>(0.0, 0.0);
      if (e < nE) {
        int i, j;
        tri_index(e, i, j);
        ri[q] = i;
        rj[q] = j;
        double re = (gram(i, j) + gram(W + i, W + j)) * invL;
        double im = (gram(W + i, j) - gram(W + j, i)) * invL;
        if (i == j) {
          re += delta;
          im = 0.0;
        }
        rv[q] = c2<double>(re, im);
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kXEnt; ++q)
      if (ri[q] >= 0) R[ri[q] * lay.RS + rj[q]] = rv[q];
    __syncthreads();
  }

  int fail;
  if constexpr (WCAP <= 16) {
    __shared__ int s_fail;
    if (tid < 64) {
      const int f = ldl_reg_solve_w(R, lay.RS, W, av, wv);
      if (tid == 0) s_fail = f;
    }
    __syncthreads();
    fail = s_fail;
  } else {
    fail = ldl_lds<TH>(R, lay.RS, W);
    if (!fail) ldl_solve(R, lay.RS, W, av, wv);
  }
  apply_chunks<PRE, TH, CH, MF, EXT>(Yw, a, k, woff, W, map, off, aligned, pre, z, zf, wv, red,
                                     fail, out + pair * a.Lt, prel, ro);
  if (wout) {
    for (int i = tid; i < a.wmax; i += TH) {
      float2 v = make_float2(0.f, 0.f);
      if (!fail && i < W) v = make_float2((float)wv[i].x, (float)wv[i].y);
      wout[pair * a.wmax + i] = v;
    }
  }
  if (info && tid == 0) info[pair] = fail | (a.route ? (1 << 30) : 0) | ps.wflag;
}

// Matrix-core form, vector form with four waves (held to 128 VGPRs up to 40 bins: four
// workgroups per CU; a 16-bin build keeps fewer staging registers) and vector form with one
// wave per pair (up to 40 bins).
template <int WCAP>
__global__ __launch_bounds__(256) void k_mvdr_xm(PairArgs a, WindowGeom g, DevDesc d,
                                                 const float2* __restrict__ Yw,
                                                 float2* __restrict__ out,
                                                 float2* __restrict__ wout,
                                                 int* __restrict__ starts_out,
                                                 int* __restrict__ info) {
  mvdr_x_body<WCAP, true, 256, 64>(a, g, d, Yw, out, wout, starts_out, info);
}

// EXT: the windows are the extended-precision hi + lo planes (a.ywl), staged as FP64.
template <bool EXT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_mvdr_xv16(
    PairArgs a, WindowGeom g, DevDesc d, const float2* __restrict__ Yw, float2* __restrict__ out,
    float2* __restrict__ wout, int* __restrict__ starts_out, int* __restrict__ info) {
  mvdr_x_body<16, false, 256, 64, EXT>(a, g, d, Yw, out, wout, starts_out, info);
}

template <bool EXT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_mvdr_xv40(
    PairArgs a, WindowGeom g, DevDesc d, const float2* __restrict__ Yw, float2* __restrict__ out,
    float2* __restrict__ wout, int* __restrict__ starts_out, int* __restrict__ info) {
  mvdr_x_body<40, false, 256, 64, EXT>(a, g, d, Yw, out, wout, starts_out, info);
}

// two waves per SIMD: the extended-precision build would otherwise take 256 VGPRs + 48 AGPRs
// (one wave per SIMD); held to 256 registers it spills some staging registers and runs 1.6x
// faster at 64-bin windows
template <bool EXT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_mvdr_xv64(
    PairArgs a, WindowGeom g, DevDesc d, const float2* __restrict__ Yw, float2* __restrict__ out,
    float2* __restrict__ wout, int* __restrict__ starts_out, int* __restrict__ info) {
  mvdr_x_body<64, false, 256, 64, EXT>(a, g, d, Yw, out, wout, starts_out, info);
}

template <bool EXT>
__global__ __launch_bounds__(64) void k_mvdr_xw40(
    PairArgs a, WindowGeom g, DevDesc d, const float2* __restrict__ Yw, float2* __restrict__ out,
    float2* __restrict__ wout, int* __restrict__ starts_out, int* __restrict__ info) {
  mvdr_x_body<40, false, 64, 16, EXT>(a, g, d, Yw, out, wout, starts_out, info);
}

hipError_t launch_mvdr_mfma(const PairArgs& a, const WindowGeom& g, const DevDesc& d,
                            const float2* Yw, float2* out, float2* wout, int* starts, int* info,
                            hipStream_t s) {
  if (a.wmax > 64) return hipErrorInvalidValue;
  const XLds lay = x_lds_layout<true, 256, 64>(a.wmax);
  const dim3 grid(a.T * (a.kc > 0 ? a.kc : a.K)), blk(256);
  if (a.wmax <= 40)
    hipLaunchKernelGGL(k_mvdr_xm<40>, grid, blk, lay.total, s, a, g, d, Yw, out, wout, starts, info);
  else
    hipLaunchKernelGGL(k_mvdr_xm<64>, grid, blk, lay.total, s, a, g, d, Yw, out, wout, starts, info);
  return hipGetLastError();
}

template <bool EXT>
static hipError_t vector_launch(const PairArgs& a, const WindowGeom& g, const DevDesc& d,
                                const float2* Yw, float2* out, float2* wout, int* starts,
                                int* info, int threads, hipStream_t s) {
  const dim3 grid(a.T * (a.kc > 0 ? a.kc : a.K));
  if (threads == 64) {
    const XLds lay = x_lds_layout<false, 64, 16>(a.wmax, EXT);
    hipLaunchKernelGGL(k_mvdr_xw40<EXT>, grid, dim3(64), lay.total, s, a, g, d, Yw, out, wout,
                       starts, info);
    return hipGetLastError();
  }
  const XLds lay = x_lds_layout<false, 256, 64>(a.wmax, EXT);
  if (a.wmax <= 16)
    hipLaunchKernelGGL(k_mvdr_xv16<EXT>, grid, dim3(256), lay.total, s, a, g, d, Yw, out, wout,
                       starts, info);
  else if (a.wmax <= 40)
    hipLaunchKernelGGL(k_mvdr_xv40<EXT>, grid, dim3(256), lay.total, s, a, g, d, Yw, out, wout,
                       starts, info);
  else
    hipLaunchKernelGGL(k_mvdr_xv64<EXT>, grid, dim3(256), lay.total, s, a, g, d, Yw, out, wout,
                       starts, info);
  return hipGetLastError();
}

hipError_t launch_mvdr_vector(const PairArgs& a, const WindowGeom& g, const DevDesc& d,
                              const float2* Yw, float2* out, float2* wout, int* starts, int* info,
                              int threads, hipStream_t s) {
  if (a.wmax > 64 || (threads == 64 && a.wmax > 40)) return hipErrorInvalidValue;
  if (a.ywl) return vector_launch<true>(a, g, d, Yw, out, wout, starts, info, threads, s);
  return vector_launch<false>(a, g, d, Yw, out, wout, starts, info, threads, s);
}

// ------------------------------------------------------------------------------------------
// Resident pair kernel: every window row of the pair sits in LDS once loaded; the covariance,
// LDL^H, solves and beam outputs run from LDS with no further global reads.  Same arithmetic as
// the vector kernel: FP32 x FP32 products exact in FP64, FP64 sums, FP64 factorisation and
// solves.
// Resident pair kernel (small problems: w_max L <= kResPart and w_max Lt <= kResPart): the
// training rows are loaded and staged first; the test rows' loads are issued with them and stay
// in flight in registers through the covariance and the factorisation, staged only for the
// beam outputs.
constexpr int kResPre = 9;                     // elements per thread of each part (256 threads)
constexpr int kResPart = kResPre * 256;
constexpr int kResRegW = 16;                   // widest window factorised in registers

struct ResLds {
  size_t y, r, wv, av, total;
  int RS, YS;
};

// window rows [wmax][B + 1] (float2), R [wmax][wmax + 1], w and steering [wmax] (FP64)
__host__ __device__ inline ResLds res_lds_layout(int wmax, int B) {
  ResLds p;
  p.RS = wmax + 1;
  p.YS = B + 1;
  p.y = 0;
  p.r = (sizeof(float2) * (size_t)wmax * p.YS + 15) & ~(size_t)15;
  p.wv = p.r + sizeof(C2<double>) * (size_t)wmax * p.RS;
  p.av = p.wv + sizeof(C2<double>) * (size_t)wmax;
  p.total = p.av + sizeof(double2) * (size_t)wmax;
  return p;
}

// LDS of at most 40 KiB: four workgroups per compute unit
bool mvdr_resident_supported(int wmax, int L, int Lt) {
  return wmax * L <= kResPart && wmax * Lt <= kResPart &&
         res_lds_layout(wmax, L + Lt).total <= 40 * 1024;
}

__global__ __launch_bounds__(256) void k_mvdr_res(PairArgs a, WindowGeom g, DevDesc d,
                                                  const float2* __restrict__ Yw,
                                                  float2* __restrict__ out,
                                                  float2* __restrict__ wout,
                                                  int* __restrict__ starts_out,
                                                  int* __restrict__ info) {
  constexpr int TH = 256, BS = 2;
  extern __shared__ __align__(16) unsigned char smem[];
  const ResLds lay = res_lds_layout(a.wmax, a.B);
  float2* ys = reinterpret_cast<float2*>(smem + lay.y);
  C2<double>* R = reinterpret_cast<C2<double>*>(smem + lay.r);
  C2<double>* wv = reinterpret_cast<C2<double>*>(smem + lay.wv);
  double2* av = reinterpret_cast<double2*>(smem + lay.av);
  const int tid = threadIdx.x;
  const PairSetup ps = pair_setup(a, g, d);
  const int k = ps.k, W = ps.W, woff = ps.woff;
  const int64_t pair = ps.pair;
  if (a.route && !a.route[pair]) return;
  const int YS = lay.YS, RS = lay.RS;

  // every element (row i, snapshot b) of the training part [W][L], then of the test part
  // [W][Lt], b fastest: runs of TB consecutive snapshots are contiguous in the tiled layout.
  // i = e / len through a float reciprocal: e + 1/2 lies at least 1/2 from a multiple of len
  // and e < 2^12, far beyond the reciprocal's rounding.
  const int TB = 1 << a.logTB;
  const float2* base = Yw + (int64_t)k * a.nbt * a.sumW * TB + (int64_t)woff * TB;
  const int ntr = W * a.L, nte = W * a.Lt;
  const float invL = 1.0f / (float)a.L, invLt = 1.0f / (float)max(a.Lt, 1);
  if (starts_out && tid == 0) starts_out[pair] = ps.s;
  // loads without branches (an index past the part reads its last element, dropped later), so
  // that each use waits only for its own load and the test loads stay in flight
  float2 vtr[kResPre], vte[kResPre];
#pragma unroll
  for (int m = 0; m < kResPre; ++m) {
    const int e = min(tid + m * TH, ntr - 1);
    const int i = (int)(((float)e + 0.5f) * invL), b = e - i * a.L;
    vtr[m] = base[((int64_t)(b >> a.logTB) * a.sumW + i) * TB + (b & (TB - 1))];
  }
  for (int i = tid; i < W; i += TH)
    av[i] = a.abar ? a.abar[ps.pair * a.wmax + i] : window_steering(g, ps.u, ps.s, i);
#pragma unroll
  for (int m = 0; m < kResPre; ++m) {
    const int e = tid + m * TH;
    if (e < ntr) {
      const int i = (int)(((float)e + 0.5f) * invL), b = e - i * a.L;
      ys[i * YS + b] = vtr[m];
    }
  }
  __syncthreads();

  // covariance over the L training snapshots: BS x BS blocks, S interleaved snapshot slices
  {
    const int nb = (W + BS - 1) / BS, nblk = nb * (nb + 1) / 2;
    int S = 1;
    while (2 * S * nblk <= TH && S < 64) S *= 2;
    const int blk = tid / S, sg = tid & (S - 1);
    const bool act = blk < nblk;
    int bi = 0, bj = 0;
    if (act) tri_index(blk, bi, bj);
    // rows past W (odd W) read row W - 1: their sums are dropped below
    int ri[BS], rc[BS];
#pragma unroll
    for (int u = 0; u < BS; ++u) {
      ri[u] = min(bi * BS + u, W - 1) * YS;
      rc[u] = min(bj * BS + u, W - 1) * YS;
    }
    double ax[BS][BS], ay[BS][BS];
#pragma unroll
    for (int u = 0; u < BS; ++u)
#pragma unroll
      for (int w = 0; w < BS; ++w) ax[u][w] = ay[u][w] = 0.0;
    if (act) {
#pragma unroll 4
      for (int b = sg; b < a.L; b += S) {
        double rx[BS], ry[BS], cx[BS], cy[BS];
#pragma unroll
        for (int u = 0; u < BS; ++u) {
          const float2 yr = ys[ri[u] + b], yc = ys[rc[u] + b];
          rx[u] = yr.x;
          ry[u] = yr.y;
          cx[u] = yc.x;
          cy[u] = yc.y;
        }
#pragma unroll
        for (int u = 0; u < BS; ++u)
#pragma unroll
          for (int w = 0; w < BS; ++w) {
            ax[u][w] = fma(rx[u], cx[w], ax[u][w]);
            ax[u][w] = fma(ry[u], cy[w], ax[u][w]);
            ay[u][w] = fma(ry[u], cx[w], ay[u][w]);
            ay[u][w] = fma(-rx[u], cy[w], ay[u][w]);
          }
      }
    }
#pragma unroll
    for (int u = 0; u < BS; ++u)
#pragma unroll
      for (int w = 0; w < BS; ++w)
        for (int off = S >> 1; off > 0; off >>= 1) {
          ax[u][w] += __shfl_xor(ax[u][w], off);
          ay[u][w] += __shfl_xor(ay[u][w], off);
        }
    const double invL = 1.0 / (double)a.L;
    if (act && sg == 0) {
#pragma unroll
      for (int u = 0; u < BS; ++u)
#pragma unroll
        for (int w = 0; w < BS; ++w) {
          const int i = bi * BS + u, j = bj * BS + w;
          if (i < W && j <= i) {
            C2<double> r = c2<double>(ax[u][w] * invL, ay[u][w] * invL);
            if (i == j) {
              r.x += ps.delta;
              r.y = 0.0;
            }
            R[i * RS + j] = r;
          }
        }
    }
  }
  __syncthreads();
  // test rows: issued once every workgroup's training rows are in (they compete with none of
  // them), in flight through the factorisation
#pragma unroll
  for (int m = 0; m < kResPre; ++m) {
    const int e = max(min(tid + m * TH, nte - 1), 0);
    const int i = (int)(((float)e + 0.5f) * invLt), b = a.L + e - i * a.Lt;
    const int bb = nte > 0 ? b : 0;
    vte[m] = base[((int64_t)(bb >> a.logTB) * a.sumW + i) * TB + (bb & (TB - 1))];
  }
  __shared__ int s_fail;
  int fail;
  if (a.wmax <= kResRegW) {
    if (tid < 64) {
      const int f = ldl_reg_solve_w(R, RS, W, av, wv);
      if (tid == 0) s_fail = f;
    }
    __syncthreads();
    fail = s_fail;
  } else {
    fail = ldl_lds<TH, double>(R, RS, W);
    if (!fail) ldl_solve(R, RS, W, av, wv);
    __syncthreads();
  }
  // test rows (loads in flight until now) into LDS
#pragma unroll
  for (int m = 0; m < kResPre; ++m) {
    const int e = tid + m * TH;
    if (e < nte) {
      const int i = (int)(((float)e + 0.5f) * invLt), b = a.L + e - i * a.Lt;
      ys[i * YS + b] = vte[m];
    }
  }
  __syncthreads();
  // beam outputs: one test snapshot per thread, FP64 sums over the window rows
  float2* o = out + pair * a.Lt;
  for (int l = tid; l < a.Lt; l += TH) {
    double zx = 0.0, zy = 0.0;
    if (!fail) {
      for (int i = 0; i < W; ++i) {
        const float2 y = ys[i * YS + a.L + l];
        const C2<double> w = wv[i];
        zx = fma(w.x, (double)y.x, fma(w.y, (double)y.y, zx));    // conj(w) y
        zy = fma(w.x, (double)y.y, fma(-w.y, (double)y.x, zy));
      }
    }
    o[l] = make_float2((float)zx, (float)zy);
  }
  if (wout) {
    for (int i = tid; i < a.wmax; i += TH) {
      float2 vv = make_float2(0.f, 0.f);
      if (!fail && i < W) vv = make_float2((float)wv[i].x, (float)wv[i].y);
      wout[pair * a.wmax + i] = vv;
    }
  }
  if (info && tid == 0) info[pair] = fail | (a.route ? (1 << 30) : 0) | ps.wflag;
}

hipError_t launch_mvdr_resident(const PairArgs& a, const WindowGeom& g, const DevDesc& d,
                                const float2* Yw, float2* out, float2* wout, int* starts,
                                int* info, hipStream_t s) {
  if (!mvdr_resident_supported(a.wmax, a.L, a.Lt)) return hipErrorInvalidValue;
  const ResLds lay = res_lds_layout(a.wmax, a.B);
  hipLaunchKernelGGL(k_mvdr_res, dim3(a.T * (a.kc > 0 ? a.kc : a.K)), dim3(256), lay.total, s, a,
                     g, d, Yw, out, wout, starts, info);
  return hipGetLastError();
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
  const int64_t pair = (int64_t)t * a.K + k;
  const int s = a.rows ? (int)pair : starts[t * a.K + k];
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
  const int64_t pair = (int64_t)t * a.K + k;
  const int s = a.rows ? (int)pair : starts[t * a.K + k];
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
  const dim3 grid(a.T * (a.kc > 0 ? a.kc : a.K)), blk(kPlainThreads);
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
  hipError_t e = hipFuncSetAttribute((const void*)k_mvdr_xm<64>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)x_lds_layout<true, 256, 64>(64).total);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_mvdr_xv64<false>,
                          hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)x_lds_layout<false, 256, 64>(64).total);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_mvdr_xv40<true>,
                          hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)x_lds_layout<false, 256, 64>(40, true).total);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_mvdr_xv64<true>,
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)x_lds_layout<false, 256, 64>(64, true).total);
}

}  // namespace wbm

// ==========================================================================================
// Mixed-precision form.  The W x W covariance is the one dense contraction of the path: with
// Z = [Re Y; Im Y] (2W x L real) the Gram G = Z Z^T gives Re R = G11 + G22 and
// Im R = G21 - G12.  G runs on MFMA (v_mfma_f32_32x32x16_bf16, FP32 accumulation) over 32 x 32
// tiles of the lower triangle, either with the BF16-rounded snapshots (one product per tile and
// step) or with each FP32 snapshot split into BF16 hi + lo parts (hi*hi + hi*lo + lo*hi, three
// products).  The LDL^H factorisation and both triangular solves run in FP32; the residual of
// the iterative-refinement step and the normalisation a^H R^-1 a run in FP64.  A window whose
// FP32 LDL^H pivots span more than a per-form ratio (max d_j / min d_j above kRouteKappaSplit or
// kRouteKappaBf16, a condition-number estimate) is routed to the exact path instead: a second
// launch runs the exact vector pair kernel on the flagged windows only (FP64 accumulation of the
// FP32 snapshots, FP64 LDL^H); their info entry carries bit 30.  Staging,
// prefetch, pair order and the apply are those of the fused pair kernels above.
namespace wbm {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

constexpr int kMixRS = 64 + 8;             // bf16 row stride of a staged plane (144 B)
// Routing thresholds.  One BF16 product rounds every snapshot to 8 significant bits, the split
// hi + lo products to about 16: the pivot ratio up to which the mixed solve stays within 0.1 dB
// of the FP64 oracle's output SINR is correspondingly smaller for the single product.  Measured
// on the batching and precision workloads (largest SINR loss of the windows kept on the mixed
// path, by the oracle covariance's pivot ratio): one BF16 product 0.036 / 0.065 / 0.21 dB below
// 10 / 100 / 1000, split products at most 0.032 dB below 1e4.
constexpr double kRouteKappaSplit = 1.0e4;
constexpr double kRouteKappaBf16 = 1.0e2;
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
  size_t region, r32, wv, av, red, total;
  int RS, pad;
};

// region: staged BF16 planes, then the tile-packed FP32 Gram; r32: the FP32 complex R and its
// LDL^H factor; the apply stages its chunks in region.
__host__ __device__ inline MixLds mix_lds_layout(int wmax, bool split) {
  MixLds p;
  p.RS = wmax + 1;
  p.pad = (2 * wmax + 31) / 32 * 32;
  const int nt = p.pad / 32;
  const size_t planes = sizeof(__bf16) * (size_t)p.pad * kMixRS * (split ? 2 : 1);
  const size_t gram = sizeof(float) * 1024 * (size_t)(nt * (nt + 1) / 2);
  size_t a = planes > gram ? planes : gram;
  a = (a + 15) & ~(size_t)15;
  const size_t r32 = sizeof(C2<float>) * (size_t)wmax * p.RS;
  size_t big = a + r32;
  const size_t zf = sizeof(float2) * (size_t)((wmax + 3) / 4 * 4) * 65;
  if (zf > big) big = zf;
  big = (big + 15) & ~(size_t)15;
  p.region = 0;
  p.r32 = a;
  p.wv = big;
  p.av = p.wv + sizeof(C2<double>) * 64;
  p.red = p.av + sizeof(double2) * 64;
  p.total = p.red + sizeof(double2) * 4 * 64;
  return p;
}

// Registers -> BF16 planes: hi (and lo = BF16(y - hi) when split) of the real parts in rows i,
// of the imaginary parts in rows W + i.
template <int PRE, bool SPLIT>
__device__ __forceinline__ void store_bf16(int W, int pad, const int* map, const float2* pre,
                                           __bf16* zh) {
  __bf16* zl = zh + pad * kMixRS;
#pragma unroll
  for (int m = 0; m < PRE; ++m) {
    if (map[m] >= 0) {
      const int o = (map[m] >> 8) * kMixRS + (map[m] & 255);
      const __bf16 hr = to_bf16(pre[m].x), hi = to_bf16(pre[m].y);
      zh[o] = hr;
      zh[o + W * kMixRS] = hi;
      if (SPLIT) {
        zl[o] = to_bf16(pre[m].x - from_bf16(hr));
        zl[o + W * kMixRS] = to_bf16(pre[m].y - from_bf16(hi));
      }
    }
  }
}

// BF16 Gram of the training snapshots into the tile-packed FP32 P[tile][32][32]: NT tiles per
// wave (tile tg + q TG; past ntiles a stand-in tile whose sum is dropped), the four 16-snapshot
// steps of a chunk split over KS = 4 / TG slices, summed in slice order.
template <int NT, int PRE, bool SPLIT>
__device__ __forceinline__ void gram_bf16(const float2* __restrict__ Yw, const PairArgs& a,
                                          const GramArgs& ga, int pad, const int* map,
                                          const int* off, float2* pre, __bf16* zh, float* P) {
  constexpr int CH = 64;
  const int KS = 4 / ga.TG;
  const __bf16* zl = zh + pad * kMixRS;
  int ra[NT], rb[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) {
    int tile = ga.tg + q * ga.TG, ti, tj;
    if (tile >= ga.ntiles) tile = 0;
    tri_index(tile, ti, tj);
    ra[q] = (ti * 32 + (ga.lane & 31)) * kMixRS + (ga.lane >> 5) * 8;
    rb[q] = (tj * 32 + (ga.lane & 31)) * kMixRS + (ga.lane >> 5) * 8;
  }
  f32x16_t acc[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) acc[q] = f32x16_t{};
  for (int c0 = 0; c0 < a.L; c0 += CH) {
    __syncthreads();   // previous chunk consumed
    store_bf16<PRE, SPLIT>(ga.W, pad, map, pre, zh);
    __syncthreads();
    // the next training chunk, or after the last one the first test chunk: one call site,
    // so that the loads stay in flight through this chunk's Gram (two calls made the
    // compiler merge their results with copies that wait for the loads)
    if (c0 + CH < a.L || a.Lt > 0) {
      const bool more = c0 + CH < a.L;
      const int from = more ? c0 + CH : a.L, to = more ? a.L : a.L + a.Lt;
      fetch_chunk<PRE>(Yw, a, ga.k, ga.woff, map, off, ga.aligned, from, to, pre);
    }
    for (int st = ga.kq; st < CH / 16; st += KS) {
#pragma unroll
      for (int q = 0; q < NT; ++q) {
        const bf16x8_t ah = *reinterpret_cast<const bf16x8_t*>(zh + ra[q] + st * 16);
        const bf16x8_t bh = *reinterpret_cast<const bf16x8_t*>(zh + rb[q] + st * 16);
        acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc[q], 0, 0, 0);
        if (SPLIT) {
          const bf16x8_t al = *reinterpret_cast<const bf16x8_t*>(zl + ra[q] + st * 16);
          const bf16x8_t bl = *reinterpret_cast<const bf16x8_t*>(zl + rb[q] + st * 16);
          acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc[q], 0, 0, 0);
          acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc[q], 0, 0, 0);
        }
      }
    }
  }
  // C layout of the 32 x 32 MFMA: column lane % 32, row 8 (r / 4) + 4 (lane / 32) + r % 4
  for (int sl = 0; sl < KS; ++sl) {
    __syncthreads();
    if (ga.kq == sl) {
#pragma unroll
      for (int q = 0; q < NT; ++q) {
        const int tile = ga.tg + q * ga.TG;
        if (tile < ga.ntiles) {
          float* dst = P + (size_t)tile * 1024 + (ga.lane & 31);
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int row = 8 * (r >> 2) + 4 * (ga.lane >> 5) + (r & 3);
            dst[row * 32] = (sl == 0 ? 0.f : dst[row * 32]) + acc[q][r];
          }
        }
      }
    }
  }
}

// Entry (r, c) of the tile-packed Gram, r >= c tile-wise.
__device__ __forceinline__ float gram32(const float* P, int r, int c) {
  const int ti = r >> 5, tj = c >> 5;
  return P[(size_t)(ti * (ti + 1) / 2 + tj) * 1024 + (r & 31) * 32 + (c & 31)];
}

template <int WCAP, bool SPLIT>
__device__ __forceinline__ void mvdr_mixed_body(const PairArgs& a, const WindowGeom& g,
                                                const DevDesc& d, const float2* __restrict__ Yw,
                                                float2* __restrict__ out,
                                                float2* __restrict__ wout,
                                                int* __restrict__ starts_out,
                                                int* __restrict__ info, int* __restrict__ flags) {
  constexpr int TH = 256, CH = 64;
  using Cap = XCap<WCAP, TH, CH>;
  constexpr int PRE = Cap::kPre;
  constexpr int kMaxT = WCAP <= 48 ? 2 : 3;   // 32 x 32 tiles per wave
  extern __shared__ __align__(16) unsigned char smem[];
  const MixLds lay = mix_lds_layout(a.wmax, SPLIT);
  __bf16* zh = reinterpret_cast<__bf16*>(smem + lay.region);
  float* P = reinterpret_cast<float*>(smem + lay.region);
  float2* zf = reinterpret_cast<float2*>(smem + lay.region);
  C2<float>* R32 = reinterpret_cast<C2<float>*>(smem + lay.r32);
  C2<double>* wv = reinterpret_cast<C2<double>*>(smem + lay.wv);
  double2* av = reinterpret_cast<double2*>(smem + lay.av);
  double2* red = reinterpret_cast<double2*>(smem + lay.red);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const PairSetup ps = pair_setup(a, g, d);
  const int k = ps.k, W = ps.W, woff = ps.woff;
  const int64_t pair = ps.pair;
  const double delta = ps.delta;
  const int RS = lay.RS, pad = lay.pad;

  int map[PRE], off[PRE];
  chunk_map<PRE, TH, CH>(a, W, map, off);
  const bool aligned = (a.L % CH) == 0;
  float2 pre[PRE];
  fetch_chunk<PRE>(Yw, a, k, woff, map, off, aligned, 0, a.L, pre);
  for (int i = tid; i < W; i += TH)
    av[i] = a.abar ? a.abar[ps.pair * a.wmax + i] : window_steering(g, ps.u, ps.s, i);
  if (starts_out && tid == 0) starts_out[pair] = ps.s;

  const int rows = 2 * W;
  const int nt = (rows + 31) >> 5;
  const int ntiles = nt * (nt + 1) / 2;
  const int TG = mfma_tile_groups(ntiles, kMaxT);
  const int NT = (ntiles + TG - 1) / TG;
  // plane rows 2W .. 32 nt - 1 stay zero for the whole loop
  for (int e = tid; e < (nt * 32 - rows) * kMixRS; e += TH) {
    zh[rows * kMixRS + e] = to_bf16(0.f);
    if (SPLIT) zh[(pad + rows) * kMixRS + e] = to_bf16(0.f);
  }
  GramArgs ga{W, woff, k, ntiles, TG, wave % TG, wave / TG, lane, aligned};
  if (NT == 1) gram_bf16<1, PRE, SPLIT>(Yw, a, ga, pad, map, off, pre, zh, P);
  else if (NT == 2) gram_bf16<2, PRE, SPLIT>(Yw, a, ga, pad, map, off, pre, zh, P);
  else if constexpr (kMaxT >= 3) gram_bf16<3, PRE, SPLIT>(Yw, a, ga, pad, map, off, pre, zh, P);
  __syncthreads();
  // FP32 complex R (lower) from the Gram, scaled and loaded
  const float invL = 1.0f / (float)a.L;
  for (int e = tid; e < W * W; e += TH) {
    const int i = e / W, j = e - i * W;
    if (j <= i) {
      float re = (gram32(P, i, j) + gram32(P, W + i, W + j)) * invL;
      float im = (gram32(P, W + i, j) - gram32(P, W + j, i)) * invL;
      if (i == j) {
        re += (float)delta;
        im = 0.f;
      }
      R32[i * RS + j] = c2<float>(re, im);
    }
  }
  __syncthreads();
  int fail = ldl_lds<TH, float>(R32, RS, W);
  // condition estimate from the pivots: max d / min d (d = LDL^H pivots, the squared
  // Cholesky ones)
  bool route = fail != 0;
  if (!fail) {
    float dmax = 0.f, dmin = 3.0e38f;
    for (int j = 0; j < W; ++j) {
      dmax = fmaxf(dmax, R32[j * RS + j].x);
      dmin = fminf(dmin, R32[j * RS + j].x);
    }
    route = (double)dmax > (SPLIT ? kRouteKappaSplit : kRouteKappaBf16) * (double)dmin;
  }
  __syncthreads();
  if (!route) {
    // wave 0: two refinement steps x += R^-1 (a - R x), the residual in FP64 with R the
    // MFMA-formed matrix read back from the Gram, the correction from the FP32 factor; then
    // q = a^H x in FP64 and w = x / q
    if (tid < 64) {
      const float invd = (lane < W) ? 1.0f / R32[lane * RS + lane].x : 0.f;
      C2<double> x = c2<double>(0.0, 0.0);
      C2<double> b = c2<double>(0.0, 0.0);
      if (lane < W) b = c2<double>(av[lane].x, av[lane].y);
      const double iL = 1.0 / (double)a.L;
      for (int it = 0; it < 2; ++it) {
        double rx = 0.0, ry = 0.0;
        for (int j = 0; j < W; ++j) {
          const double xjx = __shfl(x.x, j), xjy = __shfl(x.y, j);
          if (lane < W) {
            const int hi = lane >= j ? lane : j, lo = lane >= j ? j : lane;
            double re = ((double)gram32(P, hi, lo) + (double)gram32(P, W + hi, W + lo)) * iL;
            double im = ((double)gram32(P, W + hi, lo) - (double)gram32(P, W + lo, hi)) * iL;
            if (lane < j) im = -im;
            if (lane == j) {
              re += delta;
              im = 0.0;
            }
            rx += re * xjx - im * xjy;
            ry += re * xjy + im * xjx;
          }
        }
        C2<float> v = c2<float>(0.f, 0.f);
        if (lane < W) v = c2<float>((float)(b.x - rx), (float)(b.y - ry));
        // L y = v, y /= d, L^H z = y (FP32, unit L with l_ij = R32_ij / d_j)
        for (int j = 0; j < W; ++j) {
          const float ivj = __shfl(invd, j);
          const float yx = __shfl(v.x, j) * ivj, yy = __shfl(v.y, j) * ivj;
          if (lane > j && lane < W) {
            const C2<float> gg = R32[lane * RS + j];
            v.x -= gg.x * yx - gg.y * yy;
            v.y -= gg.x * yy + gg.y * yx;
          }
        }
        v.x *= invd;
        v.y *= invd;
        for (int j = W - 1; j >= 0; --j) {
          const float zx = __shfl(v.x, j), zy = __shfl(v.y, j);
          if (lane < j) {
            const C2<float> gg = R32[j * RS + lane];
            v.x -= (gg.x * zx + gg.y * zy) * invd;
            v.y -= (gg.x * zy - gg.y * zx) * invd;
          }
        }
        x.x += (double)v.x;
        x.y += (double)v.y;
      }
      double qq = (lane < W) ? b.x * x.x + b.y * x.y : 0.0;
      for (int o = 32; o > 0; o >>= 1) qq += __shfl_xor(qq, o);
      if (lane < W) wv[lane] = c2<double>(x.x / qq, x.y / qq);
    }
  } else {
    // the exact FP64 path solves this window in the second launch
    if (tid == 0) {
      flags[pair] = 1;
      if (info) info[pair] = kInfoRouted | ps.wflag;
    }
    return;
  }
  if (tid == 0) flags[pair] = 0;
  apply_chunks<PRE, TH, CH, false>(Yw, a, k, woff, W, map, off, aligned, pre, nullptr, zf, wv,
                                   red, fail, out + pair * a.Lt);
  if (wout) {
    for (int i = tid; i < a.wmax; i += TH) {
      float2 v = make_float2(0.f, 0.f);
      if (!fail && i < W) v = make_float2((float)wv[i].x, (float)wv[i].y);
      wout[pair * a.wmax + i] = v;
    }
  }
  if (info && tid == 0) info[pair] = fail | ps.wflag;
}

template <int WCAP, bool SPLIT>
__global__ __launch_bounds__(256) void k_mvdr_mx(PairArgs a, WindowGeom g, DevDesc d,
                                                 const float2* __restrict__ Yw,
                                                 float2* __restrict__ out,
                                                 float2* __restrict__ wout,
                                                 int* __restrict__ starts_out,
                                                 int* __restrict__ info, int* __restrict__ flags) {
  mvdr_mixed_body<WCAP, SPLIT>(a, g, d, Yw, out, wout, starts_out, info, flags);
}

template <int WCAP, bool SPLIT>
static hipError_t mixed_launch(const PairArgs& a, const WindowGeom& g, const DevDesc& d,
                               const float2* Yw, float2* out, float2* wout, int* starts,
                               int* info, int* flags, hipStream_t s) {
  const MixLds lay = mix_lds_layout(a.wmax, SPLIT);
  if (lay.total > 64 * 1024) {
    const hipError_t e = hipFuncSetAttribute((const void*)k_mvdr_mx<WCAP, SPLIT>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)lay.total);
    if (e != hipSuccess) return e;
  }
  const dim3 grid(a.T * (a.kc > 0 ? a.kc : a.K));
  hipLaunchKernelGGL((k_mvdr_mx<WCAP, SPLIT>), grid, dim3(256), lay.total, s, a, g, d, Yw, out,
                     wout, starts, info, flags);
  return hipGetLastError();
}

hipError_t launch_mvdr_mixed(const PairArgs& a, const WindowGeom& g, const DevDesc& d,
                             const float2* Yw, float2* out, float2* wout, int* starts, int* info,
                             int* flags, bool split, hipStream_t s) {
  if (a.wmax > 64 || !flags) return hipErrorInvalidValue;
  hipError_t e;
  if (a.wmax <= 40)
    e = split ? mixed_launch<40, true>(a, g, d, Yw, out, wout, starts, info, flags, s)
              : mixed_launch<40, false>(a, g, d, Yw, out, wout, starts, info, flags, s);
  else
    e = split ? mixed_launch<64, true>(a, g, d, Yw, out, wout, starts, info, flags, s)
              : mixed_launch<64, false>(a, g, d, Yw, out, wout, starts, info, flags, s);
  if (e != hipSuccess) return e;
  // second launch: the routed windows on the exact FP64 vector kernel
  PairArgs r = a;
  r.route = flags;
  return launch_mvdr_vector(r, g, d, Yw, out, wout, starts, info, 256, s);
}

}  // namespace wbm
