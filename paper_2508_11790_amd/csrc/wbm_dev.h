// Device helpers shared by the gfx950 kernels: complex arithmetic and a batched
// in-LDS Stockham FFT (radix 8 / 4 / 2) for the channelizer and the beamspace DFT.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wbm {

constexpr int kThreads = 256;         // workgroup size of the FFT kernels (4 wave64)
constexpr int kTile = 8192;           // complex values per FFT tile in LDS (64 KiB + padding)

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by -j
__device__ __forceinline__ float2 cmul_mj(float2 a) { return make_float2(a.y, -a.x); }

__device__ __forceinline__ double2 dadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 dsub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 dmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ __forceinline__ double2 dcmulc(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 dscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }

// ---------------------------------------------------------------------------------------------
// Small DFTs in registers, forward sign: X[k] = sum_r v[r] exp(-2 pi i r k / R).

__device__ __forceinline__ void dft2(float2* v) {
  float2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  float2 t0 = cadd(a0, a2), t1 = csub(a0, a2);
  float2 t2 = cadd(a1, a3), t3 = cmul_mj(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

__device__ __forceinline__ void dft4(float2* v) { dft4(v[0], v[1], v[2], v[3]); }

__device__ __forceinline__ void dft8(float2* v) {
  // even / odd split: E = DFT4(v0, v2, v4, v6), O = DFT4(v1, v3, v5, v7)
  float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4(e0, e1, e2, e3);
  dft4(o0, o1, o2, o3);
  const float r = 0.70710678118654752440f;
  // O[k] * exp(-2 pi i k / 8)
  float2 w1 = make_float2((o1.x + o1.y) * r, (o1.y - o1.x) * r);     // (1 - i)/sqrt2
  float2 w2 = cmul_mj(o2);                                            // -i
  float2 w3 = make_float2((o3.y - o3.x) * r, -(o3.x + o3.y) * r);     // (-1 - i)/sqrt2
  v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
  v[1] = cadd(e1, w1); v[5] = csub(e1, w1);
  v[2] = cadd(e2, w2); v[6] = csub(e2, w2);
  v[3] = cadd(e3, w3); v[7] = csub(e3, w3);
}

template <int R>
__device__ __forceinline__ void dftR(float2* v) {
  if constexpr (R == 2) dft2(v);
  else if constexpr (R == 4) dft4(v);
  else dft8(v);
}

// One Stockham autosort pass of radix R over `nrows` rows of length n = 2^logn held in LDS
// (row stride rs complex).  Butterfly j of a row reads v[r] = x[j + r n/R], multiplies by
// exp(-2 pi i r (j mod Ns) / (Ns R)) (table tw[q] = exp(-2 pi i q / n)), applies the R-point
// DFT and writes v[r] to (j div Ns) Ns R + (j mod Ns) + r Ns.  All reads complete (barrier)
// before any write, so the pass works in place.  Every thread owns up to PER butterflies.
template <int R, int THREADS, int TILE>
__device__ __forceinline__ void stockham_pass(float2* lds, int nrows, int logn, int rs, int logNs,
                                              const float2* __restrict__ tw) {
  constexpr int PER = (TILE / R + THREADS - 1) / THREADS;
  constexpr int LOGR = (R == 2) ? 1 : (R == 4 ? 2 : 3);
  const int n = 1 << logn;
  const int logq = logn - LOGR;              // log2(n / R)
  const int nbf = nrows << logq;             // butterflies in the tile
  const int Ns = 1 << logNs;
  float2 v[PER][R];
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int bf = threadIdx.x + p * THREADS;
    if (bf < nbf) {
      const int row = bf >> logq, j = bf & ((1 << logq) - 1);
      const float2* src = lds + row * rs + j;
#pragma unroll
      for (int r = 0; r < R; ++r) v[p][r] = src[r << logq];
    }
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int bf = threadIdx.x + p * THREADS;
    if (bf < nbf) {
      const int row = bf >> logq, j = bf & ((1 << logq) - 1);
      const int k = j & (Ns - 1);
      if (logNs > 0) {
        // twiddle index r * k * n / (Ns R)
        const int step = k << (logn - logNs - LOGR);
#pragma unroll
        for (int r = 1; r < R; ++r) v[p][r] = cmul(v[p][r], tw[(r * step) & (n - 1)]);
      }
      dftR<R>(v[p]);
      float2* dst = lds + row * rs + (((j >> logNs) << (logNs + LOGR)) | k);
#pragma unroll
      for (int r = 0; r < R; ++r) dst[r << logNs] = v[p][r];
    }
  }
  __syncthreads();
}

// Forward DFT of `nrows` rows of length 2^logn in LDS (row stride rs), natural order in and
// out, unnormalised.  Caller must __syncthreads() after filling the rows.
template <int THREADS, int TILE>
__device__ void fft_rows(float2* lds, int nrows, int logn, int rs, const float2* __restrict__ tw) {
  int logNs = 0;
  const int rem = logn % 3;
  if (rem == 1) { stockham_pass<2, THREADS, TILE>(lds, nrows, logn, rs, logNs, tw); logNs += 1; }
  if (rem == 2) { stockham_pass<4, THREADS, TILE>(lds, nrows, logn, rs, logNs, tw); logNs += 2; }
  while (logNs < logn) { stockham_pass<8, THREADS, TILE>(lds, nrows, logn, rs, logNs, tw); logNs += 3; }
}

}  // namespace wbm
