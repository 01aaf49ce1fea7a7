// Channelizer (time DFT per element and block) and beamspace (zero-padded spatial DFT per
// subband and snapshot) kernels for gfx950.  Both are HBM-bound: each workgroup stages one
// tile of rows in LDS, transforms it with the in-LDS Stockham FFT and writes it back in the
// layout the next stage reads contiguously.
#include "wbm_dev.h"
#include "wbm_launch.h"

namespace wbm {

// x [N][S] (S = B*K) -> X [K][B][N].  Workgroup = (element tile of TE = kTile/K rows, block b).
// Rows e >= N are zero-filled and not written.  Pre-twiddle h[tau] (half-bin centres) when
// hb != nullptr.  Output scaled by K^-1/2 (unitary DFT).
__global__ __launch_bounds__(kThreads) void k_channelize(const float2* __restrict__ x,
                                                         float2* __restrict__ X, int N, int logK,
                                                         int B, int64_t S, int logTE,
                                                         const float2* __restrict__ twK,
                                                         const float2* __restrict__ hb,
                                                         float scale) {
  extern __shared__ float2 lds[];
  const int K = 1 << logK, TE = 1 << logTE;
  const int rs = K + 1;
  const int e0 = blockIdx.x << logTE;
  const int b = blockIdx.y;
  const int total = TE << logK;
  for (int idx = threadIdx.x; idx < total; idx += kThreads) {
    const int e = idx >> logK, tau = idx & (K - 1);
    float2 v = make_float2(0.f, 0.f);
    if (e0 + e < N) {
      v = x[(int64_t)(e0 + e) * S + (int64_t)b * K + tau];
      if (hb) v = cmul(v, hb[tau]);
    }
    lds[e * rs + tau] = v;
  }
  __syncthreads();
  fft_rows<kThreads, kTile>(lds, TE, logK, rs, twK);
  for (int idx = threadIdx.x; idx < total; idx += kThreads) {
    const int k = idx >> logTE, e = idx & (TE - 1);
    if (e0 + e < N) X[((int64_t)k * B + b) * N + e0 + e] = cscale(lds[e * rs + k], scale);
  }
}

// X [K][B][N] -> beamspace of a tile of TB snapshots of subband k (zero padded to M), then
//   full  : Y [K][M][B]                                         (stage output), and/or
//   window: Yw [K][nbt][sumW][TB], row r = window row (t, i) of target t, bin (s_tk + i) mod M.
// Workgroup = (snapshot tile j, subband k).
__global__ __launch_bounds__(kThreads) void k_beamspace(const float2* __restrict__ X,
                                                        float2* __restrict__ Y,
                                                        float2* __restrict__ Yw, int N, int logM,
                                                        int B, int K, int logTB,
                                                        const float2* __restrict__ twM, float scale,
                                                        const int* __restrict__ rowtab, int sumW,
                                                        const int* __restrict__ starts) {
  extern __shared__ float2 lds[];
  const int M = 1 << logM, TB = 1 << logTB;
  const int rs = M + 1;
  const int j = blockIdx.x, k = blockIdx.y;
  const int b0 = j << logTB;
  const int total = TB << logM;
  for (int idx = threadIdx.x; idx < total; idx += kThreads) {
    const int b = idx >> logM, e = idx & (M - 1);
    float2 v = make_float2(0.f, 0.f);
    if (e < N && b0 + b < B) v = X[((int64_t)k * B + b0 + b) * N + e];
    lds[b * rs + e] = v;
  }
  __syncthreads();
  fft_rows<kThreads, kTile>(lds, TB, logM, rs, twM);
  if (Y) {
    for (int idx = threadIdx.x; idx < total; idx += kThreads) {
      const int m = idx >> logTB, b = idx & (TB - 1);
      if (b0 + b < B) Y[((int64_t)k * M + m) * B + b0 + b] = cscale(lds[b * rs + m], scale);
    }
  }
  if (Yw) {
    const int nbt = (B + TB - 1) >> logTB;
    float2* dst = Yw + ((int64_t)k * nbt + j) * sumW * TB;
    const int tot = sumW << logTB;
    for (int idx = threadIdx.x; idx < tot; idx += kThreads) {
      const int r = idx >> logTB, b = idx & (TB - 1);
      const int t = rowtab[r] >> 8, i = rowtab[r] & 255;
      const int m = (starts[t * K + k] + i) & (M - 1);
      dst[idx] = cscale(lds[b * rs + m], scale);
    }
  }
}

static int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

hipError_t launch_channelize(const float2* x, float2* X, int N, int K, int B, const float2* twK,
                             const float2* hb, hipStream_t s) {
  const int logK = ilog2(K);
  int logTE = ilog2(kTile) - logK;
  while (logTE > 0 && (1 << (logTE - 1)) >= N) --logTE;   // no wider than needed
  const int TE = 1 << logTE;
  dim3 grid((N + TE - 1) / TE, B);
  const size_t shm = sizeof(float2) * (size_t)TE * (K + 1);
  hipLaunchKernelGGL(k_channelize, grid, dim3(kThreads), shm, s, x, X, N, logK, B,
                     (int64_t)B * K, logTE, twK, hb, 1.0f / sqrtf((float)K));
  return hipGetLastError();
}

int beamspace_tile_log(int M, int B) {
  int logTB = ilog2(kTile) - ilog2(M);
  if (logTB > 6) logTB = 6;                                 // at most 64 snapshots per tile
  while (logTB > 0 && (1 << (logTB - 1)) >= B) --logTB;
  return logTB;
}

hipError_t launch_beamspace(const float2* X, float2* Y, float2* Yw, int N, int M, int B, int K,
                            const float2* twM, const int* rowtab, int sumW, const int* starts,
                            hipStream_t s) {
  const int logM = ilog2(M);
  const int logTB = beamspace_tile_log(M, B);
  const int TB = 1 << logTB;
  dim3 grid((B + TB - 1) / TB, K);
  const size_t shm = sizeof(float2) * (size_t)TB * (M + 1);
  hipLaunchKernelGGL(k_beamspace, grid, dim3(kThreads), shm, s, X, Y, Yw, N, logM, B, K, logTB,
                     twM, 1.0f / sqrtf((float)M), rowtab, sumW, starts);
  return hipGetLastError();
}

}  // namespace wbm

namespace wbm {
hipError_t set_fft_attributes() {
  hipError_t e = hipFuncSetAttribute((const void*)k_channelize,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, 80 * 1024);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_beamspace, hipFuncAttributeMaxDynamicSharedMemorySize,
                             80 * 1024);
}
}  // namespace wbm
