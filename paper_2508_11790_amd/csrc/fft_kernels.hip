// Channelizer (time DFT per element and block) and beamspace (zero-padded spatial DFT per
// subband and snapshot) kernels for gfx950.  Both are HBM-bound batched FFTs: the first pass
// reads its inputs straight from HBM into registers, the passes exchange through LDS (one
// 4096-complex tile per workgroup, eight values per thread), and the last pass's LDS image
// is written out in the layout the next stage reads contiguously.
#include "wbm_dev.h"
#include "wbm_launch.h"

namespace wbm {

constexpr int kLogTileMin = 12;   // 4096 complex per workgroup tile (n <= 4096)

__host__ __device__ constexpr int fft_logtile(int logn) {
  return logn > kLogTileMin ? logn : kLogTileMin;
}
__host__ __device__ constexpr int fft_threads(int logn) { return (1 << fft_logtile(logn)) / 8; }

// x [N][S] (S = B*K) -> X [K][B][N].  Workgroup = (TE = tile/K elements, block b).  Rows
// e >= N are zero-filled and not written.  Optional pre-twiddle hb[tau] (half-bin centres).
// Output scaled by K^-1/2 (unitary DFT).
template <int LOGK>
__global__ __launch_bounds__(fft_threads(LOGK)) void k_channelize(
    const float2* __restrict__ x, float2* __restrict__ X, int N, int B, int64_t S,
    const float2* __restrict__ twK, const float2* __restrict__ hb, float scale) {
  using F = Fft<LOGK, fft_logtile(LOGK)>;
  constexpr int K = F::n, TE = F::rows;
  constexpr int LOGTE = fft_logtile(LOGK) - LOGK;
  __shared__ float2 lds[F::lds_complex];
  const int e0 = blockIdx.x * TE;
  const int b = blockIdx.y;
  float2 v[8];
#pragma unroll
  for (int p = 0; p < 8 / F::R0; ++p) {
#pragma unroll
    for (int r = 0; r < F::R0; ++r) {
      int row, tau;
      F::first_input(p, r, row, tau);
      float2 val = make_float2(0.f, 0.f);
      if (e0 + row < N) {
        val = x[(int64_t)(e0 + row) * S + (int64_t)b * K + tau];
        if (hb) val = cmul(val, hb[tau]);
      }
      v[p * F::R0 + r] = val;
    }
  }
  F::run(v, lds, twK);
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int idx = threadIdx.x + q * F::threads;
    const int k = idx >> LOGTE, e = idx & (TE - 1);
    if (e0 + e < N) X[((int64_t)k * B + b) * N + e0 + e] = cscale(lds[F::addr(e, k)], scale);
  }
}

// X [K][B][N] -> beamspace of a tile of TB = tile/M snapshots of subband k (zero padded to M):
//   full  : Y [K][M][B]                                         (stage output), and/or
//   window: Yw [K][nbt][sumW][TB], row r = window row (t, i) of target t, bin (s_tk + i) mod M.
// Workgroup = (snapshot tile j, subband k).
template <int LOGM>
__global__ __launch_bounds__(fft_threads(LOGM)) void k_beamspace(
    const float2* __restrict__ X, float2* __restrict__ Y, float2* __restrict__ Yw, int N, int B,
    int K, const float2* __restrict__ twM, float scale, const int* __restrict__ rowtab, int sumW,
    const int* __restrict__ starts) {
  using F = Fft<LOGM, fft_logtile(LOGM)>;
  constexpr int M = F::n, TB = F::rows;
  constexpr int LOGTB = fft_logtile(LOGM) - LOGM;
  __shared__ float2 lds[F::lds_complex];
  const int j = blockIdx.x, k = blockIdx.y;
  const int b0 = j * TB;
  float2 v[8];
#pragma unroll
  for (int p = 0; p < 8 / F::R0; ++p) {
#pragma unroll
    for (int r = 0; r < F::R0; ++r) {
      int row, e;
      F::first_input(p, r, row, e);
      float2 val = make_float2(0.f, 0.f);
      if (e < N && b0 + row < B) val = X[((int64_t)k * B + b0 + row) * N + e];
      v[p * F::R0 + r] = val;
    }
  }
  F::run(v, lds, twM);
  if (Y) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int idx = threadIdx.x + q * F::threads;
      const int m = idx >> LOGTB, b = idx & (TB - 1);
      if (b0 + b < B) Y[((int64_t)k * M + m) * B + b0 + b] = cscale(lds[F::addr(b, m)], scale);
    }
  }
  if (Yw) {
    const int nbt = (B + TB - 1) / TB;
    float2* dst = Yw + ((int64_t)k * nbt + j) * sumW * TB;
    const int tot = sumW * TB;
    for (int idx = threadIdx.x; idx < tot; idx += F::threads) {
      const int r = idx >> LOGTB, b = idx & (TB - 1);
      const int t = rowtab[r] >> 8, i = rowtab[r] & 255;
      const int m = (starts[t * K + k] + i) & (M - 1);
      dst[idx] = cscale(lds[F::addr(b, m)], scale);
    }
  }
}

static int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

template <int LOGK>
static hipError_t chan_launch(const float2* x, float2* X, int N, int B, const float2* twK,
                              const float2* hb, hipStream_t s) {
  using F = Fft<LOGK, fft_logtile(LOGK)>;
  dim3 grid((N + F::rows - 1) / F::rows, B);
  hipLaunchKernelGGL(k_channelize<LOGK>, grid, dim3(F::threads), 0, s, x, X, N, B,
                     (int64_t)B * F::n, twK, hb, 1.0f / sqrtf((float)F::n));
  return hipGetLastError();
}

template <int LOGM>
static hipError_t beam_launch(const float2* X, float2* Y, float2* Yw, int N, int B, int K,
                              const float2* twM, const int* rowtab, int sumW, const int* starts,
                              hipStream_t s) {
  using F = Fft<LOGM, fft_logtile(LOGM)>;
  dim3 grid((B + F::rows - 1) / F::rows, K);
  hipLaunchKernelGGL(k_beamspace<LOGM>, grid, dim3(F::threads), 0, s, X, Y, Yw, N, B, K, twM,
                     1.0f / sqrtf((float)F::n), rowtab, sumW, starts);
  return hipGetLastError();
}

#define WBM_LOG_CASES(M) M(1) M(2) M(3) M(4) M(5) M(6) M(7) M(8) M(9) M(10) M(11) M(12) M(13)

hipError_t launch_channelize(const float2* x, float2* X, int N, int K, int B, const float2* twK,
                             const float2* hb, hipStream_t s) {
  switch (ilog2(K)) {
#define C(L) \
  case L:    \
    return chan_launch<L>(x, X, N, B, twK, hb, s);
    WBM_LOG_CASES(C)
#undef C
  }
  return hipErrorInvalidValue;
}

int beamspace_tile_log(int M, int /*B*/) { return fft_logtile(ilog2(M)) - ilog2(M); }

hipError_t launch_beamspace(const float2* X, float2* Y, float2* Yw, int N, int M, int B, int K,
                            const float2* twM, const int* rowtab, int sumW, const int* starts,
                            hipStream_t s) {
  switch (ilog2(M)) {
#define C(L) \
  case L:    \
    return beam_launch<L>(X, Y, Yw, N, B, K, twM, rowtab, sumW, starts, s);
    WBM_LOG_CASES(C)
#undef C
  }
  return hipErrorInvalidValue;
}

// The FFT kernels use static LDS only (at most 8192 * 9/8 + 8 complex = 72 KiB).
hipError_t set_fft_attributes() { return hipSuccess; }

}  // namespace wbm
