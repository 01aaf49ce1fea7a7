// Channelizer (time DFT per element and block) and beamspace (zero-padded spatial DFT per
// subband and snapshot) kernels for gfx950.  Both are HBM-bound batched FFTs: the first pass
// reads its inputs straight from HBM into registers, the passes exchange through LDS (one
// 4096-complex tile per workgroup, eight values per thread), and the last pass's LDS image
// is written out in the layout the next stage reads contiguously.
#include "wbm_dev.h"
#include "wbm_launch.h"

namespace wbm {

// A workgroup transforms one tile of 2^LOGTILE complex values (rows of n = 2^LOGN points),
// eight values per thread.  LOGTILE is chosen per shape by the plan's autotuner among
// kLogTiles (clamped to at least LOGN).
__host__ __device__ constexpr int fft_tile(int logn, int logtile) {
  return logtile > logn ? logtile : logn;
}
__host__ __device__ constexpr int fft_threads(int logn, int logtile) {
  return (1 << fft_tile(logn, logtile)) / 8;
}

// LDS row padding (complex slots) of a multi-row tile: fewest modelled bank-conflict cycles
// over every pass and the kernel's output gather (channelizer: lanes walk tile rows;
// beamspace: lanes walk snapshots, then window bins), for 32- and 64-bank LDS models.
__host__ __device__ constexpr int chan_pad(int logtile, int logn) {
  return logn <= 3 ? 1 : logn == 4 ? 2 : logn == 5 ? 3 : logn == 6 ? 13
       : logtile == 11 ? (logn == 7 ? 2 : logn == 8 ? 2 : logn == 9 ? 4 : logn == 10 ? 8 : 0)
       : logtile == 12 ? (logn == 7 ? 1 : logn == 8 ? 1 : logn == 9 ? 2 : logn == 10 ? 4 : logn == 11 ? 8 : 0)
       : (logn <= 9 ? 1 : logn == 10 ? 2 : logn == 11 ? 4 : logn == 12 ? 8 : 0);
}
__host__ __device__ constexpr int beam_pad(int logtile, int logn) {
  return logn <= 3 ? 1 : logn == 4 ? 2 : logn == 5 ? 3 : logn == 6 ? 13
       : logtile == 11 ? (logn == 7 ? 1 : logn == 8 ? 14 : logn == 9 ? 12 : logn == 10 ? 5 : 0)
       : logtile == 12 ? (logn == 7 ? 1 : logn == 8 ? 1 : logn == 9 ? 14 : logn == 10 ? 8 : logn == 11 ? 5 : 0)
       : (logn <= 9 ? 1 : logn == 10 ? 14 : logn == 11 ? 8 : logn == 12 ? 5 : 0);
}

// x [N][S] (S = B*K) -> X [K][B][N].  Workgroup = (TE = tile/K elements, blocks b =
// blockIdx.y, blockIdx.y + gridDim.y, ...).  Rows e >= N are zero-filled and not written.
// Optional pre-twiddle hb[tau] (half-bin centres).  Output scaled by K^-1/2 (unitary DFT).
// The next block's samples are fetched into registers while the current block is transformed.
template <int LOGK, int LOGT>
__global__ __launch_bounds__(fft_threads(LOGK, LOGT)) void k_channelize(
    const float2* __restrict__ x, float2* __restrict__ X, int N, int B, int64_t S,
    const float2* __restrict__ twK, const float2* __restrict__ hb, float scale) {
  using F = Fft<LOGK, fft_tile(LOGK, LOGT), chan_pad(fft_tile(LOGK, LOGT), LOGK)>;
  constexpr int K = F::n, TE = F::rows;
  constexpr int LOGTE = fft_tile(LOGK, LOGT) - LOGK;
  __shared__ float2 lds[F::lds_complex];
  const int e0 = blockIdx.x * TE;
  float2 tr[F::NPA][F::NTW];
  F::load_twiddles(tr, twK);
  // half-bin pre-twiddle: one table value per first-pass butterfly (its input r = 0), the
  // other inputs' values being that times exp(-i pi r / R0)
  float2 hv[8 / F::R0];
#pragma unroll
  for (int p = 0; p < 8 / F::R0; ++p) {
    int row, tau;
    F::first_input(p, 0, row, tau);
    hv[p] = hb ? hb[tau] : make_float2(1.f, 0.f);
  }
  auto fetch = [&](int b, float2 (&v)[8]) {
#pragma unroll
    for (int p = 0; p < 8 / F::R0; ++p) {
#pragma unroll
      for (int r = 0; r < F::R0; ++r) {
        int row, tau;
        F::first_input(p, r, row, tau);
        float2 val = make_float2(0.f, 0.f);
        if (e0 + row < N) val = x[(int64_t)(e0 + row) * S + (int64_t)b * K + tau];
        v[p * F::R0 + r] = val;
      }
    }
  };
  float2 nv[8];
  int b = blockIdx.y;
  if (b < B) fetch(b, nv);
  for (; b < B; b += gridDim.y) {
    float2 v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = nv[q];
    if (b + (int)gridDim.y < B) fetch(b + gridDim.y, nv);
    if (hb) {
#pragma unroll
      for (int p = 0; p < 8 / F::R0; ++p) {
#pragma unroll
        for (int r = 0; r < F::R0; ++r)
          v[p * F::R0 + r] = rot_pi8(cmul(v[p * F::R0 + r], hv[p]), r * (8 / F::R0));
      }
    }
    F::run(v, lds, tr);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int idx = threadIdx.x + q * F::threads;
      const int k = idx >> LOGTE, e = idx & (TE - 1);
      if (e0 + e < N) X[((int64_t)k * B + b) * N + e0 + e] = cscale(lds[F::addr(e, k)], scale);
    }
    __syncthreads();   // the next block's first pass overwrites lds
  }
}

// X [K][B][N] -> beamspace of tiles of TB = tile/M snapshots of subband k (zero padded to M):
//   full  : Y [K][M][B]                                         (stage output), and/or
//   window: Yw [K][nbt][sumW][TB], row r = window row (t, i) of target t, bin (s_tk + i) mod M,
//   prof  : per-target training power profile partials [K][gridDim.x][T][64]: sum over this
//           workgroup's training snapshots (b < L) of |Y|^2 at bins c_tk - 32 .. c_tk + 31
//           (mod M), c_tk = floor(u_tk + 1/2) the target's beam bin.
// Workgroup = (first snapshot tile, subband k); it loops over tiles j, j + gridDim.x, ...,
// fetching the next tile's inputs into registers while the current one is transformed.
// With windows or profiles the first threads place the targets of subband k (same FP64
// evaluation as the steering kernel) into LDS.
// ZH: N <= M / 2, so the upper half of every zero-padded row is zero; those inputs are neither
// loaded nor added.
template <int LOGM, int LOGT, bool ZH>
__global__ __launch_bounds__(fft_threads(LOGM, LOGT)) void k_beamspace(
    const float2* __restrict__ X, float2* __restrict__ Y, float2* __restrict__ Yw, int N, int B,
    int K, const float2* __restrict__ twM, float scale, const int* __restrict__ rowtab, int sumW,
    WindowGeom g, float* __restrict__ prof, int L, int k0) {
  using F = Fft<LOGM, fft_tile(LOGM, LOGT), beam_pad(fft_tile(LOGM, LOGT), LOGM)>;
  constexpr int M = F::n, TB = F::rows;
  constexpr int LOGTB = fft_tile(LOGM, LOGT) - LOGM;
  __shared__ float2 lds[F::lds_complex];
  extern __shared__ int s_dyn[];
  int* s_start = s_dyn;                                    // [T] window starts of subband k
  int* s_center = s_dyn + g.T;                             // [T] beam bins (profile centre)
  float* s_acc = reinterpret_cast<float*>(s_dyn + 2 * g.T);  // [T][64] profile sums (prof)
  int* s_bin = s_dyn + 2 * g.T + (prof ? 64 * g.T : 0);      // [sumW] bin of window row r (Yw)
  const int k = k0 + blockIdx.y;
  const int nbt = (B + TB - 1) / TB;
  float2 tr[F::NPA][F::NTW];
  F::load_twiddles(tr, twM);
  // This thread's first-pass inputs sit at the same place in every tile: element e of the
  // tile's snapshot row `row`, byte offset 8 (row N + e) from the tile's first snapshot.  A
  // tile of TB whole snapshots with every e < N (N = M/2 under ZH, else N = M) is read
  // without predicates from a uniform base.
  uint32_t foff[8];
  int frow[8];
  bool fok[8];
#pragma unroll
  for (int p = 0; p < 8 / F::R0; ++p) {
#pragma unroll
    for (int r = 0; r < F::R0; ++r) {
      int row, e;
      F::first_input(p, r, row, e);
      const int q = p * F::R0 + r;
      frow[q] = row;
      fok[q] = e < N;
      foff[q] = (uint32_t)(row * N + e) * 8u;
    }
  }
  const bool dense = N >= (ZH ? M / 2 : M);
  auto fetch = [&](int j, float2 (&v)[8]) {
    const int b0 = j * TB;
    const char* base = reinterpret_cast<const char*>(X + ((int64_t)k * B + b0) * N);
    if (dense && b0 + TB <= B) {
#pragma unroll
      for (int q = 0; q < 8; ++q)
        v[q] = (ZH && 2 * (q % F::R0) >= F::R0)
                   ? make_float2(0.f, 0.f)
                   : *reinterpret_cast<const float2*>(base + foff[q]);
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        float2 val = make_float2(0.f, 0.f);
        if (!(ZH && 2 * (q % F::R0) >= F::R0) && fok[q] && b0 + frow[q] < B)
          val = *reinterpret_cast<const float2*>(base + foff[q]);
        v[q] = val;
      }
    }
  };
  float2 nv[8];
  if ((int)blockIdx.x < nbt) fetch(blockIdx.x, nv);
  if (Yw || prof) {
    for (int t = threadIdx.x; t < g.T; t += F::threads) {
      double u;
      int s;
      window_of(g, t, k, &u, &s);
      s_start[t] = s;
      if (prof) s_center[t] = (int)floor(u + 0.5);
    }
    if (prof)
      for (int i = threadIdx.x; i < g.T * 64; i += F::threads) s_acc[i] = 0.f;
    if (Yw) {
      __syncthreads();
      for (int r = threadIdx.x; r < sumW; r += F::threads) {
        const int t = rowtab[r] >> 8, i = rowtab[r] & 255;
        s_bin[r] = (s_start[t] + i) & (M - 1);
      }
    }
  }
  for (int j = blockIdx.x; j < nbt; j += gridDim.x) {
    const int b0 = j * TB;
    float2 v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = nv[q];
    if (j + (int)gridDim.x < nbt) fetch(j + gridDim.x, nv);
    F::template run<ZH>(v, lds, tr);
    if (Y) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int idx = threadIdx.x + q * F::threads;
        const int m = idx >> LOGTB, b = idx & (TB - 1);
        if (b0 + b < B) Y[((int64_t)k * M + m) * B + b0 + b] = cscale(lds[F::addr(b, m)], scale);
      }
    }
    if (Yw) {
      float2* dst = Yw + ((int64_t)k * nbt + j) * sumW * TB;
      const int tot = sumW * TB;
      for (int idx = threadIdx.x; idx < tot; idx += F::threads) {
        const int r = idx >> LOGTB, b = idx & (TB - 1);
        dst[idx] = cscale(lds[F::addr(b, s_bin[r])], scale);
      }
    }
    if (prof && b0 < L) {
      const int nb = min(TB, L - b0);
      // each thread owns the same (t, bin) entries on every tile: no synchronisation needed
      for (int idx = threadIdx.x; idx < g.T * 64; idx += F::threads) {
        const int t = idx >> 6, jj = idx & 63;
        const int m = (s_center[t] - 32 + jj) & (M - 1);
        float acc = 0.f;
        for (int b = 0; b < nb; ++b) {
          const float2 y = cscale(lds[F::addr(b, m)], scale);
          acc += y.x * y.x + y.y * y.y;
        }
        s_acc[idx] += acc;
      }
    }
    __syncthreads();   // the next tile's first pass overwrites lds
  }
  if (prof) {
    float* dst = prof + ((int64_t)k * gridDim.x + blockIdx.x) * g.T * 64;
    for (int idx = threadIdx.x; idx < g.T * 64; idx += F::threads) dst[idx] = s_acc[idx];
  }
}

// ---------------------------------------------------------------------------------------------
// Extended-precision forms of the channelizer and the windowed spatial DFT.  Same transforms,
// tiles and data layouts as k_channelize / k_beamspace, with FP64 arithmetic (FP64 twiddle
// tables, FP32 inputs converted exactly) and every intermediate stored as hi (FP32) + lo
// (BF16 remainder, ext_split): X as Xh [K][B][N] float2 + Xl [K][B][N] uint32, the windows
// as Ywh [K][nbt][sumW][TB] float2 + Ywl (same layout) uint32.  Rounding in these stages then
// stays near 2^-33 of each value instead of the FP32 transforms' few 2^-24, which is what
// keeps the MVDR weights of scenes with strong interferers within the FP32 weight tolerance.

template <int LOGK, int LOGT>
__global__ __launch_bounds__(fft_threads(LOGK, LOGT)) void k_channelize_x(
    const float2* __restrict__ x, float2* __restrict__ Xh, uint32_t* __restrict__ Xl, int N,
    int B, int64_t S, const double2* __restrict__ twK, const double2* __restrict__ hb,
    double scale) {
  using F = Fft<LOGK, fft_tile(LOGK, LOGT), chan_pad(fft_tile(LOGK, LOGT), LOGK), double2>;
  constexpr int K = F::n, TE = F::rows;
  constexpr int LOGTE = fft_tile(LOGK, LOGT) - LOGK;
  extern __shared__ double2 lds_x[];
  double2* lds = lds_x;
  const int e0 = blockIdx.x * TE;
  auto fetch = [&](int b, float2 (&v)[8]) {
#pragma unroll
    for (int p = 0; p < 8 / F::R0; ++p) {
#pragma unroll
      for (int r = 0; r < F::R0; ++r) {
        int row, tau;
        F::first_input(p, r, row, tau);
        float2 val = make_float2(0.f, 0.f);
        if (e0 + row < N) val = x[(int64_t)(e0 + row) * S + (int64_t)b * K + tau];
        v[p * F::R0 + r] = val;
      }
    }
  };
  // the next block's samples are fetched into registers while the current block is
  // transformed (16 registers; the kernel stays within the 128 per thread that a 1024-thread
  // workgroup allows, so nothing spills)
  double2 tr[F::NPA][F::NTW];
  F::load_twiddles(tr, twK);
  float2 nv[8];
  int b = blockIdx.y;
  if (b < B) fetch(b, nv);
  for (; b < B; b += gridDim.y) {
    double2 v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = make_double2((double)nv[q].x, (double)nv[q].y);
    if (b + (int)gridDim.y < B) fetch(b + gridDim.y, nv);
    double2 hv[8 / F::R0];     // half-bin pre-twiddle, factored as in k_channelize
#pragma unroll
    for (int p = 0; p < 8 / F::R0; ++p) {
      int row, tau;
      F::first_input(p, 0, row, tau);
      hv[p] = hb ? hb[tau] : make_double2(1.0, 0.0);
    }
    if (hb) {
#pragma unroll
      for (int p = 0; p < 8 / F::R0; ++p) {
#pragma unroll
        for (int r = 0; r < F::R0; ++r)
          v[p * F::R0 + r] = rot_pi8(cmul(v[p * F::R0 + r], hv[p]), r * (8 / F::R0));
      }
    }
    F::run(v, lds, tr);
    // output offsets from an opaque copy of the thread index: hoisted out of the loop they
    // are 64-bit values the 128-register budget spills, and the reloads miss the cache
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int idx = tid + q * F::threads;
      const int k = idx >> LOGTE, e = idx & (TE - 1);
      if (e0 + e < N) {
        float2 hi;
        uint32_t lo;
        ext_split(cscale(lds[F::addr(e, k)], scale), hi, lo);
        const int64_t o = ((int64_t)k * B + b) * N + e0 + e;
        Xh[o] = hi;
        // a workgroup's remainders of one (subband, block) row are 4 TE bytes, half a cache
        // line when TE = 16: streamed past the cache (non-temporal) these partial-line writes
        // cost less than through it
        __builtin_nontemporal_store(lo, &Xl[o]);
      }
    }
    __syncthreads();   // the next block's first pass overwrites lds
  }
}

// Windowed spatial DFT in extended precision (windows and training power profiles as in
// k_beamspace; no full-beamspace output).
template <int LOGM, int LOGT, bool ZH>
__global__ __launch_bounds__(fft_threads(LOGM, LOGT)) void k_beamspace_x(
    const float2* __restrict__ Xh, const uint32_t* __restrict__ Xl, float2* __restrict__ Ywh,
    uint32_t* __restrict__ Ywl, int N, int B, int K, const double2* __restrict__ twM,
    double scale, const int* __restrict__ rowtab, int sumW, WindowGeom g, float* __restrict__ prof,
    int L, int k0) {
  using F = Fft<LOGM, fft_tile(LOGM, LOGT), beam_pad(fft_tile(LOGM, LOGT), LOGM), double2>;
  constexpr int M = F::n, TB = F::rows;
  constexpr int LOGTB = fft_tile(LOGM, LOGT) - LOGM;
  extern __shared__ double2 lds_x[];
  double2* lds = lds_x;
  int* s_dyn = reinterpret_cast<int*>(lds_x + F::lds_complex);
  int* s_start = s_dyn;                                    // [T] window starts of subband k
  int* s_center = s_dyn + g.T;                             // [T] beam bins (profile centre)
  float* s_acc = reinterpret_cast<float*>(s_dyn + 2 * g.T);  // [T][64] profile sums (prof)
  int* s_bin = s_dyn + 2 * g.T + (prof ? 64 * g.T : 0);      // [sumW] bin of window row r
  const int k = k0 + blockIdx.y;
  const int nbt = (B + TB - 1) / TB;
  double2 tr[F::NPA][F::NTW];
  F::load_twiddles(tr, twM);
  // first-pass inputs at the same element offset in every tile (see k_beamspace)
  uint32_t foff[8];
  int frow[8];
  bool fok[8];
#pragma unroll
  for (int p = 0; p < 8 / F::R0; ++p) {
#pragma unroll
    for (int r = 0; r < F::R0; ++r) {
      int row, e;
      F::first_input(p, r, row, e);
      const int q = p * F::R0 + r;
      frow[q] = row;
      fok[q] = e < N;
      foff[q] = (uint32_t)(row * N + e);
    }
  }
  const bool dense = N >= (ZH ? M / 2 : M);
  auto fetch = [&](int j, float2 (&vh)[8], uint32_t (&vl)[8]) {
    const int b0 = j * TB;
    const int64_t base = ((int64_t)k * B + b0) * N;
    const float2* bh = Xh + base;
    const uint32_t* bl = Xl + base;
    const bool full = dense && b0 + TB <= B;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      vh[q] = make_float2(0.f, 0.f);
      vl[q] = 0u;
      const bool zero_half = ZH && 2 * (q % F::R0) >= F::R0;
      if (!zero_half && (full || (fok[q] && b0 + frow[q] < B))) {
        vh[q] = bh[foff[q]];
        vl[q] = bl[foff[q]];
      }
    }
  };
  float2 nh[8];
  uint32_t nl[8];
  if ((int)blockIdx.x < nbt) fetch(blockIdx.x, nh, nl);
  if (Ywh || prof) {
    for (int t = threadIdx.x; t < g.T; t += F::threads) {
      double u;
      int s;
      window_of(g, t, k, &u, &s);
      s_start[t] = s;
      if (prof) s_center[t] = (int)floor(u + 0.5);
    }
    if (prof)
      for (int i = threadIdx.x; i < g.T * 64; i += F::threads) s_acc[i] = 0.f;
    if (Ywh) {
      __syncthreads();
      for (int r = threadIdx.x; r < sumW; r += F::threads) {
        const int t = rowtab[r] >> 8, i = rowtab[r] & 255;
        s_bin[r] = (s_start[t] + i) & (M - 1);
      }
    }
  }
  for (int j = blockIdx.x; j < nbt; j += gridDim.x) {
    const int b0 = j * TB;
    double2 v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = ext_join(nh[q], nl[q]);
    if (j + (int)gridDim.x < nbt) fetch(j + gridDim.x, nh, nl);
    F::template run<ZH>(v, lds, tr);
    if (Ywh) {
      const int64_t o0 = ((int64_t)k * nbt + j) * sumW * TB;
      const int tot = sumW * TB;
      for (int idx = threadIdx.x; idx < tot; idx += F::threads) {
        const int r = idx >> LOGTB, b = idx & (TB - 1);
        float2 hi;
        uint32_t lo;
        ext_split(cscale(lds[F::addr(b, s_bin[r])], scale), hi, lo);
        Ywh[o0 + idx] = hi;
        Ywl[o0 + idx] = lo;
      }
    }
    if (prof && b0 < L) {
      const int nb = min(TB, L - b0);
      for (int idx = threadIdx.x; idx < g.T * 64; idx += F::threads) {
        const int t = idx >> 6, jj = idx & 63;
        const int m = (s_center[t] - 32 + jj) & (M - 1);
        float acc = 0.f;
        for (int b = 0; b < nb; ++b) {
          const double2 y = cscale(lds[F::addr(b, m)], scale);
          acc += (float)(y.x * y.x + y.y * y.y);
        }
        s_acc[idx] += acc;
      }
    }
    __syncthreads();   // the next tile's first pass overwrites lds
  }
  if (prof) {
    float* dst = prof + ((int64_t)k * gridDim.x + blockIdx.x) * g.T * 64;
    for (int idx = threadIdx.x; idx < g.T * 64; idx += F::threads) dst[idx] = s_acc[idx];
  }
}

// Fourth word of a raw (untyped, stride 0) buffer descriptor on gfx9-family chips: 32-bit data
// format; the record count is then in bytes and a load past it returns zero.
constexpr int kRawBufferFlags = 0x00020000;

// Half-bin index field of a window-row list entry of the split-half kernels (M <= 8192).
constexpr int kHalfBinBits = 12;

// Window rows of subband k for the split-half kernels, as two lists in LDS: lst[0, ne) holds
// the even-bin rows and lst[ne, sumW) the odd-bin rows, each entry (row << kHalfBinBits) |
// (bin / 2), where row is the window row in split order (each window's even-bin rows first,
// then its odd-bin ones) and ne = ebase[T] the number of even-bin rows; ebase[t] counts the
// even-bin rows of the windows before t (rowtab lists the windows in target order).  Each half
// transform then stores its own rows with every lane active.  Requires s_start filled and
// visible; ends with lst and ebase written but not yet synchronised.
template <int M>
__device__ void split_row_lists(const WindowGeom& g, const int* s_start,
                                const int* __restrict__ rowtab, int sumW, int* lst, int* ebase,
                                int nthreads) {
  static_assert(M / 2 <= (1 << kHalfBinBits), "half-bin field too narrow");
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int t = 0; t < g.T; ++t) {
      ebase[t] = acc;
      acc += (g.win[t] + ((s_start[t] & 1) ? 0 : 1)) >> 1;
    }
    ebase[g.T] = acc;
  }
  __syncthreads();
  const int ne_all = ebase[g.T];
  for (int r = threadIdx.x; r < sumW; r += nthreads) {
    const int t = rowtab[r] >> 8, i = rowtab[r] & 255;
    const int st = s_start[t], m = (st + i) & (M - 1), base = r - i;
    const int ne = (g.win[t] + ((st & 1) ? 0 : 1)) >> 1;
    const int row = base + ((m & 1) ? ne : 0) + (i >> 1);
    const int at = (m & 1) ? ne_all + (base - ebase[t]) + (i >> 1) : ebase[t] + (i >> 1);
    lst[at] = (row << kHalfBinBits) | (m >> 1);
  }
}

// Windowed spatial DFT in extended precision for M >= 8192 with N <= M / 2 (the upper half of
// every zero-padded row is zero).  The M-point transform of such a row splits into two
// H = M/2-point transforms, Y[2 m'] = sum_{e<N} X[e] w_H^(m' e) and Y[2 m' + 1] = sum_{e<N}
// (X[e] w_M^e) w_H^(m' e), computed one after the other in a 64 KiB FP64 tile (one snapshot per
// iteration, 512 threads at H = 4096): the even bins' window rows are written after the first,
// the odd bins' after the second.  The full M-point row would need a 128 KiB tile and 1024
// threads, one workgroup per compute unit.  Outputs as k_beamspace_x with one snapshot per tile
// (TB = 1), except that each window's rows are stored in split order: its even-bin rows first,
// then the odd ones (each half then writes whole runs of rows).
template <int LOGH>
__global__ __launch_bounds__(fft_threads(LOGH, LOGH)) void k_beamspace_x2(
    const float2* __restrict__ Xh, const uint32_t* __restrict__ Xl, float2* __restrict__ Ywh,
    uint32_t* __restrict__ Ywl, int N, int B, int K, const double2* __restrict__ twM,
    double scale, const int* __restrict__ rowtab, int sumW, WindowGeom g, float* __restrict__ prof,
    int L, int k0) {
  using F = Fft<LOGH, LOGH, beam_pad(LOGH, LOGH), double2>;
  constexpr int H = F::n, M = 2 * H;
  extern __shared__ double2 lds_x[];
  double2* lds = lds_x;
  int* s_dyn = reinterpret_cast<int*>(lds_x + F::lds_complex);
  int* s_start = s_dyn;
  int* s_center = s_dyn + g.T;
  float* s_acc = reinterpret_cast<float*>(s_dyn + 2 * g.T);
  int* s_bin = s_dyn + 2 * g.T + (prof ? 64 * g.T : 0);
  int* s_ebase = s_bin + sumW;
  const int k = k0 + blockIdx.y;
  double2 tr[F::NPA][F::NTW];
  F::load_twiddles(tr, twM, 2);   // the H-point twiddles: every second entry of the M table
  int fpos[8];
#pragma unroll
  for (int p = 0; p < 8 / F::R0; ++p) {
#pragma unroll
    for (int r = 0; r < F::R0; ++r) {
      int row, e;
      F::first_input(p, r, row, e);
      fpos[p * F::R0 + r] = e;
    }
  }
  auto fetch = [&](int b, float2 (&vh)[8], uint32_t (&vl)[8]) {
    const int64_t base = ((int64_t)k * B + b) * N;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      vh[q] = make_float2(0.f, 0.f);
      vl[q] = 0u;
      if (fpos[q] < N) {
        vh[q] = Xh[base + fpos[q]];
        vl[q] = Xl[base + fpos[q]];
      }
    }
  };
  float2 nh[8];
  uint32_t nl[8];
  if ((int)blockIdx.x < B) fetch(blockIdx.x, nh, nl);
  if (Ywh || prof) {
    for (int t = threadIdx.x; t < g.T; t += F::threads) {
      double u;
      int s;
      window_of(g, t, k, &u, &s);
      s_start[t] = s;
      if (prof) s_center[t] = (int)floor(u + 0.5);
    }
    if (prof)
      for (int i = threadIdx.x; i < g.T * 64; i += F::threads) s_acc[i] = 0.f;
    if (Ywh) {
      __syncthreads();
      split_row_lists<M>(g, s_start, rowtab, sumW, s_bin, s_ebase, F::threads);
    }
  }
  for (int b = blockIdx.x; b < B; b += gridDim.x) {
    float2 ch[8];
    uint32_t cl[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      ch[q] = nh[q];
      cl[q] = nl[q];
    }
    if (b + (int)gridDim.x < B) fetch(b + gridDim.x, nh, nl);
    const int64_t o0 = ((int64_t)k * B + b) * sumW;
#pragma unroll 1
    for (int par = 0; par < 2; ++par) {
      double2 v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        v[q] = ext_join(ch[q], cl[q]);
        if (par) v[q] = cmul(v[q], twM[fpos[q]]);   // X[e] w_M^e for the odd bins
      }
      F::template run<false>(v, lds, tr);
      if (Ywh) {
        const int ne = s_ebase[g.T], cnt = par ? sumW - ne : ne;
        const int* lst = s_bin + (par ? ne : 0);
        for (int q = threadIdx.x; q < cnt; q += F::threads) {
          const int pk = lst[q], r = pk >> kHalfBinBits;
          float2 hi;
          uint32_t lo;
          ext_split(cscale(lds[F::addr(0, pk & ((1 << kHalfBinBits) - 1))], scale), hi, lo);
          Ywh[o0 + r] = hi;
          Ywl[o0 + r] = lo;
        }
      }
      if (prof && b < L) {
        for (int idx = threadIdx.x; idx < g.T * 64; idx += F::threads) {
          const int t = idx >> 6, jj = idx & 63;
          const int m = (s_center[t] - 32 + jj) & (M - 1);
          if ((m & 1) == par) {
            const double2 y = cscale(lds[F::addr(0, m >> 1)], scale);
            s_acc[idx] += (float)(y.x * y.x + y.y * y.y);
          }
        }
      }
      __syncthreads();   // the next transform overwrites lds
    }
  }
  if (prof) {
    float* dst = prof + ((int64_t)k * gridDim.x + blockIdx.x) * g.T * 64;
    for (int idx = threadIdx.x; idx < g.T * 64; idx += F::threads) dst[idx] = s_acc[idx];
  }
}

// ---------------------------------------------------------------------------------------------
// 4096-point FP64 transform of one LDS-resident row by 256 threads, 16 values each: three
// radix-16 Stockham passes (sub-lengths Ns = 1, 16, 256).  Butterfly j of a pass takes
// x[j + 256 r], multiplies input r by w^(r (j mod Ns)), w = exp(-2 pi i / (16 Ns)), applies the
// 16-point DFT and stores output r at (j div Ns) 16 Ns + (j mod Ns) + r Ns.  LDS position of
// element e: e ^ ((e >> 4) & 15), so that the stride-16 stores of a pass and the stride-1 loads
// of the next each put 16 consecutive lanes on 16 distinct 16-byte bank groups.
struct Fft4k {
  static constexpr int n = 4096, threads = 256;
  __device__ __forceinline__ static int pos(int e) { return e ^ ((e >> 4) & 15); }

  // 16-point DFT in place, 4 x 4: DFT4 over p of v[q + 4p] (outputs k1 at v[q + 4 k1]),
  // twiddle by exp(-2 pi i q k1 / 16), DFT4 over q (output k1 + 4 k2 at v[4 k1 + k2]).
  __device__ __forceinline__ static void dft16(double2 (&v)[16]) {
    constexpr double c = 0.92387953251128675613, sn = 0.38268343236508977173,
                     h = 0.70710678118654752440;
#pragma unroll
    for (int q = 0; q < 4; ++q) dft4(v[q], v[q + 4], v[q + 8], v[q + 12]);
    v[5] = cmul(v[5], make_double2(c, -sn));      // w^1
    v[6] = cmul(v[6], make_double2(h, -h));       // w^2
    v[7] = cmul(v[7], make_double2(sn, -c));      // w^3
    v[9] = cmul(v[9], make_double2(h, -h));       // w^2
    v[10] = cmul_mj(v[10]);                       // w^4 = -i
    v[11] = cmul(v[11], make_double2(-h, -h));    // w^6
    v[13] = cmul(v[13], make_double2(sn, -c));    // w^3
    v[14] = cmul(v[14], make_double2(-h, -h));    // w^6
    v[15] = cmul(v[15], make_double2(-c, sn));    // w^9
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) dft4(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
  }

  // output r of the butterfly (natural order) to LDS element base + r ns
  __device__ __forceinline__ static void store(const double2 (&v)[16], double2* lds, int base,
                                               int ns) {
#pragma unroll
    for (int r = 0; r < 16; ++r) lds[pos(base + r * ns)] = v[4 * (r & 3) + (r >> 2)];
  }

  __device__ __forceinline__ static void load(double2 (&v)[16], const double2* lds, int j) {
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = lds[pos(j + 256 * r)];
  }

  // input r times w^r (FP64).  The powers follow the three-term recurrence w^r = 2 Re(w)
  // w^(r-1) - w^(r-2) of cos and sin, applied to the real and imaginary parts alike (two FMAs
  // per power against four for a complex product; for r <= 15 its rounding error stays near
  // r^2 / 2 units in the last place).
  __device__ __forceinline__ static void twiddle(double2 (&v)[16], double2 w) {
    const double c2 = 2.0 * w.x;
    double2 t0 = make_double2(1.0, 0.0), t1 = w;
    v[1] = cmul(v[1], t1);
#pragma unroll
    for (int r = 2; r < 16; ++r) {
      const double2 t2 = make_double2(fma(c2, t1.x, -t0.x), fma(c2, t1.y, -t0.y));
      v[r] = cmul(v[r], t2);
      t0 = t1;
      t1 = t2;
    }
  }

  // input r times exp(-i pi r / 16): the first pass's share of the half-bin shift (below)
  __device__ __forceinline__ static void shift_first(double2 (&v)[16]) {
    constexpr double c[9] = {1.0, 0.98078528040323044913, 0.92387953251128675613,
                             0.83146961230254523708, 0.70710678118654752440,
                             0.55557023301960222474, 0.38268343236508977173,
                             0.19509032201612826785, 0.0};
#pragma unroll
    for (int r = 1; r < 16; ++r) {
      if (r == 8) {
        v[r] = cmul_mj(v[r]);
      } else {
        // cos(pi r / 16) and sin(pi r / 16) from the first quadrant
        const double cr = r < 8 ? c[r] : -c[16 - r], sr = r < 8 ? c[8 - r] : c[r - 8];
        v[r] = cmul(v[r], make_double2(cr, -sr));
      }
    }
  }

  // v = this thread's inputs x[j + 256 r]; w1 = exp(-2 pi i (j mod 16) / 256), w2 =
  // exp(-2 pi i (j mod 256) / 4096).  On return lds holds the transform in natural order
  // (position pos(m)), visible to every thread; on entry other threads may still be reading
  // lds (the previous transform's outputs).  Each barrier sits just before the stores it
  // protects, not after the loads of the pass before: a wave then works on its first loaded
  // values while the rest are still arriving, and waves that receive theirs early do not wait
  // for the others before computing.
  //
  // Half-bin shift: the transform at frequencies m + 1/2, sum_e x[e] exp(-2 pi i e (m + 1/2) /
  // 4096), is the same three passes with input r of the first pass times exp(-i pi r / 16)
  // (shift_first) and the bases w1 = exp(-2 pi i (2 (j mod 16) + 1) / 512), w2 = exp(-2 pi i
  // (2 (j mod 256) + 1) / 8192): the factor exp(-i pi e / 4096) of element e = j + 256 r splits
  // into exp(-i pi r / 16) and a factor common to butterfly j, which commutes with its DFT and
  // moves into the next pass's twiddle base, where it leaves no common factor after the third.
  __device__ __forceinline__ static void run(double2 (&v)[16], double2* lds, double2 w1,
                                             double2 w2) {
    // The empty register constraint makes the bases opaque, which keeps their powers inside
    // the caller's loop (hoisted out of it as loop invariants they would take 60 registers per
    // pass).  It stands here, before any LDS load is in flight, because in the middle of a
    // pass it makes the compiler wait for all sixteen loads before the first product.
    asm volatile("" : "+v"(w1.x), "+v"(w1.y), "+v"(w2.x), "+v"(w2.y));
    const int j = threadIdx.x;
    dft16(v);
    __syncthreads();   // every thread is done reading lds
    store(v, lds, 16 * j, 1);
    __syncthreads();
    load(v, lds, j);
    twiddle(v, w1);
    dft16(v);
    __syncthreads();
    store(v, lds, (j >> 4) * 256 + (j & 15), 16);
    __syncthreads();
    load(v, lds, j);
    twiddle(v, w2);
    dft16(v);
    __syncthreads();
    store(v, lds, j, 256);
    __syncthreads();
  }
};

// Windowed spatial DFT in extended precision at M = 8192, N <= 4096: the split-half scheme of
// k_beamspace_x2 (even bins from the 4096-point transform of X, odd bins from that of
// X[e] w_M^e) on the Fft4k engine.  256 threads: two 64 KiB workgroups per compute unit.  The
// next snapshot's inputs are fetched into the registers of the current one as soon as the odd
// half's inputs have been formed.  Outputs as k_beamspace_x2 (one snapshot per tile, window
// rows in split order).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_beamspace_x16(
    const float2* __restrict__ Xh, const uint32_t* __restrict__ Xl, float2* __restrict__ Ywh,
    uint32_t* __restrict__ Ywl, int N, int B, int K, const double2* __restrict__ twM,
    double scale, const int* __restrict__ rowtab, int sumW, WindowGeom g, float* __restrict__ prof,
    int L, int k0) {
  constexpr int M = 8192;
  extern __shared__ double2 lds_x[];
  double2* lds = lds_x;
  int* s_dyn = reinterpret_cast<int*>(lds_x + Fft4k::n);
  int* s_start = s_dyn;
  int* s_center = s_dyn + g.T;
  float* s_acc = reinterpret_cast<float*>(s_dyn + 2 * g.T);
  int* s_bin = s_dyn + 2 * g.T + (prof ? 64 * g.T : 0);
  int* s_ebase = s_bin + sumW;
  const int k = k0 + blockIdx.y;
  const int j = threadIdx.x;
  // twiddle bases of the even-bin transform and of the odd-bin one (half-bin shift)
  const double2 w1e = twM[(j & 15) * 32], w2e = twM[(j & 255) * 2];
  const double2 w1o = twM[(2 * (j & 15) + 1) * 16], w2o = twM[2 * (j & 255) + 1];
  // one snapshot row x[e], e = j + 256 r, through buffer descriptors bounded at the row's N
  // elements: the hardware returns zero for e >= N (the zero padding), with no branch
  auto fetch = [&](int b, float2 (&vh)[16], uint32_t (&vl)[16]) {
    const int64_t base = ((int64_t)k * B + b) * N;
    const __amdgpu_buffer_rsrc_t dh =
        __builtin_amdgcn_make_buffer_rsrc((void*)(Xh + base), 0, N * 8, kRawBufferFlags);
    const __amdgpu_buffer_rsrc_t dl =
        __builtin_amdgcn_make_buffer_rsrc((void*)(Xl + base), 0, N * 4, kRawBufferFlags);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int e = j + 256 * r;
      vh[r] = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(dh, e * 8, 0, 0));
      vl[r] = __builtin_amdgcn_raw_buffer_load_b32(dl, e * 4, 0, 0);
    }
  };
  float2 rh[16];
  uint32_t rl[16];
  if ((int)blockIdx.x < B) fetch(blockIdx.x, rh, rl);
  if (Ywh || prof) {
    for (int t = threadIdx.x; t < g.T; t += Fft4k::threads) {
      double u;
      int s;
      window_of(g, t, k, &u, &s);
      s_start[t] = s;
      if (prof) s_center[t] = (int)floor(u + 0.5);
    }
    if (prof)
      for (int i = threadIdx.x; i < g.T * 64; i += Fft4k::threads) s_acc[i] = 0.f;
    if (Ywh) {
      __syncthreads();
      split_row_lists<M>(g, s_start, rowtab, sumW, s_bin, s_ebase, Fft4k::threads);
    }
  }
  for (int b = blockIdx.x; b < B; b += gridDim.x) {
    const int64_t o0 = ((int64_t)k * B + b) * sumW;
#pragma unroll 1
    for (int par = 0; par < 2; ++par) {
      double2 v[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = ext_join(rh[r], rl[r]);
      if (par) Fft4k::shift_first(v);
      if (par && b + (int)gridDim.x < B) fetch(b + gridDim.x, rh, rl);
      Fft4k::run(v, lds, par ? w1o : w1e, par ? w2o : w2e);
      if (Ywh) {
        const int ne = s_ebase[g.T], cnt = par ? sumW - ne : ne;
        const int* lst = s_bin + (par ? ne : 0);
        // GB = 2 list entries per thread and pass, each pass's LDS reads issued together (the
        // entries, then the bins they name): two LDS round trips per pass instead of two per
        // entry, in registers the transform no longer holds (256 per thread; four entries per
        // pass spill)
        constexpr int GB = 2;
        for (int q0 = 0; q0 < cnt; q0 += GB * Fft4k::threads) {
          int pk[GB];
#pragma unroll
          for (int i = 0; i < GB; ++i) {
            const int q = q0 + i * Fft4k::threads + (int)threadIdx.x;
            pk[i] = q < cnt ? lst[q] : -1;
          }
          double2 y[GB];
#pragma unroll
          for (int i = 0; i < GB; ++i)
            if (pk[i] >= 0) y[i] = lds[Fft4k::pos(pk[i] & ((1 << kHalfBinBits) - 1))];
#pragma unroll
          for (int i = 0; i < GB; ++i) {
            if (pk[i] >= 0) {
              const int r = pk[i] >> kHalfBinBits;
              float2 hi;
              uint32_t lo;
              ext_split(cscale(y[i], scale), hi, lo);
              Ywh[o0 + r] = hi;
              Ywl[o0 + r] = lo;
            }
          }
        }
      }
      if (prof && b < L) {
        for (int idx = threadIdx.x; idx < g.T * 64; idx += Fft4k::threads) {
          const int t = idx >> 6, jj = idx & 63;
          const int m = (s_center[t] - 32 + jj) & (M - 1);
          if ((m & 1) == par) {
            const double2 y = cscale(lds[Fft4k::pos(m >> 1)], scale);
            s_acc[idx] += (float)(y.x * y.x + y.y * y.y);
          }
        }
      }
    }
  }
  if (prof) {
    float* dst = prof + ((int64_t)k * gridDim.x + blockIdx.x) * g.T * 64;
    for (int idx = threadIdx.x; idx < g.T * 64; idx += Fft4k::threads) dst[idx] = s_acc[idx];
  }
}

// Subband synthesis, the inverse of the channelizer per block: Z [T][K][Lt] (beam outputs of
// every subband on the test blocks) -> z [T][Lt*K], z[t][b K + tau] = K^-1/2 conj(h[tau])
// sum_k Z[t][k][b] exp(+j 2 pi tau k / K), computed as the conjugate of the forward transform
// of conj(Z).  Workgroup = (tiles of TB = tile/K blocks, target t): the block-contiguous
// inputs are staged through LDS (reads run along the blocks), the output rows are written
// time-contiguous.
template <int LOGK>
__global__ __launch_bounds__(fft_threads(LOGK, 11)) void k_synth(
    const float2* __restrict__ Z, float2* __restrict__ z, int Lt, const float2* __restrict__ twK,
    const float2* __restrict__ hb, float scale) {
  using F = Fft<LOGK, fft_tile(LOGK, 11), chan_pad(fft_tile(LOGK, 11), LOGK)>;
  constexpr int K = F::n, TB = F::rows;
  constexpr int LOGTB = fft_tile(LOGK, 11) - LOGK;
  __shared__ float2 lds[F::lds_complex];
  float2 tr[F::NPA][F::NTW];
  F::load_twiddles(tr, twK);
  const float2* Zt = Z + (int64_t)blockIdx.y * K * Lt;
  float2* zt = z + (int64_t)blockIdx.y * Lt * K;
  for (int b0 = blockIdx.x * TB; b0 < Lt; b0 += gridDim.x * TB) {
    for (int idx = threadIdx.x; idx < K * TB; idx += F::threads) {
      const int k = idx >> LOGTB, r = idx & (TB - 1);
      float2 val = make_float2(0.f, 0.f);
      if (b0 + r < Lt) {
        const float2 u = Zt[(int64_t)k * Lt + b0 + r];
        val = make_float2(u.x, -u.y);
      }
      lds[F::addr(r, k)] = val;
    }
    __syncthreads();
    float2 v[8];
#pragma unroll
    for (int p = 0; p < 8 / F::R0; ++p) {
#pragma unroll
      for (int r = 0; r < F::R0; ++r) {
        int row, pos;
        F::first_input(p, r, row, pos);
        v[p * F::R0 + r] = lds[F::addr(row, pos)];
      }
    }
    __syncthreads();
    F::run(v, lds, tr);
    for (int idx = threadIdx.x; idx < TB * K; idx += F::threads) {
      const int row = idx >> LOGK, i = idx & (K - 1);
      if (b0 + row < Lt) {
        const float2 u = lds[F::addr(row, i)];
        float2 y = make_float2(u.x * scale, -u.y * scale);
        if (hb) y = cmul(y, make_float2(hb[i].x, -hb[i].y));
        zt[(int64_t)(b0 + row) * K + i] = y;
      }
    }
    __syncthreads();   // the next tile's staging overwrites lds
  }
}

// Range compression of a pulse train (matched filter within each pulse, linear correlation):
// z [T][>= P R] -> r [T][P][R], r[p][d] = sum_{m < Lp, d + m < R} conj(c[m]) z[p R + d + m],
// computed per pulse as the inverse F-point DFT of Z conj(C) (F >= R + Lp - 1, so no product
// wraps): Z = DFT of the pulse zero-padded to F, C = the chirp's spectrum cf (unscaled DFT of
// the chirp zero-padded to F).  With cf == nullptr the kernel instead writes the spectrum of
// the single row z (the chirp) into r.  Workgroup = (tiles of F-point rows, target).
template <int LOGF>
__global__ __launch_bounds__(fft_threads(LOGF, 11)) void k_range_compress(
    const float2* __restrict__ z, int64_t zstride, int R, int P, const float2* __restrict__ cf,
    int Lp, float2* __restrict__ r, const float2* __restrict__ twF) {
  using F = Fft<LOGF, fft_tile(LOGF, 11), chan_pad(fft_tile(LOGF, 11), LOGF)>;
  constexpr int NF = F::n, TB = F::rows;
  __shared__ float2 lds[F::lds_complex];
  float2 tr[F::NPA][F::NTW];
  F::load_twiddles(tr, twF);
  const float2* zt = z + (int64_t)blockIdx.y * zstride;
  float2* rt = r + (int64_t)blockIdx.y * P * R;
  const int len = cf ? R : Lp;   // nonzero samples per row
  const int rows = cf ? P : 1;
  for (int p0 = blockIdx.x * TB; p0 < rows; p0 += gridDim.x * TB) {
    for (int idx = threadIdx.x; idx < TB * NF; idx += F::threads) {
      const int row = idx >> LOGF, n = idx & (NF - 1);
      float2 v = make_float2(0.f, 0.f);
      if (p0 + row < rows && n < len) v = zt[(int64_t)(p0 + row) * R + n];
      lds[F::addr(row, n)] = v;
    }
    __syncthreads();
    float2 v[8];
#pragma unroll
    for (int q = 0; q < 8 / F::R0; ++q)
#pragma unroll
      for (int rr = 0; rr < F::R0; ++rr) {
        int row, pos;
        F::first_input(q, rr, row, pos);
        v[q * F::R0 + rr] = lds[F::addr(row, pos)];
      }
    __syncthreads();
    F::run(v, lds, tr);
    if (!cf) {   // the chirp's spectrum
      for (int i = threadIdx.x; i < NF; i += F::threads) rt[i] = lds[F::addr(0, i)];
      return;
    }
    // inverse transform of Z conj(C): conj(DFT(conj(Z conj(C)))) / F
#pragma unroll
    for (int q = 0; q < 8 / F::R0; ++q)
#pragma unroll
      for (int rr = 0; rr < F::R0; ++rr) {
        int row, pos;
        F::first_input(q, rr, row, pos);
        const float2 a = lds[F::addr(row, pos)], c = cf[pos];
        // conj(a conj(c)) = conj(a) c
        v[q * F::R0 + rr] = make_float2(a.x * c.x + a.y * c.y, a.x * c.y - a.y * c.x);
      }
    __syncthreads();
    F::run(v, lds, tr);
    const float inv = 1.0f / (float)NF;
    for (int idx = threadIdx.x; idx < TB * NF; idx += F::threads) {
      const int row = idx >> LOGF, d = idx & (NF - 1);
      if (p0 + row < P && d < R) {
        const float2 u = lds[F::addr(row, d)];
        rt[(int64_t)(p0 + row) * R + d] = make_float2(u.x * inv, -u.y * inv);
      }
    }
    __syncthreads();
  }
}

// Doppler processing: r [T][P][R] -> power [T][R][P] = |RD|^2, RD[d][v] = P^-1/2 sum_p
// r[p][d] exp(-j 2 pi p v / P).  Workgroup = (tiles of TB range bins, target): the pulses of
// TB consecutive range bins are staged through LDS (reads run along range), one P-point row
// per range bin, powers written velocity-contiguous.
template <int LOGP>
__global__ __launch_bounds__(fft_threads(LOGP, 11)) void k_doppler(
    const float2* __restrict__ r, int R, float* __restrict__ power,
    const float2* __restrict__ twP) {
  using F = Fft<LOGP, fft_tile(LOGP, 11), chan_pad(fft_tile(LOGP, 11), LOGP)>;
  constexpr int P = F::n, TB = F::rows;
  constexpr int LOGTB = fft_tile(LOGP, 11) - LOGP;
  __shared__ float2 lds[F::lds_complex];
  float2 tr[F::NPA][F::NTW];
  F::load_twiddles(tr, twP);
  const float2* rt = r + (int64_t)blockIdx.y * P * R;
  float* pt = power + (int64_t)blockIdx.y * R * P;
  for (int d0 = blockIdx.x * TB; d0 < R; d0 += gridDim.x * TB) {
    for (int idx = threadIdx.x; idx < TB * P; idx += F::threads) {
      const int p = idx >> LOGTB, j = idx & (TB - 1);
      float2 v = make_float2(0.f, 0.f);
      if (d0 + j < R) v = rt[(int64_t)p * R + d0 + j];
      lds[F::addr(j, p)] = v;
    }
    __syncthreads();
    float2 v[8];
#pragma unroll
    for (int q = 0; q < 8 / F::R0; ++q)
#pragma unroll
      for (int rr = 0; rr < F::R0; ++rr) {
        int row, pos;
        F::first_input(q, rr, row, pos);
        v[q * F::R0 + rr] = lds[F::addr(row, pos)];
      }
    __syncthreads();
    F::run(v, lds, tr);
    const float inv = 1.0f / (float)P;
    for (int idx = threadIdx.x; idx < TB * P; idx += F::threads) {
      const int j = idx >> LOGP, vb = idx & (P - 1);
      if (d0 + j < R) {
        const float2 u = lds[F::addr(j, vb)];
        pt[(int64_t)(d0 + j) * P + vb] = (u.x * u.x + u.y * u.y) * inv;
      }
    }
    __syncthreads();
  }
}

// Cell-averaging CFAR along range for every velocity bin: noise = mean power of the cells
// guard < |d' - d| <= guard + train inside [0, R); detection when power > alpha noise (FP32).
// One thread per (d, v), consecutive threads along v.
__global__ __launch_bounds__(256) void k_cfar(const float* __restrict__ power, int R, int P,
                                              int guard, int train, float alpha,
                                              unsigned char* __restrict__ det) {
  const int64_t t = blockIdx.y;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= R * P) return;
  const int d = idx / P, v = idx - d * P;
  const float* pt = power + t * R * P;
  float sum = 0.f;
  int cnt = 0;
  for (int o = guard + 1; o <= guard + train; ++o) {
    if (d - o >= 0) {
      sum += pt[(int64_t)(d - o) * P + v];
      ++cnt;
    }
    if (d + o < R) {
      sum += pt[(int64_t)(d + o) * P + v];
      ++cnt;
    }
  }
  det[t * R * P + idx] = (cnt > 0 && pt[idx] > alpha * (sum / (float)cnt)) ? 1 : 0;
}

static int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// Workgroups the device holds at once for a kernel (occupancy x compute units), cached per
// instantiation; the FFT kernels loop over their tiles with a grid of about this size.
template <class KERN>
static int resident_blocks(KERN kernel, int threads, size_t dyn_shm, int* cache) {
  if (*cache > 0) return *cache;
  int per_cu = 0, cus = 0, dev = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, dyn_shm) !=
          hipSuccess || per_cu < 1 || cus < 1) {
    (void)hipGetLastError();
    return 2048;
  }
  *cache = per_cu * cus;
  return *cache;
}

template <int LOGK, int LOGT>
static hipError_t chan_launch(const float2* x, float2* X, int N, int B, const float2* twK,
                              const float2* hb, hipStream_t s) {
  using F = Fft<LOGK, fft_tile(LOGK, LOGT), chan_pad(fft_tile(LOGK, LOGT), LOGK)>;
  static int resident = 0;
  const int gx = (N + F::rows - 1) / F::rows;
  const int cap = resident_blocks(k_channelize<LOGK, LOGT>, F::threads, 0, &resident);
  int gy = (cap + gx - 1) / gx;
  if (gy > B) gy = B;
  if (gy < 1) gy = 1;
  hipLaunchKernelGGL((k_channelize<LOGK, LOGT>), dim3(gx, gy), dim3(F::threads), 0, s, x, X, N,
                     B, (int64_t)B * F::n, twK, hb, 1.0f / sqrtf((float)F::n));
  return hipGetLastError();
}

// LDS bytes of a spatial DFT launch's per-call tables beside its transform tile: window
// starts and beam centres (2 ints per target), the profile accumulators (64 floats per target),
// the window-row list (one int per row; the split-half kernels also the even-row offsets, T + 1
// ints).  The launchers and beamspace_lds_bytes share it.
static size_t beam_table_bytes(int T, int sumW, bool windows, bool prof, bool split) {
  size_t b = 0;
  if (windows || prof) b += sizeof(int) * 2 * (size_t)T;
  if (prof) b += sizeof(float) * 64 * (size_t)T;
  if (windows) b += sizeof(int) * ((size_t)sumW + (split ? (size_t)T + 1 : 0));
  return b;
}

template <int LOGM, int LOGT, bool ZH>
static hipError_t beam_launch_zh(const float2* X, float2* Y, float2* Yw, int N, int B, int K,
                                 const float2* twM, const int* rowtab, int sumW,
                                 const WindowGeom& g, float* prof, int L, int G, int k0, int kc,
                                 hipStream_t s) {
  using F = Fft<LOGM, fft_tile(LOGM, LOGT), beam_pad(fft_tile(LOGM, LOGT), LOGM)>;
  const int nbt = (B + F::rows - 1) / F::rows;
  if (prof && (G < 1 || G > nbt)) return hipErrorInvalidValue;
  const size_t shm = beam_table_bytes(g.T, sumW, Yw != nullptr, prof != nullptr, false);
  if (sizeof(float2) * (size_t)F::lds_complex + shm > kLdsBytes) return hipErrorInvalidValue;
  if (sizeof(float2) * (size_t)F::lds_complex + shm > 64 * 1024) {
    // beyond the default 64 KiB per workgroup: ask for exactly the dynamic part
    hipError_t e = hipFuncSetAttribute((const void*)k_beamspace<LOGM, LOGT, ZH>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
  }
  int gx = G;
  if (!prof) {
    static int resident = 0;
    const int cap = resident_blocks(k_beamspace<LOGM, LOGT, ZH>, F::threads, shm, &resident);
    gx = (cap + kc - 1) / kc;
    if (gx > nbt) gx = nbt;
    if (gx < 1) gx = 1;
  }
  hipLaunchKernelGGL((k_beamspace<LOGM, LOGT, ZH>), dim3(gx, kc), dim3(F::threads), shm, s, X, Y,
                     Yw, N, B, K, twM, 1.0f / sqrtf((float)F::n), rowtab, sumW, g, prof, L, k0);
  return hipGetLastError();
}

template <int LOGM, int LOGT>
static hipError_t beam_launch(const float2* X, float2* Y, float2* Yw, int N, int B, int K,
                              const float2* twM, const int* rowtab, int sumW,
                              const WindowGeom& g, float* prof, int L, int G, int k0, int kc,
                              hipStream_t s) {
  if (2 * N <= (1 << LOGM))
    return beam_launch_zh<LOGM, LOGT, true>(X, Y, Yw, N, B, K, twM, rowtab, sumW, g, prof, L, G,
                                            k0, kc, s);
  return beam_launch_zh<LOGM, LOGT, false>(X, Y, Yw, N, B, K, twM, rowtab, sumW, g, prof, L, G,
                                           k0, kc, s);
}

template <int LOGK, int LOGT>
static hipError_t chan_launch_x(const float2* x, float2* Xh, uint32_t* Xl, int N, int B,
                                const double2* twK, const double2* hb, hipStream_t s) {
  using F = Fft<LOGK, fft_tile(LOGK, LOGT), chan_pad(fft_tile(LOGK, LOGT), LOGK), double2>;
  const size_t shm = sizeof(double2) * (size_t)F::lds_complex;
  if (shm > kLdsBytes) return hipErrorInvalidValue;
  if (shm > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)k_channelize_x<LOGK, LOGT>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
  }
  static int resident = 0;
  const int gx = (N + F::rows - 1) / F::rows;
  const int cap = resident_blocks(k_channelize_x<LOGK, LOGT>, F::threads, shm, &resident);
  int gy = (cap + gx - 1) / gx;
  if (gy > B) gy = B;
  if (gy < 1) gy = 1;
  hipLaunchKernelGGL((k_channelize_x<LOGK, LOGT>), dim3(gx, gy), dim3(F::threads), shm, s, x, Xh,
                     Xl, N, B, (int64_t)B * F::n, twK, hb, 1.0 / sqrt((double)F::n));
  return hipGetLastError();
}

template <int LOGM, int LOGT, bool ZH>
static hipError_t beam_launch_x_zh(const float2* Xh, const uint32_t* Xl, float2* Ywh,
                                   uint32_t* Ywl, int N, int B, int K, const double2* twM,
                                   const int* rowtab, int sumW, const WindowGeom& g, float* prof,
                                   int L, int G, int k0, int kc, hipStream_t s) {
  using F = Fft<LOGM, fft_tile(LOGM, LOGT), beam_pad(fft_tile(LOGM, LOGT), LOGM), double2>;
  const int nbt = (B + F::rows - 1) / F::rows;
  if (prof && (G < 1 || G > nbt)) return hipErrorInvalidValue;
  size_t shm = sizeof(double2) * (size_t)F::lds_complex;
  shm += beam_table_bytes(g.T, sumW, Ywh != nullptr, prof != nullptr, false);
  if (shm > kLdsBytes) return hipErrorInvalidValue;
  if (shm > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)k_beamspace_x<LOGM, LOGT, ZH>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
  }
  int gx = G;
  if (!prof) {
    static int resident = 0;
    const int cap = resident_blocks(k_beamspace_x<LOGM, LOGT, ZH>, F::threads, shm, &resident);
    gx = (cap + kc - 1) / kc;
    if (gx > nbt) gx = nbt;
    if (gx < 1) gx = 1;
  }
  hipLaunchKernelGGL((k_beamspace_x<LOGM, LOGT, ZH>), dim3(gx, kc), dim3(F::threads), shm, s, Xh,
                     Xl, Ywh, Ywl, N, B, K, twM, 1.0 / sqrt((double)F::n), rowtab, sumW, g, prof,
                     L, k0);
  return hipGetLastError();
}

// Split-half form (k_beamspace_x2) for M = 2^(LOGH + 1), one snapshot per tile.
template <int LOGH>
static hipError_t beam_launch_x2(const float2* Xh, const uint32_t* Xl, float2* Ywh,
                                 uint32_t* Ywl, int N, int B, int K, const double2* twM,
                                 const int* rowtab, int sumW, const WindowGeom& g, float* prof,
                                 int L, int G, int k0, int kc, hipStream_t s) {
  using F = Fft<LOGH, LOGH, beam_pad(LOGH, LOGH), double2>;
  if (prof && (G < 1 || G > B)) return hipErrorInvalidValue;
  size_t shm = sizeof(double2) * (size_t)F::lds_complex;
  shm += beam_table_bytes(g.T, sumW, Ywh != nullptr, prof != nullptr, true);
  if (shm > kLdsBytes) return hipErrorInvalidValue;
  if (shm > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)k_beamspace_x2<LOGH>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
  }
  int gx = G;
  if (!prof) {
    static int resident = 0;
    const int cap = resident_blocks(k_beamspace_x2<LOGH>, F::threads, shm, &resident);
    gx = (cap + kc - 1) / kc;
    if (gx > B) gx = B;
    if (gx < 1) gx = 1;
  }
  hipLaunchKernelGGL((k_beamspace_x2<LOGH>), dim3(gx, kc), dim3(F::threads), shm, s, Xh, Xl, Ywh,
                     Ywl, N, B, K, twM, 1.0 / sqrt((double)(2 * F::n)), rowtab, sumW, g, prof, L,
                     k0);
  return hipGetLastError();
}

static hipError_t beam_launch_x16(const float2* Xh, const uint32_t* Xl, float2* Ywh,
                                  uint32_t* Ywl, int N, int B, int K, const double2* twM,
                                  const int* rowtab, int sumW, const WindowGeom& g, float* prof,
                                  int L, int G, int k0, int kc, hipStream_t s) {
  if (N > 4096) return hipErrorInvalidValue;
  if (prof && (G < 1 || G > B)) return hipErrorInvalidValue;
  size_t shm = sizeof(double2) * (size_t)Fft4k::n;
  shm += beam_table_bytes(g.T, sumW, Ywh != nullptr, prof != nullptr, true);
  if (shm > kLdsBytes) return hipErrorInvalidValue;
  if (shm > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)k_beamspace_x16,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
  }
  int gx = G;
  if (!prof) {
    static int resident = 0;
    const int cap = resident_blocks(k_beamspace_x16, Fft4k::threads, shm, &resident);
    gx = (cap + kc - 1) / kc;
    if (gx > B) gx = B;
    if (gx < 1) gx = 1;
  }
  hipLaunchKernelGGL(k_beamspace_x16, dim3(gx, kc), dim3(Fft4k::threads), shm, s, Xh, Xl, Ywh,
                     Ywl, N, B, K, twM, 1.0 / sqrt(8192.0), rowtab, sumW, g, prof, L, k0);
  return hipGetLastError();
}

template <int LOGM, int LOGT>
static hipError_t beam_launch_x(const float2* Xh, const uint32_t* Xl, float2* Ywh, uint32_t* Ywl,
                                int N, int B, int K, const double2* twM, const int* rowtab,
                                int sumW, const WindowGeom& g, float* prof, int L, int G, int k0,
                                int kc, hipStream_t s) {
  if constexpr (LOGM >= 13) {
    // a full FP64 row no longer fits a 64 KiB tile: split halves whenever the upper half is zero
    if (beamspace_x_split_rows(N, 1 << LOGM)) {
      if constexpr (LOGM == 13) {
        if (LOGT == 13)   // the radix-16 engine (tile 2^13: both halves of one snapshot)
          return beam_launch_x16(Xh, Xl, Ywh, Ywl, N, B, K, twM, rowtab, sumW, g, prof, L, G, k0,
                                 kc, s);
      }
      return beam_launch_x2<LOGM - 1>(Xh, Xl, Ywh, Ywl, N, B, K, twM, rowtab, sumW, g, prof, L,
                                      G, k0, kc, s);
    }
  }
  if (2 * N <= (1 << LOGM))
    return beam_launch_x_zh<LOGM, LOGT, true>(Xh, Xl, Ywh, Ywl, N, B, K, twM, rowtab, sumW, g,
                                              prof, L, G, k0, kc, s);
  return beam_launch_x_zh<LOGM, LOGT, false>(Xh, Xl, Ywh, Ywl, N, B, K, twM, rowtab, sumW, g,
                                             prof, L, G, k0, kc, s);
}

// Planar-array beamspace (Eq. 16-17): X [K][B][N], N = Nz Nx (element ix Nz + iz) ->
//   full  : Y [K][Mz Mx][B], beam mx Mz + mz                              (stage output), and/or
//   window: Yw [K][nbt][sumW][TB] in the layout of the linear-array kernel (TB = 2^logTB
//           snapshots per tile block), row r = cell i of target t's Wz x Wx window.
// The Kronecker transform factors into a zero-padded Mx-point FFT along x of every (snapshot,
// iz) row, tiles of 2^11 values through LDS as in the linear-array kernel (rows of one
// snapshot are Pz = 2^logPz >= Nz apart, the rows iz >= Nz zero), followed by the Nz-term
// DFT along z of the bins the kernel writes.  Workgroup = (first tile, subband k), looping
// over tiles of TB2 = 2^11 / (Pz Mx) snapshots.  ZH: 2 Nx <= Mx.
constexpr int kUpaLogTile = 11;

template <int LOGMX, bool ZH>
__global__ __launch_bounds__(fft_threads(LOGMX, kUpaLogTile)) void k_beamspace_upa(
    const float2* __restrict__ X, float2* __restrict__ Y, float2* __restrict__ Yw, int logPz,
    int logMz, int B, const float2* __restrict__ twM, float scale,
    const int* __restrict__ rowtab, int sumW, UpaGeom g, int logTB, int nbt) {
  using F = Fft<LOGMX, fft_tile(LOGMX, kUpaLogTile), beam_pad(fft_tile(LOGMX, kUpaLogTile), LOGMX)>;
  constexpr int Mx = F::n;
  const int Nz = g.Nz, Nx = g.Nx, N = Nz * Nx;
  const int Mz = 1 << logMz;
  const int logTB2 = fft_tile(LOGMX, kUpaLogTile) - LOGMX - logPz;
  const int TB2 = 1 << logTB2;
  const int nbt2 = (B + TB2 - 1) >> logTB2;
  const int TB = 1 << logTB;
  const int lw = logTB < logTB2 ? logTB : logTB2;
  __shared__ float2 lds[F::lds_complex];
  extern __shared__ int s_dyn[];
  float2* s_twz = reinterpret_cast<float2*>(s_dyn);        // [Mz] exp(-j 2 pi q / Mz)
  int* s_sz = reinterpret_cast<int*>(s_twz + Mz);          // [T] window starts along z
  int* s_sx = s_sz + g.T;                                  // [T] along x
  int* s_bin = s_sx + g.T;                                 // [sumW] beam of window row r
  const int k = blockIdx.y;
  float2 tr[F::NPA][F::NTW];
  F::load_twiddles(tr, twM, Mz);                           // Mx-point table = twM[q Mz]
  // This thread's first-pass inputs sit at the same place in every tile: element (iz, ix) of
  // the tile's snapshot bb, byte offset 8 (bb N + ix Nz + iz) from the tile's first snapshot.
  // A tile of TB2 whole snapshots with every slot inside the array (Nz = Pz, Nx = Mx/2 under ZH,
  // else Nx = Mx) is read without predicates from a uniform base.
  uint32_t foff[8];
  int fbb[8];
  bool fok[8];
#pragma unroll
  for (int p = 0; p < 8 / F::R0; ++p) {
#pragma unroll
    for (int r = 0; r < F::R0; ++r) {
      int row, ix;
      F::first_input(p, r, row, ix);
      const int iz = row & ((1 << logPz) - 1), bb = row >> logPz, q = p * F::R0 + r;
      fbb[q] = bb;
      fok[q] = ix < Nx && iz < Nz;
      foff[q] = (uint32_t)(bb * N + ix * Nz + iz) * 8u;
    }
  }
  const bool dense = Nz == (1 << logPz) && Nx >= (ZH ? Mx / 2 : Mx);
  auto fetch = [&](int j, float2 (&v)[8]) {
    const int b0 = j * TB2;
    const char* base = reinterpret_cast<const char*>(X + ((int64_t)k * B + b0) * N);
    if (dense && b0 + TB2 <= B) {
#pragma unroll
      for (int q = 0; q < 8; ++q)
        v[q] = (ZH && 2 * (q % F::R0) >= F::R0)
                   ? make_float2(0.f, 0.f)
                   : *reinterpret_cast<const float2*>(base + foff[q]);
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        float2 val = make_float2(0.f, 0.f);
        if (!(ZH && 2 * (q % F::R0) >= F::R0) && fok[q] && b0 + fbb[q] < B)
          val = *reinterpret_cast<const float2*>(base + foff[q]);
        v[q] = val;
      }
    }
  };
  float2 nv[8];
  if ((int)blockIdx.x < nbt2) fetch(blockIdx.x, nv);
  for (int q = threadIdx.x; q < Mz; q += F::threads) s_twz[q] = twM[q << LOGMX];
  if (Yw) {
    for (int t = threadIdx.x; t < g.T; t += F::threads) {
      double uz, ux;
      upa_window_of(g, t, k, &uz, &s_sz[t], &ux, &s_sx[t]);
    }
    __syncthreads();
    for (int r = threadIdx.x; r < sumW; r += F::threads) {
      const int t = rowtab[r] >> 8, i = rowtab[r] & 255;
      const int Wz = g.wz[t], ixw = i / Wz, izw = i - ixw * Wz;
      s_bin[r] = (((s_sx[t] + ixw) & (Mx - 1)) << logMz) | ((s_sz[t] + izw) & (Mz - 1));
    }
  }
  __syncthreads();
  // beam m of tile snapshot bb: the z-DFT of the x-transformed rows, each twiddle
  // exp(-j 2 pi mz iz / Mz) read from the table (index mz iz mod Mz), so that its error does
  // not grow with Nz as powers formed by repeated products would
  auto beam = [&](int m, int bb) {
    const int mx = m >> logMz, mz = m & (Mz - 1);
    float2 acc = lds[F::addr(bb << logPz, mx)];
    int q = mz;
    for (int iz = 1; iz < Nz; ++iz) {
      const float2 v = lds[F::addr((bb << logPz) + iz, mx)];
      const float2 w = s_twz[q];
      acc.x += v.x * w.x - v.y * w.y;
      acc.y += v.x * w.y + v.y * w.x;
      q = (q + mz) & (Mz - 1);
    }
    return cscale(acc, scale);
  };
  for (int j = blockIdx.x; j < nbt2; j += gridDim.x) {
    const int b0 = j * TB2;
    float2 v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = nv[q];
    if (j + (int)gridDim.x < nbt2) fetch(j + gridDim.x, nv);
    F::template run<ZH>(v, lds, tr);
    if (Y) {
      const int M = Mz << LOGMX;
      for (int idx = threadIdx.x; idx < (M << logTB2); idx += F::threads) {
        const int m = idx >> logTB2, bb = idx & (TB2 - 1);
        if (b0 + bb < B) Y[((int64_t)k * M + m) * B + b0 + bb] = beam(m, bb);
      }
    }
    if (Yw) {
      // per run of 2^lw = min(TB, TB2) snapshots: the [sumW][2^lw] block it fills, written
      // contiguously (window row, then snapshot); snapshots past B (zero inputs) fill the
      // padding of the last tile block
      for (int bq = 0; bq < (TB2 >> lw); ++bq) {
        const int b1 = b0 + (bq << lw);
        if (b1 >= nbt * TB) break;
        float2* dst = Yw + ((int64_t)k * nbt + (b1 >> logTB)) * sumW * TB + (b1 & (TB - 1));
        for (int idx = threadIdx.x; idx < (sumW << lw); idx += F::threads) {
          const int r = idx >> lw, blo = idx & ((1 << lw) - 1);
          dst[r * TB + blo] = beam(s_bin[r], (bq << lw) | blo);
        }
      }
    }
    __syncthreads();   // the next tile's first pass overwrites lds
  }
}

template <int LOGMX, bool ZH>
static hipError_t beam_upa_launch(const float2* X, float2* Y, float2* Yw, int logPz, int logMz,
                                  int B, int K, const float2* twM, const int* rowtab, int sumW,
                                  const UpaGeom& g, int logTB, int nbt, hipStream_t s) {
  using F = Fft<LOGMX, fft_tile(LOGMX, kUpaLogTile), beam_pad(fft_tile(LOGMX, kUpaLogTile), LOGMX)>;
  const int logTB2 = fft_tile(LOGMX, kUpaLogTile) - LOGMX - logPz;
  if (logTB2 < 0) return hipErrorInvalidValue;
  const int nbt2 = (B + (1 << logTB2) - 1) >> logTB2;
  const size_t shm = sizeof(float2) * ((size_t)1 << logMz) +
                     sizeof(int) * (2 * (size_t)g.T + (size_t)sumW);
  if (sizeof(float2) * (size_t)F::lds_complex + shm > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)k_beamspace_upa<LOGMX, ZH>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
  }
  static int resident = 0;
  const int cap = resident_blocks(k_beamspace_upa<LOGMX, ZH>, F::threads, shm, &resident);
  int gx = (cap + K - 1) / K;
  if (gx > nbt2) gx = nbt2;
  if (gx < 1) gx = 1;
  hipLaunchKernelGGL((k_beamspace_upa<LOGMX, ZH>), dim3(gx, K), dim3(F::threads), shm, s, X, Y,
                     Yw, logPz, logMz, B, twM, 1.0f / sqrtf((float)((size_t)F::n << logMz)),
                     rowtab, sumW, g, logTB, nbt);
  return hipGetLastError();
}

#define WBM_LOG_CASES(M, T) \
  M(1, T) M(2, T) M(3, T) M(4, T) M(5, T) M(6, T) M(7, T) M(8, T) M(9, T) M(10, T) M(11, T) \
  M(12, T) M(13, T)

int fft_tile_log(int logn, int logtile) { return fft_tile(logn, logtile); }

bool fft_logtile_supported(int logtile) { return logtile >= 11 && logtile <= 13; }

hipError_t launch_channelize(const float2* x, float2* X, int N, int K, int B, const float2* twK,
                             const float2* hb, int logtile, hipStream_t s) {
  const int lk = ilog2(K);
#define C(L, T)                                     \
  case L:                                           \
    return chan_launch<L, T>(x, X, N, B, twK, hb, s);
  switch (logtile) {
    case 11:
      switch (lk) { WBM_LOG_CASES(C, 11) }
      break;
    case 12:
      switch (lk) { WBM_LOG_CASES(C, 12) }
      break;
    case 13:
      switch (lk) { WBM_LOG_CASES(C, 13) }
      break;
  }
#undef C
  return hipErrorInvalidValue;
}

bool fft_x_logtile_supported(int logtile) { return logtile >= 10 && logtile <= 13; }

bool beamspace_x_split_rows(int N, int M) { return M >= 8192 && 2 * N <= M; }

hipError_t launch_channelize_x(const float2* x, float2* Xh, uint32_t* Xl, int N, int K, int B,
                               const double2* twK, const double2* hb, int logtile,
                               hipStream_t s) {
  const int lk = ilog2(K);
#define C(L, T)                                     \
  case L:                                           \
    return chan_launch_x<L, T>(x, Xh, Xl, N, B, twK, hb, s);
  switch (logtile) {
    case 10:
      switch (lk) { WBM_LOG_CASES(C, 10) }
      break;
    case 11:
      switch (lk) { WBM_LOG_CASES(C, 11) }
      break;
    case 12:
      switch (lk) { WBM_LOG_CASES(C, 12) }
      break;
    case 13:
      switch (lk) { WBM_LOG_CASES(C, 13) }
      break;
  }
#undef C
  return hipErrorInvalidValue;
}

hipError_t launch_beamspace_x(const float2* Xh, const uint32_t* Xl, float2* Ywh, uint32_t* Ywl,
                              int N, int M, int B, int K, const double2* twM, const int* rowtab,
                              int sumW, const WindowGeom& g, int logtile, hipStream_t s,
                              float* prof, int L, int G, int k0, int kc) {
  const int lm = ilog2(M);
  if (kc < 0) kc = K - k0;
  if (k0 < 0 || kc < 1 || k0 + kc > K) return hipErrorInvalidValue;
#define C(LG, T)                                                                           \
  case LG:                                                                                 \
    return beam_launch_x<LG, T>(Xh, Xl, Ywh, Ywl, N, B, K, twM, rowtab, sumW, g, prof, L, G, \
                                k0, kc, s);
  switch (logtile) {
    case 10:
      switch (lm) { WBM_LOG_CASES(C, 10) }
      break;
    case 11:
      switch (lm) { WBM_LOG_CASES(C, 11) }
      break;
    case 12:
      switch (lm) { WBM_LOG_CASES(C, 12) }
      break;
    case 13:
      switch (lm) { WBM_LOG_CASES(C, 13) }
      break;
  }
#undef C
  return hipErrorInvalidValue;
}

hipError_t launch_synth(const float2* Z, float2* z, int K, int Lt, int T, const float2* twK,
                        const float2* hb, hipStream_t s) {
  if (Lt < 1 || T < 1) return hipSuccess;
  const int lk = ilog2(K);
  if ((1 << lk) != K) return hipErrorInvalidValue;
#define C(L, unused)                                                                          \
  case L: {                                                                                   \
    constexpr int TB = (1 << fft_tile(L, 11)) >> L;                                           \
    const int gx = (Lt + TB - 1) / TB;                                                        \
    hipLaunchKernelGGL((k_synth<L>), dim3(gx, T), dim3(fft_threads(L, 11)), 0, s, Z, z, Lt,   \
                       twK, hb, 1.0f / sqrtf((float)K));                                      \
    return hipGetLastError();                                                                 \
  }
  switch (lk) { WBM_LOG_CASES(C, 0) }
#undef C
  return hipErrorInvalidValue;
}

// tw[q] = exp(-j 2 pi q / n), q < n, evaluated in FP64 (as the plan's own tables)
__global__ void k_twiddles(float2* __restrict__ tw, int n) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  double sn, cs;
  sincospi(-2.0 * (double)q / (double)n, &sn, &cs);
  tw[q] = make_float2((float)cs, (float)sn);
}

int range_doppler_fft_log(int R, int Lp) {
  int lf = 0;
  while ((1 << lf) < R + Lp - 1) ++lf;
  return lf < 1 ? 1 : lf;
}

// work: [T][P][R] compressed pulses, then the chirp spectrum and the F- and P-point twiddle
// tables (F = 2^range_doppler_fft_log(R, Lp)): T P R + 2 F + P complex.
hipError_t launch_range_doppler(const float2* z, int64_t zstride, int T, const float2* chirp,
                                int Lp, int R, int P, int guard, int train, float alpha,
                                float2* work, float* power, unsigned char* det, hipStream_t s) {
  const int lf = range_doppler_fft_log(R, Lp);
  const int lp = ilog2(P);
  if ((1 << lp) != P || lf > 13 || lp > 13 || lp < 1) return hipErrorInvalidValue;
  const int NF = 1 << lf;
  float2* cf = work + (int64_t)T * P * R;   // chirp spectrum
  float2* twF = cf + NF;
  float2* twP = twF + NF;
  hipLaunchKernelGGL(k_twiddles, dim3((NF + 255) / 256), dim3(256), 0, s, twF, NF);
  hipLaunchKernelGGL(k_twiddles, dim3((P + 255) / 256), dim3(256), 0, s, twP, P);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  switch (lf) {
#define C(L, unused)                                                                           \
  case L: {                                                                                    \
    constexpr int TB = (1 << fft_tile(L, 11)) >> L;                                            \
    hipLaunchKernelGGL((k_range_compress<L>), dim3(1, 1), dim3(fft_threads(L, 11)), 0, s,      \
                       chirp, (int64_t)0, Lp, 1, (const float2*)nullptr, Lp, cf, twF);         \
    if ((e = hipGetLastError()) != hipSuccess) return e;                                       \
    hipLaunchKernelGGL((k_range_compress<L>), dim3((P + TB - 1) / TB, T),                      \
                       dim3(fft_threads(L, 11)), 0, s, z, zstride, R, P, (const float2*)cf, Lp, \
                       work, twF);                                                             \
    if ((e = hipGetLastError()) != hipSuccess) return e;                                       \
    break;                                                                                     \
  }
    WBM_LOG_CASES(C, 0)
#undef C
    default: return hipErrorInvalidValue;
  }
  switch (lp) {
#define C(L, unused)                                                                           \
  case L: {                                                                                    \
    constexpr int TB = (1 << fft_tile(L, 11)) >> L;                                            \
    hipLaunchKernelGGL((k_doppler<L>), dim3((R + TB - 1) / TB, T), dim3(fft_threads(L, 11)), 0, \
                       s, work, R, power, twP);                                                \
    if ((e = hipGetLastError()) != hipSuccess) return e;                                       \
    break;                                                                                     \
  }
    WBM_LOG_CASES(C, 0)
#undef C
    default: return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(k_cfar, dim3((R * P + 255) / 256, T), dim3(256), 0, s, power, R, P, guard,
                     train, alpha, det);
  return hipGetLastError();
}

int beamspace_tile_log(int M, int logtile) { return fft_tile(ilog2(M), logtile) - ilog2(M); }

int beamspace_tiles(int M, int B, int logtile) {
  const int tb = 1 << beamspace_tile_log(M, logtile);
  return (B + tb - 1) / tb;
}

template <int LOGK, int LOGT, typename V>
static size_t chan_tile_bytes() {
  using F = Fft<LOGK, fft_tile(LOGK, LOGT), chan_pad(fft_tile(LOGK, LOGT), LOGK), V>;
  return sizeof(V) * (size_t)F::lds_complex;
}

size_t channelize_lds_bytes(bool ext, int K, int logtile) {
  if (!(ext ? fft_x_logtile_supported(logtile) : fft_logtile_supported(logtile)) || K < 2 ||
      K > 8192 || (K & (K - 1)))
    return SIZE_MAX;
  const int lk = ilog2(K);
  size_t bytes = SIZE_MAX;
#define C(LG, TT)                                                                     \
  case LG:                                                                            \
    bytes = ext ? chan_tile_bytes<LG, TT, double2>() : chan_tile_bytes<LG, TT, float2>(); \
    break;
  switch (logtile) {
    case 10:
      switch (lk) { WBM_LOG_CASES(C, 10) }
      break;
    case 11:
      switch (lk) { WBM_LOG_CASES(C, 11) }
      break;
    case 12:
      switch (lk) { WBM_LOG_CASES(C, 12) }
      break;
    case 13:
      switch (lk) { WBM_LOG_CASES(C, 13) }
      break;
  }
#undef C
  return bytes;
}

template <int LOGM, int LOGT>
static size_t beam_tile_bytes_f32() {
  using F = Fft<LOGM, fft_tile(LOGM, LOGT), beam_pad(fft_tile(LOGM, LOGT), LOGM)>;
  return sizeof(float2) * (size_t)F::lds_complex;
}

// the transform tile of the kernel beam_launch_x runs; *split: a split-half kernel, whose row
// tables carry T + 1 more ints
template <int LOGM, int LOGT>
static size_t beam_tile_bytes_x(int N, bool* split) {
  *split = false;
  if constexpr (LOGM >= 13) {
    if (beamspace_x_split_rows(N, 1 << LOGM)) {
      *split = true;
      if constexpr (LOGM == 13) {
        if (LOGT == 13) return sizeof(double2) * (size_t)Fft4k::n;
      }
      using H = Fft<LOGM - 1, LOGM - 1, beam_pad(LOGM - 1, LOGM - 1), double2>;
      return sizeof(double2) * (size_t)H::lds_complex;
    }
  }
  using F = Fft<LOGM, fft_tile(LOGM, LOGT), beam_pad(fft_tile(LOGM, LOGT), LOGM), double2>;
  return sizeof(double2) * (size_t)F::lds_complex;
}

size_t beamspace_lds_bytes(bool ext, int N, int M, int logtile, int T, int sumW, bool windows,
                           bool prof) {
  if (!(ext ? fft_x_logtile_supported(logtile) : fft_logtile_supported(logtile)) || M < 2 ||
      M > 8192 || (M & (M - 1)))
    return SIZE_MAX;
  const int lm = ilog2(M);
  size_t tile = 0;
  bool split = false;
  if (ext) {
#define C(LG, TT)                                \
  case LG:                                       \
    tile = beam_tile_bytes_x<LG, TT>(N, &split); \
    break;
    switch (logtile) {
      case 10:
        switch (lm) { WBM_LOG_CASES(C, 10) }
        break;
      case 11:
        switch (lm) { WBM_LOG_CASES(C, 11) }
        break;
      case 12:
        switch (lm) { WBM_LOG_CASES(C, 12) }
        break;
      case 13:
        switch (lm) { WBM_LOG_CASES(C, 13) }
        break;
    }
#undef C
  } else {
#define C(LG, TT)                              \
  case LG:                                     \
    tile = beam_tile_bytes_f32<LG, TT>();      \
    break;
    switch (logtile) {
      case 11:
        switch (lm) { WBM_LOG_CASES(C, 11) }
        break;
      case 12:
        switch (lm) { WBM_LOG_CASES(C, 12) }
        break;
      case 13:
        switch (lm) { WBM_LOG_CASES(C, 13) }
        break;
    }
#undef C
  }
  if (!tile) return SIZE_MAX;
  return tile + beam_table_bytes(T, sumW, windows, prof, split);
}

hipError_t launch_beamspace(const float2* X, float2* Y, float2* Yw, int N, int M, int B, int K,
                            const float2* twM, const int* rowtab, int sumW, const WindowGeom& g,
                            int logtile, hipStream_t s, float* prof, int L, int G, int k0,
                            int kc) {
  const int lm = ilog2(M);
  if (kc < 0) kc = K - k0;
  if (k0 < 0 || kc < 1 || k0 + kc > K) return hipErrorInvalidValue;
#define C(LG, T)                                                                          \
  case LG:                                                                                \
    return beam_launch<LG, T>(X, Y, Yw, N, B, K, twM, rowtab, sumW, g, prof, L, G, k0, kc, s);
  switch (logtile) {
    case 11:
      switch (lm) { WBM_LOG_CASES(C, 11) }
      break;
    case 12:
      switch (lm) { WBM_LOG_CASES(C, 12) }
      break;
    case 13:
      switch (lm) { WBM_LOG_CASES(C, 13) }
      break;
  }
#undef C
  return hipErrorInvalidValue;
}

hipError_t launch_beamspace_upa(const float2* X, float2* Y, float2* Yw, int B, const float2* twM,
                                const int* rowtab, int sumW, const UpaGeom& g, int logTB, int nbt,
                                hipStream_t s) {
  const int lmx = ilog2(g.Mx), lmz = ilog2(g.Mz), lpz = ilog2(g.Nz);
  if ((1 << lmx) != g.Mx || (1 << lmz) != g.Mz || g.Nx > g.Mx || g.Nz > g.Mz || lmx < 1 ||
      lmx + lpz > kUpaLogTile)
    return hipErrorInvalidValue;
  const bool zh = 2 * g.Nx <= g.Mx;
#define C(LG, unused)                                                                           \
  case LG:                                                                                      \
    return zh ? beam_upa_launch<LG, true>(X, Y, Yw, lpz, lmz, B, g.K, twM, rowtab, sumW, g,     \
                                          logTB, nbt, s)                                        \
              : beam_upa_launch<LG, false>(X, Y, Yw, lpz, lmz, B, g.K, twM, rowtab, sumW, g,    \
                                           logTB, nbt, s);
  switch (lmx) { C(1, 0) C(2, 0) C(3, 0) C(4, 0) C(5, 0) C(6, 0) C(7, 0) C(8, 0) C(9, 0) C(10, 0) C(11, 0) }
#undef C
  return hipErrorInvalidValue;
}

// Static LDS is at most 128 rows x (64 + 13) complex = 77 KiB (64-point rows in an 8192 tile);
// the beamspace kernel adds 8 + 256 bytes per target (window starts, beam bins, profile sums)
// and 4 per window row, requested at launch when the total passes 64 KiB.
hipError_t set_fft_attributes() { return hipSuccess; }

}  // namespace wbm
