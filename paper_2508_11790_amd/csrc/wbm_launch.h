// Host-side launchers of the gfx950 kernels (internal to the library; the public
// interface is include/wbmvdr.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wbm_dev.h"

namespace wbm {

// Per-call description of the targets, uploaded to the device before the kernels run.
struct DevDesc {
  const double* sin_az;   // [T]
  const int* win;         // [T]
  const int* woff;        // [T] first window row of target t (prefix sum of win)
  const int* rowtab;      // [sumW] window row r -> (t << 8) | i
  const int* torder;      // [T] targets by window width, widest first (pair kernels' order)
  const double* cz;       // [T] planar array: sin(el) (sin_az then holds cos(el) sin(az))
  const int* wz;          // [T] planar array: window rows along z (win = Wz * Wx)
};

// FFT tile sizes the kernels are built for (log2 complex per workgroup tile).
bool fft_logtile_supported(int logtile);
// log2 of the snapshots per beamspace tile for M and a tile size.
int beamspace_tile_log(int M, int logtile);

// Time-DFT channelizer: x [N][B*K] -> X [K][B][N].
hipError_t launch_channelize(const float2* x, float2* X, int N, int K, int B, const float2* twK,
                             const float2* hb, int logtile, hipStream_t s);
// Zero-padded spatial DFT: X [K][B][N] -> Y [K][M][B] (if Y) and windows Yw (if Yw; the
// kernel places the windows of subband k itself from g).  With prof, G workgroups per
// subband each loop over snapshot tiles and write training power-profile partials
// prof [K][G][T][64] (64 bins centred on each target's beam bin, snapshots b < L).
// Subbands k0 .. k0 + kc - 1 only (kc < 0: through K - 1).
hipError_t launch_beamspace(const float2* X, float2* Y, float2* Yw, int N, int M, int B, int K,
                            const float2* twM, const int* rowtab, int sumW, const WindowGeom& g,
                            int logtile, hipStream_t s, float* prof = nullptr, int L = 0,
                            int G = 0, int k0 = 0, int kc = -1);
// Snapshot tiles of the beamspace kernel for M, B at a tile size.
int beamspace_tiles(int M, int B, int logtile);

// LDS a workgroup may use (gfx950: 160 KiB per compute unit, all of it to one workgroup).
constexpr size_t kLdsBytes = 160 * 1024;
// LDS bytes of one workgroup of the channelizer (launch_channelize / _x) at this tile; SIZE_MAX
// for a tile the precision does not support.
size_t channelize_lds_bytes(bool ext, int K, int logtile);
// LDS bytes of one workgroup of the spatial DFT that launch_beamspace (ext = false) or
// launch_beamspace_x (ext = true) runs at this tile: the transform tile, and for a call with T
// targets and sumW window rows the window-row tables (windows) and the profile accumulators
// (prof).  SIZE_MAX for a tile the precision does not support.
size_t beamspace_lds_bytes(bool ext, int N, int M, int logtile, int T, int sumW, bool windows,
                           bool prof);

// Extended-precision channelizer and windowed spatial DFT (FP64 arithmetic, hi + lo storage:
// X as Xh / Xl [K][B][N], windows as Ywh / Ywl [K][nbt][sumW][TB]); tiles of 2^10 .. 2^13
// complex (fft_x_logtile_supported), the beamspace tile in snapshots as for launch_beamspace.
bool fft_x_logtile_supported(int logtile);
hipError_t launch_channelize_x(const float2* x, float2* Xh, uint32_t* Xl, int N, int K, int B,
                               const double2* twK, const double2* hb, int logtile,
                               hipStream_t s);
hipError_t launch_beamspace_x(const float2* Xh, const uint32_t* Xl, float2* Ywh, uint32_t* Ywl,
                              int N, int M, int B, int K, const double2* twM, const int* rowtab,
                              int sumW, const WindowGeom& g, int logtile, hipStream_t s,
                              float* prof = nullptr, int L = 0, int G = 0, int k0 = 0,
                              int kc = -1);

// Window starts [T][K] and windowed steering abar [T][K][wmax] (FP64).
hipError_t launch_steer(const WindowGeom& g, int wmax, int* starts, double2* abar, hipStream_t s);

// Planar array: window starts [T][K][2] (s_z, s_x; optional), windowed steering abar
// [T][K][wmax] (FP64) and, if rows, the beam index mx Mz + mz of every window cell [T][K][wmax].
hipError_t launch_steer_upa(const UpaGeom& g, int wmax, int* starts, double2* abar,
                            hipStream_t s, int* rows = nullptr);
// Planar-array beamspace X [K][B][Nz Nx] -> Y [K][Mz Mx][B] (if Y) and the Wz x Wx windows Yw
// [K][nbt][sumW][2^logTB] (if Yw) for every subband.  Needs Mx, Mz powers of two,
// Nx <= Mx, Nz <= Mz, 2 <= Mx and next_pow2(Nz) Mx <= 2048.
hipError_t launch_beamspace_upa(const float2* X, float2* Y, float2* Yw, int B, const float2* twM,
                                const int* rowtab, int sumW, const UpaGeom& g, int logTB, int nbt,
                                hipStream_t s);

struct PairArgs {
  int T, K, M, L, Lt, B, wmax;
  int logTB, nbt, sumW;          // windowed layout (fused form)
  double delta;
  // optional per-pair window width [T][K] (a sub-window of the gathered one, same parity)
  // and per-pair loading [T][K]; nullptr = the target's window / delta
  const int* pw = nullptr;
  const float* pdelta = nullptr;
  // optional [T][K] flags: when set, the fused pair kernels solve only the flagged pairs (the
  // mixed forms' windows routed to FP64) and mark their info with bit 30
  const int* route = nullptr;
  // subbands k0 .. k0 + kc - 1 only (kc = 0: all K); the grid is T * kc workgroups
  int k0 = 0, kc = 0;
  // optional windowed steering [T][K][wmax] (the planar array's); nullptr = the pair kernels
  // evaluate the linear array's from the window geometry
  const double2* abar = nullptr;
  // plain form on the planar array: beam index of every window cell [T][K][wmax] in the full
  // beamspace (nullptr = bins (s + i) mod M)
  const int* rows = nullptr;
  // extended-precision windows: the BF16 remainder plane of the windows (same layout as the
  // FP32 plane passed as Yw); nullptr = FP32 windows.  Vector pair kernels only.
  const uint32_t* ywl = nullptr;
  // window rows stored in the split-half spatial DFT's order (even-bin rows of each gathered
  // window first, then the odd ones; beamspace_x_split_rows)
  int split_rows = 0;
};
// Whether the extended-precision spatial DFT at this N, M runs its split-half form, which
// stores every window's rows in split order (even bins first).
bool beamspace_x_split_rows(int N, int M);
// Fused per-pair window/steering -> covariance (FP64 accumulation) -> LDL^H (FP64) -> solve
// -> apply, reading the window rows written by the beamspace kernel.
// threads = kPairMfma (four waves, FP64 matrix-core covariance), kPairResident (below), 64 (one
// wave per pair on the vector units, windows up to 40 bins) or 256 (four waves per pair on the
// vector units).
constexpr int kPairMfma = 1;
// kPairResident: four waves, the pair's whole window data resident in LDS (small problems,
// mvdr_resident_supported)
constexpr int kPairResident = 2;
bool mvdr_resident_supported(int wmax, int L, int Lt);
hipError_t launch_mvdr_fused(const PairArgs& a, const WindowGeom& g, const DevDesc& d,
                             const float2* Yw, float2* out, float2* wout, int* starts, int* info,
                             int threads, hipStream_t s);
bool mvdr_wave_supported(int wmax);
// Mixed-precision pair kernel: MFMA BF16 covariance (split = BF16 hi/lo, three products;
// else one BF16 product) with FP32 accumulation, FP32 LDL^H and solves, FP64 refinement
// residual and normalisation; ill-conditioned windows routed to FP64 (info bit 30).
// flags: [T][K] int scratch written by the first launch (1 = routed), read by the second.
hipError_t launch_mvdr_mixed(const PairArgs& a, const WindowGeom& g, const DevDesc& d,
                             const float2* Yw, float2* out, float2* wout, int* starts, int* info,
                             int* flags, bool split, hipStream_t s);
// Plain per-stage FP32 form reading the full beamspace Y [K][M][B]: gather + covariance,
// Cholesky + solve, apply -- three launches with R and w in HBM.
hipError_t launch_mvdr_plain(const PairArgs& a, const DevDesc& d, const float2* Y,
                             const int* starts, const double2* abar, float2* R32, float2* w32,
                             float2* out, float2* wout, int* info, hipStream_t s);

struct FullArgs {
  int N, K, L, Lt, B, T, k0, nk;  // subbands k0 .. k0 + nk - 1
  double delta, beta, dl;
  int half_bin;
};
// Full-dimensional element-space MVDR for subbands k0..k0+nk-1 (workspace: R [nk][N][N],
// V [nk][N][T], q [nk][T], wtmp [nk][T][N], FP64).
hipError_t launch_full_mvdr(const FullArgs& a, const DevDesc& d, const float2* X, double2* R,
                            double2* V, double* q, double2* wtmp, float2* out, float2* wout,
                            int* info, hipStream_t s);

// Subband synthesis (inverse channelizer per block): Z [T][K][Lt] -> z [T][Lt*K].
hipError_t launch_synth(const float2* Z, float2* z, int K, int Lt, int T, const float2* twK,
                        const float2* hb, hipStream_t s);
// Lifted correlators c^ [pairs][N] from window weights [pairs][wmax] and starts [pairs]
// (Eq. 21); twM = the M-entry table exp(-j 2 pi q / M).
hipError_t launch_lift(const float2* w, const int* starts, int pairs, int wmax, int N, int M,
                       const float2* twM, float2* c_hat, hipStream_t s);
// Beam outputs out [T][K][Lt] = c^^H X_k[:, L + l] from X [K][B][N] and c^ [T][K][N].
hipError_t launch_lift_apply(const float2* X, const float2* c_hat, float2* out, int N, int K,
                             int B, int L, int Lt, int T, hipStream_t s);

// Planar lifted correlators c^ [T][K][Nz Nx] from window weights [T][K][wmax], starts
// [T][K][2] (s_z, s_x) and window rows wz [T] (device); twM = the M-entry table, M = Mz Mx.
hipError_t launch_lift_upa(const float2* w, const int* starts, const int* wz, int T, int K,
                           int wmax, int Nz, int Nx, int Mz, int Mx, const float2* twM,
                           float2* c_hat, hipStream_t s);
// Planar beam patterns of correlators c [pairs][Nz Nx] (Nz Nx <= 4096) at omega [Q][2]
// = (Omega_z, Omega_x) (device FP64) -> pattern [pairs][Q].
hipError_t launch_beam_pattern_upa(const float2* c, int pairs, int Nz, int Nx,
                                   const double* omega, int Q, float* pattern, hipStream_t s);

// Beam patterns (Eq. 22) of correlators c [pairs][N] (N <= 4096) at angles omega [Q]
// (device FP64) -> pattern [pairs][Q].
hipError_t launch_beam_pattern(const float2* c, int pairs, int N, const double* omega, int Q,
                               float* pattern, hipStream_t s);

// Range-Doppler map and CFAR of pulse trains z [T] (row stride zstride, P pulses of R
// samples), chirp [Lp] (device): power [T][R][P] = |RD|^2, det [T][R][P] in {0, 1};
// work = T P R + 2 F + P complex, F = 2^range_doppler_fft_log(R, Lp) (at most 2^13).
int range_doppler_fft_log(int R, int Lp);
hipError_t launch_range_doppler(const float2* z, int64_t zstride, int T, const float2* chirp,
                                int Lp, int R, int P, int guard, int train, float alpha,
                                float2* work, float* power, unsigned char* det, hipStream_t s);

hipError_t set_fft_attributes();
hipError_t set_pair_attributes();
hipError_t set_full_attributes();

}  // namespace wbm
