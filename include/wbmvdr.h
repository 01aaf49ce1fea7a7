/*
 * wbmvdr.h -- C ABI of the windowed beamspace MVDR library for AMD MI355X (gfx950).
 *
 * The library implements the per-subband windowed beamspace MVDR beamformer of
 * "Scaling Wideband Massive MIMO Radar via Beamspace Dimension Reduction"
 * (Noroozi, Han, Tang, Zhang, Madhow), for a uniform linear array:
 *
 *   element samples x[e][t]          (Sec. II-A, Eq. 9: y[n] per subband)
 *     -> FFT channelizer into K subbands               (Sec. III-A, Fig. 2)
 *     -> zero-padded M-point spatial DFT (beamspace)   (Sec. III-B, Eq. 14-17)
 *     -> W-bin window around each target's beam bin   (Sec. III-B, Eq. 18-19)
 *     -> loaded W x W sample covariance               (Sec. II-B Eq. 11, Sec. III-C)
 *     -> MVDR correlator c = R^-1 a / (a^H R^-1 a)     (Eq. 13, Eq. 20)
 *     -> beam output c^H y on the test snapshots       (Sec. II-B, below Eq. 13)
 *
 * and, as the comparison, full-dimensional element-space MVDR (Sec. II-B, Eq. 11-13).
 *
 * Conventions for every entry point
 * ---------------------------------
 * - Complex data are interleaved float pairs (wbm_c32, identical to torch.complex64)
 *   or double pairs (wbm_c64).  Array pointers documented as "device" must be HIP
 *   device memory; "host" pointers are read synchronously before the call returns.
 *   The caller owns every array it passes; the plan owns its workspace.
 * - Every call validates its arguments before anything is enqueued and returns a
 *   wbm_status; no exception crosses the ABI.  On failure nothing was enqueued and
 *   wbm_last_error() returns a message (thread-local).
 * - Work is enqueued on the given HIP stream (NULL = default stream) and the call
 *   returns without waiting; synchronise the stream before reading outputs.
 * - Numerical failure of one (target, subband) solve does not fail the call: its
 *   info entry is set to j > 0 (factorisation pivot j-1 was not positive/finite),
 *   and its outputs are zero.
 * - A plan is not thread safe; independent plans may be used concurrently.
 *
 * Shapes (ULA, paper's 2-D names in brackets): N elements [N = N_z N_x], M-point
 * spatial DFT [M = M_z M_x], K subbands [the paper's L], L training and Lt test
 * snapshots (blocks of K samples) per subband [n_t], T targets [the paper's K],
 * window widths W_t <= w_max <= 64 [W = W_z W_x].  B = L + Lt, S = B * K.
 */
#ifndef WBMVDR_H
#define WBMVDR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { float re, im; } wbm_c32;
typedef struct { double re, im; } wbm_c64;

typedef enum {
  WBM_OK = 0,
  WBM_ERR_ARG = 1,          /* null pointer / value out of range */
  WBM_ERR_SHAPE = 2,        /* sizes inconsistent with the plan */
  WBM_ERR_NOMEM = 3,        /* device or pinned allocation failed */
  WBM_ERR_HIP = 4,          /* a HIP runtime call failed (text in wbm_last_error) */
  WBM_ERR_UNSUPPORTED = 5   /* valid request the library does not implement */
} wbm_status;

/* wbm_config.flags */
#define WBM_HALF_BIN 1      /* subband centres of Eq. 1: f_c + ((l - 1/2)/K) f_s (pre-twiddle
                               exp(-j pi tau / K) on every block); default: plain FFT bins */

/* form argument of wbm_beamform */
#define WBM_FORM_PLAIN 0    /* per-stage kernels, FP32 arithmetic, one launch per stage, full
                               beamspace written to HBM and gathered per pair */
#define WBM_FORM_FUSED 1    /* beamspace FFT writes only the windows; one fused per-pair
                               covariance -> LDL^H -> solves -> apply launch; FP64
                               accumulation of the covariance and FP64 LDL^H.  Both transforms
                               run in FP64 and store X and the windows in extended precision
                               (an FP32 value plus its BF16-rounded remainder, relative error
                               about 2^-33), so that FP32 rounding of the transforms does not
                               move the weights of scenes with strong interferers */
#define WBM_FORM_GRAPH 2    /* WBM_FORM_FUSED with the launch sequence replayed from a
                               HIP graph (captured on first use for a given argument set) */
#define WBM_FORM_MIXED 3    /* fused sequence with the window covariance on MFMA: each FP32
                               snapshot split into BF16 hi + lo (three BF16 products, FP32
                               accumulation), FP32 LDL^H and solves, one FP64-residual
                               refinement step and FP64 normalisation a^H R^-1 a; windows whose
                               LDL^H pivots span a ratio max d / min d above 1e4 take the FP64
                               path instead and report info bit 30 (info & (1 << 30)) */
#define WBM_FORM_MIXED_BF16 4  /* as WBM_FORM_MIXED with one BF16 product per step (snapshots
                               rounded to BF16); windows are routed to the FP64 path above a
                               pivot ratio of 1e2 (one BF16 product keeps 8 significant bits) */
#define WBM_FORM_FUSED_F32 5   /* WBM_FORM_FUSED with FP32 transforms and FP32 X and windows
                               (fewer bytes; the transforms' rounding then moves the weights
                               by about 0.1 eps32 times the input's dynamic range over the
                               noise floor: fine at moderate interference, not at 50-60 dB
                               jammers on thousands of elements).  The mixed forms also use
                               these FP32 transforms. */
#define WBM_FORM_GRAPH_F32 6   /* WBM_FORM_FUSED_F32 replayed from a HIP graph */
#define WBM_INFO_ROUTED (1 << 30)
#define WBM_INFO_WIDTH (1 << 29)   /* wbm_beamform_pairs: the pair's per-pair width was rejected */

typedef struct {
  int32_t n_elem;           /* N >= 1 */
  int32_t m_fft;            /* M: power of two, max(2, N) <= M <= 8192 */
  int32_t k_sub;            /* K: power of two, 2 <= K <= 8192 */
  int32_t l_train;          /* L >= 1 training snapshots per subband */
  int32_t l_test;           /* Lt >= 0 test snapshots per subband */
  int32_t max_targets;      /* T_max >= 1: capacity for targets per call;
                               T_max * w_max * max(64, 8192 / M) * 8 < 2^32 */
  int32_t w_max;            /* 1 <= w_max <= 64, <= M: largest window width */
  int32_t flags;            /* WBM_HALF_BIN or 0 */
  double beta;              /* fractional bandwidth f_s / f_c, 0 <= beta < 2 */
  double d_over_lambda;     /* element spacing over the centre wavelength (0.5) */
} wbm_config;

typedef struct wbm_plan wbm_plan;

/* Create a plan: validates cfg, allocates the device workspace for the largest
 * problem cfg allows (channelized and beamspace buffers, tables).  *out receives
 * the plan, or NULL on failure. */
wbm_status wbm_plan_create(const wbm_config* cfg, wbm_plan** out);
/* Free a plan and its workspace (synchronises the device first).  NULL is a no-op. */
wbm_status wbm_plan_destroy(wbm_plan* plan);
/* Bytes of device workspace the plan holds. */
int64_t wbm_plan_workspace_bytes(const wbm_plan* plan);

/* Pair kernels of the fused form (values of pair_kernel below). */
#define WBM_PAIR_MFMA 1    /* four waves, covariance on the FP64 matrix cores */
#define WBM_PAIR_WAVE 64   /* one wave per pair on the vector units, w_max <= 40 */
#define WBM_PAIR_BLOCK 256 /* four waves per pair on the vector units */
#define WBM_PAIR_RESIDENT 2 /* four waves, the pair's window data held whole in LDS;
                               w_max * L <= 2304 and w_max * Lt <= 2304 */

/* Precision of the fused sequence a launch configuration applies to. */
#define WBM_PREC_EXT 0     /* WBM_FORM_FUSED / GRAPH, wbm_beamform_pairs, wbm_beamform_learned,
                              wbm_profiles: extended-precision transforms and windows */
#define WBM_PREC_F32 1     /* WBM_FORM_FUSED_F32 / GRAPH_F32, the mixed forms' transforms and the
                              planar-array path */
#define WBM_PREC_MIXED 2      /* wbm_stage_times only: the WBM_FORM_MIXED sequence */
#define WBM_PREC_MIXED_BF16 3 /* wbm_stage_times only: the WBM_FORM_MIXED_BF16 sequence */

/* Launch configuration of the fused form in one precision.  Without a call to
 * wbm_plan_set_tuning the first call of that precision times the candidates on the caller's
 * data (FFT tiles of 2^11..2^13 complex per workgroup for the channelizer and the spatial DFT,
 * 2^10..2^13 in extended precision; the pair kernels; the number of subband chunks over which
 * the spatial DFT and the pair kernel overlap on two streams) and keeps the fastest, cached on
 * disk per device, shape and precision.  Setting pins the choice and skips that search; every
 * choice computes the same quantities (Eq. 4-20), differing only in rounding order.
 *   precision                   WBM_PREC_EXT or WBM_PREC_F32.
 *   chan_logtile, beam_logtile  11, 12 or 13 (WBM_PREC_EXT: 10 .. 13).
 *   pair_kernel                 WBM_PAIR_MFMA, WBM_PAIR_WAVE (needs w_max <= 40),
 *                               WBM_PAIR_BLOCK or WBM_PAIR_RESIDENT (needs
 *                               w_max * L and w_max * Lt <= 2304); WBM_PREC_EXT takes
 *                               WBM_PAIR_WAVE or WBM_PAIR_BLOCK only.
 *   overlap_chunks              1 (no overlap), 2, 4 or 8; K must be a multiple of 8 x chunks.
 * Errors: WBM_ERR_ARG for a NULL plan or a value outside those sets, WBM_ERR_UNSUPPORTED for
 * a pair kernel the precision or the shape does not allow, a chunk count K does not allow, or
 * a tile whose transform needs more than the 160 KiB of LDS of a compute unit at this K or M
 * (the extended channelizer's 2^13 tile at K = 2).  A call whose window rows do not fit beside
 * the pinned spatial-DFT tile runs at, and moves the plan to, the largest smaller tile where
 * they do (see wbm_beamform).
 * A pinned choice drops a captured graph (recaptured on the next graph call); the WBM_PREC_F32
 * choice also fixes the pair kernel of the planar-array path (wbm_beamform_upa).
 * wbm_plan_get_tuning writes the current choice of a precision (NULL pointers skipped). */
wbm_status wbm_plan_set_tuning(wbm_plan* plan, int32_t precision, int32_t chan_logtile,
                               int32_t beam_logtile, int32_t pair_kernel,
                               int32_t overlap_chunks);
wbm_status wbm_plan_get_tuning(const wbm_plan* plan, int32_t precision, int32_t* chan_logtile,
                               int32_t* beam_logtile, int32_t* pair_kernel,
                               int32_t* overlap_chunks);

/* Windowed beamspace MVDR for every (target, subband) pair (Sec. III, Eq. 11-20).
 *   x       device [N][S] wbm_c32: element samples, time contiguous per element.
 *   az_rad  host [T] azimuth of each target from broadside (radians), Eq. 2.
 *   win     host [T] window width W_t per target, 1 <= W_t <= w_max.
 *   T       number of targets, 1 <= T <= max_targets.
 *   loading diagonal loading delta >= 0 added to the 1/L-scaled covariance.
 *   form    WBM_FORM_PLAIN / FUSED / GRAPH / MIXED / MIXED_BF16 / FUSED_F32 / GRAPH_F32.
 *   out     device [T][K][Lt] wbm_c32: beam outputs c^H y on test snapshots L..L+Lt-1.
 *   weights device [T][K][w_max] wbm_c32 or NULL: correlators c~ in window-bin order
 *           (bins (s + i) mod M, i < W_t), zero padded to w_max.
 *   starts  device [T][K] int32 or NULL: first window bin s of every pair (may be
 *           negative; the bins are taken mod M).
 *   info    device [T][K] int32 or NULL: 0, or j > 0 when the pair's factorisation failed at
 *           pivot j-1 (mixed forms: plus WBM_INFO_ROUTED when the FP64 path was taken).
 *   stream  hipStream_t or NULL.
 * Window rows: the windowed spatial DFT of every form but WBM_FORM_PLAIN holds the call's
 * window-row tables in LDS beside its transform tile (4 bytes per window row, 8 per target, 4
 * more per target with M = 8192, N <= 4096 in extended precision; 256 more per target for the
 * learned form's profiles).  A call whose tables do not fit beside the tuned tile runs at, and
 * moves the plan to, the largest smaller tile where they do; at M = 8192 (FP32, or extended
 * with N <= 4096) every tile is 64 KiB, which leaves room for about 24 000 rows.
 * Errors: WBM_ERR_ARG for NULL pointers or a value outside the ranges above, WBM_ERR_SHAPE for T
 * outside [1, max_targets] or window rows that fit no tile (nothing is launched). */
wbm_status wbm_beamform(wbm_plan* plan, const wbm_c32* x, const double* az_rad,
                        const int32_t* win, int32_t T, double loading, int32_t form,
                        wbm_c32* out, wbm_c32* weights, int32_t* starts, int32_t* info,
                        void* stream);

/* Stage: FFT channelizer (Sec. III-A).  x device [N][S] -> X device [K][B][N],
 * X[k][b][e] = K^-1/2 sum_tau x[e][bK + tau] h[tau] exp(-j 2 pi tau k / K),
 * h = 1 or exp(-j pi tau / K) with WBM_HALF_BIN. */
wbm_status wbm_channelize(wbm_plan* plan, const wbm_c32* x, wbm_c32* X, void* stream);

/* Stage: zero-padded spatial DFT (Eq. 14-17).  X device [K][B][N] -> Y device [K][M][B],
 * Y[k][m][b] = M^-1/2 sum_{e<N} X[k][b][e] exp(-j 2 pi m e / M). */
wbm_status wbm_beamspace(wbm_plan* plan, const wbm_c32* X, wbm_c32* Y, void* stream);

/* Lifted correlators (Eq. 21): c^_tk = D^H S_tk^T c~_tk, every pair's windowed weights mapped
 * back to the N elements, c^[n] = M^-1/2 sum_i c~_i exp(+j 2 pi n m_i / M), m_i = (s + i) mod M.
 *   weights device [T][K][w_max] wbm_c32: window-bin order from the pair's start, zero past its
 *           width (as wbm_beamform / wbm_beamform_pairs write them).
 *   starts  device [T][K] int32: each pair's first window bin (may be negative).
 *   c_hat   device [T][K][N] wbm_c32, written.
 * Errors: WBM_ERR_ARG for NULL pointers or T outside [1, max_targets]. */
wbm_status wbm_lift(wbm_plan* plan, const wbm_c32* weights, const int32_t* starts, int32_t T,
                    wbm_c32* c_hat, void* stream);

/* Beam outputs from lifted correlators applied in element space (the remark after Eq. 21: no
 * spatial transform and no window gather): channelizes x into the plan's workspace and writes
 * out[t][k][l] = c^_tk^H X_k[:, L + l] for the Lt test snapshots.
 *   x      device [N][S] wbm_c32 as for wbm_beamform.
 *   c_hat  device [T][K][N] wbm_c32 (e.g. from wbm_lift).
 *   out    device [T][K][Lt] wbm_c32, written.
 * Errors: WBM_ERR_ARG for NULL pointers or T outside [1, max_targets]. */
wbm_status wbm_apply_lifted(wbm_plan* plan, const wbm_c32* x, const wbm_c32* c_hat, int32_t T,
                            wbm_c32* out, void* stream);

/* Beam pattern diagnostic (Eq. 22): for every correlator and angle, the cosine similarity
 * |<c, a(Omega)>| / (||c|| ||a(Omega)||) with the element steering a(Omega)_e = exp(j Omega e).
 *   c       device [pairs][N] wbm_c32 (element-space correlators, e.g. from wbm_lift, or
 *           full-dimensional weights), N = the plan's element count, at most 4096.
 *   omega   device [Q] double: electrical angles Omega (radians per element).
 *   pattern device [pairs][Q] float, written.
 * Errors: WBM_ERR_ARG for NULL pointers or pairs / Q < 1; WBM_ERR_UNSUPPORTED for N > 4096. */
wbm_status wbm_beam_pattern(wbm_plan* plan, const wbm_c32* c, int32_t pairs, const double* omega,
                            int32_t Q, float* pattern, void* stream);

/* Range-Doppler map and 1-D CFAR of beamformed pulse trains (the processing after synthesis,
 * Sec. II and IV; readings of the unstated parameters in the design notes):
 *   z       device [T][z_stride] wbm_c32: per target, P pulses of R samples (z[p R + n]),
 *           e.g. the output of wbm_synthesize; z_stride >= P R.
 *   chirp   device [Lp] wbm_c32: the transmitted pulse, 1 <= Lp <= R.
 *   power   device [T][R][P] float: |RD|^2, RD[d][v] = P^-1/2 sum_p r[p][d] exp(-j 2 pi p v / P)
 *           with r[p][d] = sum_{m < Lp, d + m < R} conj(chirp[m]) z[p R + d + m].
 *   det     device [T][R][P] uint8: 1 where power > 10^(threshold_db / 10) times the mean power
 *           of the cells guard < |d' - d| <= guard + train (inside [0, R)) of the same
 *           velocity bin, else 0.
 *   work    device scratch of T P R + 2 F + P wbm_c32, F = the smallest power of two
 *           >= R + Lp - 1 (at most 8192).
 * Errors: WBM_ERR_ARG for NULL pointers or out-of-range sizes (P must be a power of two in
 * [2, 8192]); WBM_ERR_UNSUPPORTED when F would exceed 8192. */
wbm_status wbm_range_doppler(wbm_plan* plan, const wbm_c32* z, int32_t T, int64_t z_stride,
                             const wbm_c32* chirp, int32_t Lp, int32_t R, int32_t P,
                             int32_t guard, int32_t train, double threshold_db, wbm_c32* work,
                             float* power, uint8_t* det, void* stream);

/* Subband synthesis (the inverse FFT across subbands that recovers the wideband beam output,
 * Sec. II and IV-B): the inverse of the channelizer per test block,
 *   z[t][b K + tau] = K^-1/2 conj(h[tau]) sum_k out[t][k][b] exp(+j 2 pi tau k / K),
 * h as for wbm_channelize, b < Lt.
 *   out device [T][K][Lt] wbm_c32 (beam outputs, e.g. from wbm_beamform).
 *   z   device [T][Lt*K] wbm_c32, written.
 * Errors: WBM_ERR_ARG for NULL pointers or T outside [1, max_targets]. */
wbm_status wbm_synthesize(wbm_plan* plan, const wbm_c32* out, int32_t T, wbm_c32* z,
                          void* stream);

/* Stage: window placement and windowed steering (Eq. 18-19; a~ = S D a below Eq. 20).
 *   starts device [T][K] int32: s = floor(u - (W_t-1)/2 + 1/2), u = M (d/lambda) sin(az) f_k/f_c
 *          evaluated in IEEE double as ((M * dl) * sin(az)) * ratio, ratio = 1 + (beta*(ks+h))/K,
 *          ks the signed bin index, h = 1/2 with WBM_HALF_BIN else 0.
 *   abar   device [T][K][w_max] wbm_c64: a~_i = M^-1/2 sum_{e<N} e^{j Omega e} e^{-j 2 pi m_i e / M}. */
wbm_status wbm_steer(wbm_plan* plan, const double* az_rad, const int32_t* win, int32_t T,
                     int32_t* starts, wbm_c64* abar, void* stream);

/* Planar array (Sec. II-A, Sec. III-B, Eq. 6 and 14-19).  The plan's n_elem = Nz * Nx and
 * m_fft = Mz * Mx describe an Nz x Nx array with an Mz x Mx beam grid; each call names
 *   nz = Nz (dividing n_elem) and mz = Mz (a power of two, Nz <= Mz; Mx = m_fft / mz must
 *   satisfy Nx <= Mx, 2 <= Mx and next_pow2(Nz) * Mx <= 2048).
 * Vectorisation: element (iz, ix) is x row ix Nz + iz (a = a_x kron a_z, Eq. 6); beam
 * (mz, mx) is index mx Mz + mz (D = D_h^T kron D_v, Eq. 16); window cell (iz_w, ix_w) is
 * index ix_w Wz + iz_w of the Wz x Wx window (Eq. 18).  Per axis the window starts at
 * s = floor(u - (W-1)/2 + 1/2) with u_z = Mz (d/lambda) sin(el) f_k/f_c and
 * u_x = Mx (d/lambda) cos(el) sin(az) f_k/f_c (FP64, evaluated as for the linear array from
 * the direction cosines cos(el) * sin(az) and sin(el)), bins mod Mz and Mx.
 * Errors: WBM_ERR_SHAPE for a geometry outside those limits or T outside [1, max_targets],
 * WBM_ERR_ARG for NULL pointers, non-finite angles or windows outside [1, Mz] x [1, Mx] or
 * above w_max. */

/* Windowed beamspace MVDR on the planar array for every (target, subband) pair: as
 * wbm_beamform with the 2-D transform and windows.
 *   az_rad, el_rad  host [T] azimuth and elevation of each target from broadside (radians).
 *   win_z, win_x    host [T] window rows Wz and columns Wx, Wz * Wx <= w_max.
 *   form            WBM_FORM_PLAIN (full planar beamspace in HBM, window cells gathered
 *                   through a beam table, FP32 covariance / Cholesky / apply), WBM_FORM_FUSED,
 *                   WBM_FORM_MIXED or WBM_FORM_MIXED_BF16 (WBM_FORM_GRAPH:
 *                   WBM_ERR_UNSUPPORTED).  The first fused call of a plan times the pair
 *                   kernels on its windows, and the channelizer tiles if the plan is neither
 *                   tuned nor pinned (WBM_AUTOTUNE=0: tile 2^12, the matrix-core kernel);
 *                   wbm_plan_set_tuning pins both.
 *   weights         device [T][K][w_max] or NULL, in window-cell order.
 *   starts          device [T][K][2] int32 or NULL: (s_z, s_x) of every pair.
 *   out, info       as for wbm_beamform. */
wbm_status wbm_beamform_upa(wbm_plan* plan, const wbm_c32* x, int32_t nz, int32_t mz,
                            const double* az_rad, const double* el_rad, const int32_t* win_z,
                            const int32_t* win_x, int32_t T, double loading, int32_t form,
                            wbm_c32* out, wbm_c32* weights, int32_t* starts, int32_t* info,
                            void* stream);

/* Stage: planar beamspace (Eq. 16-17).  X device [K][B][N] -> Y device [K][Mz Mx][B],
 * Y[k][mx Mz + mz][b] = (Mz Mx)^-1/2 sum_{ix<Nx, iz<Nz} X[k][b][ix Nz + iz]
 *                       exp(-j 2 pi (mz iz / Mz + mx ix / Mx)). */
wbm_status wbm_beamspace_upa(wbm_plan* plan, const wbm_c32* X, int32_t nz, int32_t mz,
                             wbm_c32* Y, void* stream);

/* Stage: planar window placement and windowed steering.
 *   starts device [T][K][2] int32 or NULL: (s_z, s_x).
 *   abar   device [T][K][w_max] wbm_c64: a~ = S D a (a of Eq. 6), zero past Wz * Wx. */
wbm_status wbm_steer_upa(wbm_plan* plan, int32_t nz, int32_t mz, const double* az_rad,
                         const double* el_rad, const int32_t* win_z, const int32_t* win_x,
                         int32_t T, int32_t* starts, wbm_c64* abar, void* stream);

/* Planar lifted correlators (Eq. 21 with D = D_h^T kron D_v): every pair's window weights
 * mapped back to the Nz x Nx elements,
 *   c^[ix Nz + iz] = M^-1/2 sum_i c~_i exp(+j 2 pi (mz_i iz / Mz + mx_i ix / Mx)),
 * window cell i = ix_w Wz + iz_w at beam (mz_i, mx_i) = ((s_z + iz_w) mod Mz, (s_x + ix_w) mod Mx).
 *   weights device [T][K][w_max] wbm_c32 (as wbm_beamform_upa writes them, zero past Wz * Wx).
 *   starts  device [T][K][2] int32 (s_z, s_x), as wbm_beamform_upa writes them.
 *   win_z   device [T] int32: each target's window rows Wz.
 *   c_hat   device [T][K][N] wbm_c32, written.  Apply it with wbm_apply_lifted.
 * Errors: WBM_ERR_ARG for NULL pointers or T outside [1, max_targets], WBM_ERR_SHAPE for a
 * geometry outside the planar limits. */
wbm_status wbm_lift_upa(wbm_plan* plan, const wbm_c32* weights, const int32_t* starts,
                        int32_t nz, int32_t mz, const int32_t* win_z, int32_t T, wbm_c32* c_hat,
                        void* stream);

/* Planar beam pattern (Eq. 22 with a = a_x(Omega_x) kron a_z(Omega_z), Eq. 6): for every
 * correlator and direction, |<c, a>| / (||c|| ||a||).
 *   c       device [pairs][N] wbm_c32 (element (iz, ix) at ix Nz + iz), N <= 4096.
 *   omega   device [Q][2] double: (Omega_z, Omega_x) per direction.
 *   pattern device [pairs][Q] float, written.
 * Errors: WBM_ERR_ARG for NULL pointers or pairs / Q < 1, WBM_ERR_SHAPE when nz does not
 * divide N, WBM_ERR_UNSUPPORTED for N > 4096. */
wbm_status wbm_beam_pattern_upa(wbm_plan* plan, const wbm_c32* c, int32_t pairs, int32_t nz,
                                const double* omega, int32_t Q, float* pattern, void* stream);

/* Full-dimensional element-space MVDR per subband (Sec. II-B, Eq. 11-13): the
 * comparison method.  R = (1/L) sum_{b<L} X_b X_b^H + loading I_N (N x N, FP64
 * accumulation), c_t = R^-1 a_t / (a_t^H R^-1 a_t) with a_t the element steering
 * vector of target t at the subband centre (Eq. 7-8), out = c_t^H X_b for the Lt
 * test blocks.  N <= 4096.  Subbands k0 .. k0 + nk - 1 only (nk = 0: all of them; the
 * channelizer still runs over every subband); entries of other subbands are not written.
 *   out device [T][K][Lt]; weights device [T][K][N] or NULL; info device [K] or NULL.
 * Errors: WBM_ERR_ARG for NULL x / out or a subband range outside [0, K). */
wbm_status wbm_full_mvdr(wbm_plan* plan, const wbm_c32* x, const double* az_rad, int32_t T,
                         double loading, int32_t k0, int32_t nk, wbm_c32* out,
                         wbm_c32* weights, int32_t* info, void* stream);

/* Per-stage timing of the fused sequence (same arguments as wbm_beamform with
 * form = WBM_FORM_FUSED for precision WBM_PREC_EXT, WBM_FORM_FUSED_F32 for WBM_PREC_F32,
 * WBM_FORM_MIXED / MIXED_BF16 for WBM_PREC_MIXED / MIXED_BF16; outputs go to plan-internal
 * scratch): launches each stage of it (steer, channelize, windowed beamspace, pair kernel --
 * for the mixed forms the MFMA pair kernel and the FP64 re-solve of the routed windows) once
 * untimed and then `reps` times back to back on `stream` between two HIP events, and writes the
 * average milliseconds per launch to stage_ms (host [4]).  Blocks until the stream has
 * drained.  Window rows as in wbm_beamform (WBM_ERR_SHAPE when they fit no tile). */
wbm_status wbm_stage_times(wbm_plan* plan, const wbm_c32* x, const double* az_rad,
                           const int32_t* win, int32_t T, double loading, int32_t precision,
                           int32_t reps, double* stage_ms, void* stream);

/* ------------------------------------------------------------------------------------
 * Loading / window predictor.  The paper fixes the diagonal loading and the window width;
 * this library adds a small network that picks both per (target, subband) pair from the
 * pair's beamspace power profile, trained on sweeps of the fixed method scored by output
 * SINR.  The fixed method stays the fallback.
 *   Network: 64 -> 128 -> 128 -> 2 multilayer perceptron, GELU (exact erf) after both
 *   hidden layers.  Parameters: one device array of WBM_MLP_PARAMS FP32 values in the order
 *   W1 [128][64], b1 [128], W2 [128][128], b2 [128], W3 [2][128], b3 [2] (row-major, out x in),
 *   used rounded to BF16 (round to nearest even) with FP32 activations and accumulation.
 *   Input: log10(P_j / sigma^2 + 1e-30), P_j the mean power over the L training snapshots of
 *   beamspace bin c - 32 + j (mod M), j < 64, c = floor(u + 1/2) the target's beam bin.
 *   Outputs: out0 = ln(delta / sigma^2), out1 = log2(W - 1); decision delta = sigma^2 *
 *   exp(clamp(out0, ln 0.1, ln 1e4)), W = 2^clamp(rint(out1), 2, 5) + 1 in {5, 9, 17, 33}. */
#define WBM_MLP_PARAMS 25090
#define WBM_PROFILE_BINS 64

/* Training power profiles of every pair: feat device [T][K][64] float (the network input).
 * noise_power = sigma^2 > 0.  The spatial DFT keeps 264 bytes per target in LDS beside its
 * tile; WBM_ERR_SHAPE, with nothing launched, when they fit no tile (as in wbm_beamform). */
wbm_status wbm_profiles(wbm_plan* plan, const wbm_c32* x, const double* az_rad, int32_t T,
                        double noise_power, float* feat, void* stream);

/* Windowed MVDR with a window width and a loading per pair.  Target t's window of win[t]
 * bins (host, as in wbm_beamform) is gathered once; pair (t, k) uses its centred sub-window
 * of pair_win[t][k] bins (device int32) and the loading pair_loading[t][k] (device float,
 * >= 0).  A width outside [1, win[t]] or of the other parity than win[t] is rejected: that
 * pair solves the full window of win[t] bins and its info entry carries WBM_INFO_WIDTH.
 * Outputs, window rows and errors as in wbm_beamform. */
wbm_status wbm_beamform_pairs(wbm_plan* plan, const wbm_c32* x, const double* az_rad,
                              const int32_t* win, int32_t T, const int32_t* pair_win,
                              const float* pair_loading, wbm_c32* out, wbm_c32* weights,
                              int32_t* starts, int32_t* info, void* stream);

/* Learned form: profiles -> network -> per-pair (delta, W) -> windowed MVDR, one call.
 * Needs w_max >= 33.  params device [WBM_MLP_PARAMS].  A pair whose network output is not
 * finite uses fallback_win / fallback_loading (odd fallback_win <= 33).  pair_win,
 * pair_loading (device [T][K], may be NULL) receive the decisions; fallback (device [T][K]
 * int32, may be NULL) is 1 where the fallback was used.  Window rows (33 per target) and the
 * profiles' LDS as in wbm_beamform and wbm_profiles: WBM_ERR_SHAPE when they fit no tile. */
wbm_status wbm_beamform_learned(wbm_plan* plan, const wbm_c32* x, const double* az_rad,
                                int32_t T, const float* params, double noise_power,
                                int32_t fallback_win, double fallback_loading, wbm_c32* out,
                                wbm_c32* weights, int32_t* pair_win, float* pair_loading,
                                int32_t* fallback, int32_t* starts, int32_t* info,
                                void* stream);

/* Output SINR of weights (device [T][K][w_max], window-bin order starting at starts[t][k],
 * width pair_win[t][k] or win[t] if pair_win is NULL; a width wbm_beamform_pairs rejects
 * counts as win[t], and no width counts past w_max) against the exact covariance of white
 * noise sigma^2 plus J white jammers (host jam_az [J] radians, jam_inr [J] linear per
 * element): |w^H a~|^2 / (w^H (S D R_in D^H S^T) w).  sinr device [T][K] float. */
wbm_status wbm_sinr(wbm_plan* plan, const double* az_rad, const int32_t* win, int32_t T,
                    const wbm_c32* weights, const int32_t* pair_win, const int32_t* starts,
                    const double* jam_az, const double* jam_inr, int32_t J, double noise_power,
                    float* sinr, void* stream);

typedef struct wbm_mlp wbm_mlp;
/* Network workspace for batches of up to max_batch samples. */
wbm_status wbm_mlp_create(int32_t max_batch, wbm_mlp** out);
wbm_status wbm_mlp_destroy(wbm_mlp* mlp);
/* out device [n][2] = network(in device [n][64]). */
wbm_status wbm_mlp_forward(wbm_mlp* mlp, const float* params, const float* in, int32_t n,
                           float* out, void* stream);
/* grad device [WBM_MLP_PARAMS] and loss device [1] of the mean squared error over the n
 * samples and both outputs against target device [n][2]; deterministic reduction order. */
wbm_status wbm_mlp_grad(wbm_mlp* mlp, const float* params, const float* in, const float* target,
                        int32_t n, float* grad, float* loss, void* stream);
/* wbm_mlp_grad without a network workspace, for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * gradient and loss partials live in a static device array of the library (about 25.7 MB
 * per device, held until the process ends) instead of a wbm_mlp.  No allocation happens in
 * the call; the first call on a device looks up the array's address there (not a stream
 * operation; make that first call before capturing).  Same kernels and reduction order as
 * wbm_mlp_grad, so the same results bit for bit.  loss may be NULL.  Calls that overlap on
 * one device (other streams, other threads) share the array and race: serialise them.
 * Errors: WBM_ERR_ARG for NULL params / in / target / grad, WBM_ERR_SHAPE for n outside
 * [1, WBM_MLP_STATIC_MAX_BATCH]; nothing is enqueued then. */
#define WBM_MLP_STATIC_MAX_BATCH 4096
wbm_status wbm_mlp_grad_static(const float* params, const float* in, const float* target,
                               int32_t n, float* grad, float* loss, void* stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8; step counts from 1) on params with moment
 * arrays m, v (device [WBM_MLP_PARAMS]). */
wbm_status wbm_mlp_adam(wbm_mlp* mlp, float* params, float* m, float* v, const float* grad,
                        int32_t step, double lr, void* stream);
/* Labels of a sweep: sinr device [nd * nw][npairs] (row c = id * nw + iw for loading
 * deltas[id] and width widths[iw], host arrays) -> label device [npairs][2] =
 * (ln(delta / sigma^2), log2(W - 1)) of the best SINR; ties go to the smaller width, then to
 * the larger loading.  nd, nw <= 64. */
wbm_status wbm_sweep_labels(wbm_mlp* mlp, const float* sinr, int32_t npairs, const double* deltas,
                            int32_t nd, const int32_t* widths, int32_t nw, double noise_power,
                            float* label, void* stream);

const char* wbm_status_str(wbm_status s);
const char* wbm_last_error(void);
/* Library version string. */
const char* wbm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* WBMVDR_H */
