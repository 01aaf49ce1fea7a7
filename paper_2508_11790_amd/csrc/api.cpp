// C ABI of the windowed beamspace MVDR library: argument validation, plan / workspace
// management, per-call target description upload and the launch sequences.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <sys/stat.h>
#include <vector>

#include "wbm_launch.h"
#include "wbm_learned.h"
#include "wbmvdr.h"

namespace {

thread_local std::string g_err;

wbm_status fail(wbm_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

wbm_status hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return WBM_ERR_HIP;
}

#define WBM_HIP(call, what)                  \
  do {                                       \
    hipError_t e_ = (call);                  \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

int ilog2i(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

constexpr int kMaxOverlap = 8;

struct GraphKey {
  int prec = 0;
  const void* x = nullptr;
  void* out = nullptr;
  void* weights = nullptr;
  void* info = nullptr;
  void* starts = nullptr;
  int T = 0, sumW = 0;
  double loading = 0.0;
  bool valid = false;
  bool operator==(const GraphKey& o) const {
    return valid && o.valid && prec == o.prec && x == o.x && out == o.out && weights == o.weights && info == o.info &&
           starts == o.starts && T == o.T && sumW == o.sumW && loading == o.loading;
  }
};

}  // namespace

// Precision of the fused sequence's intermediates: extended (FP64 transforms, hi + lo storage
// of X and the windows) or FP32.
constexpr int kExt = 0, kF32 = 1;

// Launch configuration of the fused sequence in one precision.
struct Tuning {
  int chan_logtile = 12, beam_logtile = 12;
  int logTB = 0, TB = 0, nbt = 0;     // beamspace tile (snapshots per workgroup)
  int pair_threads = WBM_PAIR_BLOCK;  // pair kernel: WBM_PAIR_*
  int overlap = 1;                    // subband chunks overlapping beamspace and pair kernels
  bool tuned = false;                 // timed by the autotuner or pinned
};

struct wbm_plan {
  wbm_config cfg;
  int B = 0;
  int64_t S = 0;
  Tuning tune[2];                     // [kExt], [kF32]
  int upa_pair = WBM_PAIR_MFMA;       // pair kernel of the planar-array path (timed on first use)
  bool upa_tuned = false;
  // second stream of the overlapped fused sequence and its fork / join events
  hipStream_t side_stream = nullptr;
  hipEvent_t chunk_evt[kMaxOverlap + 1] = {};
  int device = 0;
  // tables
  float2* twK = nullptr;
  float2* twM = nullptr;
  float2* hb = nullptr;
  double2* twK64 = nullptr;  // FP64 tables of the extended-precision transforms (first use)
  double2* twM64 = nullptr;
  double2* hb64 = nullptr;
  // per-call target description: device copy + pinned staging
  unsigned char* desc_dev = nullptr;
  unsigned char* desc_host = nullptr;
  size_t desc_bytes = 0;
  hipEvent_t desc_evt = nullptr;
  bool desc_evt_recorded = false;
  // the descriptor last uploaded and the stream it went on: an identical descriptor (the same
  // targets as the previous call) is not uploaded again
  std::vector<unsigned char> desc_next, desc_last;
  hipStream_t desc_stream = nullptr;
  wbm::DevDesc dd{};
  // workspace
  float2* X = nullptr;       // [K][B][N] (extended precision: the FP32 hi part)
  float2* Yw = nullptr;      // [K][nbt][T_max*w_max][TB] (extended precision: hi part)
  uint32_t* Xl = nullptr;    // [K][B][N] BF16 remainders of X (extended precision, first use)
  uint32_t* Ywl = nullptr;   // BF16 remainders of the windows, Yw's layout (first use)
  float2* Y = nullptr;       // [K][M][B]      (plain form, allocated on first use)
  float2* R32 = nullptr;     // [T_max*K][w_max^2] (plain form)
  float2* w32 = nullptr;     // [T_max*K][w_max]   (plain form)
  int* starts = nullptr;     // [T_max][K]
  double2* abar = nullptr;   // [T_max][K][w_max]
  double2* fullR = nullptr;  // [nk_full][N][N] (full-dimensional MVDR, first use)
  double2* fullW = nullptr;  // [nk_full][T_max][N]
  double2* fullV = nullptr;  // [nk_full][N][T_max] (blocked solves)
  double* fullQ = nullptr;   // [nk_full][T_max]
  int* full_info = nullptr;  // [K]
  int nk_full = 0;
  int64_t ws_bytes = 0;
  size_t yw_elems = 0;       // complex entries of Yw (and of Ywl)
  // graph replay of the fused sequence
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec = nullptr;
  GraphKey gkey;
  // scratch outputs of wbm_stage_times
  float2* prof_out = nullptr;
  float2* prof_w = nullptr;
  int* prof_info = nullptr;
  int* route = nullptr;      // [T_max][K] mixed forms: windows routed to the FP64 kernel
  int* upa_rows = nullptr;   // [T_max][K][w_max] planar plain form: beam of every window cell
  // loading / window predictor buffers (first use)
  float* pprof = nullptr;    // [K][G][T_max][64] power-profile partials
  float* feat = nullptr;     // [T_max][K][64]
  float* nnout = nullptr;    // [T_max][K][2]
  int* pw = nullptr;         // [T_max][K]
  float* pdelta = nullptr;   // [T_max][K]
  int prof_G = 0;
  // jammer list for SINR scoring: device + pinned staging
  double* jam_dev = nullptr;
  double* jam_host = nullptr;
  hipEvent_t jam_evt = nullptr;
  bool jam_evt_recorded = false;
};

struct wbm_mlp {
  int max_batch = 0;
  float* part = nullptr;       // [workgroups][params]
  float* loss_part = nullptr;  // [workgroups]
  unsigned char* tab_dev = nullptr;   // label sweep tables: 64 floats + 64 ints
  unsigned char* tab_host = nullptr;
  hipEvent_t tab_evt = nullptr;
  bool tab_evt_recorded = false;
  int device = 0;
};

namespace {

template <typename T>
wbm_status dev_alloc(wbm_plan* p, T** ptr, size_t count, const char* what) {
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, sizeof(T) * (count ? count : 1));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(WBM_ERR_NOMEM, std::string("hipMalloc failed for ") + what + " (" +
                                   std::to_string(sizeof(T) * count) + " bytes)");
  }
  *ptr = static_cast<T*>(q);
  p->ws_bytes += (int64_t)(sizeof(T) * count);
  return WBM_OK;
}

wbm_status upload_twiddles(float2* dst, int n, double sign_frac) {
  // dst[q] = exp(-2 pi i q / n) (sign_frac = 1) or the half-bin pre-twiddle exp(-i pi q / n)
  std::vector<float2> h(n);
  for (int q = 0; q < n; ++q) {
    const double ang = -2.0 * M_PI * (double)q / (double)n * sign_frac;
    h[q] = make_float2((float)std::cos(ang), (float)std::sin(ang));
  }
  WBM_HIP(hipMemcpy(dst, h.data(), sizeof(float2) * n, hipMemcpyHostToDevice), "twiddle upload");
  return WBM_OK;
}

wbm_status upload_twiddles64(double2* dst, int n, double sign_frac) {
  // the FP64 tables of the extended-precision transforms, from long double sin / cos
  std::vector<double2> h(n);
  for (int q = 0; q < n; ++q) {
    const long double ang = -2.0L * 3.141592653589793238462643383279502884L * (long double)q /
                            (long double)n * (long double)sign_frac;
    h[q] = make_double2((double)std::cos(ang), (double)std::sin(ang));
  }
  WBM_HIP(hipMemcpy(dst, h.data(), sizeof(double2) * n, hipMemcpyHostToDevice), "twiddle upload");
  return WBM_OK;
}

// Byte offsets of the per-call descriptor: FP64 arrays first, then the int arrays.
struct DescLayout {
  size_t sin_az, cz, win, woff, rowtab, torder, wz, bytes;
};

DescLayout desc_layout(int Tm, int wmax) {
  DescLayout l;
  l.sin_az = 0;
  l.cz = l.sin_az + sizeof(double) * Tm;
  l.win = l.cz + sizeof(double) * Tm;
  l.woff = l.win + sizeof(int) * Tm;
  l.rowtab = l.woff + sizeof(int) * Tm;
  l.torder = l.rowtab + sizeof(int) * (size_t)Tm * wmax;
  l.wz = l.torder + sizeof(int) * Tm;
  l.bytes = l.wz + sizeof(int) * Tm;
  return l;
}

// Window offsets, window-row table and pair order of the staged descriptor from the widths
// already in it; returns sumW.
int desc_rows(wbm_plan* p, int T) {
  const DescLayout l = desc_layout(p->cfg.max_targets, p->cfg.w_max);
  unsigned char* buf = p->desc_next.data();
  const int* wv = reinterpret_cast<const int*>(buf + l.win);
  int* woff = reinterpret_cast<int*>(buf + l.woff);
  int* rowtab = reinterpret_cast<int*>(buf + l.rowtab);
  int* torder = reinterpret_cast<int*>(buf + l.torder);
  int sumW = 0;
  for (int t = 0; t < T; ++t) {
    woff[t] = sumW;
    for (int i = 0; i < wv[t]; ++i) rowtab[sumW + i] = (t << 8) | i;
    sumW += wv[t];
    torder[t] = t;
  }
  // pair kernels take the widest windows first (longest-processing-time order): workgroups
  // are handed out in index order, so the expensive pairs start early and spread evenly
  std::stable_sort(torder, torder + T, [wv](int x, int y) { return wv[x] > wv[y]; });
  return sumW;
}

// Upload the staged descriptor, unless the device copy already holds these bytes (the same
// targets as the previous call, on the same stream, outside graph capture).
wbm_status commit_desc(wbm_plan* p, hipStream_t st) {
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  WBM_HIP(hipStreamIsCapturing(st, &cap), "capture query");
  if (p->desc_evt_recorded && st == p->desc_stream && cap == hipStreamCaptureStatusNone &&
      p->desc_next == p->desc_last) {
    // the device copy already holds these bytes (or will, in this stream's order)
    return WBM_OK;
  }
  if (p->desc_evt_recorded) {
    WBM_HIP(hipEventSynchronize(p->desc_evt), "descriptor staging wait");
  }
  std::memcpy(p->desc_host, p->desc_next.data(), p->desc_bytes);
  WBM_HIP(hipMemcpyAsync(p->desc_dev, p->desc_host, p->desc_bytes, hipMemcpyHostToDevice, st),
          "descriptor upload");
  WBM_HIP(hipEventRecord(p->desc_evt, st), "descriptor event");
  p->desc_evt_recorded = true;
  p->desc_last.swap(p->desc_next);
  p->desc_stream = st;
  return WBM_OK;
}

// Validate the per-call targets and upload their description; returns sumW.
wbm_status upload_desc(wbm_plan* p, const double* az_rad, const int32_t* win, int T,
                       hipStream_t st, int* sumW_out) {
  const wbm_config& c = p->cfg;
  if (!az_rad) return fail(WBM_ERR_ARG, "az_rad is NULL");
  if (T < 1 || T > c.max_targets)
    return fail(WBM_ERR_SHAPE, "T=" + std::to_string(T) + " outside [1, max_targets=" +
                                   std::to_string(c.max_targets) + "]");
  for (int t = 0; t < T; ++t) {
    if (!std::isfinite(az_rad[t])) return fail(WBM_ERR_ARG, "az_rad[" + std::to_string(t) + "] not finite");
    if (win) {
      const int W = win[t];
      if (W < 1 || W > c.w_max)
        return fail(WBM_ERR_ARG, "win[" + std::to_string(t) + "]=" + std::to_string(W) +
                                     " outside [1, w_max=" + std::to_string(c.w_max) + "]");
    }
  }
  const DescLayout l = desc_layout(c.max_targets, c.w_max);
  p->desc_next.assign(p->desc_bytes, 0);
  unsigned char* buf = p->desc_next.data();
  double* sin_az = reinterpret_cast<double*>(buf + l.sin_az);
  int* wv = reinterpret_cast<int*>(buf + l.win);
  for (int t = 0; t < T; ++t) {
    sin_az[t] = std::sin(az_rad[t]);
    wv[t] = win ? win[t] : c.w_max;
  }
  *sumW_out = desc_rows(p, T);
  return commit_desc(p, st);
}

// Planar array: validate the geometry (nz rows, mz-point vertical DFT) and the targets, and
// upload their description (direction cosines, Wz * Wx windows); returns sumW.
wbm_status check_upa_shape(const wbm_plan* p, int nz, int mz) {
  const wbm_config& c = p->cfg;
  if (nz < 1 || c.n_elem % nz != 0)
    return fail(WBM_ERR_SHAPE, "nz=" + std::to_string(nz) + " must divide n_elem=" +
                                   std::to_string(c.n_elem));
  if (!is_pow2(mz) || mz < nz || c.m_fft % mz != 0)
    return fail(WBM_ERR_SHAPE, "mz=" + std::to_string(mz) +
                                   " must be a power of two with nz <= mz, dividing m_fft");
  const int nx = c.n_elem / nz, mx = c.m_fft / mz;
  int pz = 1;
  while (pz < nz) pz <<= 1;
  if (mx < 2 || mx < nx || (int64_t)pz * mx > 2048)
    return fail(WBM_ERR_SHAPE, "need 2 <= m_fft/mz, n_elem/nz <= m_fft/mz and next_pow2(nz) * "
                               "(m_fft/mz) <= 2048 (got nx=" + std::to_string(nx) + ", mx=" +
                               std::to_string(mx) + ")");
  return WBM_OK;
}

wbm_status upload_desc_upa(wbm_plan* p, int nz, int mz, const double* az_rad,
                           const double* el_rad, const int32_t* win_z, const int32_t* win_x,
                           int T, hipStream_t st, int* sumW_out) {
  const wbm_config& c = p->cfg;
  wbm_status s = check_upa_shape(p, nz, mz);
  if (s) return s;
  const int mx = c.m_fft / mz;
  if (!az_rad || !el_rad || !win_z || !win_x)
    return fail(WBM_ERR_ARG, "az_rad / el_rad / win_z / win_x is NULL");
  if (T < 1 || T > c.max_targets)
    return fail(WBM_ERR_SHAPE, "T=" + std::to_string(T) + " outside [1, max_targets=" +
                                   std::to_string(c.max_targets) + "]");
  for (int t = 0; t < T; ++t) {
    const std::string ts = "[" + std::to_string(t) + "]";
    if (!std::isfinite(az_rad[t]) || !std::isfinite(el_rad[t]))
      return fail(WBM_ERR_ARG, "az_rad / el_rad" + ts + " not finite");
    if (win_z[t] < 1 || win_z[t] > mz || win_x[t] < 1 || win_x[t] > mx ||
        win_z[t] * win_x[t] > c.w_max)
      return fail(WBM_ERR_ARG, "window" + ts + " = " + std::to_string(win_z[t]) + " x " +
                                   std::to_string(win_x[t]) + " outside [1, mz] x [1, m_fft/mz]"
                                   " or above w_max=" + std::to_string(c.w_max));
  }
  const DescLayout l = desc_layout(c.max_targets, c.w_max);
  p->desc_next.assign(p->desc_bytes, 0);
  unsigned char* buf = p->desc_next.data();
  double* cx = reinterpret_cast<double*>(buf + l.sin_az);
  double* cz = reinterpret_cast<double*>(buf + l.cz);
  int* wv = reinterpret_cast<int*>(buf + l.win);
  int* wz = reinterpret_cast<int*>(buf + l.wz);
  for (int t = 0; t < T; ++t) {
    cx[t] = std::cos(el_rad[t]) * std::sin(az_rad[t]);
    cz[t] = std::sin(el_rad[t]);
    wv[t] = win_z[t] * win_x[t];
    wz[t] = win_z[t];
  }
  *sumW_out = desc_rows(p, T);
  return commit_desc(p, st);
}

wbm_status ensure_plain(wbm_plan* p) {
  if (p->Y) return WBM_OK;
  const wbm_config& c = p->cfg;
  wbm_status s = dev_alloc(p, &p->Y, (size_t)c.k_sub * c.m_fft * p->B, "beamspace Y");
  if (s) return s;
  const size_t pairs = (size_t)c.max_targets * c.k_sub;
  s = dev_alloc(p, &p->R32, pairs * c.w_max * c.w_max, "plain covariances");
  if (s) return s;
  return dev_alloc(p, &p->w32, pairs * c.w_max, "plain weights");
}

// scratch outputs for timing runs (autotuner, wbm_stage_times)
wbm_status ensure_prof(wbm_plan* p) {
  if (p->prof_out) return WBM_OK;
  const wbm_config& c = p->cfg;
  const size_t pairs = (size_t)c.max_targets * c.k_sub;
  wbm_status s;
  if ((s = dev_alloc(p, &p->prof_out, pairs * (size_t)(c.l_test ? c.l_test : 1), "timing outputs")))
    return s;
  if ((s = dev_alloc(p, &p->prof_w, pairs * (size_t)c.w_max, "timing weights"))) return s;
  return dev_alloc(p, &p->prof_info, pairs, "timing info");
}

wbm::PairArgs pair_args(const wbm_plan* p, int prec, int T, int sumW, double loading) {
  wbm::PairArgs a;
  a.T = T;
  a.K = p->cfg.k_sub;
  a.M = p->cfg.m_fft;
  a.L = p->cfg.l_train;
  a.Lt = p->cfg.l_test;
  a.B = p->B;
  a.wmax = p->cfg.w_max;
  a.logTB = p->tune[prec].logTB;
  a.nbt = p->tune[prec].nbt;
  a.sumW = sumW;
  a.delta = loading;
  a.ywl = prec == kExt ? p->Ywl : nullptr;
  a.split_rows = (prec == kExt && wbm::beamspace_x_split_rows(p->cfg.n_elem, p->cfg.m_fft)) ? 1 : 0;
  return a;
}

wbm::WindowGeom geom(const wbm_plan* p, int T) {
  wbm::WindowGeom g;
  g.T = T;
  g.K = p->cfg.k_sub;
  g.M = p->cfg.m_fft;
  g.N = p->cfg.n_elem;
  g.half_bin = (p->cfg.flags & WBM_HALF_BIN) ? 1 : 0;
  g.beta = p->cfg.beta;
  g.dl = p->cfg.d_over_lambda;
  g.sin_az = p->dd.sin_az;
  g.win = p->dd.win;
  return g;
}

// Geometry of a planar-array call (nz, mz validated by upload_desc_upa or check_upa_shape).
wbm::UpaGeom upa_geom(const wbm_plan* p, int T, int nz, int mz) {
  wbm::UpaGeom g;
  g.T = T;
  g.K = p->cfg.k_sub;
  g.Nz = nz;
  g.Nx = p->cfg.n_elem / nz;
  g.Mz = mz;
  g.Mx = p->cfg.m_fft / mz;
  g.half_bin = (p->cfg.flags & WBM_HALF_BIN) ? 1 : 0;
  g.beta = p->cfg.beta;
  g.dl = p->cfg.d_over_lambda;
  g.cx = p->dd.sin_az;
  g.cz = p->dd.cz;
  g.win = p->dd.win;
  g.wz = p->dd.wz;
  return g;
}

bool resident_ok(const wbm_plan* p) {
  return wbm::mvdr_resident_supported(p->cfg.w_max, p->cfg.l_train, p->cfg.l_test);
}

void set_beam_tile(wbm_plan* p, int prec, int logtile) {
  Tuning& t = p->tune[prec];
  t.beam_logtile = logtile;
  t.logTB = wbm::beamspace_tile_log(p->cfg.m_fft, logtile);
  t.TB = 1 << t.logTB;
  t.nbt = (p->B + t.TB - 1) / t.TB;
}

// LDS of the windowed spatial DFT at this tile for a call with T targets and sumW window rows.
size_t beam_lds(const wbm_plan* p, int prec, int logtile, int T, int sumW, bool windows,
                bool prof) {
  return wbm::beamspace_lds_bytes(prec == kExt, p->cfg.n_elem, p->cfg.m_fft, logtile, T, sumW,
                                  windows, prof);
}

// The spatial DFT holds a call's window-row tables in LDS beside its transform tile: keep the
// tuned tile if they fit there, else move the plan to the largest smaller tile where they do
// (the pair kernels follow the tile's window layout); WBM_ERR_SHAPE if none does.
wbm_status fit_beam_tile(wbm_plan* p, int prec, int T, int sumW, bool windows, bool prof) {
  const int cur = p->tune[prec].beam_logtile;
  if (beam_lds(p, prec, cur, T, sumW, windows, prof) <= wbm::kLdsBytes) return WBM_OK;
  for (int lt = cur - 1; lt >= (prec == kExt ? 10 : 11); --lt) {
    if (beam_lds(p, prec, lt, T, sumW, windows, prof) <= wbm::kLdsBytes) {
      set_beam_tile(p, prec, lt);
      return WBM_OK;
    }
  }
  return fail(WBM_ERR_SHAPE, "the window rows of this call (" + std::to_string(sumW) +
                                 " rows of " + std::to_string(T) +
                                 " targets) do not fit the spatial DFT's LDS at any tile");
}

bool logtile_ok(int prec, int logtile) {
  return prec == kExt ? wbm::fft_x_logtile_supported(logtile)
                      : wbm::fft_logtile_supported(logtile);
}

// Workspace of the extended-precision intermediates: the BF16 remainder planes of X and the
// windows, and the FP64 twiddle tables.
wbm_status ensure_ext(wbm_plan* p) {
  if (p->Xl) return WBM_OK;
  const wbm_config& c = p->cfg;
  wbm_status s;
  if ((s = dev_alloc(p, &p->twK64, c.k_sub, "FP64 twiddles K"))) return s;
  if ((s = dev_alloc(p, &p->twM64, c.m_fft, "FP64 twiddles M"))) return s;
  if ((s = dev_alloc(p, &p->hb64, c.k_sub, "FP64 half-bin twiddles"))) return s;
  if ((s = upload_twiddles64(p->twK64, c.k_sub, 1.0))) return s;
  if ((s = upload_twiddles64(p->twM64, c.m_fft, 1.0))) return s;
  if ((s = upload_twiddles64(p->hb64, c.k_sub, 0.5))) return s;
  if ((s = dev_alloc(p, &p->Ywl, p->yw_elems, "window remainders"))) return s;
  return dev_alloc(p, &p->Xl, (size_t)c.n_elem * p->S, "X remainders");
}

hipError_t enqueue_channelize(wbm_plan* p, int prec, const float2* x, hipStream_t st) {
  const wbm_config& c = p->cfg;
  const bool hb = (c.flags & WBM_HALF_BIN) != 0;
  if (prec == kExt)
    return wbm::launch_channelize_x(x, p->X, p->Xl, c.n_elem, c.k_sub, p->B, p->twK64,
                                    hb ? p->hb64 : nullptr, p->tune[kExt].chan_logtile, st);
  return wbm::launch_channelize(x, p->X, c.n_elem, c.k_sub, p->B, p->twK, hb ? p->hb : nullptr,
                                p->tune[kF32].chan_logtile, st);
}

// Windowed spatial DFT of subbands k0 .. k0 + kc - 1 (kc < 0: all), optionally with the
// training power-profile partials (prof, G workgroups per subband).
hipError_t enqueue_beamspace_windows(wbm_plan* p, int prec, int T, int sumW, hipStream_t st,
                                     int k0 = 0, int kc = -1, bool windows = true,
                                     float* prof = nullptr, int G = 0) {
  const wbm_config& c = p->cfg;
  const Tuning& t = p->tune[prec];
  const int L = prof ? c.l_train : 0;
  if (prec == kExt)
    return wbm::launch_beamspace_x(p->X, p->Xl, windows ? p->Yw : nullptr,
                                   windows ? p->Ywl : nullptr, c.n_elem, c.m_fft, p->B, c.k_sub,
                                   p->twM64, p->dd.rowtab, sumW, geom(p, T), t.beam_logtile, st,
                                   prof, L, G, k0, kc);
  return wbm::launch_beamspace(p->X, nullptr, windows ? p->Yw : nullptr, c.n_elem, c.m_fft, p->B,
                               c.k_sub, p->twM, p->dd.rowtab, sumW, geom(p, T), t.beam_logtile,
                               st, prof, L, G, k0, kc);
}

bool overlap_supported(const wbm_plan* p, int chunks) {
  return chunks == 1 || (chunks >= 2 && chunks <= kMaxOverlap && (chunks & (chunks - 1)) == 0 &&
                         p->cfg.k_sub % (8 * chunks) == 0);
}


// Channelize -> windowed beamspace -> fused MVDR on stream st (the beamspace and pair
// kernels place the windows themselves).  With C > 1 overlap chunks the subbands are split in
// C ranges: the pair kernel of range c runs on the plan's second stream while the beamspace
// kernel of range c + 1 streams on st (the first is HBM-bound, the second latency- or
// FP64-bound), joined back into st at the end; under graph capture this becomes a fork / join.
hipError_t enqueue_fused(wbm_plan* p, int prec, const float2* x, int T, int sumW,
                         double loading, float2* out, float2* wout, int* starts, int* info,
                         hipStream_t st, int chunks) {
  hipError_t e = enqueue_channelize(p, prec, x, st);
  if (e != hipSuccess) return e;
  const wbm_config& c = p->cfg;
  const int thr = p->tune[prec].pair_threads;
  if (chunks <= 1 || !overlap_supported(p, chunks)) {
    e = enqueue_beamspace_windows(p, prec, T, sumW, st);
    if (e != hipSuccess) return e;
    return wbm::launch_mvdr_fused(pair_args(p, prec, T, sumW, loading), geom(p, T), p->dd, p->Yw,
                                  out, wout, starts, info, thr, st);
  }
  // the side stream and its events exist from plan creation on: nothing is created here, where
  // st may be capturing
  const int kc = c.k_sub / chunks;
  for (int ch = 0; ch < chunks && e == hipSuccess; ++ch) {
    e = enqueue_beamspace_windows(p, prec, T, sumW, st, ch * kc, kc);
    if (e == hipSuccess) e = hipEventRecord(p->chunk_evt[ch], st);
    if (e == hipSuccess) e = hipStreamWaitEvent(p->side_stream, p->chunk_evt[ch], 0);
    if (e == hipSuccess) {
      wbm::PairArgs a = pair_args(p, prec, T, sumW, loading);
      a.k0 = ch * kc;
      a.kc = kc;
      e = wbm::launch_mvdr_fused(a, geom(p, T), p->dd, p->Yw, out, wout, starts, info, thr,
                                 p->side_stream);
    }
  }
  if (e == hipSuccess) e = hipEventRecord(p->chunk_evt[chunks], p->side_stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(st, p->chunk_evt[chunks], 0);
  return e;
}

hipError_t enqueue_fused(wbm_plan* p, int prec, const float2* x, int T, int sumW,
                         double loading, float2* out, float2* wout, int* starts, int* info,
                         hipStream_t st) {
  return enqueue_fused(p, prec, x, T, sumW, loading, out, wout, starts, info, st,
                       p->tune[prec].overlap);
}

// ---------------------------------------------------------------------------------------------
// Autotuner: times every supported tile size of the channelizer and the windowed beamspace
// kernel, every pair kernel and the overlap chunk counts on the plan's own shape (HIP events,
// time_best) and keeps the fastest.  Results are cached in a JSON file keyed by device and
// shape ($WBM_AUTOTUNE_CACHE, default ~/.cache/wbmvdr/autotune.json); WBM_AUTOTUNE=0
// disables tuning (tile 2^12).

std::string tune_key(const wbm_plan* p, int prec) {
  hipDeviceProp_t prop;
  std::string arch = "gpu";
  if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) arch = prop.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch = arch.substr(0, colon);
  const wbm_config& c = p->cfg;
  std::ostringstream os;
  os << arch << "/N" << c.n_elem << "/M" << c.m_fft << "/K" << c.k_sub << "/B" << p->B << "/L"
     << c.l_train << "/T" << c.max_targets << "/W" << c.w_max
     << (prec == kExt ? "/x1" : "/f7");
  return os.str();
}

std::string cache_path() {
  const char* env = std::getenv("WBM_AUTOTUNE_CACHE");
  if (env && *env) return env;
  const char* home = std::getenv("HOME");
  return std::string(home ? home : "/tmp") + "/.cache/wbmvdr/autotune.json";
}

// The cache file is a flat JSON object
// {"key": [chan_logtile, beam_logtile, pair_kernel, overlap_chunks], ...}
// (pair_kernel: 1 = FP64 matrix-core kernel, 2 = LDS-resident kernel, 64 / 256 = vector kernel
// with that many threads).
bool cache_lookup(const std::string& key, int prec, int* chan, int* beam, int* thr, int* ovl) {
  std::ifstream f(cache_path());
  if (!f) return false;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string txt = ss.str();
  const std::string pat = "\"" + key + "\": [";
  const size_t pos = txt.find(pat);
  if (pos == std::string::npos) return false;
  int a = 0, b = 0, c = 0, o = 0;
  if (std::sscanf(txt.c_str() + pos + pat.size(), "%d, %d, %d, %d", &a, &b, &c, &o) != 4)
    return false;
  if (!logtile_ok(prec, a) || !logtile_ok(prec, b)) return false;
  if (c != WBM_PAIR_WAVE && c != WBM_PAIR_BLOCK &&
      (prec == kExt || (c != WBM_PAIR_MFMA && c != WBM_PAIR_RESIDENT)))
    return false;
  *chan = a;
  *beam = b;
  *thr = c;
  *ovl = o;
  return true;
}

void cache_store(const std::string& key, int chan, int beam, int thr, int ovl) {
  const std::string path = cache_path();
  std::string txt;
  {
    std::ifstream f(path);
    if (f) {
      std::stringstream ss;
      ss << f.rdbuf();
      txt = ss.str();
    }
  }
  const size_t open = txt.find('{'), close = txt.rfind('}');
  std::string body = (open != std::string::npos && close != std::string::npos && close > open)
                         ? txt.substr(open + 1, close - open - 1) : std::string();
  while (!body.empty() && (body.back() == '\n' || body.back() == ' ')) body.pop_back();
  std::ostringstream os;
  os << "{" << body << (body.empty() ? "" : ",") << "\n  \"" << key << "\": [" << chan << ", "
     << beam << ", " << thr << ", " << ovl << "]\n}\n";
  const size_t slash = path.rfind('/');
  if (slash != std::string::npos) {
    std::string dir = path.substr(0, slash);
    for (size_t i = 1; i <= dir.size(); ++i)
      if (i == dir.size() || dir[i] == '/') mkdir(dir.substr(0, i).c_str(), 0755);
  }
  std::ofstream out(path);
  if (out) out << os.str();
}

// Time a candidate: one warm-up launch, then the best of four samples of three back-to-back
// launches (per launch), so that candidates a few percent apart are ordered reliably.
template <class F>
hipError_t time_best(F launch, hipStream_t st, float* best_ms) {
  constexpr int kSamples = 4, kPerSample = 3;
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e != hipSuccess) return e;
  e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    return e;
  }
  *best_ms = 1e30f;
  e = launch();
  for (int r = 0; r < kSamples && e == hipSuccess; ++r) {
    e = hipEventRecord(e0, st);
    for (int q = 0; q < kPerSample && e == hipSuccess; ++q) e = launch();
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && ms / kPerSample < *best_ms) *best_ms = ms / kPerSample;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return e;
}

// Pair kernels each precision can run: the extended-precision windows need the vector kernels.
bool pair_ok(const wbm_plan* p, int prec, int thr) {
  if (thr == WBM_PAIR_WAVE) return wbm::mvdr_wave_supported(p->cfg.w_max);
  if (thr == WBM_PAIR_BLOCK) return true;
  if (prec == kExt) return false;
  if (thr == WBM_PAIR_RESIDENT) return resident_ok(p);
  return thr == WBM_PAIR_MFMA;
}

hipError_t autotune(wbm_plan* p, int prec, const float2* x, int T, int sumW, double loading,
                    hipStream_t st) {
  Tuning& tn = p->tune[prec];
  tn.tuned = true;
  const char* env = std::getenv("WBM_AUTOTUNE");
  if (env && std::strcmp(env, "0") == 0) return hipSuccess;
  const std::string key = tune_key(p, prec);
  int chan = 12, beam = 12, thr = WBM_PAIR_BLOCK, ovl = 1;
  if (cache_lookup(key, prec, &chan, &beam, &thr, &ovl) && overlap_supported(p, ovl) &&
      pair_ok(p, prec, thr) &&
      wbm::channelize_lds_bytes(prec == kExt, p->cfg.k_sub, chan) <= wbm::kLdsBytes) {
    tn.chan_logtile = chan;
    set_beam_tile(p, prec, beam);
    tn.pair_threads = thr;
    tn.overlap = ovl;
    return hipSuccess;
  }
  float best_c = 1e30f, best_b = 1e30f;
  const int lt0 = prec == kExt ? 10 : 11;
  // tiles beyond the LDS at this shape (the extended channelizer at K = 2; a spatial DFT whose
  // tile leaves no room for this call's window rows) are not candidates
  for (int lt = lt0; lt <= 13; ++lt) {
    float ms;
    if (wbm::channelize_lds_bytes(prec == kExt, p->cfg.k_sub, lt) <= wbm::kLdsBytes) {
      tn.chan_logtile = lt;
      hipError_t e = time_best([&]() { return enqueue_channelize(p, prec, x, st); }, st, &ms);
      if (e != hipSuccess) return e;
      if (ms < best_c) {
        best_c = ms;
        chan = lt;
      }
    }
    if (beam_lds(p, prec, lt, T, sumW, true, false) <= wbm::kLdsBytes) {
      set_beam_tile(p, prec, lt);
      hipError_t e =
          time_best([&]() { return enqueue_beamspace_windows(p, prec, T, sumW, st); }, st, &ms);
      if (e != hipSuccess) return e;
      if (ms < best_b) {
        best_b = ms;
        beam = lt;
      }
    }
  }
  tn.chan_logtile = chan;
  set_beam_tile(p, prec, beam);
  // pair kernel: each candidate timed in the whole fused sequence (channelize, windows, pair
  // kernel), where it reads windows the spatial DFT has just written
  hipError_t e = hipSuccess;
  float best_p = 1e30f;
  for (int thr_c : {WBM_PAIR_MFMA, WBM_PAIR_BLOCK, WBM_PAIR_WAVE, WBM_PAIR_RESIDENT}) {
    if (!pair_ok(p, prec, thr_c)) continue;
    float ms;
    tn.pair_threads = thr_c;
    e = time_best([&]() {
      return enqueue_fused(p, prec, x, T, sumW, loading, p->prof_out, p->prof_w, nullptr,
                           p->prof_info, st, 1);
    }, st, &ms);
    if (e != hipSuccess) return e;
    if (ms < best_p) {
      best_p = ms;
      thr = thr_c;
    }
  }
  tn.pair_threads = thr;
  // subband chunks overlapping the beamspace and pair kernels: the whole fused sequence
  float best_o = 1e30f;
  for (int ch = 1; ch <= kMaxOverlap; ch <<= 1) {
    if (!overlap_supported(p, ch)) continue;
    float ms;
    e = time_best([&]() {
      return enqueue_fused(p, prec, x, T, sumW, loading, p->prof_out, p->prof_w, nullptr,
                           p->prof_info, st, ch);
    }, st, &ms);
    if (e != hipSuccess) return e;
    if (ms < best_o) {
      best_o = ms;
      ovl = ch;
    }
  }
  tn.overlap = ovl;
  cache_store(key, chan, beam, thr, ovl);
  return hipSuccess;
}

// The workspace and the launch configuration of the fused sequence in precision prec, tuned
// on this call's data on first use.
wbm_status ready_fused(wbm_plan* p, int prec, const float2* x, int T, int sumW, double loading,
                       hipStream_t st, bool prof = false) {
  wbm_status s;
  if (prec == kExt && (s = ensure_ext(p))) return s;
  if ((s = fit_beam_tile(p, prec, T, sumW, true, prof))) return s;
  if (!p->tune[prec].tuned) {
    if ((s = ensure_prof(p))) return s;
    WBM_HIP(autotune(p, prec, x, T, sumW, loading, st), "autotune");
  }
  return fit_beam_tile(p, prec, T, sumW, true, prof);
}

static_assert(WBM_PAIR_MFMA == wbm::kPairMfma && WBM_PAIR_RESIDENT == wbm::kPairResident,
              "pair kernel ids");

wbm_status check_plan(const wbm_plan* p) {
  if (!p) return fail(WBM_ERR_ARG, "plan is NULL");
  hipError_t e = hipSetDevice(p->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  return WBM_OK;
}

}  // namespace

extern "C" {

const char* wbm_version(void) { return "wbmvdr 0.1 (gfx950)"; }

const char* wbm_last_error(void) { return g_err.c_str(); }

const char* wbm_status_str(wbm_status s) {
  switch (s) {
    case WBM_OK: return "ok";
    case WBM_ERR_ARG: return "invalid argument";
    case WBM_ERR_SHAPE: return "shape mismatch";
    case WBM_ERR_NOMEM: return "out of memory";
    case WBM_ERR_HIP: return "HIP runtime error";
    case WBM_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

int64_t wbm_plan_workspace_bytes(const wbm_plan* p) { return p ? p->ws_bytes : 0; }

wbm_status wbm_plan_set_tuning(wbm_plan* p, int32_t precision, int32_t chan, int32_t beam,
                               int32_t pair, int32_t overlap) {
  if (!p) return fail(WBM_ERR_ARG, "plan is NULL");
  if (precision != WBM_PREC_EXT && precision != WBM_PREC_F32)
    return fail(WBM_ERR_ARG, "precision must be WBM_PREC_EXT or WBM_PREC_F32");
  const int prec = precision == WBM_PREC_EXT ? kExt : kF32;
  if (!logtile_ok(prec, chan) || !logtile_ok(prec, beam))
    return fail(WBM_ERR_ARG, prec == kExt ? "FFT tile log2 must be 10, 11, 12 or 13"
                                          : "FFT tile log2 must be 11, 12 or 13");
  if (pair != WBM_PAIR_MFMA && pair != WBM_PAIR_WAVE && pair != WBM_PAIR_BLOCK &&
      pair != WBM_PAIR_RESIDENT)
    return fail(WBM_ERR_ARG,
                "pair_kernel must be WBM_PAIR_MFMA, WBM_PAIR_WAVE, WBM_PAIR_BLOCK or "
                "WBM_PAIR_RESIDENT");
  if (pair == WBM_PAIR_WAVE && !wbm::mvdr_wave_supported(p->cfg.w_max))
    return fail(WBM_ERR_UNSUPPORTED, "the one-wave pair kernel needs w_max <= 40");
  if (prec == kExt && (pair == WBM_PAIR_MFMA || pair == WBM_PAIR_RESIDENT))
    return fail(WBM_ERR_UNSUPPORTED,
                "the extended-precision windows run on WBM_PAIR_BLOCK or WBM_PAIR_WAVE");
  if (pair == WBM_PAIR_RESIDENT && !resident_ok(p))
    return fail(WBM_ERR_UNSUPPORTED,
                "the resident pair kernel needs w_max * L <= 2304 and w_max * Lt <= 2304");
  if (overlap != 1 && overlap != 2 && overlap != 4 && overlap != 8)
    return fail(WBM_ERR_ARG, "overlap_chunks must be 1, 2, 4 or 8");
  if (!overlap_supported(p, overlap))
    return fail(WBM_ERR_UNSUPPORTED, "overlap_chunks needs K to be a multiple of 8 * chunks");
  if (wbm::channelize_lds_bytes(prec == kExt, p->cfg.k_sub, chan) > wbm::kLdsBytes ||
      beam_lds(p, prec, beam, 0, 0, false, false) > wbm::kLdsBytes)
    return fail(WBM_ERR_UNSUPPORTED, "this FFT tile needs more LDS than a compute unit has at "
                                     "this K / M and precision");
  Tuning& tn = p->tune[prec];
  tn.chan_logtile = chan;
  set_beam_tile(p, prec, beam);
  tn.pair_threads = pair;
  tn.overlap = overlap;
  tn.tuned = true;
  if (prec == kF32) {
    p->upa_pair = pair;
    p->upa_tuned = true;
  }
  p->gkey.valid = false;
  return WBM_OK;
}

wbm_status wbm_plan_get_tuning(const wbm_plan* p, int32_t precision, int32_t* chan,
                               int32_t* beam, int32_t* pair, int32_t* overlap) {
  if (!p) return fail(WBM_ERR_ARG, "plan is NULL");
  if (precision != WBM_PREC_EXT && precision != WBM_PREC_F32)
    return fail(WBM_ERR_ARG, "precision must be WBM_PREC_EXT or WBM_PREC_F32");
  const Tuning& tn = p->tune[precision == WBM_PREC_EXT ? kExt : kF32];
  if (chan) *chan = tn.chan_logtile;
  if (beam) *beam = tn.beam_logtile;
  if (pair) *pair = tn.pair_threads;
  if (overlap) *overlap = tn.overlap;
  return WBM_OK;
}

wbm_status wbm_plan_destroy(wbm_plan* p) {
  if (!p) return WBM_OK;
  (void)hipSetDevice(p->device);
  (void)hipDeviceSynchronize();
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  if (p->side_stream) (void)hipStreamDestroy(p->side_stream);
  for (hipEvent_t ev : p->chunk_evt)
    if (ev) (void)hipEventDestroy(ev);
  if (p->desc_evt) (void)hipEventDestroy(p->desc_evt);
  if (p->desc_host) (void)hipHostFree(p->desc_host);
  if (p->jam_evt) (void)hipEventDestroy(p->jam_evt);
  if (p->jam_host) (void)hipHostFree(p->jam_host);
  void* bufs[] = {p->twK, p->twM, p->hb, p->twK64, p->twM64, p->hb64, p->Xl, p->Ywl,
                  p->desc_dev, p->X, p->Yw, p->Y, p->R32,
                  p->w32, p->starts, p->abar, p->fullR, p->fullW, p->fullV, p->fullQ, p->full_info,
                  p->prof_out, p->prof_w, p->prof_info, p->pprof, p->feat, p->nnout,
                  p->pw, p->pdelta, p->jam_dev, p->route, p->upa_rows};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  delete p;
  return WBM_OK;
}

wbm_status wbm_plan_create(const wbm_config* cfg, wbm_plan** out) {
  if (!out) return fail(WBM_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!cfg) return fail(WBM_ERR_ARG, "cfg is NULL");
  const wbm_config& c = *cfg;
  if (c.n_elem < 1) return fail(WBM_ERR_ARG, "n_elem must be >= 1");
  if (!is_pow2(c.m_fft) || c.m_fft < 2 || c.m_fft < c.n_elem || c.m_fft > 8192)
    return fail(WBM_ERR_ARG, "m_fft must be a power of two with max(2, n_elem) <= m_fft <= 8192");
  if (!is_pow2(c.k_sub) || c.k_sub < 2 || c.k_sub > 8192)
    return fail(WBM_ERR_ARG, "k_sub must be a power of two in [2, 8192]");
  if (c.l_train < 1 || c.l_test < 0) return fail(WBM_ERR_ARG, "need l_train >= 1 and l_test >= 0");
  if (c.max_targets < 1 || c.max_targets > (1 << 20)) return fail(WBM_ERR_ARG, "max_targets out of range");
  if (c.w_max < 1 || c.w_max > 64 || c.w_max > c.m_fft)
    return fail(WBM_ERR_ARG, "w_max must be in [1, min(64, m_fft)]");
  if (!(c.beta >= 0.0 && c.beta < 2.0)) return fail(WBM_ERR_ARG, "beta must be in [0, 2)");
  if (!(c.d_over_lambda > 0.0 && std::isfinite(c.d_over_lambda)))
    return fail(WBM_ERR_ARG, "d_over_lambda must be positive");
  if (c.flags & ~WBM_HALF_BIN) return fail(WBM_ERR_ARG, "unknown flags");
  const int64_t B = (int64_t)c.l_train + c.l_test;
  if (B > 65535) return fail(WBM_ERR_ARG, "l_train + l_test must be <= 65535");
  // the pair kernels address one chunk of a subband's window tiles with 32-bit byte offsets:
  // at most max_targets * w_max rows of the largest snapshot tile block (or 64 snapshots)
  {
    const int64_t tb = std::max<int64_t>(64, (int64_t)1 << wbm::beamspace_tile_log(c.m_fft, 13));
    if ((int64_t)c.max_targets * c.w_max * tb * 8 >= ((int64_t)1 << 32))
      return fail(WBM_ERR_ARG, "max_targets * w_max too large for this m_fft (window tiles "
                               "beyond 32-bit offsets)");
  }

  int ndev = 0;
  hipError_t he = hipGetDeviceCount(&ndev);
  if (he != hipSuccess || ndev < 1) {
    (void)hipGetLastError();
    return fail(WBM_ERR_HIP, "no HIP device available");
  }
  wbm_plan* p = new wbm_plan();
  p->cfg = c;
  (void)hipGetDevice(&p->device);
  p->B = (int)B;
  p->S = B * c.k_sub;
  set_beam_tile(p, kExt, 12);
  set_beam_tile(p, kF32, 12);
  p->tune[kF32].pair_threads = WBM_PAIR_MFMA;

  auto bail = [&](wbm_status s) {
    std::string keep = g_err;
    wbm_plan_destroy(p);
    g_err = keep;
    return s;
  };
  wbm_status s;
  if ((s = dev_alloc(p, &p->twK, c.k_sub, "twiddles K"))) return bail(s);
  if ((s = dev_alloc(p, &p->twM, c.m_fft, "twiddles M"))) return bail(s);
  if ((s = dev_alloc(p, &p->hb, c.k_sub, "half-bin twiddles"))) return bail(s);
  if ((s = upload_twiddles(p->twK, c.k_sub, 1.0))) return bail(s);
  if ((s = upload_twiddles(p->twM, c.m_fft, 1.0))) return bail(s);
  if ((s = upload_twiddles(p->hb, c.k_sub, 0.5))) return bail(s);

  const int Tm = c.max_targets;
  const DescLayout dl = desc_layout(Tm, c.w_max);
  p->desc_bytes = dl.bytes;
  if ((s = dev_alloc(p, &p->desc_dev, p->desc_bytes, "descriptor"))) return bail(s);
  if (hipHostMalloc((void**)&p->desc_host, p->desc_bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return bail(fail(WBM_ERR_NOMEM, "pinned descriptor allocation failed"));
  }
  std::memset(p->desc_host, 0, p->desc_bytes);
  if (hipEventCreateWithFlags(&p->desc_evt, hipEventDisableTiming) != hipSuccess)
    return bail(fail(WBM_ERR_HIP, "hipEventCreate failed"));
  p->dd.sin_az = reinterpret_cast<const double*>(p->desc_dev + dl.sin_az);
  p->dd.cz = reinterpret_cast<const double*>(p->desc_dev + dl.cz);
  p->dd.win = reinterpret_cast<const int*>(p->desc_dev + dl.win);
  p->dd.woff = reinterpret_cast<const int*>(p->desc_dev + dl.woff);
  p->dd.rowtab = reinterpret_cast<const int*>(p->desc_dev + dl.rowtab);
  p->dd.torder = reinterpret_cast<const int*>(p->desc_dev + dl.torder);
  p->dd.wz = reinterpret_cast<const int*>(p->desc_dev + dl.wz);

  const size_t NS = (size_t)c.n_elem * p->S;
  if ((s = dev_alloc(p, &p->X, NS, "channelized X"))) return bail(s);
  // room for the snapshot padding of the largest beamspace tile the autotuner may pick
  const size_t tb_max = (size_t)1 << wbm::beamspace_tile_log(c.m_fft, 13);
  const size_t b_pad = ((size_t)p->B + tb_max - 1) / tb_max * tb_max;
  p->yw_elems = (size_t)c.k_sub * b_pad * (size_t)Tm * c.w_max;
  if ((s = dev_alloc(p, &p->Yw, p->yw_elems, "windows Yw"))) return bail(s);
  if ((s = dev_alloc(p, &p->starts, (size_t)Tm * c.k_sub, "starts"))) return bail(s);
  if ((s = dev_alloc(p, &p->abar, (size_t)Tm * c.k_sub * c.w_max, "steering"))) return bail(s);
  if ((s = dev_alloc(p, &p->full_info, (size_t)c.k_sub, "full info"))) return bail(s);

  he = wbm::set_fft_attributes();
  if (he != hipSuccess) return bail(hip_fail(he, "hipFuncSetAttribute (FFT kernels)"));
  he = wbm::set_pair_attributes();
  if (he != hipSuccess) return bail(hip_fail(he, "hipFuncSetAttribute (pair kernels)"));
  he = wbm::set_full_attributes();
  if (he != hipSuccess) return bail(hip_fail(he, "hipFuncSetAttribute (full-dimensional kernels)"));
  if (hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) != hipSuccess)
    return bail(fail(WBM_ERR_HIP, "capture stream creation failed"));
  // the overlapped fused sequence's second stream and its fork / join events: created here,
  // never while a stream may be capturing
  if (hipStreamCreateWithFlags(&p->side_stream, hipStreamNonBlocking) != hipSuccess)
    return bail(fail(WBM_ERR_HIP, "side stream creation failed"));
  for (int i = 0; i <= kMaxOverlap; ++i)
    if (hipEventCreateWithFlags(&p->chunk_evt[i], hipEventDisableTiming) != hipSuccess)
      return bail(fail(WBM_ERR_HIP, "event creation failed"));
  *out = p;
  return WBM_OK;
}

wbm_status wbm_steer(wbm_plan* p, const double* az_rad, const int32_t* win, int32_t T,
                     int32_t* starts, wbm_c64* abar, void* stream) {
  wbm_status s = check_plan(p);
  if (s) return s;
  if (!starts || !abar) return fail(WBM_ERR_ARG, "starts / abar is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  int sumW = 0;
  if ((s = upload_desc(p, az_rad, win, T, st, &sumW))) return s;
  WBM_HIP(wbm::launch_steer(geom(p, T), p->cfg.w_max, starts, reinterpret_cast<double2*>(abar), st),
          "steer launch");
  return WBM_OK;
}

wbm_status wbm_channelize(wbm_plan* p, const wbm_c32* x, wbm_c32* X, void* stream) {
  wbm_status s = check_plan(p);
  if (s) return s;
  if (!x || !X) return fail(WBM_ERR_ARG, "x / X is NULL");
  const wbm_config& c = p->cfg;
  WBM_HIP(wbm::launch_channelize(reinterpret_cast<const float2*>(x), reinterpret_cast<float2*>(X),
                                 c.n_elem, c.k_sub, p->B, p->twK,
                                 (c.flags & WBM_HALF_BIN) ? p->hb : nullptr,
                                 p->tune[kF32].chan_logtile, static_cast<hipStream_t>(stream)),
          "channelize launch");
  return WBM_OK;
}

wbm_status wbm_lift(wbm_plan* p, const wbm_c32* weights, const int32_t* starts, int32_t T,
                    wbm_c32* c_hat, void* stream) {
  wbm_status s = check_plan(p);
  if (s) return s;
  if (!weights || !starts || !c_hat) return fail(WBM_ERR_ARG, "weights / starts / c_hat is NULL");
  const wbm_config& c = p->cfg;
  if (T < 1 || T > c.max_targets) return fail(WBM_ERR_ARG, "T outside [1, max_targets]");
  WBM_HIP(wbm::launch_lift(reinterpret_cast<const float2*>(weights), starts, T * c.k_sub,
                           c.w_max, c.n_elem, c.m_fft, p->twM, reinterpret_cast<float2*>(c_hat),
                           static_cast<hipStream_t>(stream)),
          "lift launch");
  return WBM_OK;
}

wbm_status wbm_apply_lifted(wbm_plan* p, const wbm_c32* x, const wbm_c32* c_hat, int32_t T,
                            wbm_c32* out, void* stream) {
  wbm_status s = check_plan(p);
  if (s) return s;
  if (!x || !c_hat || !out) return fail(WBM_ERR_ARG, "x / c_hat / out is NULL");
  const wbm_config& c = p->cfg;
  if (T < 1 || T > c.max_targets) return fail(WBM_ERR_ARG, "T outside [1, max_targets]");
  hipStream_t st = static_cast<hipStream_t>(stream);
  WBM_HIP(enqueue_channelize(p, kF32, reinterpret_cast<const float2*>(x), st),
          "channelize launch");
  WBM_HIP(wbm::launch_lift_apply(p->X, reinterpret_cast<const float2*>(c_hat),
                                 reinterpret_cast<float2*>(out), c.n_elem, c.k_sub, p->B,
                                 c.l_train, c.l_test, T, st),
          "lifted apply launch");
  return WBM_OK;
}

wbm_status wbm_beam_pattern(wbm_plan* p, const wbm_c32* c, int32_t pairs, const double* omega,
                            int32_t Q, float* pattern, void* stream) {
  wbm_status s = check_plan(p);
  if (s) return s;
  if (!c || !omega || !pattern) return fail(WBM_ERR_ARG, "c / omega / pattern is NULL");
  if (pairs < 1 || Q < 1) return fail(WBM_ERR_ARG, "need pairs >= 1 and Q >= 1");
  if (p->cfg.n_elem > 4096) return fail(WBM_ERR_UNSUPPORTED, "beam patterns need N <= 4096");
  WBM_HIP(wbm::launch_beam_pattern(reinterpret_cast<const float2*>(c), pairs, p->cfg.n_elem, omega,
                                   Q, pattern, static_cast<hipStream_t>(stream)),
          "beam pattern launch");
  return WBM_OK;
}

wbm_status wbm_lift_upa(wbm_plan* p, const wbm_c32* weights, const int32_t* starts, int32_t nz,
                        int32_t mz, const int32_t* win_z, int32_t T, wbm_c32* c_hat,
                        void* stream) {
  wbm_status s = check_plan(p);
  if (s) return s;
  if (!weights || !starts || !win_z || !c_hat)
    return fail(WBM_ERR_ARG, "weights / starts / win_z / c_hat is NULL");
  if ((s = check_upa_shape(p, nz, mz))) return s;
  const wbm_config& c = p->cfg;
  if (T < 1 || T > c.max_targets) return fail(WBM_ERR_ARG, "T outside [1, max_targets]");
  WBM_HIP(wbm::launch_lift_upa(reinterpret_cast<const float2*>(weights), starts, win_z, T,
                               c.k_sub, c.w_max, nz, c.n_elem / nz, mz, c.m_fft / mz, p->twM,
                               reinterpret_cast<float2*>(c_hat),
                               static_cast<hipStream_t>(stream)),
          "planar lift launch");
  return WBM_OK;
}

wbm_status wbm_beam_pattern_upa(wbm_plan* p, const wbm_c32* c, int32_t pairs, int32_t nz,
                                const double* omega, int32_t Q, float* pattern, void* stream) {
  wbm_status s = check_plan(p);
  if (s) return s;
  if (!c || !omega || !pattern) return fail(WBM_ERR_ARG, "c / omega / pattern is NULL");
  if (pairs < 1 || Q < 1) return fail(WBM_ERR_ARG, "need pairs >= 1 and Q >= 1");
  if (nz < 1 || p->cfg.n_elem % nz != 0)
    return fail(WBM_ERR_SHAPE, "nz must divide n_elem");
  if (p->cfg.n_elem > 4096) return fail(WBM_ERR_UNSUPPORTED, "beam patterns need N <= 4096");
  WBM_HIP(wbm::launch_beam_pattern_upa(reinterpret_cast<const float2*>(c), pairs, nz,
                                       p->cfg.n_elem / nz, omega, Q, pattern,
                                       static_cast<hipStream_t>(stream)),
          "planar beam pattern launch");
  return WBM_OK;
}

wbm_status wbm_range_doppler(wbm_plan* p, const wbm_c32* z, int32_t T, int64_t z_stride,
                             const wbm_c32* chirp, int32_t Lp, int32_t R, int32_t P,
                             int32_t guard, int32_t train, double threshold_db, wbm_c32* work,
                             float* power, uint8_t* det, void* stream) {
  wbm_status s = check_plan(p);
  if (s) return s;
  if (!z || !chirp || !work || !power || !det) return fail(WBM_ERR_ARG, "NULL pointer argument");
  if (T < 1 || Lp < 1 || R < Lp) return fail(WBM_ERR_ARG, "need T >= 1 and 1 <= Lp <= R");
  if (P < 2 || P > 8192 || (P & (P - 1)) != 0)
    return fail(WBM_ERR_ARG, "P must be a power of two in [2, 8192]");
  if (z_stride < (int64_t)P * R) return fail(WBM_ERR_ARG, "z_stride must be >= P * R");
  if (guard < 0 || train < 1) return fail(WBM_ERR_ARG, "need guard >= 0 and train >= 1");
  if (!std::isfinite(threshold_db)) return fail(WBM_ERR_ARG, "threshold_db must be finite");
  if (wbm::range_doppler_fft_log(R, Lp) > 13)
    return fail(WBM_ERR_UNSUPPORTED, "R + Lp - 1 must be at most 8192");
  const float alpha = (float)std::pow(10.0, threshold_db / 10.0);
  WBM_HIP(wbm::launch_range_doppler(reinterpret_cast<const float2*>(z), z_stride, T,
                                    reinterpret_cast<const float2*>(chirp), Lp, R, P, guard,
                                    train, alpha, reinterpret_cast<float2*>(work), power, det,
                                    static_cast<hipStream_t>(stream)),
          "range-Doppler launch");
  return WBM_OK;
}

wbm_status wbm_synthesize(wbm_plan* p, const wbm_c32* out, int32_t T, wbm_c32* z, void* stream) {
  wbm_status s = check_plan(p);
  if (s) return s;
  if (!out || !z) return fail(WBM_ERR_ARG, "out / z is NULL");
  const wbm_config& c = p->cfg;
  if (T < 1 || T > c.max_targets) return fail(WBM_ERR_ARG, "T outside [1, max_targets]");
  WBM_HIP(wbm::launch_synth(reinterpret_cast<const float2*>(out), reinterpret_cast<float2*>(z),
                            c.k_sub, c.l_test, T, p->twK,
                            (c.flags & WBM_HALF_BIN) ? p->hb : nullptr,
                            static_cast<hipStream_t>(stream)),
          "synthesis launch");
  return WBM_OK;
}

wbm_status wbm_beamspace(wbm_plan* p, const wbm_c32* X, wbm_c32* Y, void* stream) {
  wbm_status s = check_plan(p);
  if (s) return s;
  if (!X || !Y) return fail(WBM_ERR_ARG, "X / Y is NULL");
  const wbm_config& c = p->cfg;
  WBM_HIP(wbm::launch_beamspace(reinterpret_cast<const float2*>(X), reinterpret_cast<float2*>(Y),
                                nullptr, c.n_elem, c.m_fft, p->B, c.k_sub, p->twM, nullptr, 0,
                                geom(p, 0), p->tune[kF32].beam_logtile,
                                static_cast<hipStream_t>(stream)),
          "beamspace launch");
  return WBM_OK;
}

wbm_status wbm_beamform(wbm_plan* p, const wbm_c32* x, const double* az_rad, const int32_t* win,
                        int32_t T, double loading, int32_t form, wbm_c32* out, wbm_c32* weights,
                        int32_t* starts, int32_t* info, void* stream) {
  wbm_status s = check_plan(p);
  if (s) return s;
  const wbm_config& c = p->cfg;
  if (!x) return fail(WBM_ERR_ARG, "x is NULL");
  if (!out && c.l_test > 0) return fail(WBM_ERR_ARG, "out is NULL");
  if (!(loading >= 0.0 && std::isfinite(loading))) return fail(WBM_ERR_ARG, "loading must be finite and >= 0");
  if (form < WBM_FORM_PLAIN || form > WBM_FORM_GRAPH_F32) return fail(WBM_ERR_ARG, "unknown form");
  hipStream_t st = static_cast<hipStream_t>(stream);
  int sumW = 0;
  if ((s = upload_desc(p, az_rad, win, T, st, &sumW))) return s;
  float2* o = reinterpret_cast<float2*>(out);
  float2* w = reinterpret_cast<float2*>(weights);
  const float2* xx = reinterpret_cast<const float2*>(x);
  // the fused forms' intermediates: extended precision, or FP32 (the *_F32 forms and the mixed
  // forms, whose covariance is formed at lower precision still)
  const int prec = (form == WBM_FORM_FUSED || form == WBM_FORM_GRAPH) ? kExt : kF32;
  if (form != WBM_FORM_PLAIN && (s = ready_fused(p, prec, xx, T, sumW, loading, st))) return s;
  if (form == WBM_FORM_PLAIN) {
    if ((s = ensure_plain(p))) return s;
    WBM_HIP(wbm::launch_steer(geom(p, T), c.w_max, p->starts, p->abar, st), "steer launch");
    WBM_HIP(enqueue_channelize(p, kF32, xx, st), "channelize launch");
    WBM_HIP(wbm::launch_beamspace(p->X, p->Y, nullptr, c.n_elem, c.m_fft, p->B, c.k_sub, p->twM,
                                  nullptr, 0, geom(p, T), 12, st),
            "beamspace launch");
    WBM_HIP(wbm::launch_mvdr_plain(pair_args(p, kF32, T, sumW, loading), p->dd, p->Y, p->starts,
                                   p->abar, p->R32, p->w32, o, w, info, st),
            "plain MVDR launch");
    if (starts) {
      WBM_HIP(hipMemcpyAsync(starts, p->starts, sizeof(int) * (size_t)T * c.k_sub,
                             hipMemcpyDeviceToDevice, st),
              "starts copy");
    }
  } else if (form == WBM_FORM_FUSED || form == WBM_FORM_FUSED_F32) {
    WBM_HIP(enqueue_fused(p, prec, xx, T, sumW, loading, o, w, starts, info, st), "fused launch");
  } else if (form == WBM_FORM_MIXED || form == WBM_FORM_MIXED_BF16) {
    WBM_HIP(enqueue_channelize(p, kF32, xx, st), "channelize launch");
    WBM_HIP(enqueue_beamspace_windows(p, kF32, T, sumW, st), "beamspace launch");
    if (!p->route) {
      wbm_status rs = dev_alloc(p, &p->route, (size_t)c.max_targets * c.k_sub, "route flags");
      if (rs) return rs;
    }
    WBM_HIP(wbm::launch_mvdr_mixed(pair_args(p, kF32, T, sumW, loading), geom(p, T), p->dd, p->Yw,
                                   o, w, starts, info, p->route, form == WBM_FORM_MIXED, st),
            "mixed MVDR launch");
  } else {
    GraphKey key;
    key.prec = prec;
    key.x = x;
    key.out = out;
    key.weights = weights;
    key.info = info;
    key.starts = starts;
    key.T = T;
    key.sumW = sumW;
    key.loading = loading;
    key.valid = true;
    if (!(key == p->gkey)) {
      if (p->gexec) {
        WBM_HIP(hipGraphExecDestroy(p->gexec), "graph destroy");
        p->gexec = nullptr;
      }
      p->gkey.valid = false;
      hipGraph_t g = nullptr;
      WBM_HIP(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
      hipError_t le = enqueue_fused(p, prec, xx, T, sumW, loading, o, w, starts, info,
                                    p->cap_stream);
      hipError_t ce = hipStreamEndCapture(p->cap_stream, &g);
      if (le != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(le, "launch during capture");
      }
      if (ce != hipSuccess) return hip_fail(ce, "end capture");
      hipError_t ie = hipGraphInstantiate(&p->gexec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ie != hipSuccess) {
        p->gexec = nullptr;
        return hip_fail(ie, "graph instantiate");
      }
      p->gkey = key;
    }
    WBM_HIP(hipGraphLaunch(p->gexec, st), "graph launch");
  }
  return WBM_OK;
}

wbm_status wbm_steer_upa(wbm_plan* p, int32_t nz, int32_t mz, const double* az_rad,
                         const double* el_rad, const int32_t* win_z, const int32_t* win_x,
                         int32_t T, int32_t* starts, wbm_c64* abar, void* stream) {
  wbm_status s = check_plan(p);
  if (s) return s;
  if (!abar) return fail(WBM_ERR_ARG, "abar is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  int sumW = 0;
  if ((s = upload_desc_upa(p, nz, mz, az_rad, el_rad, win_z, win_x, T, st, &sumW))) return s;
  WBM_HIP(wbm::launch_steer_upa(upa_geom(p, T, nz, mz), p->cfg.w_max, starts,
                                reinterpret_cast<double2*>(abar), st),
          "planar steer launch");
  return WBM_OK;
}

wbm_status wbm_beamspace_upa(wbm_plan* p, const wbm_c32* X, int32_t nz, int32_t mz, wbm_c32* Y,
                             void* stream) {
  wbm_status s = check_plan(p);
  if (s) return s;
  if (!X || !Y) return fail(WBM_ERR_ARG, "X / Y is NULL");
  if ((s = check_upa_shape(p, nz, mz))) return s;
  WBM_HIP(wbm::launch_beamspace_upa(reinterpret_cast<const float2*>(X),
                                    reinterpret_cast<float2*>(Y), nullptr, p->B, p->twM, nullptr,
                                    0, upa_geom(p, 0, nz, mz), p->tune[kF32].logTB,
                                    p->tune[kF32].nbt,
                                    static_cast<hipStream_t>(stream)),
          "planar beamspace launch");
  return WBM_OK;
}

}  // extern "C"

namespace {

// Channelize -> planar beamspace windows for the uploaded targets (steering already in abar).
hipError_t enqueue_upa_windows(wbm_plan* p, const float2* x, int T, int sumW,
                               const wbm::UpaGeom& g, hipStream_t st) {
  hipError_t e = enqueue_channelize(p, kF32, x, st);
  if (e != hipSuccess) return e;
  return wbm::launch_beamspace_upa(p->X, nullptr, p->Yw, p->B, p->twM, p->dd.rowtab, sumW, g,
                                   p->tune[kF32].logTB, p->tune[kF32].nbt, st);
}

// First planar-array call of a plan: the channelizer tile (unless already tuned or pinned)
// and the pair kernel of the fused form are timed on this call's data (each pair-kernel
// candidate with the channelizer and planar spatial DFT before it; time_best, as the linear
// array's autotuner); WBM_AUTOTUNE=0 keeps the defaults (tile 2^12, matrix-core kernel).
hipError_t tune_upa(wbm_plan* p, const float2* x, int T, int sumW, const wbm::UpaGeom& g,
                    double loading, hipStream_t st) {
  p->upa_tuned = true;
  const char* env = std::getenv("WBM_AUTOTUNE");
  if (env && std::strcmp(env, "0") == 0) return hipSuccess;
  hipError_t e = hipSuccess;
  Tuning& tn = p->tune[kF32];
  if (!tn.tuned) {
    float best_c = 1e30f;
    int chan = tn.chan_logtile;
    for (int lt = 11; lt <= 13; ++lt) {
      float ms;
      tn.chan_logtile = lt;
      e = time_best([&]() { return enqueue_channelize(p, kF32, x, st); }, st, &ms);
      if (e != hipSuccess) return e;
      if (ms < best_c) {
        best_c = ms;
        chan = lt;
      }
    }
    tn.chan_logtile = chan;
  }
  wbm::PairArgs pa = pair_args(p, kF32, T, sumW, loading);
  pa.abar = p->abar;
  float best = 1e30f;
  for (int thr : {WBM_PAIR_MFMA, WBM_PAIR_BLOCK, WBM_PAIR_WAVE, WBM_PAIR_RESIDENT}) {
    if (thr == WBM_PAIR_WAVE && !wbm::mvdr_wave_supported(p->cfg.w_max)) continue;
    if (thr == WBM_PAIR_RESIDENT && !resident_ok(p)) continue;
    float ms;
    e = time_best([&]() {
      hipError_t le = enqueue_upa_windows(p, x, T, sumW, g, st);
      if (le != hipSuccess) return le;
      return wbm::launch_mvdr_fused(pa, geom(p, T), p->dd, p->Yw, p->prof_out, p->prof_w, nullptr,
                                    p->prof_info, thr, st);
    }, st, &ms);
    if (e != hipSuccess) return e;
    if (ms < best) {
      best = ms;
      p->upa_pair = thr;
    }
  }
  return hipSuccess;
}

}  // namespace

extern "C" {

wbm_status wbm_beamform_upa(wbm_plan* p, const wbm_c32* x, int32_t nz, int32_t mz,
                            const double* az_rad, const double* el_rad, const int32_t* win_z,
                            const int32_t* win_x, int32_t T, double loading, int32_t form,
                            wbm_c32* out, wbm_c32* weights, int32_t* starts, int32_t* info,
                            void* stream) {
  wbm_status s = check_plan(p);
  if (s) return s;
  const wbm_config& c = p->cfg;
  if (!x) return fail(WBM_ERR_ARG, "x is NULL");
  if (!out && c.l_test > 0) return fail(WBM_ERR_ARG, "out is NULL");
  if (!(loading >= 0.0 && std::isfinite(loading))) return fail(WBM_ERR_ARG, "loading must be finite and >= 0");
  if (form != WBM_FORM_PLAIN && form != WBM_FORM_FUSED && form != WBM_FORM_MIXED &&
      form != WBM_FORM_MIXED_BF16)
    return fail(WBM_ERR_UNSUPPORTED, "the planar array runs the plain, fused and mixed forms");
  hipStream_t st = static_cast<hipStream_t>(stream);
  int sumW = 0;
  if ((s = upload_desc_upa(p, nz, mz, az_rad, el_rad, win_z, win_x, T, st, &sumW))) return s;
  if (sizeof(float2) * (size_t)mz + sizeof(int) * (2 * (size_t)T + sumW) > 96 * 1024)
    return fail(WBM_ERR_SHAPE, "too many window rows for the planar beamspace kernel");
  const wbm::UpaGeom g = upa_geom(p, T, nz, mz);
  const float2* xx = reinterpret_cast<const float2*>(x);
  float2* o = reinterpret_cast<float2*>(out);
  float2* w = reinterpret_cast<float2*>(weights);
  if (form == WBM_FORM_PLAIN) {
    // per-stage FP32 baseline: full planar beamspace in HBM, the window cells gathered from it
    // through the beam table, covariance / Cholesky / apply as three launches
    if ((s = ensure_plain(p))) return s;
    if (!p->upa_rows &&
        (s = dev_alloc(p, &p->upa_rows, (size_t)c.max_targets * c.k_sub * c.w_max, "beam table")))
      return s;
    WBM_HIP(wbm::launch_steer_upa(g, c.w_max, starts, p->abar, st, p->upa_rows),
            "planar steer launch");
    WBM_HIP(enqueue_channelize(p, kF32, xx, st), "channelize launch");
    WBM_HIP(wbm::launch_beamspace_upa(p->X, p->Y, nullptr, p->B, p->twM, nullptr, 0, g,
                                      p->tune[kF32].logTB, p->tune[kF32].nbt, st),
            "planar beamspace launch");
    wbm::PairArgs pp = pair_args(p, kF32, T, sumW, loading);
    pp.rows = p->upa_rows;
    WBM_HIP(wbm::launch_mvdr_plain(pp, p->dd, p->Y, p->starts, p->abar, p->R32, p->w32, o, w, info,
                                   st),
            "plain MVDR launch");
    return WBM_OK;
  }
  WBM_HIP(wbm::launch_steer_upa(g, c.w_max, starts, p->abar, st), "planar steer launch");
  if (form == WBM_FORM_FUSED && !p->upa_tuned) {
    if ((s = ensure_prof(p))) return s;
    WBM_HIP(tune_upa(p, xx, T, sumW, g, loading, st), "planar pair kernel tuning");
  }
  WBM_HIP(enqueue_upa_windows(p, xx, T, sumW, g, st), "planar beamspace launch");
  wbm::PairArgs pa = pair_args(p, kF32, T, sumW, loading);
  pa.abar = p->abar;
  if (form == WBM_FORM_FUSED) {
    WBM_HIP(wbm::launch_mvdr_fused(pa, geom(p, T), p->dd, p->Yw, o, w, nullptr, info, p->upa_pair,
                                   st),
            "fused MVDR launch");
  } else {
    if (!p->route) {
      wbm_status rs = dev_alloc(p, &p->route, (size_t)c.max_targets * c.k_sub, "route flags");
      if (rs) return rs;
    }
    WBM_HIP(wbm::launch_mvdr_mixed(pa, geom(p, T), p->dd, p->Yw, o, w, nullptr, info, p->route,
                                   form == WBM_FORM_MIXED, st),
            "mixed MVDR launch");
  }
  return WBM_OK;
}

wbm_status wbm_stage_times(wbm_plan* p, const wbm_c32* x, const double* az_rad,
                           const int32_t* win, int32_t T, double loading, int32_t precision,
                           int32_t reps, double* stage_ms, void* stream) {
  wbm_status s = check_plan(p);
  if (s) return s;
  const wbm_config& c = p->cfg;
  if (!x || !stage_ms) return fail(WBM_ERR_ARG, "x / stage_ms is NULL");
  if (reps < 1) return fail(WBM_ERR_ARG, "reps must be >= 1");
  if (!(loading >= 0.0 && std::isfinite(loading))) return fail(WBM_ERR_ARG, "loading must be finite and >= 0");
  hipStream_t st = static_cast<hipStream_t>(stream);
  int sumW = 0;
  if (precision < WBM_PREC_EXT || precision > WBM_PREC_MIXED_BF16)
    return fail(WBM_ERR_ARG, "precision must be WBM_PREC_EXT, _F32, _MIXED or _MIXED_BF16");
  const int prec = precision == WBM_PREC_EXT ? kExt : kF32;
  const bool mixed = precision == WBM_PREC_MIXED || precision == WBM_PREC_MIXED_BF16;
  if ((s = upload_desc(p, az_rad, win, T, st, &sumW))) return s;
  if ((s = ensure_prof(p))) return s;
  if (mixed && !p->route &&
      (s = dev_alloc(p, &p->route, (size_t)c.max_targets * c.k_sub, "route flags")))
    return s;
  const float2* xx = reinterpret_cast<const float2*>(x);
  if ((s = ready_fused(p, prec, xx, T, sumW, loading, st))) return s;
  hipEvent_t ev[2];
  for (int i = 0; i < 2; ++i) WBM_HIP(hipEventCreate(&ev[i]), "event create");
  // each stage launched `reps` times back to back between two events (every launch rewrites
  // the same output from the same input), after one untimed launch; stages in pipeline order
  hipError_t e = hipSuccess;
  auto stage = [&](int i) -> hipError_t {
    switch (i) {
      case 0: return wbm::launch_steer(geom(p, T), c.w_max, p->starts, p->abar, st);
      case 1: return enqueue_channelize(p, prec, xx, st);
      case 2: return enqueue_beamspace_windows(p, prec, T, sumW, st);
      default:
        if (mixed)
          return wbm::launch_mvdr_mixed(pair_args(p, kF32, T, sumW, loading), geom(p, T), p->dd,
                                        p->Yw, p->prof_out, p->prof_w, nullptr, p->prof_info,
                                        p->route, precision == WBM_PREC_MIXED, st);
        return wbm::launch_mvdr_fused(pair_args(p, prec, T, sumW, loading), geom(p, T), p->dd,
                                      p->Yw, p->prof_out, p->prof_w, nullptr, p->prof_info,
                                      p->tune[prec].pair_threads, st);
    }
  };
  for (int i = 0; i < 4 && e == hipSuccess; ++i) {
    e = stage(i);
    if (e == hipSuccess) e = hipEventRecord(ev[0], st);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = stage(i);
    if (e == hipSuccess) e = hipEventRecord(ev[1], st);
    if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
    stage_ms[i] = ms / reps;
  }
  for (int i = 0; i < 2; ++i) (void)hipEventDestroy(ev[i]);
  if (e != hipSuccess) return hip_fail(e, "stage timing");
  return WBM_OK;
}

wbm_status wbm_full_mvdr(wbm_plan* p, const wbm_c32* x, const double* az_rad, int32_t T,
                         double loading, int32_t k_first, int32_t nk_req, wbm_c32* out,
                         wbm_c32* weights, int32_t* info, void* stream) {
  wbm_status s = check_plan(p);
  if (s) return s;
  const wbm_config& c = p->cfg;
  if (!x) return fail(WBM_ERR_ARG, "x is NULL");
  if (!out && c.l_test > 0) return fail(WBM_ERR_ARG, "out is NULL");
  if (!(loading >= 0.0 && std::isfinite(loading))) return fail(WBM_ERR_ARG, "loading must be finite and >= 0");
  if (c.n_elem > 4096) return fail(WBM_ERR_UNSUPPORTED, "full-dimensional MVDR supports N <= 4096");
  if (nk_req == 0) {
    k_first = 0;
    nk_req = c.k_sub;
  }
  if (k_first < 0 || nk_req < 0 || k_first + nk_req > c.k_sub)
    return fail(WBM_ERR_ARG, "subband range outside [0, K)");
  const int k_end = k_first + nk_req;
  hipStream_t st = static_cast<hipStream_t>(stream);
  int sumW = 0;
  if ((s = upload_desc(p, az_rad, nullptr, T, st, &sumW))) return s;
  const size_t NN = (size_t)c.n_elem * c.n_elem;
  if (!p->fullR) {
    const size_t budget = (size_t)8 << 30;
    size_t nk = budget / (sizeof(double2) * NN);
    if (nk < 1) nk = 1;
    if (nk > (size_t)c.k_sub) nk = c.k_sub;
    p->nk_full = (int)nk;
    if ((s = dev_alloc(p, &p->fullR, nk * NN, "full covariance"))) return s;
    if ((s = dev_alloc(p, &p->fullW, nk * (size_t)c.max_targets * c.n_elem, "full weights"))) return s;
    if ((s = dev_alloc(p, &p->fullV, nk * (size_t)c.max_targets * c.n_elem, "full solves"))) return s;
    if ((s = dev_alloc(p, &p->fullQ, nk * (size_t)c.max_targets, "full norms"))) return s;
  }
  WBM_HIP(enqueue_channelize(p, kF32, reinterpret_cast<const float2*>(x), st),
          "channelize launch");
  int* inf = info ? info : p->full_info;
  for (int k0 = k_first; k0 < k_end; k0 += p->nk_full) {
    wbm::FullArgs a;
    a.N = c.n_elem;
    a.K = c.k_sub;
    a.L = c.l_train;
    a.Lt = c.l_test;
    a.B = p->B;
    a.T = T;
    a.k0 = k0;
    a.nk = std::min(p->nk_full, k_end - k0);
    a.delta = loading;
    a.beta = c.beta;
    a.dl = c.d_over_lambda;
    a.half_bin = (c.flags & WBM_HALF_BIN) ? 1 : 0;
    WBM_HIP(wbm::launch_full_mvdr(a, p->dd, p->X, p->fullR, p->fullV, p->fullQ, p->fullW,
                                  reinterpret_cast<float2*>(out), reinterpret_cast<float2*>(weights),
                                  inf, st),
            "full MVDR launch");
  }
  return WBM_OK;
}

// ============================================================================================
// Loading / window predictor

}  // extern "C"

namespace {

constexpr int kMaxJam = 64;
constexpr double kLearnedWin = 33.0;

wbm_status ensure_learned(wbm_plan* p) {
  if (p->pprof) return WBM_OK;
  const wbm_config& c = p->cfg;
  const size_t pairs = (size_t)c.max_targets * c.k_sub;
  const int nbt_max = wbm::beamspace_tiles(c.m_fft, p->B, 11);
  int G = (1024 + c.k_sub - 1) / c.k_sub;
  if (G > 16) G = 16;
  if (G < 1) G = 1;
  p->prof_G = G;
  (void)nbt_max;
  wbm_status s;
  if ((s = dev_alloc(p, &p->pprof, (size_t)c.k_sub * 16 * c.max_targets * 64, "profile partials")))
    return s;
  if ((s = dev_alloc(p, &p->feat, pairs * 64, "features"))) return s;
  if ((s = dev_alloc(p, &p->nnout, pairs * 2, "network outputs"))) return s;
  if ((s = dev_alloc(p, &p->pw, pairs, "pair windows"))) return s;
  return dev_alloc(p, &p->pdelta, pairs, "pair loadings");
}

// Channelize + beamspace (windows if Yw) + profile partials -> features (into feat).
hipError_t enqueue_profiles(wbm_plan* p, const float2* x, int T, int sumW, bool windows,
                            float noise, float* feat, hipStream_t st) {
  const wbm_config& c = p->cfg;
  hipError_t e = enqueue_channelize(p, kExt, x, st);
  if (e != hipSuccess) return e;
  const int nbt = p->tune[kExt].nbt;
  const int G = p->prof_G < nbt ? p->prof_G : nbt;
  e = enqueue_beamspace_windows(p, kExt, T, sumW, st, 0, -1, windows, p->pprof, G);
  if (e != hipSuccess) return e;
  return wbm::launch_features(p->pprof, T, c.k_sub, G, c.l_train, noise, feat, st);
}

wbm_status check_mlp(const wbm_mlp* m) {
  if (!m) return fail(WBM_ERR_ARG, "mlp is NULL");
  hipError_t e = hipSetDevice(m->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  return WBM_OK;
}

}  // namespace

extern "C" {

wbm_status wbm_profiles(wbm_plan* p, const wbm_c32* x, const double* az_rad, int32_t T,
                        double noise_power, float* feat, void* stream) {
  wbm_status s = check_plan(p);
  if (s) return s;
  if (!x || !feat) return fail(WBM_ERR_ARG, "x / feat is NULL");
  if (!(noise_power > 0.0 && std::isfinite(noise_power)))
    return fail(WBM_ERR_ARG, "noise_power must be positive");
  hipStream_t st = static_cast<hipStream_t>(stream);
  int sumW = 0;
  if ((s = upload_desc(p, az_rad, nullptr, T, st, &sumW))) return s;
  if ((s = ensure_learned(p))) return s;
  if ((s = ensure_ext(p))) return s;
  if ((s = fit_beam_tile(p, kExt, T, sumW, false, true))) return s;
  WBM_HIP(enqueue_profiles(p, reinterpret_cast<const float2*>(x), T, sumW, false,
                           (float)noise_power, feat, st),
          "profile launch");
  return WBM_OK;
}

wbm_status wbm_beamform_pairs(wbm_plan* p, const wbm_c32* x, const double* az_rad,
                              const int32_t* win, int32_t T, const int32_t* pair_win,
                              const float* pair_loading, wbm_c32* out, wbm_c32* weights,
                              int32_t* starts, int32_t* info, void* stream) {
  wbm_status s = check_plan(p);
  if (s) return s;
  const wbm_config& c = p->cfg;
  if (!x) return fail(WBM_ERR_ARG, "x is NULL");
  if (!pair_win || !pair_loading) return fail(WBM_ERR_ARG, "pair_win / pair_loading is NULL");
  if (!out && c.l_test > 0) return fail(WBM_ERR_ARG, "out is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  int sumW = 0;
  if ((s = upload_desc(p, az_rad, win, T, st, &sumW))) return s;
  const float2* xx = reinterpret_cast<const float2*>(x);
  if ((s = ready_fused(p, kExt, xx, T, sumW, 0.0, st))) return s;
  WBM_HIP(enqueue_channelize(p, kExt, xx, st), "channelize launch");
  WBM_HIP(enqueue_beamspace_windows(p, kExt, T, sumW, st), "beamspace launch");
  wbm::PairArgs a = pair_args(p, kExt, T, sumW, 0.0);
  a.pw = pair_win;
  a.pdelta = pair_loading;
  WBM_HIP(wbm::launch_mvdr_fused(a, geom(p, T), p->dd, p->Yw, reinterpret_cast<float2*>(out),
                                 reinterpret_cast<float2*>(weights), starts, info,
                                 p->tune[kExt].pair_threads, st),
          "pair MVDR launch");
  return WBM_OK;
}

wbm_status wbm_beamform_learned(wbm_plan* p, const wbm_c32* x, const double* az_rad,
                                int32_t T, const float* params, double noise_power,
                                int32_t fallback_win, double fallback_loading, wbm_c32* out,
                                wbm_c32* weights, int32_t* pair_win, float* pair_loading,
                                int32_t* fallback, int32_t* starts, int32_t* info,
                                void* stream) {
  wbm_status s = check_plan(p);
  if (s) return s;
  const wbm_config& c = p->cfg;
  if (!x || !params) return fail(WBM_ERR_ARG, "x / params is NULL");
  if (!out && c.l_test > 0) return fail(WBM_ERR_ARG, "out is NULL");
  if (c.w_max < (int)kLearnedWin) return fail(WBM_ERR_SHAPE, "the learned form needs w_max >= 33");
  if (fallback_win < 1 || fallback_win > (int)kLearnedWin || (fallback_win & 1) == 0)
    return fail(WBM_ERR_ARG, "fallback_win must be odd and <= 33");
  if (!(fallback_loading >= 0.0 && std::isfinite(fallback_loading)))
    return fail(WBM_ERR_ARG, "fallback_loading must be finite and >= 0");
  if (!(noise_power > 0.0 && std::isfinite(noise_power)))
    return fail(WBM_ERR_ARG, "noise_power must be positive");
  if (T < 1 || T > c.max_targets) return fail(WBM_ERR_SHAPE, "T outside [1, max_targets]");
  std::vector<int32_t> win(T, (int)kLearnedWin);
  hipStream_t st = static_cast<hipStream_t>(stream);
  int sumW = 0;
  if ((s = upload_desc(p, az_rad, win.data(), T, st, &sumW))) return s;
  if ((s = ensure_learned(p))) return s;
  const float2* xx = reinterpret_cast<const float2*>(x);
  if ((s = ready_fused(p, kExt, xx, T, sumW, fallback_loading, st, true))) return s;
  const int n = T * c.k_sub;
  int* pw = pair_win ? pair_win : p->pw;
  float* pd = pair_loading ? pair_loading : p->pdelta;
  WBM_HIP(enqueue_profiles(p, xx, T, sumW, true, (float)noise_power, p->feat, st), "profiles");
  WBM_HIP(wbm::launch_mlp_forward(params, p->feat, n, p->nnout, st), "network forward");
  WBM_HIP(wbm::launch_decide(p->nnout, n, (float)noise_power, (float)fallback_loading,
                             fallback_win, pw, pd, fallback, st),
          "decision");
  wbm::PairArgs a = pair_args(p, kExt, T, sumW, fallback_loading);
  a.pw = pw;
  a.pdelta = pd;
  WBM_HIP(wbm::launch_mvdr_fused(a, geom(p, T), p->dd, p->Yw, reinterpret_cast<float2*>(out),
                                 reinterpret_cast<float2*>(weights), starts, info,
                                 p->tune[kExt].pair_threads, st),
          "pair MVDR launch");
  return WBM_OK;
}

wbm_status wbm_sinr(wbm_plan* p, const double* az_rad, const int32_t* win, int32_t T,
                    const wbm_c32* weights, const int32_t* pair_win, const int32_t* starts,
                    const double* jam_az, const double* jam_inr, int32_t J, double noise_power,
                    float* sinr, void* stream) {
  wbm_status s = check_plan(p);
  if (s) return s;
  if (!weights || !starts || !sinr) return fail(WBM_ERR_ARG, "weights / starts / sinr is NULL");
  if (J < 0 || J > kMaxJam) return fail(WBM_ERR_ARG, "J outside [0, 64]");
  if (J > 0 && (!jam_az || !jam_inr)) return fail(WBM_ERR_ARG, "jam_az / jam_inr is NULL");
  if (!(noise_power > 0.0 && std::isfinite(noise_power)))
    return fail(WBM_ERR_ARG, "noise_power must be positive");
  hipStream_t st = static_cast<hipStream_t>(stream);
  int sumW = 0;
  if ((s = upload_desc(p, az_rad, win, T, st, &sumW))) return s;
  if (!p->jam_dev) {
    if ((s = dev_alloc(p, &p->jam_dev, 2 * kMaxJam, "jammer list"))) return s;
    if (hipHostMalloc((void**)&p->jam_host, sizeof(double) * 2 * kMaxJam, hipHostMallocDefault) !=
        hipSuccess) {
      (void)hipGetLastError();
      return fail(WBM_ERR_NOMEM, "pinned jammer staging allocation failed");
    }
    WBM_HIP(hipEventCreateWithFlags(&p->jam_evt, hipEventDisableTiming), "event create");
  }
  if (p->jam_evt_recorded) WBM_HIP(hipEventSynchronize(p->jam_evt), "jammer staging wait");
  for (int j = 0; j < J; ++j) {
    if (!std::isfinite(jam_az[j]) || !(jam_inr[j] >= 0.0))
      return fail(WBM_ERR_ARG, "jammer " + std::to_string(j) + " not finite / negative INR");
    p->jam_host[j] = std::sin(jam_az[j]);
    p->jam_host[kMaxJam + j] = jam_inr[j];
  }
  WBM_HIP(hipMemcpyAsync(p->jam_dev, p->jam_host, sizeof(double) * 2 * kMaxJam,
                         hipMemcpyHostToDevice, st),
          "jammer upload");
  WBM_HIP(hipEventRecord(p->jam_evt, st), "jammer event");
  p->jam_evt_recorded = true;
  WBM_HIP(wbm::launch_sinr(geom(p, T), reinterpret_cast<const float2*>(weights), p->cfg.w_max,
                           pair_win, starts, p->jam_dev, p->jam_dev + kMaxJam, J, noise_power, sinr,
                           st),
          "SINR launch");
  return WBM_OK;
}

wbm_status wbm_mlp_create(int32_t max_batch, wbm_mlp** out) {
  if (!out) return fail(WBM_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (max_batch < 1 || max_batch > (1 << 24)) return fail(WBM_ERR_ARG, "max_batch out of range");
  wbm_mlp* m = new wbm_mlp();
  m->max_batch = max_batch;
  (void)hipGetDevice(&m->device);
  const int nwg = wbm::mlp_backward_workgroups(max_batch);
  auto bail = [&](const char* what) {
    (void)hipGetLastError();
    wbm_mlp_destroy(m);
    return fail(WBM_ERR_NOMEM, what);
  };
  if (hipMalloc((void**)&m->part, sizeof(float) * (size_t)nwg * wbm::mlp_param_count()) != hipSuccess)
    return bail("gradient partials allocation failed");
  if (hipMalloc((void**)&m->loss_part, sizeof(float) * (size_t)nwg) != hipSuccess)
    return bail("loss partials allocation failed");
  if (hipMalloc((void**)&m->tab_dev, 512) != hipSuccess) return bail("table allocation failed");
  if (hipHostMalloc((void**)&m->tab_host, 512, hipHostMallocDefault) != hipSuccess)
    return bail("pinned table allocation failed");
  if (hipEventCreateWithFlags(&m->tab_evt, hipEventDisableTiming) != hipSuccess)
    return bail("event creation failed");
  *out = m;
  return WBM_OK;
}

wbm_status wbm_mlp_destroy(wbm_mlp* m) {
  if (!m) return WBM_OK;
  (void)hipSetDevice(m->device);
  (void)hipDeviceSynchronize();
  if (m->tab_evt) (void)hipEventDestroy(m->tab_evt);
  if (m->tab_host) (void)hipHostFree(m->tab_host);
  if (m->tab_dev) (void)hipFree(m->tab_dev);
  if (m->part) (void)hipFree(m->part);
  if (m->loss_part) (void)hipFree(m->loss_part);
  delete m;
  return WBM_OK;
}

wbm_status wbm_mlp_forward(wbm_mlp* m, const float* params, const float* in, int32_t n,
                           float* out, void* stream) {
  wbm_status s = check_mlp(m);
  if (s) return s;
  if (!params || !in || !out) return fail(WBM_ERR_ARG, "params / in / out is NULL");
  if (n < 0) return fail(WBM_ERR_ARG, "n < 0");
  WBM_HIP(wbm::launch_mlp_forward(params, in, n, out, static_cast<hipStream_t>(stream)), "forward");
  return WBM_OK;
}

wbm_status wbm_mlp_grad(wbm_mlp* m, const float* params, const float* in, const float* target,
                        int32_t n, float* grad, float* loss, void* stream) {
  wbm_status s = check_mlp(m);
  if (s) return s;
  if (!params || !in || !target || !grad) return fail(WBM_ERR_ARG, "NULL argument");
  if (n < 1 || n > m->max_batch) return fail(WBM_ERR_SHAPE, "n outside [1, max_batch]");
  WBM_HIP(wbm::launch_mlp_backward(params, in, target, n, m->part, m->loss_part, grad, loss,
                                   static_cast<hipStream_t>(stream)),
          "backward");
  return WBM_OK;
}

wbm_status wbm_mlp_grad_static(const float* params, const float* in, const float* target,
                               int32_t n, float* grad, float* loss, void* stream) {
  if (!params || !in || !target || !grad) return fail(WBM_ERR_ARG, "NULL argument");
  if (n < 1 || n > WBM_MLP_STATIC_MAX_BATCH)
    return fail(WBM_ERR_SHAPE, "n outside [1, WBM_MLP_STATIC_MAX_BATCH = " +
                                   std::to_string(WBM_MLP_STATIC_MAX_BATCH) + "]");
  float* part = nullptr;
  float* loss_part = nullptr;
  WBM_HIP(wbm::mlp_static_scratch(&part, &loss_part), "static scratch address");
  WBM_HIP(wbm::launch_mlp_backward(params, in, target, n, part, loss_part, grad, loss,
                                   static_cast<hipStream_t>(stream)),
          "backward");
  return WBM_OK;
}

wbm_status wbm_mlp_adam(wbm_mlp* m, float* params, float* mom, float* var, const float* grad,
                        int32_t step, double lr, void* stream) {
  wbm_status s = check_mlp(m);
  if (s) return s;
  if (!params || !mom || !var || !grad) return fail(WBM_ERR_ARG, "NULL argument");
  if (step < 1) return fail(WBM_ERR_ARG, "step must be >= 1");
  if (!(lr > 0.0 && std::isfinite(lr))) return fail(WBM_ERR_ARG, "lr must be positive");
  const double c1 = 1.0 - std::pow(0.9, step), c2 = 1.0 - std::pow(0.999, step);
  WBM_HIP(wbm::launch_adam(params, mom, var, grad, (float)lr, 0.9f, 0.999f, 1e-8f, (float)c1,
                           (float)c2, static_cast<hipStream_t>(stream)),
          "adam");
  return WBM_OK;
}

wbm_status wbm_sweep_labels(wbm_mlp* m, const float* sinr, int32_t npairs, const double* deltas,
                            int32_t nd, const int32_t* widths, int32_t nw, double noise_power,
                            float* label, void* stream) {
  wbm_status s = check_mlp(m);
  if (s) return s;
  if (!sinr || !deltas || !widths || !label) return fail(WBM_ERR_ARG, "NULL argument");
  if (nd < 1 || nd > 64 || nw < 1 || nw > 64) return fail(WBM_ERR_ARG, "nd, nw must be in [1, 64]");
  if (npairs < 1) return fail(WBM_ERR_ARG, "npairs < 1");
  if (!(noise_power > 0.0)) return fail(WBM_ERR_ARG, "noise_power must be positive");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (m->tab_evt_recorded) WBM_HIP(hipEventSynchronize(m->tab_evt), "table staging wait");
  float* fd = reinterpret_cast<float*>(m->tab_host);
  int* iw = reinterpret_cast<int*>(m->tab_host + 256);
  for (int i = 0; i < nd; ++i) {
    if (!(deltas[i] > 0.0)) return fail(WBM_ERR_ARG, "deltas must be positive");
    fd[i] = (float)deltas[i];
  }
  for (int i = 0; i < nw; ++i) {
    if (widths[i] < 2) return fail(WBM_ERR_ARG, "widths must be >= 2");
    iw[i] = widths[i];
  }
  WBM_HIP(hipMemcpyAsync(m->tab_dev, m->tab_host, 512, hipMemcpyHostToDevice, st), "table upload");
  WBM_HIP(hipEventRecord(m->tab_evt, st), "table event");
  m->tab_evt_recorded = true;
  WBM_HIP(wbm::launch_label(sinr, npairs, reinterpret_cast<const float*>(m->tab_dev), nd,
                            reinterpret_cast<const int*>(m->tab_dev + 256), nw, (float)noise_power,
                            label, st),
          "label launch");
  return WBM_OK;
}

}  // extern "C"
