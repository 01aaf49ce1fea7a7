// Drives every entry point of the C ABI through the library's real host code, linked against
// the host-only HIP stand-in (hip_stub.cpp), under AddressSanitizer and UBSan.  Shapes are small;
// outputs are not checked (no kernel runs); what is checked is that the host logic -- argument
// validation, descriptor staging, workspace sizing, the autotuner and its cache, graph capture
// with a forked overlap stream, two plans in one process, the static scratch -- makes no invalid
// memory access, no undefined operation and no call the capture rules forbid, and that invalid
// arguments return the documented status.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "wbmvdr.h"

#pragma clang diagnostic ignored "-Wunused-value"
#pragma clang diagnostic ignored "-Wunused-result"

extern "C" long hip_stub_launches();
extern "C" int hip_stub_open_captures();

static int g_fail = 0;
#define EXPECT(call, want)                                                                 \
  do {                                                                                     \
    const int got_ = (int)(call);                                                          \
    if (got_ != (int)(want)) {                                                             \
      std::fprintf(stderr, "line %d: %s returned %d (%s), expected %d\n", __LINE__, #call, \
                   got_, wbm_last_error(), (int)(want));                                   \
      g_fail = 1;                                                                          \
    }                                                                                      \
  } while (0)

template <typename T>
static T* dev(size_t n) {
  void* p = nullptr;
  if (hipMalloc(&p, sizeof(T) * (n ? n : 1)) != hipSuccess) std::abort();
  return static_cast<T*>(p);
}

static wbm_config config(int N, int M, int K, int L, int Lt, int T, int wmax, int flags) {
  wbm_config c{};
  c.n_elem = N; c.m_fft = M; c.k_sub = K; c.l_train = L; c.l_test = Lt;
  c.max_targets = T; c.w_max = wmax; c.flags = flags; c.beta = 0.2; c.d_over_lambda = 0.5;
  return c;
}

static void linear_plan(int flags, hipStream_t st) {
  const int N = 16, M = 32, K = 16, L = 8, Lt = 8, T = 4, W = 9, B = L + Lt;
  const long S = (long)B * K;
  wbm_config cfg = config(N, M, K, L, Lt, T, W, flags);
  wbm_plan* p = nullptr;
  EXPECT(wbm_plan_create(&cfg, &p), WBM_OK);
  if (!p) return;
  auto* x = dev<wbm_c32>((size_t)N * S);
  auto* out = dev<wbm_c32>((size_t)T * K * Lt);
  auto* w = dev<wbm_c32>((size_t)T * K * W);
  auto* starts = dev<int32_t>((size_t)T * K);
  auto* info = dev<int32_t>((size_t)T * K);
  double az[T] = {-0.5, 0.1, 0.3, 0.7};
  int32_t win[T] = {9, 5, 3, 9};
  // every form, twice each (the second call of a form replays its graph or reuses its tuning),
  // a target change between calls, then the same targets again
  for (int rep = 0; rep < 2; ++rep)
    for (int form = 0; form <= 6; ++form)
      EXPECT(wbm_beamform(p, x, az, win, T, 10.0, form, out, w, starts, info, st), WBM_OK);
  double az2[2] = {0.2, -0.2};
  int32_t win2[2] = {5, 7};
  EXPECT(wbm_beamform(p, x, az2, win2, 2, 10.0, WBM_FORM_GRAPH, out, w, starts, info, st), WBM_OK);
  EXPECT(wbm_beamform(p, x, az2, win2, 2, 10.0, WBM_FORM_GRAPH, out, w, nullptr, nullptr, st), WBM_OK);
  EXPECT(wbm_beamform(p, x, az, win, T, 10.0, WBM_FORM_GRAPH, out, w, starts, info, nullptr), WBM_OK);
  // pinned tunings, including overlapped subband chunks (a forked stream inside the capture)
  for (int prec = WBM_PREC_EXT; prec <= WBM_PREC_F32; ++prec) {
    for (int chunks : {1, 2}) {
      const int pair = prec == WBM_PREC_EXT ? WBM_PAIR_BLOCK : WBM_PAIR_MFMA;
      EXPECT(wbm_plan_set_tuning(p, prec, 12, 12, pair, chunks), WBM_OK);
      const int gform = prec == WBM_PREC_EXT ? WBM_FORM_GRAPH : WBM_FORM_GRAPH_F32;
      const int fform = prec == WBM_PREC_EXT ? WBM_FORM_FUSED : WBM_FORM_FUSED_F32;
      EXPECT(wbm_beamform(p, x, az, win, T, 10.0, gform, out, w, starts, info, st), WBM_OK);
      EXPECT(wbm_beamform(p, x, az, win, T, 10.0, gform, out, w, starts, info, st), WBM_OK);
      EXPECT(wbm_beamform(p, x, az, win, T, 10.0, fform, out, w, starts, info, st), WBM_OK);
    }
    int32_t c = 0, b = 0, pk = 0, ov = 0;
    EXPECT(wbm_plan_get_tuning(p, prec, &c, &b, &pk, &ov), WBM_OK);
  }
  EXPECT(wbm_plan_set_tuning(p, WBM_PREC_F32, 11, 11, WBM_PAIR_RESIDENT, 1), WBM_OK);
  EXPECT(wbm_beamform(p, x, az, win, T, 10.0, WBM_FORM_GRAPH_F32, out, w, starts, info, st), WBM_OK);
  // stage entry points and timing
  auto* X = dev<wbm_c32>((size_t)K * B * N);
  auto* Y = dev<wbm_c32>((size_t)K * M * B);
  auto* abar = dev<wbm_c64>((size_t)T * K * W);
  EXPECT(wbm_channelize(p, x, X, st), WBM_OK);
  EXPECT(wbm_beamspace(p, X, Y, st), WBM_OK);
  EXPECT(wbm_steer(p, az, win, T, starts, abar, st), WBM_OK);
  double ms[4];
  for (int prec = 0; prec <= 3; ++prec)
    EXPECT(wbm_stage_times(p, x, az, win, T, 10.0, prec, 2, ms, st), WBM_OK);
  // full-dimensional MVDR on all and on a range of subbands
  auto* fw = dev<wbm_c32>((size_t)T * K * N);
  auto* finfo = dev<int32_t>(K);
  EXPECT(wbm_full_mvdr(p, x, az, T, 10.0, 0, 0, out, fw, finfo, st), WBM_OK);
  EXPECT(wbm_full_mvdr(p, x, az, T, 10.0, 3, 5, out, nullptr, nullptr, st), WBM_OK);
  // beside the path
  auto* chat = dev<wbm_c32>((size_t)T * K * N);
  EXPECT(wbm_lift(p, w, starts, T, chat, st), WBM_OK);
  EXPECT(wbm_apply_lifted(p, x, chat, T, out, st), WBM_OK);
  auto* omega = dev<double>(64);
  auto* pat = dev<float>((size_t)T * K * 64);
  EXPECT(wbm_beam_pattern(p, chat, T * K, omega, 64, pat, st), WBM_OK);
  auto* z = dev<wbm_c32>((size_t)T * Lt * K);
  EXPECT(wbm_synthesize(p, out, T, z, st), WBM_OK);
  const int R = 32, P = 4, Lp = 8, F = 64;
  auto* chirp = dev<wbm_c32>(Lp);
  auto* work = dev<wbm_c32>((size_t)T * P * R + 2 * F + P);
  auto* power = dev<float>((size_t)T * R * P);
  auto* det = dev<uint8_t>((size_t)T * R * P);
  EXPECT(wbm_range_doppler(p, z, T, (int64_t)Lt * K, chirp, Lp, R, P, 2, 8, 10.0, work, power,
                           det, st), WBM_OK);
  // invalid arguments: documented statuses, nothing enqueued
  EXPECT(wbm_beamform(p, nullptr, az, win, T, 10.0, WBM_FORM_FUSED, out, w, starts, info, st), WBM_ERR_ARG);
  EXPECT(wbm_beamform(p, x, az, win, 0, 10.0, WBM_FORM_FUSED, out, w, starts, info, st), WBM_ERR_SHAPE);
  EXPECT(wbm_beamform(p, x, az, win, T + 1, 10.0, WBM_FORM_FUSED, out, w, starts, info, st), WBM_ERR_SHAPE);
  EXPECT(wbm_beamform(p, x, az, win, T, 10.0, 99, out, w, starts, info, st), WBM_ERR_ARG);
  EXPECT(wbm_beamform(p, x, az, win, T, -1.0, WBM_FORM_FUSED, out, w, starts, info, st), WBM_ERR_ARG);
  int32_t badwin[T] = {9, 10, 3, 9};
  EXPECT(wbm_beamform(p, x, az, badwin, T, 10.0, WBM_FORM_FUSED, out, w, starts, info, st), WBM_ERR_ARG);
  EXPECT(wbm_plan_set_tuning(p, WBM_PREC_EXT, 9, 12, WBM_PAIR_BLOCK, 1), WBM_ERR_ARG);
  EXPECT(wbm_plan_set_tuning(p, WBM_PREC_EXT, 12, 12, WBM_PAIR_BLOCK, 3), WBM_ERR_ARG);
  EXPECT(wbm_full_mvdr(p, x, az, T, 10.0, 10, 7, out, nullptr, nullptr, st), WBM_ERR_ARG);
  EXPECT(wbm_plan_destroy(p), WBM_OK);
  hipFree(x); hipFree(out); hipFree(w); hipFree(starts); hipFree(info); hipFree(X); hipFree(Y);
  hipFree(abar); hipFree(fw); hipFree(finfo); hipFree(chat); hipFree(omega); hipFree(pat);
  hipFree(z); hipFree(chirp); hipFree(work); hipFree(power); hipFree(det);
}

// a second plan whose first call is the learned form (its own first tuning), beside the pair
// and SINR entry points and the predictor network
static void learned_plan(hipStream_t st) {
  const int N = 32, M = 64, K = 16, L = 8, Lt = 8, T = 3, W = 33, B = L + Lt;
  const long S = (long)B * K;
  wbm_config cfg = config(N, M, K, L, Lt, T, W, 0);
  wbm_plan* p = nullptr;
  EXPECT(wbm_plan_create(&cfg, &p), WBM_OK);
  if (!p) return;
  auto* x = dev<wbm_c32>((size_t)N * S);
  auto* params = dev<float>(WBM_MLP_PARAMS);
  auto* out = dev<wbm_c32>((size_t)T * K * Lt);
  auto* w = dev<wbm_c32>((size_t)T * K * W);
  auto* pw = dev<int32_t>((size_t)T * K);
  auto* pd = dev<float>((size_t)T * K);
  auto* fb = dev<int32_t>((size_t)T * K);
  auto* starts = dev<int32_t>((size_t)T * K);
  auto* info = dev<int32_t>((size_t)T * K);
  double az[T] = {-0.4, 0.0, 0.5};
  EXPECT(wbm_beamform_learned(p, x, az, T, params, 1.0, 9, 10.0, out, w, pw, pd, fb, starts, info, st), WBM_OK);
  EXPECT(wbm_beamform_learned(p, x, az, T, params, 1.0, 9, 10.0, out, w, nullptr, nullptr, nullptr, nullptr, nullptr, st), WBM_OK);
  int32_t win[T] = {33, 33, 33};
  EXPECT(wbm_beamform_pairs(p, x, az, win, T, pw, pd, out, w, starts, info, st), WBM_OK);
  auto* feat = dev<float>((size_t)T * K * WBM_PROFILE_BINS);
  EXPECT(wbm_profiles(p, x, az, T, 1.0, feat, st), WBM_OK);
  double jaz[2] = {-0.2, 0.6}, jinr[2] = {1e3, 1e4};
  auto* sinr = dev<float>((size_t)T * K);
  EXPECT(wbm_sinr(p, az, win, T, w, pw, starts, jaz, jinr, 2, 1.0, sinr, st), WBM_OK);
  EXPECT(wbm_sinr(p, az, win, T, w, nullptr, starts, jaz, jinr, 0, 1.0, sinr, st), WBM_OK);
  EXPECT(wbm_beamform_learned(p, x, az, T, params, 0.0, 9, 10.0, out, w, pw, pd, fb, starts, info, st), WBM_ERR_ARG);
  // predictor network
  wbm_mlp* m = nullptr;
  EXPECT(wbm_mlp_create(64, &m), WBM_OK);
  const int n = 40;
  auto* in = dev<float>((size_t)n * 64);
  auto* tgt = dev<float>((size_t)n * 2);
  auto* o = dev<float>((size_t)n * 2);
  auto* g = dev<float>(WBM_MLP_PARAMS);
  auto* mm = dev<float>(WBM_MLP_PARAMS);
  auto* vv = dev<float>(WBM_MLP_PARAMS);
  auto* loss = dev<float>(1);
  EXPECT(wbm_mlp_forward(m, params, in, n, o, st), WBM_OK);
  EXPECT(wbm_mlp_grad(m, params, in, tgt, n, g, loss, st), WBM_OK);
  EXPECT(wbm_mlp_grad(m, params, in, tgt, 65, g, loss, st), WBM_ERR_SHAPE);
  for (int step = 1; step <= 3; ++step)
    EXPECT(wbm_mlp_adam(m, params, mm, vv, g, step, 1e-3, st), WBM_OK);
  EXPECT(wbm_mlp_adam(m, params, mm, vv, g, 0, 1e-3, st), WBM_ERR_ARG);
  double deltas[3] = {0.1, 1.0, 10.0};
  int32_t widths[2] = {5, 9};
  auto* sw = dev<float>((size_t)6 * T * K);
  auto* label = dev<float>((size_t)T * K * 2);
  EXPECT(wbm_sweep_labels(m, sw, T * K, deltas, 3, widths, 2, 1.0, label, st), WBM_OK);
  EXPECT(wbm_sweep_labels(m, sw, T * K, deltas, 3, widths, 2, 1.0, label, st), WBM_OK);
  EXPECT(wbm_mlp_destroy(m), WBM_OK);
  // the allocation-free gradient: the largest batch, then a smaller one, then one too large
  const int nmax = WBM_MLP_STATIC_MAX_BATCH;
  auto* inb = dev<float>((size_t)nmax * 64);
  auto* tgtb = dev<float>((size_t)nmax * 2);
  EXPECT(wbm_mlp_grad_static(params, inb, tgtb, nmax, g, loss, st), WBM_OK);
  EXPECT(wbm_mlp_grad_static(params, in, tgt, n, g, nullptr, st), WBM_OK);
  EXPECT(wbm_mlp_grad_static(params, inb, tgtb, nmax + 1, g, loss, st), WBM_ERR_SHAPE);
  EXPECT(wbm_mlp_grad_static(nullptr, in, tgt, n, g, loss, st), WBM_ERR_ARG);
  EXPECT(wbm_plan_destroy(p), WBM_OK);
  for (void* q : {(void*)x, (void*)params, (void*)out, (void*)w, (void*)pw, (void*)pd, (void*)fb,
                  (void*)starts, (void*)info, (void*)feat, (void*)sinr, (void*)in, (void*)tgt,
                  (void*)o, (void*)g, (void*)mm, (void*)vv, (void*)loss, (void*)sw, (void*)label,
                  (void*)inb, (void*)tgtb})
    hipFree(q);
}

// the planar array: 2 x 8 elements, 4 x 16 beams
static void planar_plan(hipStream_t st) {
  const int nz = 2, mz = 4, N = 16, M = 64, K = 8, L = 6, Lt = 3, T = 3, W = 12, B = L + Lt;
  const long S = (long)B * K;
  wbm_config cfg = config(N, M, K, L, Lt, T, W, WBM_HALF_BIN);
  wbm_plan* p = nullptr;
  EXPECT(wbm_plan_create(&cfg, &p), WBM_OK);
  if (!p) return;
  auto* x = dev<wbm_c32>((size_t)N * S);
  auto* out = dev<wbm_c32>((size_t)T * K * Lt);
  auto* w = dev<wbm_c32>((size_t)T * K * W);
  auto* starts = dev<int32_t>((size_t)T * K * 2);
  auto* info = dev<int32_t>((size_t)T * K);
  double az[T] = {-0.3, 0.2, 0.6}, el[T] = {0.1, 0.3, 0.0};
  int32_t wz[T] = {2, 1, 3}, wx[T] = {4, 5, 4};
  for (int form : {WBM_FORM_PLAIN, WBM_FORM_FUSED, WBM_FORM_MIXED, WBM_FORM_MIXED_BF16, WBM_FORM_FUSED})
    EXPECT(wbm_beamform_upa(p, x, nz, mz, az, el, wz, wx, T, 10.0, form, out, w, starts, info, st), WBM_OK);
  EXPECT(wbm_beamform_upa(p, x, nz, mz, az, el, wz, wx, T, 10.0, WBM_FORM_GRAPH, out, w, starts, info, st), WBM_ERR_UNSUPPORTED);
  EXPECT(wbm_beamform_upa(p, x, 3, mz, az, el, wz, wx, T, 10.0, WBM_FORM_FUSED, out, w, starts, info, st), WBM_ERR_SHAPE);
  int32_t wbig[T] = {4, 1, 3};
  EXPECT(wbm_beamform_upa(p, x, nz, mz, az, el, wbig, wx, T, 10.0, WBM_FORM_FUSED, out, w, starts, info, st), WBM_ERR_ARG);
  auto* X = dev<wbm_c32>((size_t)K * B * N);
  auto* Y = dev<wbm_c32>((size_t)K * M * B);
  EXPECT(wbm_beamspace_upa(p, X, nz, mz, Y, st), WBM_OK);
  auto* abar = dev<wbm_c64>((size_t)T * K * W);
  EXPECT(wbm_steer_upa(p, nz, mz, az, el, wz, wx, T, starts, abar, st), WBM_OK);
  auto* wzd = dev<int32_t>(T);
  hipMemcpy(wzd, wz, sizeof(wz), hipMemcpyHostToDevice);
  auto* chat = dev<wbm_c32>((size_t)T * K * N);
  EXPECT(wbm_lift_upa(p, w, starts, nz, mz, wzd, T, chat, st), WBM_OK);
  auto* omega = dev<double>(2 * 16);
  auto* pat = dev<float>((size_t)T * K * 16);
  EXPECT(wbm_beam_pattern_upa(p, chat, T * K, nz, omega, 16, pat, st), WBM_OK);
  // a linear call on the same plan between planar ones
  int32_t win[T] = {5, 7, 9};
  EXPECT(wbm_beamform(p, x, az, win, T, 10.0, WBM_FORM_GRAPH, out, w, nullptr, info, st), WBM_OK);
  EXPECT(wbm_beamform_upa(p, x, nz, mz, az, el, wz, wx, T, 10.0, WBM_FORM_FUSED, out, w, starts, info, st), WBM_OK);
  EXPECT(wbm_plan_destroy(p), WBM_OK);
  for (void* q : {(void*)x, (void*)out, (void*)w, (void*)starts, (void*)info, (void*)X, (void*)Y,
                  (void*)abar, (void*)wzd, (void*)chat, (void*)omega, (void*)pat})
    hipFree(q);
}

// Extreme and unusual shapes: every form once (no autotuning), full-dimensional MVDR where
// N <= 4096, so that each launcher's grid, block and LDS request is checked at the limits.
static void shape_sweep(hipStream_t st) {
  struct Shape { int N, M, K, L, Lt, T, W; };
  const Shape shapes[] = {
      {1, 2, 2, 1, 1, 1, 1},            // one element, the smallest spatial DFT
      {2, 2, 2, 1, 1, 2, 2},            // W = M = N = 2
      {3, 4, 2, 2, 0, 2, 3},            // no test snapshots
      {5, 8, 4, 3, 1, 3, 8},            // windows as wide as M
      {33, 64, 8192, 1, 1, 2, 5},       // the most subbands
      {100, 128, 16, 5, 3, 7, 33},      // N not a power of two
      {2048, 8192, 2, 2, 2, 2, 64},     // split-half extended spatial DFT (2N <= M = 8192)
      {4096, 8192, 2, 1, 1, 2, 64},     // the largest array
      {3000, 4096, 4, 2, 1, 3, 17},     // N > M / 2: no zero-half skip
      {64, 64, 32, 4, 4, 40, 64},       // many targets, W = M = N
  };
  setenv("WBM_AUTOTUNE", "0", 1);
  for (const Shape& sh : shapes) {
    const int fail_before = g_fail;
    g_fail = 0;
    wbm_config cfg = config(sh.N, sh.M, sh.K, sh.L, sh.Lt, sh.T, sh.W, 0);
    wbm_plan* p = nullptr;
    EXPECT(wbm_plan_create(&cfg, &p), WBM_OK);
    if (!p) continue;
    const long S = (long)(sh.L + sh.Lt) * sh.K;
    auto* x = dev<wbm_c32>((size_t)sh.N * S);
    auto* out = dev<wbm_c32>((size_t)sh.T * sh.K * (sh.Lt ? sh.Lt : 1));
    auto* w = dev<wbm_c32>((size_t)sh.T * sh.K * sh.W);
    auto* starts = dev<int32_t>((size_t)sh.T * sh.K);
    auto* info = dev<int32_t>((size_t)sh.T * sh.K);
    std::vector<double> az(sh.T);
    std::vector<int32_t> win(sh.T);
    for (int t = 0; t < sh.T; ++t) {
      az[t] = -1.2 + 2.4 * t / (sh.T > 1 ? sh.T - 1 : 1);
      win[t] = 1 + (t * 7) % sh.W;
    }
    win[0] = sh.W;
    for (int form = 0; form <= 6; ++form)
      EXPECT(wbm_beamform(p, x, az.data(), win.data(), sh.T, 10.0, form, out, w, starts, info, st), WBM_OK);
    auto* fw = dev<wbm_c32>((size_t)sh.T * sh.K * sh.N);
    auto* finfo = dev<int32_t>(sh.K);
    EXPECT(wbm_full_mvdr(p, x, az.data(), sh.T, 10.0, 0, sh.K < 4 ? sh.K : 4, out, fw, finfo, st), WBM_OK);
    EXPECT(wbm_plan_destroy(p), WBM_OK);
    for (void* q : {(void*)x, (void*)out, (void*)w, (void*)starts, (void*)info, (void*)fw, (void*)finfo})
      hipFree(q);
    if (g_fail)
      std::fprintf(stderr, "  (shape N=%d M=%d K=%d L=%d Lt=%d T=%d W=%d)\n", sh.N, sh.M, sh.K,
                   sh.L, sh.Lt, sh.T, sh.W);
    g_fail |= fail_before;
  }
  unsetenv("WBM_AUTOTUNE");
}

// Planar geometries at their limits: one row, one column, the longest z-DFT, the widest x-FFT.
static void planar_sweep(hipStream_t st) {
  struct Geo { int Nz, Nx, Mz, Mx, K, T, Wz, Wx; };
  const Geo geos[] = {
      {1, 16, 1, 32, 4, 2, 1, 5},       // one row
      {8, 1, 16, 2, 2, 2, 3, 1},        // one column
      {100, 4, 128, 16, 2, 2, 4, 3},    // longest z-DFT the tile allows
      {2, 300, 2, 1024, 2, 2, 2, 8},    // widest x-FFT of a two-row array
      {4, 4, 4, 4, 8, 3, 4, 4},         // no zero padding, window = whole grid
  };
  setenv("WBM_AUTOTUNE", "0", 1);
  for (const Geo& g : geos) {
    const int fail_before = g_fail;
    g_fail = 0;
    const int N = g.Nz * g.Nx, M = g.Mz * g.Mx, L = 3, Lt = 2, W = g.Wz * g.Wx;
    wbm_config cfg = config(N, M, g.K, L, Lt, g.T, W, 0);
    wbm_plan* p = nullptr;
    EXPECT(wbm_plan_create(&cfg, &p), WBM_OK);
    if (!p) continue;
    const long S = (long)(L + Lt) * g.K;
    auto* x = dev<wbm_c32>((size_t)N * S);
    auto* out = dev<wbm_c32>((size_t)g.T * g.K * Lt);
    auto* w = dev<wbm_c32>((size_t)g.T * g.K * W);
    auto* starts = dev<int32_t>((size_t)g.T * g.K * 2);
    auto* info = dev<int32_t>((size_t)g.T * g.K);
    std::vector<double> az(g.T), el(g.T);
    std::vector<int32_t> wz(g.T, g.Wz), wx(g.T, g.Wx);
    for (int t = 0; t < g.T; ++t) {
      az[t] = -0.8 + 1.6 * t / (g.T - 1);
      el[t] = 0.1 * t;
    }
    for (int form : {WBM_FORM_PLAIN, WBM_FORM_FUSED, WBM_FORM_MIXED, WBM_FORM_MIXED_BF16})
      EXPECT(wbm_beamform_upa(p, x, g.Nz, g.Mz, az.data(), el.data(), wz.data(), wx.data(), g.T,
                              10.0, form, out, w, starts, info, st), WBM_OK);
    auto* wzd = dev<int32_t>(g.T);
    hipMemcpy(wzd, wz.data(), sizeof(int32_t) * g.T, hipMemcpyHostToDevice);
    auto* chat = dev<wbm_c32>((size_t)g.T * g.K * N);
    EXPECT(wbm_lift_upa(p, w, starts, g.Nz, g.Mz, wzd, g.T, chat, st), WBM_OK);
    auto* omega = dev<double>(2 * 8);
    auto* pat = dev<float>((size_t)g.T * g.K * 8);
    EXPECT(wbm_beam_pattern_upa(p, chat, g.T * g.K, g.Nz, omega, 8, pat, st), WBM_OK);
    EXPECT(wbm_apply_lifted(p, x, chat, g.T, out, st), WBM_OK);
    EXPECT(wbm_plan_destroy(p), WBM_OK);
    for (void* q : {(void*)x, (void*)out, (void*)w, (void*)starts, (void*)info, (void*)wzd,
                    (void*)chat, (void*)omega, (void*)pat})
      hipFree(q);
    if (g_fail)
      std::fprintf(stderr, "  (planar Nz=%d Nx=%d Mz=%d Mx=%d K=%d)\n", g.Nz, g.Nx, g.Mz, g.Mx, g.K);
    g_fail |= fail_before;
  }
  unsetenv("WBM_AUTOTUNE");
}

// Self-checks of the seam itself (each must end the process with a report): a stream created
// while a capture is open, and a write one element past a buffer from hipMalloc.
static int plant(const char* what) {
  hipStream_t a = nullptr, b = nullptr;
  hipStreamCreateWithFlags(&a, hipStreamNonBlocking);
  if (std::string(what) == "capture") {
    hipStreamBeginCapture(a, hipStreamCaptureModeThreadLocal);
    hipStreamCreateWithFlags(&b, hipStreamNonBlocking);
  } else if (std::string(what) == "oob") {
    auto* q = dev<float>(16);
    volatile float* v = q;
    v[16] = 1.0f;
    hipFree(q);
  }
  std::printf("planted %s: not caught\n", what);
  return 0;
}

// Calls whose window-row tables outgrow the spatial DFT's LDS: a call that fits only smaller
// tiles than the tuned (or pinned) one runs at the largest that fits, and the plan reports it;
// a call that fits none is rejected with WBM_ERR_SHAPE before any launch; the autotuner leaves
// out the tiles that cannot hold the call's rows.
static void window_row_limits(hipStream_t st) {
  const int N = 64, M = 2048, K = 2, L = 2, Lt = 1, TMAX = 1100, W = 64;
  const long S = (long)(L + Lt) * K;
  for (int tuned = 0; tuned < 2; ++tuned) {
    if (!tuned) setenv("WBM_AUTOTUNE", "0", 1);
    wbm_config cfg = config(N, M, K, L, Lt, TMAX, W, 0);
    wbm_plan* p = nullptr;
    EXPECT(wbm_plan_create(&cfg, &p), WBM_OK);
    if (!p) return;
    auto* x = dev<wbm_c32>((size_t)N * S);
    auto* out = dev<wbm_c32>((size_t)TMAX * K * Lt);
    auto* w = dev<wbm_c32>((size_t)TMAX * K * W);
    auto* starts = dev<int32_t>((size_t)TMAX * K);
    auto* info = dev<int32_t>((size_t)TMAX * K);
    auto* feat = dev<float>((size_t)TMAX * K * 64);
    std::vector<double> az(TMAX);
    std::vector<int32_t> win(TMAX, W);
    for (int t = 0; t < TMAX; ++t) az[t] = -1.2 + 2.4 * t / (TMAX - 1);
    // 320 targets x 64 bins = 20480 rows: the extended tile 2^13 (128 KiB transform tile) cannot
    // hold them, 2^12 can
    const int T1 = 320;
    if (!tuned) {
      // K = 2: the extended channelizer's 2^13 tile (4096 two-point rows, padded) exceeds 160 KiB
      EXPECT(wbm_plan_set_tuning(p, WBM_PREC_EXT, 13, 12, WBM_PAIR_BLOCK, 1), WBM_ERR_UNSUPPORTED);
      EXPECT(wbm_plan_set_tuning(p, WBM_PREC_EXT, 12, 13, WBM_PAIR_BLOCK, 1), WBM_OK);
      EXPECT(wbm_plan_set_tuning(p, WBM_PREC_F32, 12, 13, WBM_PAIR_BLOCK, 1), WBM_OK);
    }
    for (int form : {WBM_FORM_FUSED, WBM_FORM_GRAPH, WBM_FORM_FUSED_F32, WBM_FORM_MIXED})
      EXPECT(wbm_beamform(p, x, az.data(), win.data(), T1, 10.0, form, out, w, starts, info, st), WBM_OK);
    int32_t chan = 0, beam = 0, pair = 0, ovl = 0;
    EXPECT(wbm_plan_get_tuning(p, WBM_PREC_EXT, &chan, &beam, &pair, &ovl), WBM_OK);
    if (beam > 12) {
      std::fprintf(stderr, "line %d: extended beam tile %d holds 20480 window rows\n", __LINE__, beam);
      g_fail = 1;
    }
    if (!tuned) {   // FP32 at 2^13 (64 KiB tile) holds them: the pinned tile stays
      EXPECT(wbm_plan_get_tuning(p, WBM_PREC_F32, &chan, &beam, &pair, &ovl), WBM_OK);
      if (beam != 13) {
        std::fprintf(stderr, "line %d: FP32 beam tile moved to %d\n", __LINE__, beam);
        g_fail = 1;
      }
    }
    // 1100 x 64 = 70400 rows fit no tile: rejected, nothing launched
    const long before = hip_stub_launches();
    for (int form = WBM_FORM_FUSED; form <= WBM_FORM_GRAPH_F32; ++form)
      EXPECT(wbm_beamform(p, x, az.data(), win.data(), TMAX, 10.0, form, out, w, starts, info, st),
             WBM_ERR_SHAPE);
    EXPECT(wbm_profiles(p, x, az.data(), TMAX, 1.0, feat, st), WBM_ERR_SHAPE);
    std::vector<float> params(WBM_MLP_PARAMS, 0.f);
    auto* dparams = dev<float>(WBM_MLP_PARAMS);
    EXPECT(wbm_beamform_learned(p, x, az.data(), TMAX, dparams, 1.0, 9, 10.0, out, w, nullptr,
                                nullptr, nullptr, starts, info, st),
           WBM_ERR_SHAPE);
    if (hip_stub_launches() != before) {
      std::fprintf(stderr, "line %d: %ld launches for rejected calls\n", __LINE__,
                   hip_stub_launches() - before);
      g_fail = 1;
    }
    // and the plan still serves calls that fit
    EXPECT(wbm_beamform(p, x, az.data(), win.data(), 8, 10.0, WBM_FORM_GRAPH, out, w, starts, info, st), WBM_OK);
    EXPECT(wbm_plan_destroy(p), WBM_OK);
    for (void* q : {(void*)x, (void*)out, (void*)w, (void*)starts, (void*)info, (void*)feat, (void*)dparams})
      hipFree(q);
    if (!tuned) unsetenv("WBM_AUTOTUNE");
  }
}

int main(int argc, char** argv) {
  if (argc > 2 && std::string(argv[1]) == "--plant") return plant(argv[2]);
  if (argc > 1) setenv("WBM_AUTOTUNE_CACHE", argv[1], 1);
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return 2;
  wbm_config bad = config(16, 24, 16, 8, 8, 4, 9, 0);          // M not a power of two
  wbm_plan* none = nullptr;
  EXPECT(wbm_plan_create(&bad, &none), WBM_ERR_ARG);
  bad = config(1, 1, 2, 1, 1, 1, 1, 0);                         // a one-point spatial DFT
  EXPECT(wbm_plan_create(&bad, &none), WBM_ERR_ARG);
  EXPECT(wbm_plan_create(nullptr, &none), WBM_ERR_ARG);
  linear_plan(0, st);
  linear_plan(WBM_HALF_BIN, st);
  learned_plan(st);
  planar_plan(st);
  shape_sweep(st);
  planar_sweep(st);
  window_row_limits(st);
  EXPECT(wbm_plan_destroy(nullptr), WBM_OK);
  hipStreamDestroy(st);
  if (hip_stub_open_captures() != 0) {
    std::fprintf(stderr, "a stream capture was left open\n");
    g_fail = 1;
  }
  std::printf("host seam: %ld kernel launches checked, %s\n", hip_stub_launches(),
              g_fail ? "FAILED" : "ok");
  return g_fail;
}
