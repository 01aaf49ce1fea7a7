// Launchers of the loading / window predictor kernels (internal).
#pragma once
#include <hip/hip_runtime.h>

#include "wbm_dev.h"

namespace wbm {

hipError_t launch_features(const float* prof, int T, int K, int G, int L, float noise,
                           float* feat, hipStream_t s);
hipError_t launch_mlp_forward(const float* P, const float* in, int n, float* out, hipStream_t s);
int mlp_backward_workgroups(int n);
int mlp_param_count();
hipError_t launch_mlp_backward(const float* P, const float* in, const float* tgt, int n,
                               float* part, float* loss_part, float* grad, float* loss,
                               hipStream_t s);
// Device addresses (current device) of the static scratch of wbm_mlp_grad_static: gradient
// partials [WBM_MLP_STATIC_MAX_BATCH / 16][params] and loss partials after them.
hipError_t mlp_static_scratch(float** part, float** loss_part);
hipError_t launch_adam(float* P, float* m, float* v, const float* grad, float lr, float beta1,
                       float beta2, float eps, float c1, float c2, hipStream_t s);
hipError_t launch_decide(const float* out, int n, float noise, float fb_delta, int fb_win, int* pw,
                         float* pdelta, int* fallback, hipStream_t s);
hipError_t launch_sinr(const WindowGeom& g, const float2* w, int wmax, const int* pw,
                       const int* starts, const double* jam_sin, const double* jam_inr, int J,
                       double noise, float* sinr, hipStream_t s);
hipError_t launch_label(const float* sinr, int npairs, const float* deltas, int nd,
                        const int* widths, int nw, float noise, float* label, hipStream_t s);

}  // namespace wbm
