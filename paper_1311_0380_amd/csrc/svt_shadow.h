// Internal declarations of the float-shadow kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace svt {

struct ShadowCall {
    const float *x;        // [n][6]
    const float *tau;      // [n][3]
    const int32_t *off;    // [n_sectors + 1]
    int32_t n_tracks, n_sectors;
    float w[3];
    const float *coef;     // [S][6][6]
    const float *offset;   // [S][6]
    float *y;              // optional [n][6]
    double *loss;          // [1]
    double *g_coef;        // [S][6][6]
    double *g_off;         // [S][6]
    float *g_coef32;       // optional
    float *g_off32;        // optional
};

int shadow_slices(int32_t n_tracks, int32_t n_sectors);
size_t shadow_scratch_bytes(int32_t n_tracks, int32_t n_sectors);
hipError_t launch_shadow_forward(const ShadowCall &c, double *scratch, hipStream_t st);
hipError_t launch_shadow_backward(const ShadowCall &c, const double *scale, double *scratch, hipStream_t st);
hipError_t launch_shadow_penalty(const float *coef, int32_t n_sectors, double lam, double *value,
                                 double *g_coef, float *g_coef32, hipStream_t st);
hipError_t launch_adam(int32_t n, float *p, const double *g, float *m, float *v, float lr, float b1,
                       float b2, float eps, int32_t step, hipStream_t st);
hipError_t launch_requantize(const float *coef, const float *offset, int32_t n_sectors,
                             int32_t max_abs, int32_t *coef_i, int32_t *off_i, int32_t *shift,
                             int32_t *status, hipStream_t st);

}  // namespace svt
