// Float shadow of the SVT fit for calibrating the sector constants.
//
// The shadow evaluates the same linearized fit as the integer path (every
// fit row a scalar product of per-sector constants with the input words plus
// an offset, Sec. 2) on unquantized fp32 words.  Loss of a batch of N tracks:
//     L_data = (1/N) sum_t [ sum_{k<3} w_k (y_k - tau_k)^2 + sum_{k>=3} y_k^2 ]
// plus an orthonormality penalty lambda sum_s ||C_s C_s^T - I||^2 on the
// constraint rows C_s.  Rows are computed in fp32 (fma chains); every sum over
// tracks is accumulated in fp64 with a fixed reduction order, so results are
// bit-reproducible.
//
// Tracks are grouped by sector (CSR sector_offsets).  Pass 1 runs one block
// per (sector, slice) with the sector's constants in scalar registers; pass 2
// reduces the slices of each sector in order.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "svt.h"
#include "svt_shadow.h"

namespace svt {
namespace {

constexpr int kSBlock = 256;
constexpr int kSWaves = kSBlock / 64;
constexpr int kNG = 43;   // 36 coefficient sums, 6 offset sums, 1 loss

struct SArgs {
    const float *x;
    const float *tau;
    const int32_t *off;
    int32_t n_tracks, n_sectors, slices;
    float w0, w1, w2;
    const float *coef;
    const float *offset;
    float *y;             // optional [n][6]
    double *part;         // [n_sectors * slices][kNG]
};

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ void slice_range(const SArgs &a, int &t0, int &t1, int &s)
{
    s = blockIdx.x / a.slices;
    const int i = blockIdx.x - s * a.slices;
    int lo = a.off[s], hi = a.off[s + 1];
    lo = lo < 0 ? 0 : (lo > a.n_tracks ? a.n_tracks : lo);
    hi = hi < lo ? lo : (hi > a.n_tracks ? a.n_tracks : hi);
    const int64_t len = hi - lo;
    t0 = lo + (int)(len * i / a.slices);
    t1 = lo + (int)(len * (i + 1) / a.slices);
}

// y = A x + b for one track, fp32.
__device__ __forceinline__ void rows(const float *A, const float *b, const float *x, float *y)
{
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        float v = b[k];
#pragma unroll
        for (int j = 0; j < 6; ++j) v = fmaf(A[k * 6 + j], x[j], v);
        y[k] = v;
    }
}

// Block-level fixed-order sum of NV doubles per thread into part[0..NV).
template <int NV>
__device__ void block_store_sums(double (&v)[NV], double *part)
{
    __shared__ double s_w[kSWaves][NV];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = wave_sum(v[q]);
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) s_w[wid][q] = v[q];
    }
    __syncthreads();
    for (int q = threadIdx.x; q < NV; q += kSBlock) {
        double t = 0.0;
        for (int w = 0; w < kSWaves; ++w) t += s_w[w][q];
        part[q] = t;
    }
}

__global__ void __launch_bounds__(kSBlock) shadow_fwd(SArgs a)
{
    int t0, t1, s;
    slice_range(a, t0, t1, s);
    float A[36], b[6];
#pragma unroll
    for (int q = 0; q < 36; ++q) A[q] = a.coef[s * 36 + q];
#pragma unroll
    for (int q = 0; q < 6; ++q) b[q] = a.offset[s * 6 + q];
    double loss = 0.0;
    for (int t = t0 + threadIdx.x; t < t1; t += kSBlock) {
        float x[6], y[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) x[j] = a.x[(int64_t)t * 6 + j];
        rows(A, b, x, y);
        if (a.y) {
#pragma unroll
            for (int k = 0; k < 6; ++k) a.y[(int64_t)t * 6 + k] = y[k];
        }
        const float r0 = y[0] - a.tau[(int64_t)t * 3 + 0];
        const float r1 = y[1] - a.tau[(int64_t)t * 3 + 1];
        const float r2 = y[2] - a.tau[(int64_t)t * 3 + 2];
        double l = (double)a.w0 * (double)r0 * (double)r0;
        l = fma((double)a.w1 * (double)r1, (double)r1, l);
        l = fma((double)a.w2 * (double)r2, (double)r2, l);
        l = fma((double)y[3], (double)y[3], l);
        l = fma((double)y[4], (double)y[4], l);
        l = fma((double)y[5], (double)y[5], l);
        loss += l;
    }
    double v[1] = {loss};
    block_store_sums<1>(v, a.part + (size_t)blockIdx.x * kNG + 42);
}

__global__ void __launch_bounds__(kSBlock) shadow_bwd(SArgs a)
{
    int t0, t1, s;
    slice_range(a, t0, t1, s);
    float A[36], b[6];
#pragma unroll
    for (int q = 0; q < 36; ++q) A[q] = a.coef[s * 36 + q];
#pragma unroll
    for (int q = 0; q < 6; ++q) b[q] = a.offset[s * 6 + q];
    const float wk[6] = {a.w0, a.w1, a.w2, 1.f, 1.f, 1.f};
    double g[42];
#pragma unroll
    for (int q = 0; q < 42; ++q) g[q] = 0.0;
    for (int t = t0 + threadIdx.x; t < t1; t += kSBlock) {
        float x[6], y[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) x[j] = a.x[(int64_t)t * 6 + j];
        rows(A, b, x, y);
        float r[6];
        r[0] = wk[0] * (y[0] - a.tau[(int64_t)t * 3 + 0]);
        r[1] = wk[1] * (y[1] - a.tau[(int64_t)t * 3 + 1]);
        r[2] = wk[2] * (y[2] - a.tau[(int64_t)t * 3 + 2]);
        r[3] = y[3];
        r[4] = y[4];
        r[5] = y[5];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const double rk = (double)r[k];
#pragma unroll
            for (int j = 0; j < 6; ++j) g[k * 6 + j] = fma(rk, (double)x[j], g[k * 6 + j]);
            g[36 + k] += rk;
        }
    }
    block_store_sums<42>(g, a.part + (size_t)blockIdx.x * kNG);
}

// Pass 2 of the backward: per sector, the slices in order; scaled by
// scale * 2 / N.  One thread per (sector, value).
__global__ void shadow_bwd_reduce(const double *part, int32_t n_sectors, int32_t slices,
                                  double factor, const double *scale, double *g_coef,
                                  double *g_off, float *g_coef32, float *g_off32)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_sectors * 42) return;
    const int s = i / 42, q = i - s * 42;
    double t = 0.0;
    for (int k = 0; k < slices; ++k) t += part[((size_t)s * slices + k) * kNG + q];
    t *= factor * (scale ? scale[0] : 1.0);
    if (q < 36) {
        g_coef[s * 36 + q] = t;
        if (g_coef32) g_coef32[s * 36 + q] = (float)t;
    } else {
        g_off[s * 6 + (q - 36)] = t;
        if (g_off32) g_off32[s * 6 + (q - 36)] = (float)t;
    }
}

// Pass 2 of the forward: one block; thread i sums blocks i, i + 256, ... in
// order, then a fixed shuffle tree and the waves in order.
__global__ void __launch_bounds__(kSBlock) shadow_fwd_reduce(const double *part, int32_t n_blocks,
                                                             double inv_n, double *loss)
{
    __shared__ double s_w[kSWaves];
    double t = 0.0;
    for (int k = threadIdx.x; k < n_blocks; k += kSBlock) t += part[(size_t)k * kNG + 42];
    t = wave_sum(t);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        double u = 0.0;
        for (int w = 0; w < kSWaves; ++w) u += s_w[w];
        loss[0] = u * inv_n;
    }
}

// Orthonormality penalty of the constraint rows, one thread per sector, then
// a fixed-order sum by thread 0 of block 0 (n_sectors <= 256: one block).
__global__ void shadow_penalty(const float *coef, int32_t n_sectors, double lam, double *value,
                               double *g_coef, float *g_coef32)
{
    __shared__ double s_val[256];
    const int s = threadIdx.x;
    double val = 0.0;
    if (s < n_sectors) {
        double C[3][6];
        for (int k = 0; k < 3; ++k)
            for (int j = 0; j < 6; ++j) C[k][j] = (double)coef[s * 36 + (3 + k) * 6 + j];
        double G[3][3];
        for (int k = 0; k < 3; ++k)
            for (int m = 0; m < 3; ++m) {
                double d = 0.0;
                for (int j = 0; j < 6; ++j) d = fma(C[k][j], C[m][j], d);
                G[k][m] = d - (k == m ? 1.0 : 0.0);
                val = fma(G[k][m], G[k][m], val);
            }
        for (int k = 0; k < 3; ++k)
            for (int j = 0; j < 6; ++j) {
                double d = 0.0;
                for (int m = 0; m < 3; ++m) d = fma(G[k][m], C[m][j], d);
                const double add = 4.0 * lam * d;
                const int idx = s * 36 + (3 + k) * 6 + j;
                g_coef[idx] += add;
                if (g_coef32) g_coef32[idx] = (float)g_coef[idx];
            }
    }
    s_val[s] = lam * val;
    __syncthreads();
    if (s == 0) {
        double t = 0.0;
        for (int k = 0; k < n_sectors; ++k) t += s_val[k];
        value[0] = t;
    }
}

__global__ void adam_step(int32_t n, float *p, const double *g, float *m, float *v, float lr,
                          float b1, float b2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = (float)g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Per sector: the largest shift S in [-30, 30] with every |rint(A 2^S)| <
// max_abs and every row within the int32 bound of the integer fit.
__global__ void requantize_k(const float *coef, const float *offset, int32_t n_sectors,
                             int32_t max_abs, int32_t *coef_i, int32_t *off_i, int32_t *shift,
                             int32_t *status)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_sectors) return;
    for (int S = 30; S >= -30; --S) {
        bool ok = true;
        for (int k = 0; k < 6 && ok; ++k) {
            double row = fabs(rint(ldexp((double)offset[s * 6 + k], S)));
            for (int j = 0; j < 6; ++j) {
                const double q = rint(ldexp((double)coef[s * 36 + k * 6 + j], S));
                if (fabs(q) >= (double)max_abs) ok = false;
                row += fabs(q) * 4095.0;
            }
            if (row > 2147483647.0) ok = false;
        }
        if (!ok) continue;
        for (int q = 0; q < 36; ++q) coef_i[s * 36 + q] = (int32_t)rint(ldexp((double)coef[s * 36 + q], S));
        for (int k = 0; k < 6; ++k) off_i[s * 6 + k] = (int32_t)rint(ldexp((double)offset[s * 6 + k], S));
        shift[s] = S;
        return;
    }
    shift[s] = INT32_MIN;
    atomicExch(status, 1);
}

}  // namespace

int shadow_slices(int32_t n_tracks, int32_t n_sectors)
{
    // about 2048 tracks per block, at least one slice, at most 64
    const int64_t per = n_sectors > 0 ? ((int64_t)n_tracks + n_sectors - 1) / n_sectors : 0;
    int sl = (int)((per + 2047) / 2048);
    if (sl < 1) sl = 1;
    if (sl > 64) sl = 64;
    return sl;
}

size_t shadow_scratch_bytes(int32_t n_tracks, int32_t n_sectors)
{
    return (size_t)n_sectors * shadow_slices(n_tracks, n_sectors) * kNG * sizeof(double);
}

hipError_t launch_shadow_forward(const ShadowCall &c, double *scratch, hipStream_t st)
{
    SArgs a{c.x, c.tau, c.off, c.n_tracks, c.n_sectors, shadow_slices(c.n_tracks, c.n_sectors),
            c.w[0], c.w[1], c.w[2], c.coef, c.offset, c.y, scratch};
    const int nb = c.n_sectors * a.slices;
    hipLaunchKernelGGL(shadow_fwd, dim3(nb), dim3(kSBlock), 0, st, a);
    hipLaunchKernelGGL(shadow_fwd_reduce, dim3(1), dim3(kSBlock), 0, st, scratch, nb,
                       c.n_tracks > 0 ? 1.0 / c.n_tracks : 0.0, c.loss);
    return hipGetLastError();
}

hipError_t launch_shadow_backward(const ShadowCall &c, const double *scale, double *scratch,
                                  hipStream_t st)
{
    SArgs a{c.x, c.tau, c.off, c.n_tracks, c.n_sectors, shadow_slices(c.n_tracks, c.n_sectors),
            c.w[0], c.w[1], c.w[2], c.coef, c.offset, nullptr, scratch};
    const int nb = c.n_sectors * a.slices;
    hipLaunchKernelGGL(shadow_bwd, dim3(nb), dim3(kSBlock), 0, st, a);
    const double factor = c.n_tracks > 0 ? 2.0 / c.n_tracks : 0.0;
    const int n = c.n_sectors * 42;
    hipLaunchKernelGGL(shadow_bwd_reduce, dim3((n + 255) / 256), dim3(256), 0, st, scratch,
                       c.n_sectors, a.slices, factor, scale, c.g_coef, c.g_off, c.g_coef32,
                       c.g_off32);
    return hipGetLastError();
}

hipError_t launch_shadow_penalty(const float *coef, int32_t n_sectors, double lam, double *value,
                                 double *g_coef, float *g_coef32, hipStream_t st)
{
    hipLaunchKernelGGL(shadow_penalty, dim3(1), dim3(256), 0, st, coef, n_sectors, lam, value,
                       g_coef, g_coef32);
    return hipGetLastError();
}

hipError_t launch_adam(int32_t n, float *p, const double *g, float *m, float *v, float lr, float b1,
                       float b2, float eps, int32_t step, hipStream_t st)
{
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(adam_step, dim3((n + 255) / 256), dim3(256), 0, st, n, p, g, m, v, lr, b1,
                       b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_requantize(const float *coef, const float *offset, int32_t n_sectors,
                             int32_t max_abs, int32_t *coef_i, int32_t *off_i, int32_t *shift,
                             int32_t *status, hipStream_t st)
{
    hipLaunchKernelGGL(requantize_k, dim3((n_sectors + 63) / 64), dim3(64), 0, st, coef, offset,
                       n_sectors, max_abs, coef_i, off_i, shift, status);
    return hipGetLastError();
}

}  // namespace svt
