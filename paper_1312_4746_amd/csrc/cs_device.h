// Device helpers shared by the library's kernels (FP64 patch arithmetic in a
// fixed evaluation order, BF16 rounding).  Library-internal.
#pragma once
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cs {

// Symmetric border reflection that repeats the edge pixel: -1 -> 0, n -> n-1.
__device__ __forceinline__ int reflect_idx(int i, int n) {
    return i < 0 ? -i - 1 : (i >= n ? 2 * n - i - 1 : i);
}

// Gray value, FP64, order (0.299 R + 0.587 G) + 0.114 B.
__device__ __forceinline__ double gray64(const float *rgb, int64_t N, int64_t idx) {
#pragma clang fp contract(off)
    double r = (double)rgb[idx], g = (double)rgb[N + idx], b = (double)rgb[2 * N + idx];
    return (0.299 * r + 0.587 * g) + 0.114 * b;
}

// sum_t O_jt s_t, sequential in t, no FMA.
__device__ __noinline__ inline double dot64(const float *om, const double *s, int n) {
#pragma clang fp contract(off)
    double acc = 0.0;
    for (int t = 0; t < n; ++t) acc = acc + (double)om[t] * s[t];
    return acc;
}

// Exact normalised patch of one pixel from global memory: q_t = w_t g_t,
// mu = sum_t q_t / n, z = q - mu, nu2 = sum_t z_t^2, s = z / sqrt(nu2) (or 0),
// every sum sequential in t.  Same operations as the LDS path of the
// analysis kernel.
__device__ __noinline__ inline void patch_s64(const float *rgb, int H, int W, int p,
                                              const double *wmask, int64_t pix, double *s) {
#pragma clang fp contract(off)
    const int64_t N = (int64_t)H * W;
    const int h = (p - 1) / 2, n = p * p;
    const int row = (int)(pix / W), col = (int)(pix - (int64_t)(pix / W) * W);
    for (int t = 0; t < n; ++t) {
        int u = t / p, v = t - u * p;
        int rr = reflect_idx(row + u - h, H), cc = reflect_idx(col + v - h, W);
        s[t] = wmask[t] * gray64(rgb, N, (int64_t)rr * W + cc);
    }
    double sum = 0.0;
    for (int t = 0; t < n; ++t) sum = sum + s[t];
    double mu = sum / (double)n;
    for (int t = 0; t < n; ++t) s[t] = s[t] - mu;
    double nu2 = 0.0;
    for (int t = 0; t < n; ++t) nu2 = nu2 + s[t] * s[t];
    if (nu2 == 0.0) {
        for (int t = 0; t < n; ++t) s[t] = 0.0;
        return;
    }
    double nu = sqrt(nu2);
    for (int t = 0; t < n; ++t) s[t] = s[t] / nu;
}

// Per-row decision margin: the given absolute margin when >= 0, else the
// proven bound coef * ||O_j||_2 of the rounded analysed vector (unit-norm
// patch) with a relative safety factor for the FP64 evaluation of the bound
// itself and a tiny absolute term for flushed subnormal products.
__device__ __forceinline__ double row_margin(const float *omega, int j, int n, double margin, double coef) {
#pragma clang fp contract(off)
    if (margin >= 0.0) return margin;
    double ss = 0.0;
    for (int t = 0; t < n; ++t) {
        const double o = (double)omega[(int64_t)j * n + t];
        ss = ss + o * o;
    }
    return coef * sqrt(ss) * (1.0 + 0x1p-20) + 0x1p-100;
}

__device__ __forceinline__ short bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

}  // namespace cs
