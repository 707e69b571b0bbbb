// Device helpers shared by the library's kernels (FP64 patch arithmetic in a
// fixed evaluation order, BF16 rounding).  Library-internal.
#pragma once
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include <cstdint>

#include "cs_internal.h"

namespace cs {

// Symmetric border reflection that repeats the edge pixel: -1 -> 0, n -> n-1.
__device__ __forceinline__ int reflect_idx(int i, int n) {
    return i < 0 ? -i - 1 : (i >= n ? 2 * n - i - 1 : i);
}

// Gray value, FP64, order (0.299 R + 0.587 G) + 0.114 B.
__device__ __forceinline__ double gray64_of(float r, float g, float b) {
#pragma clang fp contract(off)
    return (0.299 * (double)r + 0.587 * (double)g) + 0.114 * (double)b;
}
__device__ __forceinline__ double gray64(const float *rgb, int64_t N, int64_t idx) {
    return gray64_of(rgb[idx], rgb[N + idx], rgb[2 * N + idx]);
}

// Exact FP64 a_j = sum_t O_jt s_t of pixel pix (om = row j of O): the
// normalised Gaussian-masked gray patch rebuilt from the image in the
// oracle's operation order, q_t = w_t g_t, s_t = (q_t - mu) / sqrt(nu2) (0 when
// nu2 = 0), every sum sequential in t and no contraction.  mu = sum_t q_t / n
// and nu2 = sum_t (q_t - mu)^2 come from stats[2 pix], stats[2 pix + 1] (the
// analysis kernel's exact values, the same operations) when stats is
// non-null, else they are computed here.  One lane per entry: loads are
// issued eight elements at a time.
__device__ __noinline__ inline double exact_entry(const float *rgb, int H, int W, int p, const double *wmask,
                                                  const float *om, int64_t pix, const double *stats) {
#pragma clang fp contract(off)
    const int64_t N = (int64_t)H * W;
    const int h = (p - 1) / 2, n = p * p;
    const int row = (int)(pix / W), col = (int)(pix - (int64_t)row * W);
    auto q_at = [&](int t) {
        const int u = t / p, v = t - u * p;
        const int rr = reflect_idx(row + u - h, H), cc = reflect_idx(col + v - h, W);
        return wmask[t] * gray64(rgb, N, (int64_t)rr * W + cc);
    };
    double mu, nu2;
    if (stats) {
        mu = stats[2 * pix];
        nu2 = stats[2 * pix + 1];
    } else {
        double sum = 0.0;
        for (int t0 = 0; t0 < n; t0 += 8) {
            double qv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) qv[u] = q_at(t0 + u < n ? t0 + u : n - 1);
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (t0 + u < n) sum = sum + qv[u];
        }
        mu = sum / (double)n;
        nu2 = 0.0;
        for (int t0 = 0; t0 < n; t0 += 8) {
            double qv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) qv[u] = q_at(t0 + u < n ? t0 + u : n - 1);
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (t0 + u < n) {
                    const double z = qv[u] - mu;
                    nu2 = nu2 + z * z;
                }
        }
    }
    if (nu2 == 0.0) return 0.0;
    const double nu = sqrt(nu2);
    double acc = 0.0;
    for (int t0 = 0; t0 < n; t0 += 8) {
        double qv[8];
        float ov[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int t = t0 + u < n ? t0 + u : n - 1;
            qv[u] = q_at(t);
            ov[u] = om[t];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (t0 + u < n) acc = acc + (double)ov[u] * ((qv[u] - mu) / nu);
    }
    return acc;
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

// Radix selection helpers (256-thread workgroups).
// The digit holding the remaining rank in a complete kHistBins-bin histogram
// (parallel prefix over the bins): the prefix with that digit set and the
// rank left inside it, returned to every thread.
__device__ __forceinline__ void tau_pick_digit(const unsigned int *hist, int shift, unsigned int prefix_in,
                                               unsigned long long rank_in, unsigned int &prefix_out,
                                               unsigned long long &rank_out) {
    constexpr int per = kHistBins / 256;
    __shared__ unsigned long long scan[256];
    __shared__ unsigned int s_pfx;
    __shared__ unsigned long long s_rank;
    const int t = threadIdx.x;
    unsigned int loc[per];
    unsigned long long sum = 0;
#pragma unroll
    for (int i = 0; i < per; ++i) {
        loc[i] = hist[t * per + i];
        sum += loc[i];
    }
    scan[t] = sum;
    if (t == 0) {
        s_pfx = prefix_in;
        s_rank = rank_in;
    }
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const unsigned long long v = t >= off ? scan[t - off] : 0ull;
        __syncthreads();
        scan[t] += v;
        __syncthreads();
    }
    const unsigned long long before = scan[t] - sum;
    if (rank_in >= before && rank_in < scan[t]) {
        unsigned long long rr = rank_in - before;
        for (int i = 0; i < per; ++i) {
            if (rr < loc[i]) {
                s_pfx = prefix_in | ((unsigned int)(t * per + i) << shift);
                s_rank = rr;
                break;
            }
            rr -= loc[i];
        }
    }
    __syncthreads();
    prefix_out = s_pfx;
    rank_out = s_rank;
}

// Set-up of a folded selection by one 256-thread workgroup: per-row margins
// and their maximum, the state (digit 0: empty prefix, the target rank) and
// three cleared histograms.
__device__ __forceinline__ void tau_setup(TauState *st, unsigned int *hist3, const float *omega, int k, int n,
                                          double coef, unsigned long long rank0, double *margins,
                                          double *max_margin) {
    __shared__ double red[4];
    const int t = threadIdx.x;
    double m = 0.0;
    for (int j = t; j < k; j += 256) {
        const double mj = row_margin(omega, j, n, -1.0, coef);
        margins[j] = mj;
        m = fmax(m, mj);
    }
    for (int off = 1; off < 64; off <<= 1) m = fmax(m, __shfl_xor(m, off));
    if ((t & 63) == 0) red[t >> 6] = m;
    for (int i = t; i < 3 * kHistBins; i += 256) hist3[i] = 0u;
    __syncthreads();
    if (t == 0) {
        *max_margin = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
        st->rank0 = rank0;
        st->rank = rank0;
        st->prefix = 0;
        for (int d = 0; d < 4; ++d) {
            st->pfx[d] = 0;
            st->rk[d] = rank0;
        }
        st->nparts = 0;
        st->below = 0;
        st->ncand = 0;
        st->n_d = 0;
        st->n_r = 0;
        st->lo = st->hi = 0.0;
        st->median = 0.0;
        st->tau = 0.0;
    }
}

__device__ __forceinline__ short bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

}  // namespace cs
