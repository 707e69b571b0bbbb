// Exact selection of the co-support threshold tau = frac * median|a| on
// gfx950.  The threshold stands in for the exact-zero test of the Sec. 2
// co-support definition; the median is the lower median over all N*k entries
// of the FP64 analysed vectors.
//
// 1. Radix select (11/11/10-bit digits, LDS-privatised histograms) finds the
//    float value v of the target rank among the rounded |a| (the |a| bit
//    patterns order like unsigned integers).
// 2. Every rounded |a| is within the proven margin m of its exact value, so
//    the exact median lies in [v - m, v + m]; entries whose rounded value lies
//    in [v - 2m, v + 2m] are gathered as candidates and the entries below that
//    window are counted.
// 3. The candidates are recomputed in FP64 (same operation order as the
//    oracle's patch and product) and a single-workgroup radix select over their
//    64-bit patterns picks the rank that remains after the count below.
#pragma clang fp contract(off)

#include "cs_internal.h"
#include "cs_device.h"

namespace cs {

constexpr int kHistBins = 2048;

__global__ void k_tau_init(TauState *st, unsigned long long rank0) {
    st->rank0 = rank0;
    st->rank = rank0;
    st->prefix = 0;
    st->below = 0;
    st->ncand = 0;
    st->lo = st->hi = 0.0;
    st->median = 0.0;
    st->tau = 0.0;
}

__global__ __launch_bounds__(256) void k_tau_hist(const float *alpha, int64_t count, int shift,
                                                   unsigned int pmask, const TauState *st,
                                                   unsigned int *hist) {
    __shared__ unsigned int lh[kHistBins];
    for (int i = threadIdx.x; i < kHistBins; i += 256) lh[i] = 0;
    __syncthreads();
    const unsigned int pval = st->prefix & pmask;
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < count; e += stride) {
        const unsigned int key = __float_as_uint(alpha[e]) & 0x7FFFFFFFu;
        if ((key & pmask) == pval) atomicAdd(&lh[(key >> shift) & (kHistBins - 1)], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kHistBins; i += 256)
        if (lh[i]) atomicAdd(&hist[i], lh[i]);
}

// Pick the digit holding the remaining rank, then clear the histogram.
__global__ __launch_bounds__(256) void k_tau_pick(unsigned int *hist, int shift, TauState *st) {
    if (threadIdx.x == 0) {
        unsigned long long r = st->rank;
        for (int b = 0; b < kHistBins; ++b) {
            if (r < hist[b]) {
                st->prefix |= (unsigned int)b << shift;
                break;
            }
            r -= hist[b];
        }
        st->rank = r;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kHistBins; i += 256) hist[i] = 0;
}

__global__ __launch_bounds__(256) void k_tau_clear(unsigned int *hist) {
    for (int i = threadIdx.x; i < kHistBins; i += 256) hist[i] = 0;
}

hipError_t tau_select_float(const LaunchCtx &lc, const float *alpha, int64_t count,
                            unsigned int *hist, TauState *st) {
    hipLaunchKernelGGL(k_tau_init, dim3(1), dim3(1), 0, lc.stream, st,
                       (unsigned long long)((count - 1) / 2));
    const int shifts[3] = {21, 10, 0};
    const unsigned int pmasks[3] = {0u, 0xFFE00000u, 0xFFFFFC00u};
    int64_t blocks = (count + 255) / 256;
    const int64_t cap = (int64_t)lc.num_cu * 16;
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_tau_clear, dim3(1), dim3(256), 0, lc.stream, hist);
    for (int pass = 0; pass < 3; ++pass) {
        hipLaunchKernelGGL(k_tau_hist, dim3((unsigned)blocks), dim3(256), 0, lc.stream, alpha, count,
                           shifts[pass], pmasks[pass], st, hist);
        hipLaunchKernelGGL(k_tau_pick, dim3(1), dim3(256), 0, lc.stream, hist, shifts[pass], st);
    }
    return hipGetLastError();
}

__global__ void k_tau_reset(TauState *st) {
    st->below = 0;
    st->ncand = 0;
}

hipError_t tau_reset_gather(const LaunchCtx &lc, TauState *st) {
    hipLaunchKernelGGL(k_tau_reset, dim3(1), dim3(1), 0, lc.stream, st);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_tau_gather(const float *alpha, int64_t count,
                                                     const double *max_margin, TauState *st,
                                                     int64_t *cand, int64_t cap) {
    __shared__ unsigned long long red[256];
    // The three digit passes left the selected float's bit pattern in prefix.
    const double v = (double)__uint_as_float(st->prefix);
    const double w = 2.0 * (*max_margin);
    const double lo = v - w, hi = v + w;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->lo = lo;
        st->hi = hi;
    }
    unsigned long long below = 0;
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < count; e += stride) {
        const double x = (double)fabsf(alpha[e]);
        if (x < lo) {
            ++below;
        } else if (x <= hi) {
            unsigned long long slot = atomicAdd(&st->ncand, 1ull);
            if ((int64_t)slot < cap) cand[slot] = e;
        }
    }
    red[threadIdx.x] = below;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0 && red[0]) atomicAdd(&st->below, red[0]);
}

hipError_t tau_gather(const LaunchCtx &lc, const float *alpha, int64_t count,
                      const double *max_margin, TauState *st, int64_t *cand, int64_t cap) {
    int64_t blocks = (count + 255) / 256;
    const int64_t bcap = (int64_t)lc.num_cu * 16;
    if (blocks > bcap) blocks = bcap;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_tau_gather, dim3((unsigned)blocks), dim3(256), 0, lc.stream, alpha, count,
                       max_margin, st, cand, cap);
    return hipGetLastError();
}

// FP64 recompute of each candidate entry e = pixel * k + j.
__global__ __launch_bounds__(64) void k_tau_recompute(const float *rgb, int H, int W, int p,
                                                       const double *wmask, const float *omega,
                                                       int k, const int64_t *cand, int64_t ncand,
                                                       double *vals) {
    const int64_t c = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (c >= ncand) return;
    double s[15 * 15];
    const int64_t e = cand[c];
    const int64_t pix = e / k;
    const int j = (int)(e - pix * k);
    const int n = p * p;
    patch_s64(rgb, H, W, p, wmask, pix, s);
    vals[c] = fabs(dot64(omega + (int64_t)j * n, s, n));
}

// Single-workgroup radix select of rank (rank0 - below) among the FP64
// candidate values (non-negative doubles order like their bit patterns).
__global__ __launch_bounds__(1024) void k_tau_select64(const double *vals, int64_t ncand,
                                                        double frac, TauState *st) {
    __shared__ unsigned int hist[256];
    __shared__ unsigned long long s_prefix, s_rank;
    __shared__ int s_ok;
    if (threadIdx.x == 0) {
        s_prefix = 0;
        const unsigned long long r0 = st->rank0, below = st->below;
        s_ok = (r0 >= below) && (r0 - below < (unsigned long long)ncand);
        s_rank = s_ok ? r0 - below : 0;
    }
    __syncthreads();
    if (!s_ok) {
        if (threadIdx.x == 0) {
            st->median = __longlong_as_double(0x7FF8000000000000ll);  // NaN: bound violated
            st->tau = st->median;
        }
        return;
    }
    for (int pass = 0; pass < 8; ++pass) {
        const int shift = 56 - 8 * pass;
        const unsigned long long pmask = pass == 0 ? 0ull : (~0ull << (64 - 8 * pass));
        for (int i = threadIdx.x; i < 256; i += 1024) hist[i] = 0;
        __syncthreads();
        const unsigned long long pval = s_prefix;
        for (int64_t c = threadIdx.x; c < ncand; c += 1024) {
            const unsigned long long key = (unsigned long long)__double_as_longlong(vals[c]);
            if ((key & pmask) == pval) atomicAdd(&hist[(key >> shift) & 255ull], 1u);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long r = s_rank;
            for (int b = 0; b < 256; ++b) {
                if (r < hist[b]) {
                    s_prefix |= (unsigned long long)b << shift;
                    break;
                }
                r -= hist[b];
            }
            s_rank = r;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double med = __longlong_as_double((long long)s_prefix);
        st->median = med;
        st->tau = frac * med;
    }
}

hipError_t tau_finish(const LaunchCtx &lc, const float *rgb, int H, int W, int p, int n,
                      const double *wmask, const float *omega, int k, const int64_t *cand,
                      int64_t ncand, double *vals, double frac, TauState *st) {
    (void)n;
    if (ncand > 0)
        hipLaunchKernelGGL(k_tau_recompute, dim3((unsigned)((ncand + 63) / 64)), dim3(64), 0,
                           lc.stream, rgb, H, W, p, wmask, omega, k, cand, ncand, vals);
    hipLaunchKernelGGL(k_tau_select64, dim3(1), dim3(1024), 0, lc.stream, vals, ncand, frac, st);
    return hipGetLastError();
}

}  // namespace cs
