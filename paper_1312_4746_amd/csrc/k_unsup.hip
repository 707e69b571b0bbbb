// Unsupervised data term on gfx950 (Sec. 3.1, unsupervised segmentation):
// colour classes by k-means on the pixels' colours, texture classes by
// k-medians on their co-support masks (texture similarity TSM = Hamming
// distance, component-wise median = majority), every (colour, texture) pair a
// segment class, and per pixel the class likelihoods in the form of
// eq:post_text, the data term the convex relaxation (with its label cost) then
// takes.
//
// k-means: the colour distances are FP64, summed in the order of the
// definition without contracted products, so the assignment decides as an
// FP64 evaluation does; the new centroids are FP64 means from per-workgroup
// partial sums added in a fixed order (deterministic).  k-medians: distances
// are popcounts and the medians integer counts, exact whatever the order: a
// wave turns each mask bit into a 64-lane ballot and counts it per class with
// a popcount against the class's ballot, one integer atomic per workgroup,
// class and bit.
#include "cs_internal.h"

namespace cs {

namespace {

constexpr int kUsMaxK = kUnsupMaxClasses;  // classes of one clustering
constexpr int kUsMaxWords = 4;      // 256 co-support bits

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

}  // namespace

// ---- initial centroids (caller-given pixels) ----
__global__ __launch_bounds__(64) void k_us_init(UnsupArgs a, UnsupInit init) {
    const int t = threadIdx.x;
    const int64_t N = a.N;
    if (t < a.Kc) {
        const int64_t p = init.pix[t];
        for (int ch = 0; ch < 3; ++ch) a.ccent[t * 3 + ch] = (double)a.rgb[ch * N + p];
    }
    if (t < a.Kt) {
        const int64_t p = init.pix[a.Kc + t];
        for (int q = 0; q < a.nw; ++q) a.tcent[t * a.nw + q] = a.masks[p * a.nw + q];
    }
}

// ---- k-means: assignment and per-workgroup partial sums ----
// part[blk][a][0..3] = sums of r, g, b and the pixel count of class a.
__global__ __launch_bounds__(256) void k_km_assign(UnsupArgs a, int with_sums) {
#pragma clang fp contract(off)
    __shared__ double s_c[kUsMaxK * 3];
    __shared__ double red[4][4];
    const int64_t N = a.N;
    for (int i = threadIdx.x; i < a.Kc * 3; i += 256) s_c[i] = a.ccent[i];
    __syncthreads();
    const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool in = x < N;
    double r = 0, g = 0, b = 0;
    int best = 0;
    if (in) {
        r = (double)a.rgb[x];
        g = (double)a.rgb[N + x];
        b = (double)a.rgb[2 * N + x];
        double bd = 0;
        for (int c = 0; c < a.Kc; ++c) {
            const double dr = r - s_c[3 * c], dg = g - s_c[3 * c + 1], db = b - s_c[3 * c + 2];
            const double d = (dr * dr + dg * dg) + db * db;
            if (c == 0 || d < bd) {
                bd = d;
                best = c;
            }
        }
        a.clab[x] = best;
    }
    if (!with_sums) return;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int c = 0; c < a.Kc; ++c) {
        const bool mine = in && best == c;
        const double vr = wave_sum_f64(mine ? r : 0.0), vg = wave_sum_f64(mine ? g : 0.0),
                     vb = wave_sum_f64(mine ? b : 0.0);
        const double vn = (double)__popcll(__ballot(mine));
        __syncthreads();
        if (lane == 0) {
            red[w][0] = vr;
            red[w][1] = vg;
            red[w][2] = vb;
            red[w][3] = vn;
        }
        __syncthreads();
        if (threadIdx.x < 4) {
            const int q = threadIdx.x;
            a.cpart[((int64_t)blockIdx.x * a.Kc + c) * 4 + q] = ((red[0][q] + red[1][q]) + red[2][q]) + red[3][q];
        }
    }
}

// New centroids: the partial sums of every workgroup in order; a class
// without pixels keeps its centroid.
__global__ __launch_bounds__(64) void k_km_update(UnsupArgs a, int nparts) {
#pragma clang fp contract(off)
    const int c = threadIdx.x;
    if (c >= a.Kc) return;
    double s[4] = {0, 0, 0, 0};
    for (int p = 0; p < nparts; ++p)
        for (int q = 0; q < 4; ++q) s[q] = s[q] + a.cpart[((int64_t)p * a.Kc + c) * 4 + q];
    if (s[3] > 0.0)
        for (int q = 0; q < 3; ++q) a.ccent[c * 3 + q] = s[q] / s[3];
}

// ---- k-medians: assignment and per-bit counts ----
// tcount[b * k + j]: pixels of class b with bit j set; tsize[b]: pixels of
// class b (both zero before).
__global__ __launch_bounds__(256) void k_kmed_assign(UnsupArgs a, int with_counts) {
    __shared__ uint64_t s_c[kUsMaxK * kUsMaxWords];
    __shared__ unsigned int s_cnt[kUsMaxK * kUsMaxWords * 64];
    __shared__ unsigned int s_size[kUsMaxK];
    const int64_t N = a.N;
    const int nw = a.nw, Kt = a.Kt;
    for (int i = threadIdx.x; i < Kt * nw; i += 256) s_c[i] = a.tcent[i];
    if (with_counts) {
        for (int i = threadIdx.x; i < Kt * nw * 64; i += 256) s_cnt[i] = 0;
        for (int i = threadIdx.x; i < Kt; i += 256) s_size[i] = 0;
    }
    __syncthreads();
    const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool in = x < N;
    uint64_t m[kUsMaxWords] = {0, 0, 0, 0};
    int best = -1;
    if (in) {
        for (int q = 0; q < nw; ++q) m[q] = a.masks[x * nw + q];
        int bd = 0;
        for (int c = 0; c < Kt; ++c) {
            int d = 0;
            for (int q = 0; q < nw; ++q) d += __popcll(m[q] ^ s_c[c * nw + q]);
            if (c == 0 || d < bd) {
                bd = d;
                best = c;
            }
        }
        a.tlab[x] = best;
    }
    if (!with_counts) return;
    const int lane = threadIdx.x & 63;
    uint64_t Cb[kUsMaxK];  // the wave's pixels of each class
#pragma unroll
    for (int c = 0; c < kUsMaxK; ++c) Cb[c] = c < Kt ? __ballot(best == c) : 0ull;
    // lane t ends with the counts of bit 64 q + t of each class
    for (int q = 0; q < nw; ++q) {
        unsigned int mine[kUsMaxK];
#pragma unroll
        for (int c = 0; c < kUsMaxK; ++c) mine[c] = 0;
        for (int t = 0; t < 64; ++t) {
            const uint64_t B = __ballot(in && ((m[q] >> t) & 1ull));
            if (!B) continue;
#pragma unroll
            for (int c = 0; c < kUsMaxK; ++c)
                if (c < Kt && lane == t) mine[c] = (unsigned int)__popcll(B & Cb[c]);
        }
#pragma unroll
        for (int c = 0; c < kUsMaxK; ++c)
            if (c < Kt && mine[c]) atomicAdd(&s_cnt[(c * nw + q) * 64 + lane], mine[c]);
    }
#pragma unroll
    for (int c = 0; c < kUsMaxK; ++c)
        if (c < Kt && lane == 0 && Cb[c]) atomicAdd(&s_size[c], (unsigned int)__popcll(Cb[c]));
    __syncthreads();
    for (int i = threadIdx.x; i < Kt * nw * 64; i += 256) {
        const int c = i / (nw * 64), j = i - c * nw * 64;
        if (j < a.k && s_cnt[i]) atomicAdd(&a.tcount[(int64_t)c * a.k + j], s_cnt[i]);
    }
    for (int i = threadIdx.x; i < Kt; i += 256)
        if (s_size[i]) atomicAdd(&a.tsize[i], s_size[i]);
}

// New texture centroids: bit j of class b set iff 2 count >= size (the median
// of 0/1 values, a tie in); a class without pixels keeps its centroid.  The
// counts are cleared for the next assignment.
__global__ __launch_bounds__(256) void k_kmed_update(UnsupArgs a) {
    const int c = blockIdx.x;
    const unsigned int n = a.tsize[c];
    __syncthreads();
    for (int q = threadIdx.x; q < a.nw; q += 256) {
        if (n) {
            uint64_t w = 0;
            for (int t = 0; t < 64; ++t) {
                const int j = q * 64 + t;
                if (j < a.k && 2ull * a.tcount[(int64_t)c * a.k + j] >= (uint64_t)n) w |= 1ull << t;
            }
            a.tcent[c * a.nw + q] = w;
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < a.k; j += 256) a.tcount[(int64_t)c * a.k + j] = 0;
    if (threadIdx.x == 0) a.tsize[c] = 0;
}

// ---- class likelihoods ----
// loglik[x][a Kt + b] = log P(I(x) | a) + log P(s_x | b): minus the distance
// (||I - mu_a||^2 / (2 sigma_c^2), TSM(x, c_b) / beta), normalised over all
// Kc Kt classes.
__global__ __launch_bounds__(256) void k_us_loglik(UnsupArgs a, float *loglik) {
#pragma clang fp contract(off)
    __shared__ double s_c[kUsMaxK * 3];
    __shared__ uint64_t s_t[kUsMaxK * kUsMaxWords];
    const int64_t N = a.N;
    const int nw = a.nw, Kc = a.Kc, Kt = a.Kt, L = Kc * Kt;
    for (int i = threadIdx.x; i < Kc * 3; i += 256) s_c[i] = a.ccent[i];
    for (int i = threadIdx.x; i < Kt * nw; i += 256) s_t[i] = a.tcent[i];
    __syncthreads();
    const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (x >= N) return;
    const double r = (double)a.rgb[x], g = (double)a.rgb[N + x], b = (double)a.rgb[2 * N + x];
    const double two_s2 = 2.0 * a.sigma_c * a.sigma_c;
    double ec[kUsMaxK], et[kUsMaxK];
    double mc = 0, mt = 0;
    for (int c = 0; c < Kc; ++c) {
        const double dr = r - s_c[3 * c], dg = g - s_c[3 * c + 1], db = b - s_c[3 * c + 2];
        ec[c] = -(((dr * dr + dg * dg) + db * db) / two_s2);
        mc = c == 0 ? ec[c] : (ec[c] > mc ? ec[c] : mc);
    }
    uint64_t m[kUsMaxWords] = {0, 0, 0, 0};
    for (int q = 0; q < nw; ++q) m[q] = a.masks[x * nw + q];
    for (int c = 0; c < Kt; ++c) {
        int d = 0;
        for (int q = 0; q < nw; ++q) d += __popcll(m[q] ^ s_t[c * nw + q]);
        et[c] = -((double)d / a.beta);
        mt = c == 0 ? et[c] : (et[c] > mt ? et[c] : mt);
    }
    // normaliser over all classes, in class order
    double sc = 0, st = 0;
    for (int i = 0; i < L; ++i) {
        sc = sc + exp(ec[i / Kt] - mc);
        st = st + exp(et[i % Kt] - mt);
    }
    const double lc = mc + log(sc), lt = mt + log(st);
    for (int i = 0; i < L; ++i) loglik[x * L + i] = (float)((ec[i / Kt] - lc) + (et[i % Kt] - lt));
}

// ---- launchers ----
hipError_t launch_unsup_init(const LaunchCtx &lc, const UnsupArgs &a, const UnsupInit &init) {
    hipLaunchKernelGGL(k_us_init, dim3(1), dim3(64), 0, lc.stream, a, init);
    return hipGetLastError();
}

hipError_t launch_kmeans_step(const LaunchCtx &lc, const UnsupArgs &a, bool update) {
    const unsigned nb = (unsigned)((a.N + 255) / 256);
    hipLaunchKernelGGL(k_km_assign, dim3(nb), dim3(256), 0, lc.stream, a, update ? 1 : 0);
    if (update) hipLaunchKernelGGL(k_km_update, dim3(1), dim3(64), 0, lc.stream, a, (int)nb);
    return hipGetLastError();
}

hipError_t launch_kmedians_step(const LaunchCtx &lc, const UnsupArgs &a, bool update) {
    const unsigned nb = (unsigned)((a.N + 255) / 256);
    hipLaunchKernelGGL(k_kmed_assign, dim3(nb), dim3(256), 0, lc.stream, a, update ? 1 : 0);
    if (update) hipLaunchKernelGGL(k_kmed_update, dim3((unsigned)a.Kt), dim3(256), 0, lc.stream, a);
    return hipGetLastError();
}

hipError_t launch_unsup_loglik(const LaunchCtx &lc, const UnsupArgs &a, float *loglik) {
    const unsigned nb = (unsigned)((a.N + 255) / 256);
    hipLaunchKernelGGL(k_us_loglik, dim3(nb), dim3(256), 0, lc.stream, a, loglik);
    return hipGetLastError();
}

}  // namespace cs
