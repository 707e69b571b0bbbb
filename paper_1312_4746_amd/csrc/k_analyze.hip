// Patch analysis on gfx950: normalised Gaussian-masked gray patches, the
// contraction a = O s on MFMA, and the co-support threshold epilogue.
//
// Paper: Sec. 2 (analysed vector a = O s, co-support of zero entries, bias
// and gain normalisation) and Sec. 3.1 (gray patch s_x centred at x, Gaussian
// mask applied before normalisation).
//
// One workgroup owns a row segment of TP pixels (128 for p <= 9, else 64).
// 1. The FP64 gray values of the segment and its halo are staged in LDS.
// 2. One thread per pixel computes the exact statistics of its masked patch
//    q_t = w_t g_t: mu = (sum_t q_t)/n and nu2 = sum_t (q_t - mu)^2, each sum
//    sequential in t with no FMA contraction (the oracle's operations).
// 3. The normalised patch s_t = (q_t - mu)/sqrt(nu2) is written to LDS in
//    FP32 (via the FP64 reciprocal: within one FP64 ulp of the exact quotient,
//    far inside the FP32 rounding the error bound already counts).
// 4. a = O s on MFMA with A = patches (rows = pixels, LDS) and B = O^T
//    (columns = operator rows, from L2); each wave owns every fourth 16-pixel
//    block and walks all 16-row blocks of O.
//
// Output layout of the 16x16 MFMA tile: lane l, accumulator r holds pixel
// 4*(l/16) + r of the block and operator row l%16 of the j-block, so one wave
// ballot over a predicate on accumulator r yields four 16-bit co-support
// pieces (one per pixel), which land directly in the packed mask words.
//
// Entries whose rounded |a| lies within the per-row margin of tau are
// recomputed in FP64 from the exact patch (rebuilt on the fly from the LDS
// gray values and the exact statistics, in the oracle's operation order) and
// decided exactly.
#pragma clang fp contract(off)

#include "cs_internal.h"
#include "cs_device.h"
#include "../../include/cosparse.h"

namespace cs {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short s16x4 __attribute__((ext_vector_type(4)));

template <int P>
struct AnalyzeTile {
    // ss: LDS row stride of the FP32 patches; np / 4 + 1 is odd, so lane (g, jl)
    // of an MFMA operand read (row jl, column 4 kb + g) hits bank 4 odd jl + g,
    // 64 distinct banks
    static constexpr int h = (P - 1) / 2, n = P * P, np = (n + 15) / 16 * 16, ss = np + 4;
    static constexpr int np4 = (n + 3) / 4 * 4;    // K extent of the FP32 MFMA steps
    static constexpr int TP = P <= 9 ? 128 : 64;  // pixels per workgroup
    static constexpr int hw = TP + 2 * h;
};

// Exact FP64 a_j = sum_t O_jt s_t of pixel il of the tile, the patch rebuilt
// from the LDS gray halo and the exact statistics: q_t = w_t g_t,
// s_t = (q_t - mu) / sqrt(nu2) (0 when nu2 = 0), summed in t order.
template <int P>
__device__ __noinline__ double exact_dot(const float *om, const double *gh, const double *wmask, int il,
                                         double mu, double nu2) {
#pragma clang fp contract(off)
    using T = AnalyzeTile<P>;
    const double nu = nu2 == 0.0 ? 0.0 : sqrt(nu2);
    double acc = 0.0;
    for (int t = 0; t < T::n; ++t) {
        const int u = t / P, v = t - u * P;
        const double q = wmask[t] * gh[u * T::hw + il + v];
        const double st = nu2 == 0.0 ? 0.0 : (q - mu) / nu;
        acc = acc + (double)om[t] * st;
    }
    return acc;
}

template <int PREC, int P>
__global__ __launch_bounds__(256) void k_analyze(AnalyzeArgs a) {
    using T = AnalyzeTile<P>;
    constexpr int h = T::h, n = T::n, np = T::np, ss = T::ss, TP = T::TP, hw = T::hw;
    extern __shared__ __align__(16) unsigned char smem[];
    double *gh = reinterpret_cast<double *>(smem);   // (2h+1) x hw gray halo
    double *st_mu = gh + (2 * h + 1) * hw;            // TP exact means
    double *st_nu2 = st_mu + TP;                       // TP exact squared norms
    double *st_rinv = st_nu2 + TP;                     // TP values 1/sqrt(nu2) (0 if nu2 = 0)
    double *wm = st_rinv + TP;                         // the n mask weights (read at every t)
    float *s = reinterpret_cast<float *>(wm + np);     // TP x ss FP32 patches
    uint16_t *mk = reinterpret_cast<uint16_t *>(s + TP * ss);  // TP x 4*W64 pieces
    const int W64 = (a.k + 63) / 64;

    const int row = blockIdx.y, c0 = blockIdx.x * TP;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t N = (int64_t)a.H * a.W;
    const int valid_px = min(TP, a.W - c0);

    // 1. FP64 gray halo of the segment (all colour loads issued before the
    // first is used; positions past the row end read pixel 0 and store 0).
    constexpr int kHalo = (2 * h + 1) * hw, kHaloIt = (kHalo + 255) / 256;
    const int ncols = valid_px + 2 * h;
    float hr[kHaloIt], hg[kHaloIt], hb[kHaloIt];
#pragma unroll
    for (int it = 0; it < kHaloIt; ++it) {
        const int idx = tid + 256 * it;
        const int rr = idx / hw, cc = idx - rr * hw;
        int64_t src = 0;
        if (idx < kHalo && cc < ncols)
            src = (int64_t)reflect_idx(row - h + rr, a.H) * a.W + reflect_idx(c0 - h + cc, a.W);
        hr[it] = a.rgb[src];
        hg[it] = a.rgb[N + src];
        hb[it] = a.rgb[2 * N + src];
    }
#pragma unroll
    for (int it = 0; it < kHaloIt; ++it) {
        const int idx = tid + 256 * it;
        const int cc = idx - (idx / hw) * hw;
        if (idx < kHalo) gh[idx] = cc < ncols ? gray64_of(hr[it], hg[it], hb[it]) : 0.0;
    }
    for (int t = tid; t < n; t += 256) wm[t] = a.wmask[t];
    if (a.masks)
        for (int idx = tid; idx < TP * 4 * W64; idx += 256) mk[idx] = 0;
    __syncthreads();

    // 2. exact statistics, one thread per pixel, sequential in t.
    for (int i = tid; i < TP; i += 256) {
#pragma clang fp contract(off)
        double sum = 0.0;
        for (int t = 0; t < n; ++t) {
            const int u = t / P, v = t - u * P;
            sum = sum + wm[t] * gh[u * hw + i + v];
        }
        const double mu = sum / (double)n;
        double nu2 = 0.0;
        for (int t = 0; t < n; ++t) {
            const int u = t / P, v = t - u * P;
            const double z = wm[t] * gh[u * hw + i + v] - mu;
            nu2 = nu2 + z * z;
        }
        st_mu[i] = mu;
        st_nu2[i] = nu2;
        st_rinv[i] = nu2 == 0.0 ? 0.0 : 1.0 / sqrt(nu2);
        if (a.pstats && i < valid_px) {
            double *ps = a.pstats + 2 * ((int64_t)row * a.W + c0 + i);
            ps[0] = mu;
            ps[1] = nu2;
        }
    }
    __syncthreads();

    // 3. FP32 normalised patches (zero for pixels past the row end and t >= n).
    for (int idx = tid; idx < TP * np; idx += 256) {
        const int i = idx / np, t = idx - i * np;
        float sv = 0.0f;
        if (i < valid_px && t < n) {
            const int u = t / P, v = t - u * P;
            sv = (float)((wm[t] * gh[u * hw + i + v] - st_mu[i]) * st_rinv[i]);
        }
        s[i * ss + t] = sv;
    }
    __syncthreads();

    // 4. a = O s on MFMA.  Wave w owns the operator row blocks (j-blocks)
    // w, w + 4, w + 8, ..., taken in pairs (jb, jb + 4); the B fragments of a
    // pair are loaded once (unconditional loads with clamped row and column: a
    // clamped t >= n meets a zero patch entry, rows past k give outputs that
    // are not stored), then every 16-pixel block of the tile streams its A
    // fragments from LDS past both.
    const int nblk_j = (a.k + 15) / 16;
    unsigned long long nrecomp = 0;
    // FP32 K steps.  Where padding K to np costs at most one step (11 x 11
    // and 13 x 13 patches), the K order is cut into four runs of np / 4, lane
    // group g = lane / 16 taking patch entries (np / 4) g + kb, so the lane's A
    // values are 16-byte aligned runs of its patch row: one ds_read_b128 per
    // four steps, the next one in flight while four steps are multiplied
    // (the row stride keeps a 16-lane group's reads on distinct banks).
    constexpr bool RUNS = np / 4 - T::np4 / 4 <= 1;
    constexpr int KF = RUNS ? np / 4 : T::np4 / 4, KH = np / 16;  // FP32 and BF16 K steps
    for (int jp = wave; jp < nblk_j; jp += 8) {
        const int jbs[2] = {jp, jp + 4};
        const bool pair = jp + 4 < nblk_j;
        float bf[2][KF];
        s16x4 bb[2][KH];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int jj = jbs[u] * 16 + (lane & 15);
            const float *o = a.omega + (int64_t)(jj < a.k ? jj : a.k - 1) * n;
            if (PREC == CS_FP32) {
#pragma unroll
                for (int kb = 0; kb < KF; ++kb) {
                    const int t = RUNS ? KF * (lane >> 4) + kb : kb * 4 + (lane >> 4);
                    bf[u][kb] = o[t < n ? t : n - 1];
                }
            } else {
#pragma unroll
                for (int kb = 0; kb < KH; ++kb)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int t = kb * 16 + 4 * (lane >> 4) + q;
                        bb[u][kb][q] = bf16_rne(o[t < n ? t : n - 1]);
                    }
            }
        }
        float tin[2], tout[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int j = jbs[u] * 16 + (lane & 15);
            const bool jv = j < a.k;
            tin[u] = (a.masks && jv) ? a.t_in[j] : 0.f;
            tout[u] = (a.masks && jv) ? a.t_out[j] : 0.f;
        }
        for (int rb = 0; rb < TP / 16; ++rb) {
            if (rb * 16 >= valid_px) break;
            const float *srow = s + (rb * 16 + (lane & 15)) * ss;
            f32x4 acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
            if (PREC == CS_FP32 && RUNS) {
                const float4 *arun = reinterpret_cast<const float4 *>(srow + KF * (lane >> 4));
                float4 cur = arun[0];
#pragma unroll
                for (int q = 0; q < KF / 4; ++q) {
                    const float4 nxt = arun[q + 1 < KF / 4 ? q + 1 : q];
                    const float av[4] = {cur.x, cur.y, cur.z, cur.w};
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bf[0][4 * q + i], acc[0], 0, 0, 0);
                        if (pair)
                            acc[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bf[1][4 * q + i], acc[1], 0, 0, 0);
                    }
                    cur = nxt;
                    // keep the next run's read one step ahead, not hoisted
                    __builtin_amdgcn_sched_barrier(0);
                }
            } else if (PREC == CS_FP32) {
#pragma unroll
                for (int kb = 0; kb < KF; ++kb) {
                    const float av = srow[kb * 4 + (lane >> 4)];
                    acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bf[0][kb], acc[0], 0, 0, 0);
                    if (pair) acc[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bf[1][kb], acc[1], 0, 0, 0);
                }
            } else {
#pragma unroll
                for (int kb = 0; kb < KH; ++kb) {
                    const int t0 = kb * 16 + 4 * (lane >> 4);
                    s16x4 av;
#pragma unroll
                    for (int q = 0; q < 4; ++q) av[q] = bf16_rne(srow[t0 + q]);
                    acc[0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bb[0][kb], acc[0], 0, 0, 0);
                    if (pair) acc[1] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bb[1][kb], acc[1], 0, 0, 0);
                }
            }
            // Epilogue: store a and/or decide the co-support bits.
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                if (u == 1 && !pair) break;
                const int jb = jbs[u];
                const int j = jb * 16 + (lane & 15);
                const bool jv = j < a.k;
                const float *om = a.omega + (int64_t)(jv ? j : 0) * n;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int il = rb * 16 + 4 * (lane >> 4) + r;
                    const bool pv = il < valid_px;
                    const float v = acc[u][r];
                    const int64_t pix = (int64_t)row * a.W + c0 + il;
                    if (a.alpha && pv && jv) a.alpha[pix * a.k + j] = v;
                    if (a.masks) {
                        const float av = fabsf(v);
                        bool in = av <= tin[u];
                        const bool out = av > tout[u];
                        const bool near = !in && !out && pv && jv;
                        if (near) in = fabs(exact_dot<P>(om, gh, wm, il, st_mu[il], st_nu2[il])) <= a.tau;
                        nrecomp += (unsigned long long)__popcll(__ballot(near));
                        const unsigned long long bits = __ballot(in && pv && jv);
                        if (lane < 4)
                            mk[(rb * 16 + 4 * lane + r) * (4 * W64) + jb] =
                                (uint16_t)((bits >> (16 * lane)) & 0xFFFFull);
                    }
                }
            }
        }
    }

    if (a.masks) {
        __syncthreads();
        const uint64_t *mk64 = reinterpret_cast<const uint64_t *>(mk);
        for (int idx = tid; idx < valid_px * W64; idx += 256) {
            const int i = idx / W64, w = idx - i * W64;
            a.masks[((int64_t)row * a.W + c0 + i) * W64 + w] = mk64[i * W64 + w];
        }
        if (a.recomputed && lane == 0 && nrecomp) atomicAdd(a.recomputed, nrecomp);
    }
    // the set-up of the median selection that follows this kernel
    if (a.tau_st && blockIdx.x == 0 && blockIdx.y == 0)
        tau_setup(a.tau_st, a.tau_hist3, a.omega, a.k, n, a.tau_coef, a.tau_rank0, a.tau_margins, a.tau_max_margin);
}

template <int PREC, int P>
static hipError_t launch_analyze_p(const LaunchCtx &lc, const AnalyzeArgs &a) {
    using T = AnalyzeTile<P>;
    const int W64 = (a.k + 63) / 64;
    const size_t lds = sizeof(double) * ((size_t)(2 * T::h + 1) * T::hw + 3 * (size_t)T::TP + T::np) +
                       sizeof(float) * (size_t)T::TP * T::ss + sizeof(uint16_t) * (size_t)T::TP * 4 * W64;
    dim3 grid((a.W + T::TP - 1) / T::TP, a.H);
    hipError_t e = hipFuncSetAttribute((const void *)k_analyze<PREC, P>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_analyze<PREC, P>), grid, dim3(256), lds, lc.stream, a);
    return hipGetLastError();
}

template <int PREC>
static hipError_t launch_analyze_prec(const LaunchCtx &lc, const AnalyzeArgs &a) {
    switch (a.p) {
        case 3: return launch_analyze_p<PREC, 3>(lc, a);
        case 5: return launch_analyze_p<PREC, 5>(lc, a);
        case 7: return launch_analyze_p<PREC, 7>(lc, a);
        case 9: return launch_analyze_p<PREC, 9>(lc, a);
        case 11: return launch_analyze_p<PREC, 11>(lc, a);
        case 13: return launch_analyze_p<PREC, 13>(lc, a);
        case 15: return launch_analyze_p<PREC, 15>(lc, a);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_analyze(const LaunchCtx &lc, const AnalyzeArgs &a, int precision) {
    if (precision == CS_BF16) return launch_analyze_prec<CS_BF16>(lc, a);
    return launch_analyze_prec<CS_FP32>(lc, a);
}

// Co-support masks from stored analysed vectors (the same decision as the
// analysis epilogue): bit j of pixel x is set when the rounded |a_j| is at most
// t_in[j] and clear above t_out[j]; in between the entry is recomputed in FP64
// from the exact patch (Sec. 2 co-support, Sec. 3.1 patch).  A wave takes
// blocks of kMaskPx consecutive pixels, lane = row j within a 64-bit mask
// word, so the loads are coalesced and each mask word is the ballot of one
// comparison.  The entries in between are resolved per pixel by the whole
// wave: the pixel's exact normalised patch is built in the wave's LDS slice
// (its mean and squared norm from the analysis when pstats is given, else
// summed by lane 0 in t order; LDS accesses of one wave complete in issue
// order, so the hand-offs need no barrier), then every lane recomputes all of
// its rows j = 64 w + lane that are in between in one pass over the patch.
// Persistent workgroups of kMaskWaves waves; with OML the FP32 operator is
// staged in LDS once per workgroup, so the recompute reads it there.
constexpr int kMaskPx = 8;
constexpr int kMaskWaves = 16;
// LDS bytes of the per-wave patch pairs and entry lists (the operator follows,
// 16-byte aligned).
__host__ __device__ inline size_t mask_lds_head(int n, int k) {
    const size_t b = sizeof(double) * kMaskWaves * 2 * (size_t)n + sizeof(uint16_t) * kMaskWaves * 2 * (size_t)k;
    return (b + 15) / 16 * 16;
}
template <int W64, bool OML>
__global__ __launch_bounds__(64 * kMaskWaves) void k_mask_alpha(const float *alpha, int64_t N, int k,
                                                                 const float *t_in, const float *t_out, double tau,
                                                                 const double *tau_dev, const float *rgb, int H,
                                                                 int W, int p, const double *wmask,
                                                                 const float *omega, uint64_t *masks,
                                                                 unsigned long long *recomputed,
                                                                 const double *pstats) {
#pragma clang fp contract(off)
    extern __shared__ __align__(16) unsigned char smem[];
    if (tau_dev) tau = *tau_dev;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int n = p * p, h = (p - 1) / 2;
    double *s = reinterpret_cast<double *>(smem) + wave * 2 * n;  // this wave's two patches
    uint16_t *lst = reinterpret_cast<uint16_t *>(smem + sizeof(double) * kMaskWaves * 2 * n) + wave * 2 * k;
    float *s_om = reinterpret_cast<float *>(smem + mask_lds_head(n, k));
    if constexpr (OML) {
        for (int idx = threadIdx.x; idx < k * n; idx += 64 * kMaskWaves) s_om[idx] = omega[idx];
        __syncthreads();
    }
    const int64_t NN = (int64_t)H * W;
    // pixels per block (even): fewer for long masks (their ballots are held in SGPRs)
    constexpr int PX = W64 >= 2 ? kMaskPx / 2 : kMaskPx;
    const unsigned long long lt = (1ull << lane) - 1ull;
    float tin[W64], tout[W64];
    uint64_t vmask[W64];
#pragma unroll
    for (int w = 0; w < W64; ++w) {
        const int j = 64 * w + lane;
        const bool jv = j < k;
        tin[w] = jv ? t_in[j] : 0.0f;
        tout[w] = jv ? t_out[j] : 0.0f;
        vmask[w] = __ballot(jv);
    }
    unsigned long long nrec = 0;
    const int64_t nblk = (N + PX - 1) / PX;
    for (int64_t blk = (int64_t)blockIdx.x * kMaskWaves + wave; blk < nblk;
         blk += (int64_t)gridDim.x * kMaskWaves) {
    const int64_t p0 = blk * PX;
    // loads issued unconditionally (clamped indices, all in flight together),
    // padding replaced afterwards
    float v[PX][W64];
#pragma unroll
    for (int i = 0; i < PX; ++i)
#pragma unroll
        for (int w = 0; w < W64; ++w) {
            const int j = 64 * w + lane;
            const int64_t pix = p0 + i;
            v[i][w] = alpha[(pix < N ? pix : N - 1) * k + (j < k ? j : k - 1)];
        }
#pragma unroll
    for (int i = 0; i < PX; ++i)
#pragma unroll
        for (int w = 0; w < W64; ++w) v[i][w] = (64 * w + lane < k && p0 + i < N) ? fabsf(v[i][w]) : INFINITY;
    uint64_t words[PX][W64], nearw[PX][W64];
    uint64_t anyn = 0;
#pragma unroll
    for (int i = 0; i < PX; ++i)
#pragma unroll
        for (int w = 0; w < W64; ++w) {
            const uint64_t inb = __ballot(v[i][w] <= tin[w]);
            const uint64_t outb = __ballot(v[i][w] > tout[w]);
            words[i][w] = inb & vmask[w];
            nearw[i][w] = ~(inb | outb) & vmask[w];  // NaN: neither, so recomputed
            anyn |= nearw[i][w];
        }
    if (anyn) {
        // pixels in pairs: both exact patches in the wave's LDS slice, then
        // the pair's entries in between listed (pixel, word, lane order) and
        // recomputed one per lane, the decision returned in the entry's bit 15
#pragma unroll
        for (int i0 = 0; i0 < PX; i0 += 2) {
            uint64_t any2 = 0;
#pragma unroll
            for (int w = 0; w < W64; ++w) any2 |= nearw[i0][w] | nearw[i0 + 1][w];
            if (!any2) continue;
            for (int idx = lane; idx < 2 * n; idx += 64) {
                const int ii = idx >= n ? 1 : 0, t = idx - ii * n;
                const int64_t pix = p0 + i0 + ii;
                double q = 0.0;
                if (pix < N) {
                    const int row = (int)(pix / W), col = (int)(pix - (int64_t)row * W);
                    const int u = t / p, vv = t - u * p;
                    const int rr = reflect_idx(row + u - h, H), cc = reflect_idx(col + vv - h, W);
                    q = wmask[t] * gray64(rgb, NN, (int64_t)rr * W + cc);
                }
                s[idx] = q;
            }
            double mu[2] = {0.0, 0.0}, nu2[2] = {0.0, 0.0};
#pragma unroll
            for (int ii = 0; ii < 2; ++ii) {
                const int64_t pix = p0 + i0 + ii;
                if (pix >= N) continue;
                if (pstats) {
                    mu[ii] = pstats[2 * pix];
                    nu2[ii] = pstats[2 * pix + 1];
                } else {
                    double m = 0.0, v2 = 0.0;
                    if (lane == 0) {
                        const double *sp = s + ii * n;
                        double sum = 0.0;
                        for (int t = 0; t < n; ++t) sum = sum + sp[t];
                        m = sum / (double)n;
                        for (int t = 0; t < n; ++t) {
                            const double z = sp[t] - m;
                            v2 = v2 + z * z;
                        }
                    }
                    mu[ii] = __shfl(m, 0);
                    nu2[ii] = __shfl(v2, 0);
                }
            }
            const double nu[2] = {nu2[0] == 0.0 ? 0.0 : sqrt(nu2[0]), nu2[1] == 0.0 ? 0.0 : sqrt(nu2[1])};
            for (int idx = lane; idx < 2 * n; idx += 64) {
                const int ii = idx >= n ? 1 : 0;
                s[idx] = nu2[ii] == 0.0 ? 0.0 : (s[idx] - mu[ii]) / nu[ii];
            }
            // the list: entry (ii << 8) | j
            unsigned int C = 0;
#pragma unroll
            for (int ii = 0; ii < 2; ++ii)
#pragma unroll
                for (int w = 0; w < W64; ++w) {
                    const uint64_t nm = nearw[i0 + ii][w];
                    if (!nm) continue;
                    if ((nm >> lane) & 1ull) lst[C + __popcll(nm & lt)] = (uint16_t)((ii << 8) | (64 * w + lane));
                    C += (unsigned int)__popcll(nm);
                }
            __builtin_amdgcn_wave_barrier();
            for (unsigned int r0 = 0; r0 < C; r0 += 64) {
                const unsigned int q = r0 + lane;
                if (q < C) {
                    const unsigned int e = lst[q];
                    const double *sp = s + (e >> 8) * n;
                    const float *om = (OML ? s_om : omega) + (int64_t)(e & 255u) * n;
                    double acc = 0.0;
                    for (int t0 = 0; t0 < n; t0 += 8) {
                        double sv[8];
                        float ov[8];
#pragma unroll
                        for (int u = 0; u < 8; ++u) {
                            const int t = t0 + u < n ? t0 + u : n - 1;
                            sv[u] = sp[t];
                            ov[u] = om[t];
                        }
#pragma unroll
                        for (int u = 0; u < 8; ++u)
                            if (t0 + u < n) acc = acc + (double)ov[u] * sv[u];
                    }
                    if (fabs(acc) <= tau) lst[q] = (uint16_t)(e | 0x8000u);
                }
            }
            __builtin_amdgcn_wave_barrier();
            unsigned int C2 = 0;
#pragma unroll
            for (int ii = 0; ii < 2; ++ii)
#pragma unroll
                for (int w = 0; w < W64; ++w) {
                    const uint64_t nm = nearw[i0 + ii][w];
                    if (!nm) continue;
                    const bool in = ((nm >> lane) & 1ull) && (lst[C2 + __popcll(nm & lt)] & 0x8000u);
                    words[i0 + ii][w] = (words[i0 + ii][w] & ~nm) | (__ballot(in) & nm);
                    nrec += (unsigned long long)__popcll(nm);
                    C2 += (unsigned int)__popcll(nm);
                }
            __builtin_amdgcn_wave_barrier();  // s and the list are rewritten for the next pair
        }
    }
// lane l < PX * W64 stores word (l / W64, l % W64)
    const int li = lane / W64, lw = lane - li * W64;
    uint64_t outw = 0;
#pragma unroll
    for (int i = 0; i < PX; ++i)
#pragma unroll
        for (int w = 0; w < W64; ++w)
            if (li == i && lw == w) outw = words[i][w];
    if (lane < PX * W64 && p0 + li < N) masks[(p0 + li) * W64 + lw] = outw;
    }
    if (recomputed && lane == 0 && nrec) atomicAdd(recomputed, nrec);
}

template <int W64, bool OML>
static hipError_t launch_mask_k(const LaunchCtx &lc, size_t lds, const float *alpha, int64_t N, int k,
                                const float *t_in, const float *t_out, double tau, const double *tau_dev,
                                const float *rgb, int H, int W, int p, const double *wmask, const float *omega,
                                uint64_t *masks, unsigned long long *recomputed, const double *pstats) {
    hipError_t e = hipFuncSetAttribute((const void *)k_mask_alpha<W64, OML>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_mask_alpha<W64, OML>, 64 * kMaskWaves, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    int64_t blocks = (int64_t)lc.num_cu * per_cu;
    const int64_t px = W64 >= 2 ? kMaskPx / 2 : kMaskPx;
    const int64_t need = (N + px * kMaskWaves - 1) / (px * kMaskWaves);
    if (blocks > need) blocks = need;
    hipLaunchKernelGGL((k_mask_alpha<W64, OML>), dim3((unsigned)blocks), dim3(64 * kMaskWaves), lds, lc.stream,
                       alpha, N, k, t_in, t_out, tau, tau_dev, rgb, H, W, p, wmask, omega, masks, recomputed,
                       pstats);
    return hipGetLastError();
}

hipError_t launch_mask_alpha(const LaunchCtx &lc, const float *alpha, int64_t N, int k, const float *t_in,
                             const float *t_out, double tau, const double *tau_dev, const float *rgb, int H,
                             int W, int p,
                             const double *wmask, const float *omega, uint64_t *masks,
                             unsigned long long *recomputed, const double *pstats) {
    if (N <= 0) return hipSuccess;
    const int n = p * p;
    const size_t head = mask_lds_head(n, k);
    const size_t om = sizeof(float) * (size_t)k * n;
    const bool oml = head + om <= (size_t)160 * 1024;  // operator in LDS when it fits beside the patches
    const size_t lds = head + (oml ? om : 0);
#define CS_MASK_LAUNCH(WW)                                                                                       \
    return oml ? launch_mask_k<WW, true>(lc, lds, alpha, N, k, t_in, t_out, tau, tau_dev, rgb, H, W, p, wmask,  \
                                         omega, masks, recomputed, pstats)                                      \
               : launch_mask_k<WW, false>(lc, lds, alpha, N, k, t_in, t_out, tau, tau_dev, rgb, H, W, p, wmask, \
                                          omega, masks, recomputed, pstats)
    switch ((k + 63) / 64) {
        case 1: CS_MASK_LAUNCH(1);
        case 2: CS_MASK_LAUNCH(2);
        case 3: CS_MASK_LAUNCH(3);
        default: CS_MASK_LAUNCH(4);
    }
#undef CS_MASK_LAUNCH
}

__global__ __launch_bounds__(256) void k_put_table(double *dst, MaskTable t, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = t.w[i];
}

hipError_t launch_put_table(const LaunchCtx &lc, double *dst, const MaskTable &t, int n) {
    hipLaunchKernelGGL(k_put_table, dim3(1), dim3(256), 0, lc.stream, dst, t, n);
    return hipGetLastError();
}

// Per-row decision thresholds.  One workgroup of 256 threads (k <= 256).
__global__ __launch_bounds__(256) void k_thresholds(const float *omega, int k, int n, double tau,
                                                     const double *tau_dev, double margin, double coef,
                                                     float *t_in, float *t_out, double *margins,
                                                     double *max_margin, unsigned long long *zero) {
    __shared__ double red[256];
    if (tau_dev) tau = *tau_dev;
    if (zero && threadIdx.x == 0) *zero = 0ull;
    const int j = threadIdx.x;
    double m = 0.0;
    if (j < k) {
        // Proven bound: |a_rounded - a| <= coef * sum_t |O_jt||s_t| <= coef * ||O_j||_2,
        // since ||s||_2 = 1.
        m = row_margin(omega, j, n, margin, coef);
        const double lo = tau - m, hi = tau + m;
        float fl = (float)lo;
        if ((double)fl > lo) fl = nextafterf(fl, -INFINITY);
        float fh = (float)hi;
        if ((double)fh < hi) fh = nextafterf(fh, INFINITY);
        if (t_in) t_in[j] = fl;
        if (t_out) t_out[j] = fh;
        if (margins) margins[j] = m;
    }
    red[j] = m;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (j < st) red[j] = fmax(red[j], red[j + st]);
        __syncthreads();
    }
    if (j == 0 && max_margin) *max_margin = red[0];
}

hipError_t launch_thresholds(const LaunchCtx &lc, const float *omega, int k, int n, double tau,
                             const double *tau_dev, double margin, double coef, float *t_in, float *t_out,
                             double *margins, double *max_margin, unsigned long long *zero) {
    hipLaunchKernelGGL(k_thresholds, dim3(1), dim3(256), 0, lc.stream, omega, k, n, tau, tau_dev, margin,
                       coef, t_in, t_out, margins, max_margin, zero);
    return hipGetLastError();
}

}  // namespace cs
