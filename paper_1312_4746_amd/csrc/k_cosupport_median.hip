// Co-support masks at tau = frac * median|a| with the mask decision fused
// into the candidate gather of the exact median (Sec. 2 co-support of a
// thresholded analysed vector; the threshold is a fixed fraction of the
// median magnitude).
//
// The separate path reads the N*k analysed vectors five times: three radix
// digits, the candidate gather and then the masks at the exact tau.  Here the
// gather pass decides the masks as well, and takes the place of the third
// digit: after two digits (the top 22 bits) the float median of the rounded
// |a| is known to lie in a bin [v_lo, v_hi] of 2^10 floats (at the medians
// and FP32 bounds of the 7 x 7 and 11 x 11 workloads, 0.6 and 0.25 of the
// candidate window's half-width 2m, so the window grows little), and the exact
// median lies in [v_lo - m, v_hi + m] (m the largest proven rounding bound),
// so tau lies in a short interval.  Every entry whose rounded |a| is clear of that interval by more
// than its row's margin is decided in the gather pass; the few others are
// listed and decided against the exact tau once it is selected, in FP64 where
// the rounded value is within the margin.  Masks and tau equal those of the
// separate path bit for bit.  The lists have room for every entry, so nothing
// depends on a host round trip.
#pragma clang fp contract(off)

#include "cs_internal.h"
#include "cs_device.h"

namespace cs {

namespace {
constexpr int kPx = 8;  // pixels per wave and round in the pixel-major pass
constexpr int kRoundsPerWave = 4;

}  // namespace

// The gather pass.  Each wave takes a contiguous run of rounds of kPx
// consecutive pixels (about kRoundsPerWave of them, the loads of the next in
// flight while one is decided), lane = row within a 64-bit mask word.  Its
// candidates and undecided entries go to its own region of cand and didx,
// which starts at its first entry (so it can never overflow), counted in
// ccnt and dcnt: no global atomics.  Per workgroup the count of entries below
// the candidate window goes to parts[blockIdx.x].
template <int W64>
__global__ __launch_bounds__(256) void k_median_mask_gather(const float *alpha, int64_t N, int k,
                                                            const double *max_margin, const double *margins,
                                                            double frac, TauState *st, int64_t *cand,
                                                            unsigned int *ccnt, unsigned long long *parts,
                                                            int64_t *didx, unsigned int *dcnt, uint64_t *masks,
                                                            const unsigned int *hist3) {
    static_assert(kPx * W64 <= 64, "one mask word per lane");
    __shared__ unsigned long long red[256];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // the second digit, from its complete histogram: the target rank's rounded
    // |a| has the top 22 bits prefix, so it lies in [v_lo, v_hi] (workgroup 0
    // records the digit)
    unsigned int prefix;
    unsigned long long rank;
    tau_pick_digit(hist3 + kHistBins, 10, st->pfx[1], st->rk[1], prefix, rank);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->pfx[2] = st->prefix = prefix;
        st->rk[2] = st->rank = rank;
    }
    // candidate window [v_lo - 2m, v_hi + 2m] as float bit patterns
    // (non-negative floats order like their bit patterns): an entry below it
    // is exactly below the exact median, one above it exactly above
    const double vlo = (double)__uint_as_float(prefix), vhi = (double)__uint_as_float(prefix | 0x3FFu);
    const double mm = *max_margin;
    const double wlo = vlo - 2.0 * mm, whi = vhi + 2.0 * mm;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->lo = wlo;
        st->hi = whi;
    }
    float flo = (float)wlo, fhi = (float)whi;
    if ((double)flo < wlo) flo = nextafterf(flo, INFINITY);
    if ((double)fhi > whi) fhi = nextafterf(fhi, -INFINITY);
    const uint32_t blo = wlo <= 0.0 ? 0u : __float_as_uint(flo);
    const uint32_t bhi = __float_as_uint(fhi);
    // tau = fl(frac * median) is monotone in the median, which lies in
    // [v_lo - m, v_hi + m]; both ends are widened by the rounding of the bounds
    double mlo = vlo - mm;
    mlo = mlo > 0.0 ? nextafter(mlo, 0.0) : 0.0;
    const double mhi = nextafter(vhi + mm, INFINITY);
    const double tlo = mlo > 0.0 ? nextafter(frac * mlo, 0.0) : 0.0;
    const double thi = nextafter(frac * mhi, INFINITY);
    float tin[W64], tout[W64];
#pragma unroll
    for (int w = 0; w < W64; ++w) {
        const int j = 64 * w + lane;
        const bool jv = j < k;
        const double m = jv ? margins[j] : 0.0;
        const double a = tlo - m, b = thi + m;
        float fa = (float)a;
        if ((double)fa > a) fa = nextafterf(fa, -INFINITY);
        float fb = (float)b;
        if ((double)fb < b) fb = nextafterf(fb, INFINITY);
        tin[w] = fa;
        tout[w] = fb;
    }
    unsigned long long below = 0;
    const int64_t nrounds = (N + kPx - 1) / kPx;
    const int64_t nw = (int64_t)gridDim.x * 4;
    const int64_t R = (nrounds + nw - 1) / nw;  // rounds per wave
    const int64_t gw = (int64_t)blockIdx.x * 4 + wave;
    const int64_t r_end = (gw + 1) * R < nrounds ? (gw + 1) * R : nrounds;
    const int64_t region = R * kPx * k;  // entries of a wave's run of rounds
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->rg_waves = (unsigned int)nw;
        st->rg_size = (long long)region;
    }
    int64_t *creg = cand + gw * region, *dreg = didx + gw * region;
    unsigned int nc_w = 0, nd_w = 0;  // wave-uniform counts
    const unsigned long long lt = (1ull << lane) - 1ull;
    // the keys of a round, loaded unconditionally (clamped indices: the loads
    // are in flight together; padding is replaced when the round is used)
    auto load = [&](int64_t rd, uint32_t (&kk)[kPx][W64]) {
        const int64_t p0 = rd * kPx;
#pragma unroll
        for (int i = 0; i < kPx; ++i)
#pragma unroll
            for (int w = 0; w < W64; ++w) {
                const int j = 64 * w + lane;
                const int64_t pix = p0 + i;
                kk[i][w] = __float_as_uint(alpha[(pix < N ? pix : N - 1) * k + (j < k ? j : k - 1)]);
            }
    };
    uint32_t key[kPx][W64], nkey[kPx][W64];
    int64_t rd = gw * R;
    if (rd < r_end) load(rd, key);
    for (; rd < r_end; ++rd) {
        const int64_t p0 = rd * kPx;
        if (rd + 1 < r_end) load(rd + 1, nkey);  // next round in flight
#pragma unroll
        for (int i = 0; i < kPx; ++i)
#pragma unroll
            for (int w = 0; w < W64; ++w)
                key[i][w] = (64 * w + lane < k && p0 + i < N) ? (key[i][w] & 0x7FFFFFFFu) : 0x7F800000u;
        // lane l < kPx * W64 stores word (l / W64, l % W64), picked up as the
        // words are formed (no array of ballots held in scalar registers)
        const int li = lane / W64, lw = lane - li * W64;
        uint64_t outw = 0;
#pragma unroll
        for (int i = 0; i < kPx; ++i)
#pragma unroll
            for (int w = 0; w < W64; ++w) {
                // rows past k and pixels past N hold the key of +inf, which
                // every test below rejects (not below, no candidate, not in,
                // not deferred), so no separate liveness mask is needed
                const uint32_t x = key[i][w];
                below += x < blo ? 1ull : 0ull;
                const bool is_cand = x >= blo && x <= bhi;
                const unsigned long long cm = __ballot(is_cand);
                if (cm) {
                    if (is_cand) creg[nc_w + __popcll(cm & lt)] = (p0 + i) * k + 64 * w + lane;
                    nc_w += (unsigned int)__popcll(cm);
                }
                const float f = __uint_as_float(x);
                const uint64_t inb = __ballot(f <= tin[w]);
                if (li == i && lw == w) outw = inb;
                const bool defer = !(f <= tin[w]) && !(f > tout[w]);  // NaN: deferred
                const unsigned long long dm = __ballot(defer);
                if (dm) {
                    if (defer) dreg[nd_w + __popcll(dm & lt)] = (p0 + i) * k + 64 * w + lane;
                    nd_w += (unsigned int)__popcll(dm);
                }
                // one entry at a time: keeps the ballots from piling up in
                // scalar registers
                __builtin_amdgcn_sched_barrier(0);
            }
        if (lane < kPx * W64 && p0 + li < N) masks[(p0 + li) * W64 + lw] = outw;
#pragma unroll
        for (int i = 0; i < kPx; ++i)
#pragma unroll
            for (int w = 0; w < W64; ++w) key[i][w] = nkey[i][w];
    }
    if (lane == 0 && gw < nw) {
        ccnt[gw] = nc_w;
        dcnt[gw] = nd_w;
    }
    red[threadIdx.x] = below;
    __syncthreads();
    for (int s2 = 128; s2 > 0; s2 >>= 1) {
        if ((int)threadIdx.x < s2) red[threadIdx.x] += red[threadIdx.x + s2];
        __syncthreads();
    }
    if (threadIdx.x == 0) parts[blockIdx.x] = red[0];
    if (blockIdx.x == 0 && threadIdx.x == 0) st->nparts = gridDim.x;
}

// The listed entries against the exact tau: lane = one wave region of the
// gather, its entries in order.  An entry whose rounded |a| is clear of tau
// by more than its row margin is decided at once; the few within the margin
// (or NaN) are recomputed in FP64 by their lane from the exact patch (Sec. 2
// a = O s with the Sec. 3.1 normalised, Gaussian-masked gray patch, in the
// oracle's operation order, the patch statistics from the analysis when
// given) and decided exactly.
__device__ __forceinline__ void finish_entry(int64_t e, const float *alpha, const float *rgb, int H, int W, int p,
                                             const double *wmask, const float *omega, int k, const double *margins,
                                             double tau, uint64_t *masks, const double *pstats) {
    const int64_t pix = e / k;
    const int j = (int)(e - pix * k);
    const double a = (double)fabsf(alpha[e]);
    const double m = margins[j];
    bool in = a <= tau - m;
    if (!in && !(a > tau + m))  // within the margin, or NaN
        in = fabs(exact_entry(rgb, H, W, p, wmask, omega + (int64_t)j * p * p, pix, pstats)) <= tau;
    if (in) atomicOr(reinterpret_cast<unsigned long long *>(masks + pix * ((k + 63) / 64) + (j >> 6)), 1ull << (j & 63));
}

__global__ __launch_bounds__(64) void k_median_mask_finish(const float *alpha, const float *rgb, int H, int W,
                                                           int p, const double *wmask, const float *omega, int k,
                                                           const int64_t *didx, const unsigned int *dcnt,
                                                           const int64_t *dcomp, const double *margins,
                                                           const TauState *st, uint64_t *masks,
                                                           const double *pstats) {
    const double tau = st->tau;
    const int64_t stride = (int64_t)gridDim.x * 64;
    const int64_t nd = (int64_t)st->n_d;
    if (nd <= kListCap) {  // the compact list: one lane per entry
        for (int64_t q = (int64_t)blockIdx.x * 64 + threadIdx.x; q < nd; q += stride)
            finish_entry(dcomp[q], alpha, rgb, H, W, p, wmask, omega, k, margins, tau, masks, pstats);
        return;
    }
    const int64_t nw = (int64_t)st->rg_waves, region = (int64_t)st->rg_size;
    for (int64_t r = (int64_t)blockIdx.x * 64 + threadIdx.x; r < nw; r += stride) {
        const unsigned int cnt = dcnt[r];
        const int64_t *lst = didx + r * region;
        for (unsigned int q = 0; q < cnt; ++q)
            finish_entry(lst[q], alpha, rgb, H, W, p, wmask, omega, k, margins, tau, masks, pstats);
    }
}

hipError_t median_mask_gather(const LaunchCtx &lc, const float *alpha, int64_t N, int k,
                              const double *max_margin, const double *margins, double frac, TauState *st,
                              int64_t *cand, unsigned int *ccnt, unsigned long long *parts, int64_t *didx,
                              unsigned int *dcnt, uint64_t *masks, const unsigned int *hist3) {
    if (N <= 0) return hipSuccess;
    // kRoundsPerWave rounds per wave (each prefetches the next), more where
    // the per-workgroup counts would not fit
    const int64_t blocks = median_gather_waves(N) / 4;
#define CS_MG_LAUNCH(WW)                                                                                    \
    hipLaunchKernelGGL(k_median_mask_gather<WW>, dim3((unsigned)blocks), dim3(256), 0, lc.stream, alpha, N, \
                       k, max_margin, margins, frac, st, cand, ccnt, parts, didx, dcnt, masks, hist3)
    switch ((k + 63) / 64) {
        case 1: CS_MG_LAUNCH(1); break;
        case 2: CS_MG_LAUNCH(2); break;
        case 3: CS_MG_LAUNCH(3); break;
        default: CS_MG_LAUNCH(4); break;
    }
#undef CS_MG_LAUNCH
    return hipGetLastError();
}

int64_t median_gather_waves(int64_t N) {
    int64_t blocks = (N + 4 * kPx * kRoundsPerWave - 1) / (4 * kPx * kRoundsPerWave);
    if (blocks > kTauParts) blocks = kTauParts;
    return 4 * blocks;
}

hipError_t median_mask_finish(const LaunchCtx &lc, const float *alpha, const float *rgb, int H, int W, int p,
                              const double *wmask, const float *omega, int k, const int64_t *didx,
                              const unsigned int *dcnt, const int64_t *dcomp, const double *margins,
                              const TauState *st, uint64_t *masks, const double *pstats) {
    // one lane per listed entry, or per gather wave when the list did not fit
    int64_t blocks = (int64_t)lc.num_cu * 8;
    const int64_t nw = median_gather_waves((int64_t)H * W);
    if (blocks < (nw + 63) / 64) blocks = (nw + 63) / 64;
    hipLaunchKernelGGL(k_median_mask_finish, dim3((unsigned)blocks), dim3(64), 0, lc.stream, alpha, rgb, H, W, p,
                       wmask, omega, k, didx, dcnt, dcomp, margins, st, masks, pstats);
    return hipGetLastError();
}

}  // namespace cs
