// Spatially varying Parzen sum with co-support texture factor on gfx950
// (Sec. 3.1: Parzen colour/location density with adaptive spatial bandwidth,
// texture similarity of Sec. 2 inside the sum, beta proportional to rho; the
// data term of Sec. 3.2 is its negative).
//
// For pixel x and label i with samples S_i (m_i = |S_i|):
//   e(x,y)  = -|x-y|^2 / (2 rho^2) - |I(x)-I(y)|^2 / (2 sigma_c^2) - TSM(x,y) / beta
//   l_i(x)  = log sum_y exp e(x,y) - log m_i - log(2 pi rho^2) - 1.5 log(2 pi sigma_c^2)
//
// Execution model.  A persistent grid of 64-lane waves pulls work items
// (label, 64-pixel tile) from an atomic queue, largest labels first.  Lanes
// are pixels; the samples of the label are wave-uniform, so each 64-byte
// sample record arrives through the scalar cache into SGPRs and every pair
// costs only VALU work: two coordinate and three colour differences, their
// squares, an XOR + v_bcnt per 32-bit co-support word, three FMAs combining
// the exponent in log2 units, one v_exp_f32 and one add.
//
// Log-sum-exp without a running max.  Every exponent is bounded above by
// U = -A d_min^2 (the nearest sample has the smallest |x-y|), and the nearest
// sample itself (known from the distance transform) gives an achieved value
// e*.  With the reference R = min(U, e* + 64) the sum of 2^(e-R) is at least
// 2^-64 and overflows only if some sample beats the nearest one by more than
// about 2^127 / m_i; a wave in which any lane leaves [0, 2^100] repeats the
// label with an exact max pass (counted as a fix-up).
#include "cs_internal.h"

namespace cs {

constexpr double kLog2e = 1.4426950408889634;
constexpr double kLn2 = 0.6931471805599453;
constexpr int kRefSubset = 4;
constexpr float kRefMargin = 48.0f;

template <int NW>
__device__ __forceinline__ float pair_e(float px, float py, float pr, float pg, float pb,
                                        const uint32_t (&mx)[NW], const uint32_t *rw, float nA,
                                        float nB, float nC) {
    const float dx = px - __uint_as_float(rw[0]);
    const float dy = py - __uint_as_float(rw[1]);
    const float d2 = fmaf(dy, dy, dx * dx);
    const float dr = pr - __uint_as_float(rw[2]);
    const float dg = pg - __uint_as_float(rw[3]);
    const float db = pb - __uint_as_float(rw[4]);
    const float c2 = fmaf(db, db, fmaf(dg, dg, dr * dr));
    uint32_t t = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) t = __popc(mx[w] ^ rw[8 + w]) + t;
    float e = (float)t * nB;
    e = fmaf(nC, c2, e);
    e = fmaf(nA, d2, e);
    return e;
}

// Per (label, pixel) coefficients of the pair exponent in log2 units, from
// the exact nearest-sample distance d (FP32):
//   nA = -log2(e) / (2 rho^2), nB = -log2(e) / beta, rho = alpha_rho max(d, r_f),
//   (nB = 0 when the texture factor is applied outside the sum, eq:joined),
//   K  = -log m_i - log(2 pi) - 1.5 log(2 pi sigma_c^2) - log(rho^2),
//   nR = -R with the log-sum-exp reference R = min(U, e^ + kRefMargin):
//   U = nA d^2 bounds every exponent from above, e^ is the largest exponent
//   over the nearest sample and kRefSubset strided samples of the label (an
//   achieved value, so the sum is at least 2^-kRefMargin).
// coef[l * npix + i] = {nA, nB, nR, K}; pixel i is subset[i] or i.
// Tiled layout (matrix-core path): slot i = tile * kTilePix + q, the pixel of
// fast_slot_row (the tile grid, or entry i of the subset); empty slots get
// {0, 0, -200, 0} (their terms vanish).
template <int NW>
__global__ __launch_bounds__(256) void k_coef(ParzenArgs a, float4 *__restrict__ coef) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int l = blockIdx.y;
    const int64_t nslots = a.coef_tiled ? (int64_t)a.ntiles_pad * kTilePix : a.npix;
    if (i >= nslots) return;
    const int64_t N = (int64_t)a.H * a.W;
    const int W64 = (a.k + 63) / 64;
    int64_t pix;
    if (a.coef_tiled) {
        const int t = (int)(i / kTilePix), q = (int)(i - (int64_t)t * kTilePix);
        const int64_t row = fast_slot_row(a.subset, a.npix, a.H, a.W, a.tiles_x, a.ntiles_real, t, q);
        if (row < 0) {
            coef[(int64_t)l * nslots + i] = make_float4(0.0f, 0.0f, -200.0f, 0.0f);
            return;
        }
        pix = fast_row_pixel(a.subset, row);
    } else {
        pix = a.subset ? (int64_t)a.subset[i] : i;
    }
    const uint32_t *mask32 = reinterpret_cast<const uint32_t *>(a.masks);
    const float nC = (float)(-kLog2e / (2.0 * a.sigma_c * a.sigma_c));
    const int d2min = a.d2[(int64_t)l * N + pix];
    const int64_t nearp = a.nearest[(int64_t)l * N + pix];
    // FP32 from here (the results are FP32; a few ulps against one rounding)
    const float fl2 = (float)(a.rho_floor * a.rho_floor);
    const float dm = fmaxf((float)d2min, fl2);
    const float rho2 = (float)(a.alpha_rho * a.alpha_rho) * dm;
    const float rho = sqrtf(rho2);
    const float nA = -(float)kLog2e / (2.0f * rho2);
    const float nB = a.texture_in_sum ? -(float)kLog2e / ((float)a.beta_scale * rho) : 0.0f;
    const float K = (float)a.kconst[l] - logf(rho2);
    uint32_t mx[NW], nrec[kRecWords];
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        mx[w] = mask32[pix * 2 * W64 + w];
        nrec[8 + w] = mask32[nearp * 2 * W64 + w];
    }
    nrec[0] = __float_as_uint((float)(nearp % a.W));
    nrec[1] = __float_as_uint((float)(nearp / a.W));
    nrec[2] = __float_as_uint(a.rgb[nearp]);
    nrec[3] = __float_as_uint(a.rgb[N + nearp]);
    nrec[4] = __float_as_uint(a.rgb[2 * N + nearp]);
    const float px = (float)(pix % a.W), py = (float)(pix / a.W);
    const float pr = a.rgb[pix], pg = a.rgb[N + pix], pb = a.rgb[2 * N + pix];
    float est = pair_e<NW>(px, py, pr, pg, pb, mx, nrec, nA, nB, nC);
    // Largest exponent over the nearest sample and an evenly strided subset of
    // the label's samples: an achieved value close to the maximum.
    const int s0 = a.seg_off[l], m = a.seg_off[l + 1] - s0;
    const int nsub = m < kRefSubset ? m : kRefSubset;
    const uint32_t *recw = reinterpret_cast<const uint32_t *>(a.recs);
    for (int j = 0; j < nsub; ++j) {
        const int64_t sidx = s0 + (int64_t)j * m / nsub;
        est = fmaxf(est, pair_e<NW>(px, py, pr, pg, pb, mx, recw + sidx * kRecWords, nA, nB, nC));
    }
    const float U = nA * (float)d2min;
    coef[(int64_t)l * nslots + i] = make_float4(nA, nB, -fminf(U, est + kRefMargin), K);
}

// The sample records and the outputs are separate restrict-qualified
// arguments so that the compiler can prove the records are never written in
// the kernel and fetch them with scalar loads.
template <int NW>
__global__ __launch_bounds__(256) void k_parzen(ParzenArgs a, const uint32_t *__restrict__ recw,
                                                 float *__restrict__ loglik,
                                                 unsigned int *__restrict__ work_counter,
                                                 unsigned int *__restrict__ fixups,
                                                 const float4 *__restrict__ coef) {
    const int lane = threadIdx.x & 63;
    const int64_t N = (int64_t)a.H * a.W;
    const int W64 = (a.k + 63) / 64;
    const bool fixmode = a.fixlist != nullptr;
    int total = a.tiles * a.L;
    if (fixmode) {
        const unsigned int nf = *a.fix_count;
        total = (int)(nf < (unsigned int)a.fix_cap ? nf : (unsigned int)a.fix_cap);
        if (total == 0) return;
    }
    const float nC = (float)(-kLog2e / (2.0 * a.sigma_c * a.sigma_c));
    const uint32_t *mask32 = reinterpret_cast<const uint32_t *>(a.masks);

    for (;;) {
        int item = 0;
        if (lane == 0) item = (int)atomicAdd(work_counter, 1u);
        item = __shfl(item, 0);
        item = __builtin_amdgcn_readfirstlane(item);
        if (item >= total) break;
        int l, tile;
        int64_t i, pix;
        bool valid;
        if (fixmode) {
            const int2 fx = a.fixlist[item];
            l = __builtin_amdgcn_readfirstlane(fx.x);
            tile = __builtin_amdgcn_readfirstlane(fx.y);
            // lanes 0 .. kTilePix-1 take the tile's slots (fast_slot_row)
            const int64_t row = lane < kTilePix
                                    ? fast_slot_row(a.subset, a.npix, a.H, a.W, a.tiles_x, a.ntiles_real, tile, lane)
                                    : -1;
            valid = row >= 0;
            i = valid ? row : 0;
            pix = valid ? fast_row_pixel(a.subset, row) : 0;
        } else {
            l = a.label_order[item / a.tiles];
            tile = item - (item / a.tiles) * a.tiles;
            i = (int64_t)tile * 64 + lane;
            valid = i < a.npix;
            pix = valid ? (a.subset ? (int64_t)a.subset[i] : i) : 0;
        }

        const float px = (float)(pix % a.W), py = (float)(pix / a.W);
        const float pr = a.rgb[pix], pg = a.rgb[N + pix], pb = a.rgb[2 * N + pix];
        uint32_t mx[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) mx[w] = mask32[pix * 2 * W64 + w];

        // Per (pixel, label) coefficients (see k_coef).
        const float4 cf = fixmode ? coef[((int64_t)l * a.ntiles_pad + tile) * kTilePix + (lane & (kTilePix - 1))]
                                  : coef[(int64_t)l * a.npix + i];
        const float nA = cf.x, nB = cf.y;
        float R = -cf.z;
        const double K = (double)cf.w;

        const int s0 = a.seg_off[l], s1 = a.seg_off[l + 1];
        float S = 0.0f, S1 = 0.0f;
        int s = s0;
        for (; s + 4 <= s1; s += 4) {
            const uint32_t *rw = recw + (int64_t)s * kRecWords;
            const float e0 = pair_e<NW>(px, py, pr, pg, pb, mx, rw, nA, nB, nC);
            const float e1 = pair_e<NW>(px, py, pr, pg, pb, mx, rw + kRecWords, nA, nB, nC);
            const float e2 = pair_e<NW>(px, py, pr, pg, pb, mx, rw + 2 * kRecWords, nA, nB, nC);
            const float e3 = pair_e<NW>(px, py, pr, pg, pb, mx, rw + 3 * kRecWords, nA, nB, nC);
            S += __builtin_amdgcn_exp2f(e0 - R);
            S1 += __builtin_amdgcn_exp2f(e1 - R);
            S += __builtin_amdgcn_exp2f(e2 - R);
            S1 += __builtin_amdgcn_exp2f(e3 - R);
        }
        for (; s < s1; ++s) {
            const uint32_t *rw = recw + (int64_t)s * kRecWords;
            S += __builtin_amdgcn_exp2f(pair_e<NW>(px, py, pr, pg, pb, mx, rw, nA, nB, nC) - R);
        }
        S += S1;
        const bool bad = valid && !(S <= 0x1p100f && S > 0.0f);
        if (fixmode || __ballot(bad)) {
            float E = -INFINITY;
            for (int s2 = s0; s2 < s1; ++s2) {
                const uint32_t *rw = recw + (int64_t)s2 * kRecWords;
                E = fmaxf(E, pair_e<NW>(px, py, pr, pg, pb, mx, rw, nA, nB, nC));
            }
            S = 0.0f;
            for (int s2 = s0; s2 < s1; ++s2) {
                const uint32_t *rw = recw + (int64_t)s2 * kRecWords;
                S += __builtin_amdgcn_exp2f(pair_e<NW>(px, py, pr, pg, pb, mx, rw, nA, nB, nC) - E);
            }
            R = E;
            if (lane == 0 && !fixmode) atomicAdd(fixups, 1u);
        }
        if (valid) {
            const double lg = kLn2 * ((double)R + (double)__builtin_amdgcn_logf(S)) + K;
            loglik[i * a.L + l] = (float)lg;
        }
    }
}

template <int NW>
static hipError_t launch_parzen_nw(const LaunchCtx &lc, const ParzenArgs &a) {
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_parzen<NW>, 256, 0);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    int64_t blocks = (int64_t)lc.num_cu * per_cu;
    const int64_t need = ((int64_t)a.tiles * a.L + 3) / 4;
    if (blocks > need) blocks = need;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_parzen<NW>, dim3((unsigned)blocks), dim3(256), 0, lc.stream, a,
                       reinterpret_cast<const uint32_t *>(a.recs), a.loglik, a.work_counter,
                       a.fixups, a.coef);
    return hipGetLastError();
}

template <int NW>
static hipError_t launch_coef_nw(const LaunchCtx &lc, const ParzenArgs &a, float4 *coef) {
    const int64_t nslots = a.coef_tiled ? (int64_t)a.ntiles_pad * kTilePix : a.npix;
    hipLaunchKernelGGL(k_coef<NW>, dim3((unsigned)((nslots + 255) / 256), a.L), dim3(256), 0,
                       lc.stream, a, coef);
    return hipGetLastError();
}

hipError_t launch_coef(const LaunchCtx &lc, const ParzenArgs &a, float4 *coef) {
    if (a.npix == 0) return hipSuccess;
    switch (a.nw32) {
        case 1: return launch_coef_nw<1>(lc, a, coef);
        case 2: return launch_coef_nw<2>(lc, a, coef);
        case 3: return launch_coef_nw<3>(lc, a, coef);
        case 4: return launch_coef_nw<4>(lc, a, coef);
        case 5: return launch_coef_nw<5>(lc, a, coef);
        case 6: return launch_coef_nw<6>(lc, a, coef);
        case 7: return launch_coef_nw<7>(lc, a, coef);
        default: return launch_coef_nw<8>(lc, a, coef);
    }
}

hipError_t launch_parzen(const LaunchCtx &lc, const ParzenArgs &a) {
    switch (a.nw32) {
        case 1: return launch_parzen_nw<1>(lc, a);
        case 2: return launch_parzen_nw<2>(lc, a);
        case 3: return launch_parzen_nw<3>(lc, a);
        case 4: return launch_parzen_nw<4>(lc, a);
        case 5: return launch_parzen_nw<5>(lc, a);
        case 6: return launch_parzen_nw<6>(lc, a);
        case 7: return launch_parzen_nw<7>(lc, a);
        default: return launch_parzen_nw<8>(lc, a);
    }
}

// Optional output form: l_i - log sum_i' exp l_i' per pixel (labels normalise).
__global__ __launch_bounds__(256) void k_normalise(float *loglik, int64_t npix, int L) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= npix) return;
    float *r = loglik + i * L;
    float m = -INFINITY;
    for (int l = 0; l < L; ++l) m = fmaxf(m, r[l]);
    float s = 0.0f;
    for (int l = 0; l < L; ++l) s += expf(r[l] - m);
    const float lse = m + logf(s);
    for (int l = 0; l < L; ++l) r[l] -= lse;
}

hipError_t launch_normalise(const LaunchCtx &lc, float *loglik, int64_t npix, int L) {
    if (!npix) return hipSuccess;
    hipLaunchKernelGGL(k_normalise, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, lc.stream,
                       loglik, npix, L);
    return hipGetLastError();
}

}  // namespace cs
