// Parzen sum with the co-support texture factor on gfx950, texture term on
// the matrix cores (Sec. 3.1 Parzen colour/location density with adaptive
// bandwidth; Sec. 2 texture similarity inside the sum; Sec. 3.2 data term).
//
// The texture similarity of a pixel x and a sample y is the Hamming distance
// of their co-support masks, TSM = |A| + |B| - 2 |A n B|.  It is a dot product
// of two short feature vectors, so a whole 16-pixel x 16-sample block of it is
// one MFMA: v_mfma_scale_f32_16x16x128_f8f6f4 with FP8 (E4M3) operands and
// unit scales.  Pixel features: mask bit j in {0, 1} for j < k, then
// [16 floor(|A|/16), |A| mod 16, 1, 1]; sample features: -2 x bit j, then
// [1, 1, 16 floor(|B|/16), |B| mod 16].  Every operand is an exactly
// representable FP8 value and every partial sum an integer below 2^10, so the
// FP32 accumulator holds TSM exactly.
//
// Work decomposition.  A workgroup of 4 waves owns a group of four 8x8 pixel
// tiles and one label; items come from an atomic queue, largest labels first.
// The label's samples stream through LDS in chunks of 64 (features padded
// against bank conflicts, position and colour as separate arrays), prefetched
// into registers one chunk ahead.  Per 16-sample step a wave issues 4 x
// KSTEPS MFMAs (one per 16-pixel row block and 128-feature slice) and then,
// for its 16 pixels per lane x 1 sample per lane, the VALU work: the location
// term needs one FMA per pair because the pixel offsets inside the tile are
// compile-time constants, plus three colour differences and squares, three
// FMAs combining the exponent with the log-sum-exp reference folded in, one
// v_exp_f32 and one add.
//
// The reference R = min(U, e* + 64) (U = upper bound from the nearest sample
// distance, e* = the nearest sample's exponent) keeps the sum in
// [2^-64, 2^100] unless some sample beats the nearest one by more than about
// 2^127; a wave that sees a sum outside that range queues its (label, tile)
// for the exact two-pass kernel instead of writing.
#include "cs_internal.h"

namespace cs {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

constexpr double kLog2eF = 1.4426950408889634;
constexpr double kLn2F = 0.6931471805599453;
constexpr int kChunkS = 64;       // samples per LDS chunk
constexpr float kFarAway = 1e30f;  // position of padding samples (term underflows to 0)

// E4M3 (bias 7) bit pattern of an integer 0..256 that is exactly representable
// (0..16 and multiples of 16 up to 256).
__device__ __forceinline__ uint32_t fp8_of_int(uint32_t v) {
    if (v == 0) return 0u;
    const int e = 31 - __clz(v);
    const uint32_t m = ((v << 3) >> e) & 7u;
    return ((uint32_t)(e + 7) << 3) | m;
}

// Spread the 4 bits of a nibble into the 4 bytes of a word, each byte 0 or b.
__device__ __forceinline__ uint32_t nibble_bytes(uint32_t nib, uint32_t b) {
    const uint32_t s = (nib & 1u) | ((nib & 2u) << 7) | ((nib & 4u) << 14) | ((nib & 8u) << 21);
    return s * b;
}

// Sample features in MFMA order, KP bytes per sample (built from the sorted
// sample records; see the header comment for the layout).
__global__ __launch_bounds__(256) void k_sample_features(const SampleRec *recs, int64_t M, int k,
                                                          int KP, uint8_t *feat) {
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= M) return;
    const uint32_t *rw = recs[s].w;
    uint32_t cnt = 0;
    uint32_t words[8];
    for (int w = 0; w < 8; ++w) {
        uint32_t v = rw[8 + w];
        const int lo = 32 * w;
        if (lo >= k) v = 0;
        else if (k - lo < 32) v &= (1u << (k - lo)) - 1u;
        words[w] = v;
        cnt += __popc(v);
    }
    uint32_t *out = reinterpret_cast<uint32_t *>(feat + s * KP);
    for (int q = 0; q < KP / 4; ++q) {  // 4 features per word
        const int f0 = 4 * q;
        uint32_t val = 0;
        if (f0 < 256) val = nibble_bytes((words[f0 >> 5] >> (f0 & 31)) & 0xFu, 0xC0u);  // -2.0
        for (int b = 0; b < 4; ++b) {
            const int f = f0 + b;
            uint32_t byte = 0xFFFFFFFFu;
            if (f == k || f == k + 1) byte = 0x38u;  // 1.0
            else if (f == k + 2) byte = fp8_of_int(16u * (cnt >> 4));
            else if (f == k + 3) byte = fp8_of_int(cnt & 15u);
            if (byte != 0xFFFFFFFFu) val = (val & ~(0xFFu << (8 * b))) | (byte << (8 * b));
        }
        out[q] = val;
    }
}

hipError_t launch_sample_features(const LaunchCtx &lc, const SampleRec *recs, int64_t M, int k,
                                  int KP, uint8_t *feat) {
    hipLaunchKernelGGL(k_sample_features, dim3((unsigned)((M + 255) / 256)), dim3(256), 0,
                       lc.stream, recs, M, k, KP, feat);
    return hipGetLastError();
}

template <int KSTEPS, int RB>
__global__ __launch_bounds__(256) void k_parzen_mfma(ParzenFastArgs a) {
    constexpr int KP = 128 * KSTEPS;
    constexpr int FSTRIDE = KP + 16;  // LDS row stride of the sample features (bank spread)
    __shared__ __align__(16) uint8_t s_feat[kChunkS * FSTRIDE];
    __shared__ float s_x[kChunkS], s_y[kChunkS], s_r[kChunkS], s_g[kChunkS], s_b[kChunkS];
    __shared__ int s_item;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, jl = lane & 15;
    const int64_t N = (int64_t)a.H * a.W;
    const int W64 = (a.k + 63) / 64;
    const float nC = (float)(-kLog2eF / (2.0 * a.sigma_c * a.sigma_c));
    const int total = a.ngroups * a.L;
    const uint32_t *mask32 = reinterpret_cast<const uint32_t *>(a.masks);
    const uint64_t lastmask = (a.k % 64) ? ((1ull << (a.k % 64)) - 1ull) : ~0ull;

    for (;;) {
        __syncthreads();
        if (tid == 0) s_item = (int)atomicAdd(a.work_counter, 1u);
        __syncthreads();
        const int item = s_item;
        if (item >= total) break;
        const int l = a.label_order[item / a.ngroups];
        const int tile = (item - (item / a.ngroups) * a.ngroups) * 4 + wave;
        const bool tile_ok = tile < a.ntiles;
        const int ty_t = tile_ok ? tile / a.tiles_x : 0;
        const int x0 = (tile_ok ? tile - ty_t * a.tiles_x : 0) * 8, y0 = ty_t * 2 * RB;

        // ---- pixel state: lane holds pixels (rb, r) -> (x0 + 4(g&1) + r, y0 + 2rb + (g>>1))
        float pr[RB][4], pg[RB][4], pb[RB][4], nA[RB][4], nB[RB][4], nR[RB][4], S[RB][4];
        bool anyvalid = false;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int px = x0 + 4 * (g & 1) + r, py = y0 + 2 * rb + (g >> 1);
                const bool v = tile_ok && px < a.W && py < a.H;
                anyvalid |= v;
                const int64_t pix = v ? (int64_t)py * a.W + px : 0;
                pr[rb][r] = a.rgb[pix];
                pg[rb][r] = a.rgb[N + pix];
                pb[rb][r] = a.rgb[2 * N + pix];
                const int d2min = a.d2[(int64_t)l * N + pix];
                const int64_t nearp = a.nearest[(int64_t)l * N + pix];
                const double fl2 = a.rho_floor * a.rho_floor;
                const double dm = (double)d2min > fl2 ? (double)d2min : fl2;
                const double rho2 = a.alpha_rho * a.alpha_rho * dm;
                const double rho = sqrt(rho2);
                const float fA = (float)(-kLog2eF / (2.0 * rho2));
                const float fB = (float)(-kLog2eF / (a.beta_scale * rho));
                nA[rb][r] = fA;
                nB[rb][r] = fB;
                // exponent of the nearest sample (same operations as the pair loop)
                int t = 0;
                for (int w = 0; w < W64; ++w) {
                    uint64_t m1 = a.masks[pix * W64 + w] ^ a.masks[nearp * W64 + w];
                    if (w == W64 - 1) m1 &= lastmask;
                    t += __popcll(m1);
                }
                const int nx = (int)(nearp % a.W), ny = (int)(nearp / a.W);
                const float dx = (float)(px - nx), dy = (float)(py - ny);
                const float d2n = fmaf(dx, dx, dy * dy);
                const float dr = pr[rb][r] - a.rgb[nearp], dg = pg[rb][r] - a.rgb[N + nearp],
                            db = pb[rb][r] - a.rgb[2 * N + nearp];
                const float c2n = fmaf(db, db, fmaf(dg, dg, dr * dr));
                const float estar = fmaf(fA, d2n, fmaf(nC, c2n, (float)t * fB));
                const float U = fA * (float)d2min;
                nR[rb][r] = -fminf(U, estar + 64.0f);
                S[rb][r] = 0.0f;
            }
        }

        const bool wave_active = __ballot(anyvalid) != 0ull;

        // ---- pixel features (MFMA A operand): row i = l%16 of row block rb is
        // pixel rb*16 + jl of the tile = (x0 + (jl & 7), y0 + 2rb + (jl >> 3)).
        i32x8 Aop[RB][KSTEPS];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            const int px = x0 + (jl & 7), py = y0 + 2 * rb + (jl >> 3);
            const bool v = tile_ok && px < a.W && py < a.H;
            const int64_t pix = v ? (int64_t)py * a.W + px : 0;
            uint32_t cnt = 0;
            for (int w = 0; w < 2 * W64; ++w) {
                uint32_t m = mask32[pix * 2 * W64 + w];
                const int lo = 32 * w;
                if (lo >= a.k) m = 0;
                else if (a.k - lo < 32) m &= (1u << (a.k - lo)) - 1u;
                cnt += __popc(m);
            }
#pragma unroll
            for (int q = 0; q < KSTEPS; ++q) {
                const int f0 = 128 * q + 32 * g;  // first feature of this lane's slice
                const int wi = f0 >> 5;
                uint32_t bits = 0;
                if (f0 < a.k && wi < 2 * W64) {
                    bits = mask32[pix * 2 * W64 + wi];
                    if (a.k - f0 < 32) bits &= (1u << (a.k - f0)) - 1u;
                }
#pragma unroll
                for (int vv = 0; vv < 8; ++vv) {
                    uint32_t val = nibble_bytes((bits >> (4 * vv)) & 0xFu, 0x38u);
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        const int f = f0 + 4 * vv + b;
                        uint32_t byte = 0xFFFFFFFFu;
                        if (f == a.k) byte = fp8_of_int(16u * (cnt >> 4));
                        else if (f == a.k + 1) byte = fp8_of_int(cnt & 15u);
                        else if (f == a.k + 2 || f == a.k + 3) byte = 0x38u;
                        if (byte != 0xFFFFFFFFu) val = (val & ~(0xFFu << (8 * b))) | (byte << (8 * b));
                    }
                    if (!v) val = 0;
                    Aop[rb][q][vv] = (int)val;
                }
            }
        }

        // ---- stream the label's samples
        const int s0 = a.seg_off[l], s1 = a.seg_off[l + 1];
        const int nchunk = (s1 - s0 + kChunkS - 1) / kChunkS;
        // register prefetch of one chunk: features (KP/16 uint4 per sample, 64 samples)
        constexpr int FV = kChunkS * KP / 16 / 256;  // uint4 per thread
        uint4 pf[FV];
        float pfx = kFarAway, pfy = 0.f, pfr = 0.f, pfg = 0.f, pfb = 0.f;
        auto fetch = [&](int c) {
            const int base = s0 + c * kChunkS;
#pragma unroll
            for (int u = 0; u < FV; ++u) {
                const int e = tid + 256 * u;  // uint4 index inside the chunk
                const int smp = e / (KP / 16), part = e - smp * (KP / 16);
                if (base + smp < s1)
                    pf[u] = reinterpret_cast<const uint4 *>(a.feat + (int64_t)(base + smp) * KP)[part];
                else
                    pf[u] = make_uint4(0u, 0u, 0u, 0u);
            }
            if (tid < kChunkS) {
                if (base + tid < s1) {
                    const uint32_t *rw = a.recs[base + tid].w;
                    pfx = __uint_as_float(rw[0]);
                    pfy = __uint_as_float(rw[1]);
                    pfr = __uint_as_float(rw[2]);
                    pfg = __uint_as_float(rw[3]);
                    pfb = __uint_as_float(rw[4]);
                } else {
                    pfx = kFarAway;
                    pfy = pfr = pfg = pfb = 0.f;
                }
            }
        };
        fetch(0);
        const float xl = (float)(x0 + 4 * (g & 1)), yl = (float)(y0 + (g >> 1));

        // One 16-sample step: the texture block on the matrix cores, then the
        // per-pair VALU work; returns nothing, accumulates into S and tracks
        // the largest exponent (relative to the lane's reference) in mx.
        auto step = [&](int st, float (&mx)[RB][4]) {
            const int js = st * 16 + jl;
            i32x8 Bop[KSTEPS];
#pragma unroll
            for (int q = 0; q < KSTEPS; ++q) {
                const uint4 *src = reinterpret_cast<const uint4 *>(s_feat + js * FSTRIDE + 128 * q + 32 * g);
                const uint4 lo4 = src[0], hi4 = src[1];
                Bop[q] = i32x8{(int)lo4.x, (int)lo4.y, (int)lo4.z, (int)lo4.w,
                               (int)hi4.x, (int)hi4.y, (int)hi4.z, (int)hi4.w};
            }
            f32x4 T[RB];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                T[rb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int q = 0; q < KSTEPS; ++q)
                    T[rb] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
                        Aop[rb][q], Bop[q], T[rb], 0, 0, 0, 127, 0, 127);
            }
            const float sx = s_x[js], sy = s_y[js], sr = s_r[js], sg = s_g[js], sb = s_b[js];
            const float tx = xl - sx, ty = yl - sy;
            float dx[4], dy2[RB];
#pragma unroll
            for (int r = 0; r < 4; ++r) dx[r] = tx + (float)r;
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const float dy = ty + (float)(2 * rb);
                dy2[rb] = dy * dy;
            }
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float d2 = fmaf(dx[r], dx[r], dy2[rb]);
                    const float dr = pr[rb][r] - sr, dg = pg[rb][r] - sg, db = pb[rb][r] - sb;
                    const float c2 = fmaf(db, db, fmaf(dg, dg, dr * dr));
                    float u = fmaf(T[rb][r], nB[rb][r], nR[rb][r]);
                    u = fmaf(nC, c2, u);
                    u = fmaf(nA[rb][r], d2, u);
                    mx[rb][r] = fmaxf(mx[rb][r], u);
                    S[rb][r] += __builtin_amdgcn_exp2f(u);
                }
            }
        };

        for (int c = 0; c < nchunk; ++c) {
            __syncthreads();
#pragma unroll
            for (int u = 0; u < FV; ++u) {
                const int e = tid + 256 * u;
                const int smp = e / (KP / 16), part = e - smp * (KP / 16);
                *reinterpret_cast<uint4 *>(s_feat + smp * FSTRIDE + part * 16) = pf[u];
            }
            if (tid < kChunkS) {
                s_x[tid] = pfx;
                s_y[tid] = pfy;
                s_r[tid] = pfr;
                s_g[tid] = pfg;
                s_b[tid] = pfb;
            }
            __syncthreads();
            if (c + 1 < nchunk) fetch(c + 1);
            if (!wave_active) continue;
            float Ssave[RB][4], mx[RB][4];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    Ssave[rb][r] = S[rb][r];
                    mx[rb][r] = -INFINITY;
                }
#pragma unroll 1
            for (int st = 0; st < kChunkS / 16; ++st) step(st, mx);
            // Dynamic reference: a lane whose exponents reached 2^32 above its
            // reference moves the reference up by a whole power of two (exact
            // rescale of its partial sum); above 2^100 the chunk may have
            // overflowed and is recomputed from the saved sums.
            float mall = -INFINITY;
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int r = 0; r < 4; ++r) mall = fmaxf(mall, mx[rb][r]);
            if (__ballot(mall > 32.0f)) {
                bool redo = false;
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        if (mx[rb][r] > 32.0f) {
                            const float sh = ceilf(mx[rb][r]);
                            nR[rb][r] -= sh;
                            const float f = __builtin_amdgcn_exp2f(-sh);
                            S[rb][r] *= f;
                            Ssave[rb][r] *= f;
                            if (mx[rb][r] > 100.0f) redo = true;
                        }
                    }
                if (__ballot(redo)) {
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            S[rb][r] = Ssave[rb][r];
                            mx[rb][r] = -INFINITY;
                        }
#pragma unroll 1
                    for (int st = 0; st < kChunkS / 16; ++st) step(st, mx);
                }
            }
        }

        // ---- combine the 16 lanes that share each pixel (one sample column
        // each): common reference = their largest, partial sums rescaled.
        bool bad = false;
        float Rtot[RB][4], Stot[RB][4];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float Rl = -nR[rb][r];
                float Rm = Rl;
#pragma unroll
                for (int off = 1; off < 16; off <<= 1) Rm = fmaxf(Rm, __shfl_xor(Rm, off));
                float sp = S[rb][r] * __builtin_amdgcn_exp2f(Rl - Rm);
#pragma unroll
                for (int off = 1; off < 16; off <<= 1) sp += __shfl_xor(sp, off);
                Rtot[rb][r] = Rm;
                Stot[rb][r] = sp;
                const int px = x0 + 4 * (g & 1) + r, py = y0 + 2 * rb + (g >> 1);
                const bool v = tile_ok && px < a.W && py < a.H;
                if (v && !(sp <= 0x1p126f && sp > 0.0f)) bad = true;
            }
        if (__ballot(bad)) {
            if (lane == 0) {
                const unsigned int slot = atomicAdd(a.fix_count, 1u);
                if (slot < (unsigned int)a.fix_cap) a.fixlist[slot] = make_int2(l, tile);
            }
            continue;
        }
        if (jl == 0) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int px = x0 + 4 * (g & 1) + r, py = y0 + 2 * rb + (g >> 1);
                    const bool v = tile_ok && px < a.W && py < a.H;
                    if (v) {
                        const int64_t pix = (int64_t)py * a.W + px;
                        const int d2min = a.d2[(int64_t)l * N + pix];
                        const double fl2 = a.rho_floor * a.rho_floor;
                        const double dm = (double)d2min > fl2 ? (double)d2min : fl2;
                        const double rho2 = a.alpha_rho * a.alpha_rho * dm;
                        const double K = a.kconst[l] - log(rho2);
                        const double lg = kLn2F * ((double)Rtot[rb][r] +
                                                   (double)__builtin_amdgcn_logf(Stot[rb][r])) + K;
                        a.loglik[pix * a.L + l] = (float)lg;
                    }
                }
        }
    }
}

template <int KSTEPS>
static hipError_t launch_mfma_k(const LaunchCtx &lc, const ParzenFastArgs &a) {
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_parzen_mfma<KSTEPS, kParzenRB>,
                                                                256, 0);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    int64_t blocks = (int64_t)lc.num_cu * per_cu;
    const int64_t need = (int64_t)a.ngroups * a.L;
    if (blocks > need) blocks = need;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL((k_parzen_mfma<KSTEPS, kParzenRB>), dim3((unsigned)blocks), dim3(256), 0,
                       lc.stream, a);
    return hipGetLastError();
}

hipError_t launch_parzen_mfma(const LaunchCtx &lc, const ParzenFastArgs &a) {
    switch (a.ksteps) {
        case 1: return launch_mfma_k<1>(lc, a);
        case 2: return launch_mfma_k<2>(lc, a);
        default: return launch_mfma_k<3>(lc, a);
    }
}

}  // namespace cs
