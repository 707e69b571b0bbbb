// Parzen sum with the co-support texture factor on gfx950, texture term on
// the matrix cores (Sec. 3.1 Parzen colour/location density with adaptive
// bandwidth; Sec. 2 texture similarity inside the sum; Sec. 3.2 data term).
//
// The texture similarity of a pixel x and a sample y is the Hamming distance
// of their co-support masks, TSM = |A| + |B| - 2 |A n B|.  Its sample-dependent
// part |B| - 2 |A n B| is a dot product of two short feature vectors, so a
// whole 16-pixel x 16-sample block of it is one MFMA:
// v_mfma_scale_f32_16x16x128_f8f6f4 with FP8 (E4M3) operands and unit scales.
// Pixel features: mask bit j in {0, 1} for j < k, then [1, 1]; sample
// features: -2 x bit j, then [16 floor(|B|/16), |B| mod 16].  Every operand is
// an exactly representable FP8 value and every partial sum an integer below
// 2^10, so the FP32 accumulator holds it exactly; the pixel's own |A| joins
// the location operand below.
//
// The location term nA |p - s|^2 is a second, FP32 MFMA (16x16x4): with the
// pixel and sample positions taken relative to the tile origin it is the dot
// product of nA [|p|^2, -2 px, -2 py, 1] and [1, sx, sy, |s|^2], exact in its
// integer part, and the log-sum-exp reference rides in as the accumulator
// input.  Colours are stored pre-scaled by sqrt(log2(e) / (2 sigma_c^2)), so
// per pair the VALU is left with three colour differences, four FMAs (the
// texture term onto the MFMA result and the three negated squares), one
// v_exp_f32 and one add.
//
// Work decomposition.  A workgroup of 4 waves owns four 8x4 pixel tiles (one
// per wave); a work item is such a group and one label, taken from an atomic
// queue (labels of a group by decreasing sample count).  The samples of each
// label are padded to whole chunks of 64 with samples that contribute exactly
// 0.  Chunks are copied from HBM/L2 straight into LDS with global_load_lds (no
// registers), double-buffered: chunk c+1 is in flight while chunk c is
// computed.
//
// Log-sum-exp: every lane keeps its own reference per pixel, starting at the
// per-pixel value from the coefficient kernel (an achieved exponent plus a
// margin, capped by the upper bound from the nearest sample distance).  After
// each chunk a lane sum above 2^64 moves that reference up by a whole power of
// two (exact rescale).  At the end of the item the 16 lanes that share a pixel
// (one sample column each) are combined at their largest reference.  An
// overflowed, non-finite or empty sum queues the (label, tile) for the exact
// two-pass kernel.
#include <type_traits>

#include "cs_internal.h"

namespace cs {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(3))) void lds_void;

constexpr double kLn2F = 0.6931471805599453;
constexpr double kLog2eF = 1.4426950408889634;
constexpr int kChunkS = kStreamChunk;  // samples per chunk
constexpr float kFarAway = 1e15f;      // x of padding samples: d^2 ~ 1e30, finite, term underflows to 0

// E4M3 (bias 7) bit pattern of an integer 0..256 that is exactly representable
// (0..16 and multiples of 16 up to 256).
__device__ __forceinline__ uint32_t fp8_of_int(uint32_t v) {
    if (v == 0) return 0u;
    const int e = 31 - __clz(v);
    const uint32_t m = ((v << 3) >> e) & 7u;
    return ((uint32_t)(e + 7) << 3) | m;
}

// Spread the 4 bits of a nibble into the 4 bytes of a word, each byte 0 or b:
// the copies nib << 7i do not overlap, so bit i lands alone at bit 8i.
__device__ __forceinline__ uint32_t nibble_bytes(uint32_t nib, uint32_t b) {
    return ((nib * 0x00204081u) & 0x01010101u) * b;
}

// Physical 16-byte slot of logical slot p in a sample row.  Rows are 128 B
// (or a multiple), so two consecutive rows share one 256-byte span of the 64
// LDS banks; XOR-ing the slot with (row / 2) mod 8 puts the 16 rows that one
// 16-lane group reads at the same logical slot into 16 distinct 16-byte bank
// windows.
__device__ __forceinline__ int swz(int p, int row) { return (p & ~7) | ((p & 7) ^ ((row >> 1) & 7)); }

// Padded sample stream: for every padded slot s (label segments rounded up to
// whole chunks), the FP8 feature row (swizzled) and its record; the records
// of a chunk of 64 slots take 2 KiB: 64 float4 {x, y, r, g}, then 64 floats b
// (then padding), so that 16 lanes reading 16 consecutive slots touch distinct
// LDS banks.  Padding slots have zero features and x = 1e15.
__global__ __launch_bounds__(256) void k_stream_build(const SampleRec *recs, int k, int KP, int L,
                                                       StreamSegs segs, int64_t Mpad, float cscale,
                                                       uint8_t *feat, float *rec) {
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= Mpad) return;
    int l = 0;
    while (l + 1 < L && s >= segs.pseg[l + 1]) ++l;
    const int64_t j = s - segs.pseg[l];
    const bool real = j < (int64_t)(segs.seg[l + 1] - segs.seg[l]);
    uint32_t words[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    uint32_t cnt = 0;
    const int row = (int)(s & (kChunkS - 1));
    float *rc = rec + (s - row) * 8;  // this chunk's 2 KiB of records
    float v5[5] = {kFarAway, 0.0f, 0.0f, 0.0f, 0.0f};
    if (real) {
        const uint32_t *rw = recs[segs.seg[l] + j].w;
        for (int w = 0; w < 8; ++w) {
            uint32_t v = rw[8 + w];
            const int lo = 32 * w;
            if (lo >= k) v = 0;
            else if (k - lo < 32) v &= (1u << (k - lo)) - 1u;
            words[w] = v;
            cnt += __popc(v);
        }
        for (int q = 0; q < 5; ++q) v5[q] = __uint_as_float(rw[q]);
        for (int q = 2; q < 5; ++q) v5[q] *= cscale;  // colours in units of the kernel width
    }
    for (int q = 0; q < 4; ++q) rc[4 * row + q] = v5[q];
    rc[4 * kChunkS + row] = v5[4];
    rc[5 * kChunkS + row] = 0.0f;  // padding (keeps the whole 2 KiB defined)
    rc[6 * kChunkS + row] = 0.0f;
    rc[7 * kChunkS + row] = 0.0f;
    uint32_t *fo = reinterpret_cast<uint32_t *>(feat + s * KP);
    for (int p = 0; p < KP / 16; ++p) {  // logical 16-byte slot p holds features 16p..16p+15
        uint32_t out4[4];
        for (int q = 0; q < 4; ++q) {
            const int f0 = 16 * p + 4 * q;
            uint32_t val = 0;
            if (real) {
                if (f0 < 256) val = nibble_bytes((words[f0 >> 5] >> (f0 & 31)) & 0xFu, 0xC0u);  // -2.0
                for (int b = 0; b < 4; ++b) {
                    const int f = f0 + b;
                    uint32_t byte = 0xFFFFFFFFu;
                    if (f == k) byte = fp8_of_int(16u * (cnt >> 4));
                    else if (f == k + 1) byte = fp8_of_int(cnt & 15u);
                    if (byte != 0xFFFFFFFFu) val = (val & ~(0xFFu << (8 * b))) | (byte << (8 * b));
                }
            }
            out4[q] = val;
        }
        uint32_t *dst = fo + 4 * swz(p, row);
        for (int q = 0; q < 4; ++q) dst[q] = out4[q];
    }
}

hipError_t launch_stream_build(const LaunchCtx &lc, const SampleRec *recs, int k, int KP, int L,
                               const StreamSegs &segs, int64_t Mpad, float cscale, uint8_t *feat, float *rec) {
    hipLaunchKernelGGL(k_stream_build, dim3((unsigned)((Mpad + 255) / 256)), dim3(256), 0, lc.stream,
                       recs, k, KP, L, segs, Mpad, cscale, feat, rec);
    return hipGetLastError();
}


// Register budget: four waves per SIMD (128 VGPRs) with one 128-feature MFMA
// step, two with the wider feature rows.
template <int KSTEPS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(KSTEPS == 1 ? 4 : 2)))
void k_parzen_mfma(ParzenFastArgs a) {
    constexpr int RB = kParzenRB;
    constexpr int KP = 128 * KSTEPS;
    constexpr int FEAT_B = kChunkS * KP;  // feature bytes per chunk
    // Separate LDS objects per buffer: with the buffer known at compile time the
    // compiler can tell that reads of one buffer do not depend on the copy in
    // flight into the other, and does not wait for it.
    __shared__ __align__(16) uint8_t s_feat0[FEAT_B];
    __shared__ __align__(16) uint8_t s_feat1[FEAT_B];
    __shared__ __align__(16) float s_rec0[kChunkS * 8];
    __shared__ __align__(16) float s_rec1[kChunkS * 8];
    __shared__ int s_item;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, jl = lane & 15;
    const int64_t N = (int64_t)a.H * a.W;
    const int W64 = (a.k + 63) / 64;
    // colours are scaled by sqrt(log2(e) / (2 sigma_c^2)) (samples by the
    // stream builder), so the colour term is minus the squared difference
    const float cscale = (float)sqrt(kLog2eF / (2.0 * a.sigma_c * a.sigma_c));
    const uint32_t *mask32 = reinterpret_cast<const uint32_t *>(a.masks);
    const int nitems = a.ngroups * a.L;
    const int64_t coef_label_stride = (int64_t)a.ngroups * 4 * kTilePix;
    // the lane's 32-feature slice q of the pixel features covers mask word
    // 4q + g: which of its bits are real mask bits, which are the unit features
    const int nw32 = (a.k + 31) / 32;
    const uint32_t lastmask = (a.k & 31) ? (1u << (a.k & 31)) - 1u : ~0u;
    uint32_t lowm[KSTEPS], spec[KSTEPS];
#pragma unroll
    for (int q = 0; q < KSTEPS; ++q) {
        const int wi = 4 * q + g, rel = a.k - 32 * wi;
        lowm[q] = wi < nw32 - 1 ? ~0u : wi == nw32 - 1 ? lastmask : 0u;
        spec[q] = (rel >= 0 && rel < 32 ? 1u << rel : 0u) | (rel + 1 >= 0 && rel + 1 < 32 ? 1u << (rel + 1) : 0u);
    }
    const float wc = g == 0 ? 1.0f : 0.0f, wx = g == 1 ? 1.0f : 0.0f, wy = g == 2 ? 1.0f : 0.0f,
                wq = g == 3 ? 1.0f : 0.0f;
    uint32_t n_rescale = 0;  // wave-chunks whose reference moved (wave-uniform)
    uint32_t n_overflow = 0; // (label, tile) items handed to the exact kernel on overflow

    for (;;) {
        __syncthreads();  // the previous item's LDS reads are done
        if (tid == 0) s_item = (int)atomicAdd(a.work_counter, 1u);
        __syncthreads();
        const int item = s_item;
        if (item >= nitems) break;
        // item -> (group of 4 tiles, label); labels of a group in order of
        // decreasing sample count, so the queue ends with the short items
        const int grp = item / a.L;
        const int lab = a.meta[a.L + 1 + (item - grp * a.L)];
        const int c0 = a.meta[lab], c1 = a.meta[lab + 1];
        const int tile = grp * 4 + wave;
        const bool tile_ok = tile < a.ntiles;
        const int ty_t = tile_ok ? tile / a.tiles_x : 0;
        const int x0 = (tile_ok ? tile - ty_t * a.tiles_x : 0) * 8, y0 = ty_t * 2 * RB;

        // Async copy of chunk c into a buffer pair.
        auto issue = [&](int c, uint8_t *sf, float *sr) {
            const int64_t s0 = (int64_t)c * kChunkS;
#pragma unroll
            for (int u = 0; u < FEAT_B / 4096; ++u) {
                const uint8_t *src = a.feat + s0 * KP + u * 4096 + tid * 16;
                __builtin_amdgcn_global_load_lds(src, (lds_void *)(sf + u * 4096 + wave * 1024), 16, 0, 0);
            }
            if (wave < 2) {
                const float *src = a.rec + s0 * 8 + tid * 4;
                __builtin_amdgcn_global_load_lds(src, (lds_void *)(sr + wave * 256), 16, 0, 0);
            }
        };
        issue(c0, s_feat0, s_rec0);

        // ---- pixel colours: lane holds pixels (rb, r) -> (x0 + 4(g&1) + r, y0 + 2rb + (g>>1)),
        // the rows 4g + r of the MFMA result blocks
        float pr[RB][4], pg[RB][4], pb[RB][4];
        bool anyvalid = false;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int px = x0 + 4 * (g & 1) + r, py = y0 + 2 * rb + (g >> 1);
                const bool v = tile_ok && px < a.W && py < a.H;
                anyvalid |= v;
                const int64_t pix = v ? (int64_t)py * a.W + px : 0;
                pr[rb][r] = cscale * a.rgb[pix];
                pg[rb][r] = cscale * a.rgb[N + pix];
                pb[rb][r] = cscale * a.rgb[2 * N + pix];
            }
        bool active = __ballot(anyvalid) != 0ull;  // wave-uniform
        const bool wave_valid = active;

        // ---- per-pixel coefficients of this label (log2 units)
        const float4 *cf = a.coef + (int64_t)lab * coef_label_stride + (int64_t)tile * kTilePix;
        float nB[RB][4];
        f32x4 nRv[RB];  // -reference, the accumulator input of the location MFMA
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float4 v = cf[(2 * rb + (g >> 1)) * 8 + 4 * (g & 1) + r];
                nB[rb][r] = v.y;
                nRv[rb][r] = v.z;
            }

        // ---- pixel rows of both MFMAs: row i = lane%16 of row block rb is
        // pixel rb*16 + jl of the tile = (x0 + (jl & 7), y0 + 2rb + (jl >> 3)).
        // FP8 operand: the lane's 32-feature slice of the mask bits plus the
        // two unit features at k, k+1.
        // Location operand (FP32 MFMA, K = 4), positions relative to the tile
        // origin: A[i] = [nA_i (dx^2 + dy^2) + nB_i |A_i|, -2 nA_i dx, -2 nA_i dy, nA_i]
        // against B[j] = [1, sx, sy, sx^2 + sy^2], so that (A B)[i][j] =
        // nA_i |p_i - s_j|^2 + nB_i |A_i|; the reference rides in as the
        // accumulator input.
        i32x8 Aop[RB][KSTEPS];
        float Aloc[RB];
        bool weak = false;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            const int dxi = jl & 7, dyi = 2 * rb + (jl >> 3);
            const bool v = tile_ok && x0 + dxi < a.W && y0 + dyi < a.H;
            const int64_t pix = v ? (int64_t)(y0 + dyi) * a.W + x0 + dxi : 0;
            const uint32_t *mw = mask32 + pix * 2 * W64;
            uint32_t cnt = 0;
            for (int w = 0; w < nw32; ++w) cnt += __popc(mw[w] & (w == nw32 - 1 ? lastmask : ~0u));
#pragma unroll
            for (int q = 0; q < KSTEPS; ++q) {
                const uint32_t m = lowm[q] ? mw[4 * q + g] & lowm[q] : 0u;
                const uint32_t ext = v ? (m | spec[q]) : 0u;
#pragma unroll
                for (int vv = 0; vv < 8; ++vv) Aop[rb][q][vv] = (int)nibble_bytes((ext >> (4 * vv)) & 0xFu, 0x38u);
            }
            const float4 crow = cf[rb * 16 + jl];
            const float nA = crow.x;
            const float dx = (float)dxi, dy = (float)dyi;
            Aloc[rb] = g == 0 ? fmaf(nA, fmaf(dx, dx, dy * dy), crow.y * (float)cnt)
                     : g == 1 ? -2.0f * dx * nA : g == 2 ? -2.0f * dy * nA : nA;
            // padding samples sit 1e15 px away; a bandwidth wide enough to
            // reach them (or a non-finite one) goes to the exact kernel
            weak |= v && !(nA < -1e-18f);
        }
        bool item_bad = __ballot(weak) != 0ull;
        if (item_bad) active = false;

        const float x0f = (float)x0, y0f = (float)y0;
        float S[RB][4];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int r = 0; r < 4; ++r) S[rb][r] = 0.0f;

        // One chunk computed from buffers (F, Rr) while the next one streams
        // into (Fn, Rn).
        auto process = [&](int c, const uint8_t *F, const float *Rr, uint8_t *Fn, float *Rn) {
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();  // chunk c resident in (F, Rr); the other pair is free
            if (c + 1 < c1) issue(c + 1, Fn, Rn);
            if (!active) return;
#pragma unroll 1
            for (int st = 0; st < kChunkS / 16; ++st) {
                const int js = st * 16 + jl;
                i32x8 Bop[KSTEPS];
#pragma unroll
                for (int q = 0; q < KSTEPS; ++q) {
                    const int p0 = 8 * q + 2 * g;
                    const uint4 lo4 = *reinterpret_cast<const uint4 *>(F + js * KP + 16 * swz(p0, js));
                    const uint4 hi4 = *reinterpret_cast<const uint4 *>(F + js * KP + 16 * swz(p0 + 1, js));
                    Bop[q] = i32x8{(int)lo4.x, (int)lo4.y, (int)lo4.z, (int)lo4.w,
                                   (int)hi4.x, (int)hi4.y, (int)hi4.z, (int)hi4.w};
                }
                const float4 sxyrg = *reinterpret_cast<const float4 *>(Rr + js * 4);
                const float sb = Rr[4 * kChunkS + js];
                f32x4 T[RB];
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    T[rb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int q = 0; q < KSTEPS; ++q)
                        T[rb] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(Aop[rb][q], Bop[q], T[rb], 0, 0,
                                                                                  0, 127, 0, 127);
                }
                // this lane's entry g of the location column (one-hot weights,
                // no divergent select)
                const float sx = sxyrg.x - x0f, sy = sxyrg.y - y0f;
                const float bl = fmaf(wq, fmaf(sx, sx, sy * sy), fmaf(wy, sy, fmaf(wx, sx, wc)));
                f32x4 D[RB];
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) D[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(Aloc[rb], bl, nRv[rb], 0, 0, 0);
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const float dr = pr[rb][r] - sxyrg.z, dg = pg[rb][r] - sxyrg.w, db = pb[rb][r] - sb;
                        float u = fmaf(T[rb][r], nB[rb][r], D[rb][r]);
                        u = fmaf(-dr, dr, u);
                        u = fmaf(-dg, dg, u);
                        u = fmaf(-db, db, u);
                        S[rb][r] += __builtin_amdgcn_exp2f(u);
                    }
            }
            // A lane sum above 2^64 moves that pixel's reference up by a whole
            // power of two (exact rescale).  Entering a chunk the sums are at
            // most 2^64, so an overflowed sum means terms beyond 2^128 that make
            // the earlier part negligible; such a tile goes to the exact kernel.
            bool big = false;
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int r = 0; r < 4; ++r) big |= !(S[rb][r] <= 0x1p64f);
            if (__ballot(big)) {
                ++n_rescale;
                bool over = false;
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const float s = S[rb][r];
                        if (!(s <= 0x1p64f)) {
                            if (s <= 3.0e38f) {
                                const int e = (int)((__float_as_uint(s) >> 23) & 0xFFu) - 127;
                                S[rb][r] = ldexpf(s, -e);
                                nRv[rb][r] -= (float)e;
                            } else {
                                over = true;
                            }
                        }
                    }
                if (__ballot(over)) {
                    item_bad = true;
                    active = false;
                    ++n_overflow;
                }
            }
        };
        for (int c = c0; c < c1; c += 2) {
            process(c, s_feat0, s_rec0, s_feat1, s_rec1);
            if (c + 1 < c1) process(c + 1, s_feat1, s_rec1, s_feat0, s_rec0);
        }
        if (!wave_valid) continue;

        // ---- end of item: combine the 16 lanes sharing each pixel (one sample
        // column each) at their largest reference; lane jl < 8 of each 16-lane
        // group keeps pixel (rb, r) = (jl >> 2, jl & 3) for the write
        bool bad = item_bad;
        float Rw = 0.0f, Sw = 1.0f;
        if (!bad) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float Rl = -nRv[rb][r];
                    float Rm = Rl;
#pragma unroll
                    for (int off = 1; off < 16; off <<= 1) Rm = fmaxf(Rm, __shfl_xor(Rm, off));
                    float sp = S[rb][r] * __builtin_amdgcn_exp2f(Rl - Rm);
#pragma unroll
                    for (int off = 1; off < 16; off <<= 1) sp += __shfl_xor(sp, off);
                    const int px = x0 + 4 * (g & 1) + r, py = y0 + 2 * rb + (g >> 1);
                    const bool v = tile_ok && px < a.W && py < a.H;
                    if (v && !(sp <= 0x1p126f && sp > 0.0f)) bad = true;
                    if (jl == 4 * rb + r) {
                        Rw = Rm;
                        Sw = sp;
                    }
                }
        }
        if (__ballot(bad)) {
            if (lane == 0) {
                const unsigned int slot = atomicAdd(a.fix_count, 1u);
                if (slot < (unsigned int)a.fix_cap) a.fixlist[slot] = make_int2(lab, tile);
            }
            continue;
        }
        if (jl < 4 * RB) {
            const int rb = jl >> 2, r = jl & 3;
            const int px = x0 + 4 * (g & 1) + r, py = y0 + 2 * rb + (g >> 1);
            if (tile_ok && px < a.W && py < a.H) {
                const double K = (double)cf[(2 * rb + (g >> 1)) * 8 + 4 * (g & 1) + r].w;
                const double lg = kLn2F * ((double)Rw + (double)__builtin_amdgcn_logf(Sw)) + K;
                a.loglik[((int64_t)py * a.W + px) * a.L + lab] = (float)lg;
            }
        }
    }
    if (lane == 0 && (n_rescale | n_overflow)) {
        if (n_rescale) atomicAdd(a.fix_count + 1, n_rescale);
        if (n_overflow) atomicAdd(a.fix_count + 2, n_overflow);
    }
}

template <int KSTEPS>
static hipError_t launch_mfma_k(const LaunchCtx &lc, const ParzenFastArgs &a) {
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_parzen_mfma<KSTEPS>, 256, 0);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    int64_t blocks = (int64_t)lc.num_cu * per_cu;
    const int64_t items = (int64_t)a.ngroups * a.L;
    if (blocks > items) blocks = items;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_parzen_mfma<KSTEPS>, dim3((unsigned)blocks), dim3(256), 0, lc.stream, a);
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
