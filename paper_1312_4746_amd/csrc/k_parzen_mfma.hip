// Parzen sum with the co-support texture factor on gfx950, texture term on
// the matrix cores (Sec. 3.1 Parzen colour/location density with adaptive
// bandwidth; Sec. 2 texture similarity inside the sum; Sec. 3.2 data term).
//
// The texture similarity of a pixel x and a sample y is the Hamming distance
// of their co-support masks, TSM = |A| + |B| - 2 |A n B|: a dot product of two
// short integer feature vectors, so a whole 16-pixel x 16-sample block of it
// is one matrix-core product, v_mfma_scale_f32_16x16x128_f8f6f4 with FP6
// (E2M3) operands and unit scales.  Pixel features: mask bit j in {0, 1} for
// j < k, then the base-7 digits of |A| (D slots of values 0..7 whose sum
// times 7 is 7 floor(|A|/7)), |A| mod 7, D sevens and a one; sample features:
// -2 x bit j, then D sevens, a one, the digits of |B| and |B| mod 7.  The
// product is the whole TSM.  Every operand is an integer in -7..7, exactly
// representable in E2M3, and every partial sum an integer below 2^10, so the
// FP32 accumulator holds it exactly; FP6 operands run at twice the FP8 rate.
//
// The location term nA |p - s|^2 needs the integer Q = |p - s|^2 = |p|^2 -
// 2 p.s + |s|^2 of two pixel positions.  With every coordinate below 2048 each
// factor splits into at most three BF16 pieces of 8 significant bits (exact),
// every product of pieces is exact, and every partial sum is an integer of
// magnitude at most |p|^2 + |s|^2 < 2^24, so a BF16 MFMA (16x16x32, 14 of the
// 32 K slots used) returns Q exactly in FP32 whatever its summation order.  The
// sample pieces are precomputed in the sample stream; the pixel pieces are
// set once per work item.  Colours are stored pre-scaled by
// sqrt(log2(e) / (2 sigma_c^2)), so per pair the VALU is left with the texture
// and location factors (two FMAs onto the log-sum-exp reference), three
// colour differences and three negated squares (FMAs), one v_exp_f32 and one
// add.  (An FP32 MFMA, K = 4, also fits the location term, but on gfx950 it
// holds the VALU for its whole duration; the BF16 one largely overlaps it.)
//
// Colours at n <= 255 levels per channel (8-bit images): with q = rint(c n)
// - 128 in -128..127 per channel, the squared colour distance
// |q_x|^2 - 2 q_x.q_y + |q_y|^2 is an integer below 2^18 whose every factor
// is exact in BF16 (|q|^2 < 2^16 split at bit 8), so it is a third BF16
// product, exact in FP32.  One FMA with kcol = -log2(e) / (2 sigma_c^2 n^2)
// replaces the six colour instructions: five VALU instructions per pair, one
// of them the v_exp_f32.  That form (k_parzen_mfma32, below the 16 x 16 one)
// runs the products as 32 x 32 blocks with the samples as rows and one pixel
// per lane; the 16 x 16 form (k_parzen_mfma) takes float colours.
//
// Work decomposition.  A workgroup of 4 waves owns four 8x4 pixel tiles (one
// per wave); a work item is such a group and one label.  Items come from one
// atomic queue per XCD: queue x holds the groups x, x + 8, x + 16, ... with
// the labels of a group consecutive (by decreasing sample count), and a
// workgroup takes from the queue of its own XCD first (workgroup w runs on
// XCD w mod 8), then from the others.  The ten items of a group thus run at
// about the same time on one XCD: its pixel operands are fetched into that
// XCD's L2 once, and the partial lines of its pixel-major log-likelihood rows
// are mostly merged there before they are written back.  The last
// kTailGroups groups of a queue go label by label instead, so that the queue
// ends with the items of the smallest label.  The samples of each
// label are padded to whole chunks of 64 with samples that contribute exactly
// 0.  Chunks are copied from HBM/L2 straight into LDS with global_load_lds (no
// registers), double-buffered: chunk c+1 is in flight while chunk c is
// computed.
//
// Log-sum-exp: each pixel has one reference, shared by the 16 lanes that hold
// its sample columns, starting at the per-pixel value from the coefficient
// kernel (an achieved exponent plus a margin, capped by the upper bound from
// the nearest sample distance).  After each chunk a lane sum above 2^64 moves
// the reference of that pixel up by a whole power of two, the largest needed
// by any of its 16 lanes (exact rescale); at the end of the item the 16 lane
// sums are added.  A sum that overflows within a chunk stops the pass; the
// item is computed again with the overflowed pixels' references raised (up to
// kRetries times).  A sum that still overflows, or is non-finite or empty,
// queues the (label, tile) for the exact two-pass kernel.
#include <type_traits>

#include "cs_internal.h"

namespace cs {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(3))) void lds_void;

constexpr double kLn2F = 0.6931471805599453;
constexpr double kLog2eF = 1.4426950408889634;
constexpr int kChunkS = kStreamChunk;  // samples per chunk
constexpr float kFarQ = 0x1p100f;      // location feature of padding samples: Q ~ 2^100, term underflows to 0
// Floats of one chunk's records: location pieces K 0..7 (64 x 16 B), K 8..15
// (64 x 16 B), colours (64 x float4).
constexpr int kRecChunkF = kChunkS * 12;
constexpr int kTailGroups = 64;  // groups at the end of each work queue taken label by label
constexpr int kRetries = 8;      // passes again over an item whose sums overflowed
constexpr float kRaise = 170.0f; // reference raise per retry (log2 units)

// BF16 bit pattern of a float that BF16 holds exactly.
__device__ __forceinline__ short bf16_bits(float v) { return __builtin_bit_cast(short, (__bf16)v); }

// E2M3 (bias 1) bit pattern of an integer -7..7 (all exactly representable).
__device__ __forceinline__ uint32_t fp6_of_int(int v) {
    const uint32_t a = (uint32_t)(v < 0 ? -v : v);
    // 0, 1, 2, 3 = 1.5 x 2, 4, 5 = 1.25 x 4, 6 = 1.5 x 4, 7 = 1.75 x 4
    const uint32_t code = (0x1E1C1A1814100800ull >> (8 * a)) & 0x3Fu;
    return code | (v < 0 ? 0x20u : 0u);
}

// Colour value c at n levels as a centred integer: rint(c n) clamped to
// 0..255, minus 128 (so -128..127; for c the FP32 value of a multiple of 1/n,
// c n is within two ulps of that integer and rounds to it).
__device__ __forceinline__ int colour_level(float c, int n) {
    float q = rintf(c * (float)n);
    q = fminf(fmaxf(q, 0.0f), 255.0f);  // a NaN becomes 0
    return (int)q - 128;
}

// The 32 FP6 codes of features f0 .. f0 + 31 (f0 a multiple of 32) packed as
// the lane operand of one 16x16x128 step: feature f0 + v at bits 6v .. 6v + 5
// of six dwords.  The mask-bit features of the group take a code for each set
// bit (1 for a pixel, -2 for a sample); the count features k .. k + 2D + 1
// that fall in the group are formed directly (the digits and the remainder
// of the count computed once); every other feature is zero.
template <bool PIX>
__device__ __forceinline__ void tex_pack(int f0, int k, const uint32_t *bits, uint32_t c, uint32_t (&o)[6]) {
    for (int d = 0; d < 6; ++d) o[d] = 0u;
    auto put = [&](int v, uint32_t code) {
        const int b = 6 * v, d = b >> 5, sh = b & 31;
        o[d] |= code << sh;
        if (sh > 26) o[d + 1] |= code >> (32 - sh);
    };
    if (f0 < k) {
        uint32_t w = bits[f0 >> 5];
        if (k - f0 < 32) w &= (1u << (k - f0)) - 1u;
        const uint32_t code = PIX ? fp6_of_int(1) : fp6_of_int(-2);
        // unrolled: every position a constant, so each bit is a masked OR
#pragma unroll
        for (int v = 0; v < 32; ++v)
            if ((w >> v) & 1u) put(v, code);
    }
    const int D = tex_digits(k);
    const int e0 = f0 > k ? f0 : k, e1 = f0 + 32 < k + 2 * D + 2 ? f0 + 32 : k + 2 * D + 2;
    if (e0 < e1) {
        const int q = (int)(c / 7u), r = (int)(c % 7u);
        for (int e = e0; e < e1; ++e) {
            const int x = e - k;
            const int s = x < D ? x : x - D - 1;  // digit index within its run
            int dg = q - 7 * s;
            dg = dg < 0 ? 0 : dg > 7 ? 7 : dg;
            int val;
            if (x < D) val = PIX ? dg : 7;
            else if (x == D) val = PIX ? r : 1;
            else if (x < 2 * D + 1) val = PIX ? 7 : dg;
            else val = PIX ? 1 : r;
            put(e - f0, fp6_of_int(val));
        }
    }
}

// Physical 16-byte slot of logical slot p in a sample row.  Rows are 128 B
// (or a multiple), so two consecutive rows share one 256-byte span of the 64
// LDS banks; XOR-ing the slot with (row / 2) mod 8 puts the 16 rows that one
// 16-lane group reads at the same logical slot into 16 distinct 16-byte bank
// windows.
__device__ __forceinline__ int swz(int p, int row) { return (p & ~7) | ((p & 7) ^ ((row >> 1) & 7)); }

// Padded sample stream: for every padded slot s (label segments rounded up to
// whole chunks), the FP6 feature row (swizzled; 32 bytes per 32-feature group,
// six dwords used) and its record.  The records
// of a chunk of 64 slots take 3 KiB, three planes of 64 x 16 B so that 16 lanes
// reading 16 consecutive slots touch distinct LDS banks: the BF16 location
// pieces for K 0..7 [1, 1, 1, sx_h, sx_l, sx_h, sx_l, sy_h] and K 8..15
// [sy_l, sy_h, sy_l, q_h, q_m, q_l, far, 0] (q = sx^2 + sy^2), then the
// scaled colours {r, g, b, 0}, or with colour levels the BF16 colour pieces
// for K 16..23 [-2 r, -2 g, -2 b, 1, 1, s_h, s_l, 0] of the centred integer
// colours (s = r^2 + g^2 + b^2 < 2^16, split at bit 8).  Padding slots have
// zero features and pieces except far = 2^100.
__device__ __forceinline__ void stream_build(const SampleRec *recs, int k, int KP, int L, const StreamSegs &segs,
                                             int64_t Mpad, float cscale, int levels, uint8_t *feat, float *rec,
                                             int bid) {
    const int64_t s = (int64_t)bid * 256 + threadIdx.x;
    if (s >= Mpad) return;
    int l = 0;
    while (l + 1 < L && s >= segs.pseg[l + 1]) ++l;
    const int64_t j = s - segs.pseg[l];
    const bool real = j < (int64_t)(segs.seg[l + 1] - segs.seg[l]);
    uint32_t words[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    uint32_t cnt = 0;
    const int row = (int)(s & (kChunkS - 1));
    float *rc = rec + (s / kChunkS) * kRecChunkF;  // this chunk's 3 KiB of records
    float lp[16];
    for (int q = 0; q < 16; ++q) lp[q] = 0.0f;
    float col[3] = {0.0f, 0.0f, 0.0f};
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
        const uint32_t sx = (uint32_t)__uint_as_float(rw[0]), sy = (uint32_t)__uint_as_float(rw[1]);
        const uint32_t q = sx * sx + sy * sy;
        const float sxh = (float)(sx & ~0xFFu), sxl = (float)(sx & 0xFFu);
        const float syh = (float)(sy & ~0xFFu), syl = (float)(sy & 0xFFu);
        const float v0[16] = {1.0f, 1.0f, 1.0f, sxh, sxl, sxh, sxl, syh,
                              syl, syh, syl, (float)(q & ~0xFFFFu), (float)(q & 0xFF00u), (float)(q & 0xFFu),
                              0.0f, 0.0f};
        for (int t = 0; t < 16; ++t) lp[t] = v0[t];
        for (int c = 0; c < 3; ++c) col[c] = cscale * __uint_as_float(rw[2 + c]);
    } else {
        lp[14] = kFarQ;
    }
    uint32_t pk[8];
    for (int t = 0; t < 8; ++t)
        pk[t] = (uint32_t)(uint16_t)bf16_bits(lp[2 * t]) | ((uint32_t)(uint16_t)bf16_bits(lp[2 * t + 1]) << 16);
    uint32_t *r0 = reinterpret_cast<uint32_t *>(rc) + 4 * row;
    uint32_t *r1 = reinterpret_cast<uint32_t *>(rc) + 4 * kChunkS + 4 * row;
    for (int t = 0; t < 4; ++t) {
        r0[t] = pk[t];
        r1[t] = pk[4 + t];
    }
    float *rcol = rc + 8 * kChunkS + 4 * row;
    if (levels > 0) {
        float cp[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (real) {
            const uint32_t *rw = recs[segs.seg[l] + j].w;
            int cq[3], ss = 0;
            for (int c = 0; c < 3; ++c) {
                cq[c] = colour_level(__uint_as_float(rw[2 + c]), levels);
                ss += cq[c] * cq[c];
                cp[c] = (float)(-2 * cq[c]);
            }
            cp[3] = 1.0f;
            cp[4] = 1.0f;
            cp[5] = (float)(ss & ~0xFF);
            cp[6] = (float)(ss & 0xFF);
        }
        uint32_t *rq = reinterpret_cast<uint32_t *>(rcol);
        for (int t = 0; t < 4; ++t)
            rq[t] = (uint32_t)(uint16_t)bf16_bits(cp[2 * t]) | ((uint32_t)(uint16_t)bf16_bits(cp[2 * t + 1]) << 16);
    } else {
        rcol[0] = col[0];
        rcol[1] = col[1];
        rcol[2] = col[2];
        rcol[3] = 0.0f;
    }
    uint32_t *fo = reinterpret_cast<uint32_t *>(feat + s * KP);
    for (int grp = 0; grp < KP / 32; ++grp) {  // features 32 grp .. 32 grp + 31: logical slots 2 grp, 2 grp + 1
        uint32_t o[6] = {0, 0, 0, 0, 0, 0};
        if (real) tex_pack<false>(32 * grp, k, words, cnt, o);
        uint32_t *d0 = fo + 4 * swz(2 * grp, row), *d1 = fo + 4 * swz(2 * grp + 1, row);
        d0[0] = o[0];
        d0[1] = o[1];
        d0[2] = o[2];
        d0[3] = o[3];
        d1[0] = o[4];
        d1[1] = o[5];
        d1[2] = 0u;
        d1[3] = 0u;
    }
}

// Pixel records of the matrix-core path, tiled like the coefficients
// ([tile][kTilePix], slot q of a tile as in fast_slot_row): colours scaled by
// sqrt(log2(e) / (2 sigma_c^2)) (so that the colour term is minus the squared
// difference) and the co-support size |A| as a float; zeros for empty slots.
__device__ __forceinline__ void pixel_tiles(const float *rgb, const uint64_t *masks, int H, int W, int k,
                                            int tiles_x, int ntiles, const int32_t *list, int64_t nlist,
                                            int64_t nslots, float cscale, float4 *pix4, int bid) {
    const int64_t s = (int64_t)bid * 256 + threadIdx.x;
    if (s >= nslots) return;
    const int tile = (int)(s / kTilePix), i = (int)(s - (int64_t)tile * kTilePix);
    const int64_t row = fast_slot_row(list, nlist, H, W, tiles_x, ntiles, tile, i);
    float4 out = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (row >= 0) {
        const int64_t N = (int64_t)H * W, pix = fast_row_pixel(list, row);
        const int W64 = (k + 63) / 64;
        uint32_t cnt = 0;
        for (int w = 0; w < W64; ++w) {
            uint64_t m = masks[pix * W64 + w];
            if (w == W64 - 1 && (k & 63)) m &= (1ull << (k & 63)) - 1ull;
            cnt += (uint32_t)__popcll(m);
        }
        out = make_float4(cscale * rgb[pix], cscale * rgb[N + pix], cscale * rgb[2 * N + pix], (float)cnt);
    }
    pix4[s] = out;
}

// Pixel operands of the matrix-core path, built once per call: for every
// padded tile, row block rb and lane (g, jl) of the MFMA operands, row jl is
// the tile's slot (2 rb + (jl >> 3)) * 8 + (jl & 7) (fast_slot_row).
//  * FP6 texture operand (32 B per lane and 128-feature step q, six dwords
//    used): pixel features 128 q + 32 g .. + 31 (tex_feature; zero for empty
//    slots);
//  * BF16 location operand (16 B per lane): K 0..7 [|p|^2 pieces (3), -2 px
//    pieces (2, each twice), -2 py high] for g = 0, K 8..15 [-2 py high, -2 py
//    low (twice), 1, 1, 1, 1 (far term), 0] for g = 1, zeros for g = 3 and,
//    without colour levels, for g = 2; with colour levels g = 2 holds the
//    colour pieces K 16..23 [r, g, b, s_h, s_l, 1, 1, 0] of the centred integer
//    colours (s = r^2 + g^2 + b^2 split at bit 8), so that against the sample
//    pieces the product is the squared colour distance.
__device__ __forceinline__ void pixel_operands(const float *rgb, const uint64_t *masks, int H, int W, int k,
                                               int tiles_x, int ntiles, const int32_t *list, int64_t nlist,
                                               int64_t nthreads, int ksteps, int levels, uint32_t *aop, uint4 *abf,
                                               int bid) {
    const int64_t s = (int64_t)bid * 256 + threadIdx.x;
    if (s >= nthreads) return;
    const int lane = (int)(s & 63);
    const int64_t tr = s >> 6;  // tile * RB + rb
    const int rb = (int)(tr % kParzenRB);
    const int tile = (int)(tr / kParzenRB);
    const int g = lane >> 4, jl = lane & 15;
    const int64_t row = fast_slot_row(list, nlist, H, W, tiles_x, ntiles, tile, (2 * rb + (jl >> 3)) * 8 + (jl & 7));
    const bool v = row >= 0;
    const int64_t pix = v ? fast_row_pixel(list, row) : 0;
    const int px = (int)(pix % W), py = (int)(pix / W);
    const int W64 = (k + 63) / 64;
    const uint32_t *mw = reinterpret_cast<const uint32_t *>(masks) + pix * 2 * W64;
    const int nw32 = (k + 31) / 32;
    uint32_t bits[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    uint32_t cnt = 0;
    if (v)
        for (int w = 0; w < nw32; ++w) {
            const uint32_t m = mw[w] & (w == nw32 - 1 && (k & 31) ? (1u << (k & 31)) - 1u : ~0u);
            bits[w] = m;
            cnt += __popc(m);
        }
    for (int q = 0; q < ksteps; ++q) {
        uint32_t o[6] = {0, 0, 0, 0, 0, 0};
        if (v) tex_pack<true>(128 * q + 32 * g, k, bits, cnt, o);
        uint4 *dst = reinterpret_cast<uint4 *>(aop + (((int64_t)tr * ksteps + q) * 64 + lane) * 8);
        dst[0] = make_uint4(o[0], o[1], o[2], o[3]);
        dst[1] = make_uint4(o[4], o[5], 0u, 0u);
    }
    const uint32_t p2 = (uint32_t)(px * px + py * py), X = 2u * (uint32_t)px, Y = 2u * (uint32_t)py;
    const float xh = -(float)(X & ~0xFFu), xl = -(float)(X & 0xFFu);
    const float yh = -(float)(Y & ~0xFFu), yl = -(float)(Y & 0xFFu);
    float e[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (g == 0) {
        e[0] = (float)(p2 & ~0xFFFFu); e[1] = (float)(p2 & 0xFF00u); e[2] = (float)(p2 & 0xFFu);
        e[3] = xh; e[4] = xh; e[5] = xl; e[6] = xl; e[7] = yh;
    } else if (g == 1) {
        e[0] = yh; e[1] = yl; e[2] = yl; e[3] = 1.0f; e[4] = 1.0f; e[5] = 1.0f; e[6] = 1.0f;
    } else if (g == 2 && levels > 0 && v) {
        const int64_t N = (int64_t)H * W;
        int ss = 0;
        for (int c = 0; c < 3; ++c) {
            const int cq = colour_level(rgb[c * N + pix], levels);
            ss += cq * cq;
            e[c] = (float)cq;
        }
        e[3] = (float)(ss & ~0xFF); e[4] = (float)(ss & 0xFF); e[5] = 1.0f; e[6] = 1.0f;
    }
    uint32_t pk[4];
    for (int t = 0; t < 4; ++t)
        pk[t] = (uint32_t)(uint16_t)bf16_bits(e[2 * t]) | ((uint32_t)(uint16_t)bf16_bits(e[2 * t + 1]) << 16);
    abf[s] = make_uint4(pk[0], pk[1], pk[2], pk[3]);
}

// The per-call preparation of the full-image path in one launch: workgroups
// [0, b_stream) build the sample stream, the next b_tiles the pixel records,
// the rest the pixel operands (no dependence between the three).
__global__ __launch_bounds__(256) void k_prep(PrepArgs a) {
    int b = blockIdx.x;
    if (b < a.b_stream) {
        stream_build(a.recs, a.k, a.KP, a.L, a.segs, a.Mpad, a.cscale, a.levels, a.feat, a.rec, b);
        return;
    }
    b -= a.b_stream;
    if (b < a.b_tiles) {
        pixel_tiles(a.rgb, a.masks, a.H, a.W, a.k, a.tiles_x, a.ntiles, a.list, a.nlist, a.nslots, a.cscale,
                    a.pix4, b);
        return;
    }
    b -= a.b_tiles;
    pixel_operands(a.rgb, a.masks, a.H, a.W, a.k, a.tiles_x, a.ntiles, a.list, a.nlist, a.nthreads, a.ksteps,
                   a.levels, a.aop, a.abf, b);
}

hipError_t launch_prep(const LaunchCtx &lc, PrepArgs a) {
    a.nslots = a.ntiles_pad * kTilePix;
    a.nthreads = a.ntiles_pad * kParzenRB * 64;
    a.b_stream = (int)((a.Mpad + 255) / 256);
    a.b_tiles = (int)((a.nslots + 255) / 256);
    const int64_t blocks = a.b_stream + a.b_tiles + (a.nthreads + 255) / 256;
    hipLaunchKernelGGL(k_prep, dim3((unsigned)blocks), dim3(256), 0, lc.stream, a);
    return hipGetLastError();
}

// Register budget: four waves per SIMD (128 VGPRs) with one 128-feature MFMA
// step, two with the wider feature rows.
// TEX = false: the texture factor stays out of the sum (eq:joined forms):
// no feature stream, no FP6 products, only the location and colour terms.
// This form takes float colours (colour levels go to k_parzen_mfma32).
template <int KSTEPS, bool TEX, bool LIST>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(KSTEPS == 1 ? 4 : 2)))
void k_parzen_mfma(ParzenFastArgs a) {
    constexpr int RB = kParzenRB;
    constexpr int KP = 128 * KSTEPS;
    constexpr int FEAT_B = TEX ? kChunkS * KP : 16;  // feature bytes per chunk
    // Separate LDS objects per buffer: with the buffer known at compile time the
    // compiler can tell that reads of one buffer do not depend on the copy in
    // flight into the other, and does not wait for it.
    __shared__ __align__(16) uint8_t s_feat0[FEAT_B];
    __shared__ __align__(16) uint8_t s_feat1[FEAT_B];
    __shared__ __align__(16) float s_rec0[kRecChunkF];
    __shared__ __align__(16) float s_rec1[kRecChunkF];
    // each wave's BF16 location operands (read at every step; kept here
    // rather than in registers, which the kernel has none left of)
    __shared__ __align__(16) s16x8 s_abf[4][RB][64];
    __shared__ int s_item, s_queue;
    // overflow retry: any wave of the workgroup overflowed in the last pass,
    // and per lane the pixels (bit 4 rb + r) whose sums overflowed
    __shared__ int s_ovf;
    __shared__ uint8_t s_ovp[4][64];
    // per wave, lane and pixel (4 rb + r): how often the reference was raised
    __shared__ uint32_t s_nraise[4][64];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, jl = lane & 15;
    // the wave index as a wave-uniform (scalar) value: the LDS destinations of
    // the chunk copies and the copy branch need no per-lane arithmetic
    const int wave_u = __builtin_amdgcn_readfirstlane(wave);
    const int64_t coef_label_stride = (int64_t)a.ngroups * 4 * kTilePix;
    // LDS byte offsets of the lane's operands in step 0 of a chunk buffer (step
    // st adds st * 16 rows; the swizzle depends on the row only through
    // (row / 2) mod 8, the same for rows jl and 16 st + jl)
    int foff[KSTEPS][2];
#pragma unroll
    for (int q = 0; q < KSTEPS; ++q)
#pragma unroll
        for (int h = 0; h < 2; ++h) foff[q][h] = jl * KP + 16 * swz(8 * q + 2 * g + h, jl);
    const int loff = (g & 1) * (16 * kChunkS) + 16 * jl;  // location pieces, K 0..7 or 8..15
    const int coff = 32 * kChunkS + 16 * jl;              // colours
    uint32_t n_rescale = 0;  // wave-chunks whose reference moved (wave-uniform)
    uint32_t n_overflow = 0; // (label, tile) items handed to the exact kernel on overflow

    // queue state (thread 0): current queue and how many have been emptied
    int queue = blockIdx.x % kParzenQueues, emptied = 0;
    if (tid == 0) s_ovf = 0;
    for (;;) {
        __syncthreads();  // the previous item's LDS reads are done
        if (tid == 0) {
            int it = -1;
            while (emptied < kParzenQueues) {
                // groups queue, queue + 8, ... : nq of them, L items each
                const int nq = queue < a.ngroups ? (a.ngroups - 1 - queue) / kParzenQueues + 1 : 0;
                const int t = (int)atomicAdd(a.work_counter + queue * kQueueStride, 1u);
                if (t < nq * a.L) {
                    it = t;
                    break;
                }
                queue = queue + 1 == kParzenQueues ? 0 : queue + 1;
                ++emptied;
            }
            s_item = it;
            s_queue = queue;
        }
        __syncthreads();
        const int item = s_item;
        if (item < 0) break;
        // item -> (group, label).  The labels (in order of decreasing sample
        // count) are cut into blocks of a.lblock; block by block, the groups
        // of the queue go in order with the labels of the block consecutive.
        // With one block (the label streams fit the L2 together) a group's
        // items run at about the same time, its pixel operands fetched once;
        // with several, the workgroups of an XCD share the streams of a few
        // labels at a time, which then stay in its L2.  The queue's last
        // kTailGroups groups go label by label so that the queue ends with the
        // shortest items (their operands stay in L2 meanwhile).
        const int qg = s_queue < a.ngroups ? (a.ngroups - 1 - s_queue) / kParzenQueues + 1 : 0;
        const int tg = qg < kTailGroups ? qg : kTailGroups;
        const int hg = qg - tg;
        const int head_items = hg * a.L;
        int gi, lrank;
        if (item < head_items) {
            const int nblk = (a.L + a.lblock - 1) / a.lblock;
            int b = item / (hg * a.lblock);
            if (b > nblk - 1) b = nblk - 1;
            const int bsz = b < nblk - 1 ? a.lblock : a.L - a.lblock * (nblk - 1);
            const int rr = item - hg * a.lblock * b;
            gi = rr / bsz;
            lrank = a.lblock * b + (rr - gi * bsz);
        } else {
            const int j = item - head_items;
            lrank = j / tg;
            gi = qg - tg + (j - lrank * tg);
        }
        const int grp = s_queue + kParzenQueues * gi;
        const int lab = a.meta[a.L + 1 + lrank];
        const int c0 = a.meta[lab], c1 = a.meta[lab + 1];
        const int last_steps = a.meta[2 * a.L + 1 + lab];  // 16-sample steps of the last chunk
        const int tile = grp * 4 + wave;
        // slots of the tile that hold a pixel (fast_slot_row): on the tile
        // grid those inside the image, on a list the first qlim
        const bool tile_ok = tile < a.ntiles;
        const int ty_t = tile_ok ? tile / a.tiles_x : 0;
        const int x0 = (tile_ok ? tile - ty_t * a.tiles_x : 0) * 8, y0 = ty_t * 2 * RB;
        int qlim = 0;
        if constexpr (LIST) {
            const int64_t rem = a.nlist - (int64_t)tile * kTilePix;
            qlim = rem < 0 ? 0 : rem > kTilePix ? kTilePix : (int)rem;
        }
        auto slot_ok = [&](int rb, int r) {
            if constexpr (LIST) return (2 * rb + (g >> 1)) * 8 + 4 * (g & 1) + r < qlim;
            const int px = x0 + 4 * (g & 1) + r, py = y0 + 2 * rb + (g >> 1);
            return tile_ok && px < a.W && py < a.H;
        };

        // Async copy of chunk c into a buffer pair.
        // (The lane's byte offset is rebuilt at every copy: held across the
        // chunk loop, its 64-bit address would be spilled at the register limit
        // and reloaded in front of the copies.)
        auto issue = [&](int c, uint8_t *sf, float *sr) {
            uint32_t off = (uint32_t)tid * 16u;
            __asm__ volatile("" : "+v"(off));
            if constexpr (TEX) {
                const uint8_t *fbase = a.feat + (int64_t)c * FEAT_B;
#pragma unroll
                for (int u = 0; u < FEAT_B / 4096; ++u)
                    __builtin_amdgcn_global_load_lds(fbase + u * 4096 + off,
                                                     (lds_void *)(sf + u * 4096 + wave_u * 1024), 16, 0, 0);
            }
            if (wave_u < 3) {
                const uint8_t *rbase = reinterpret_cast<const uint8_t *>(a.rec) + (int64_t)c * (kRecChunkF * 4);
                __builtin_amdgcn_global_load_lds(rbase + off, (lds_void *)(sr + wave_u * 256), 16, 0, 0);
            }
        };
        issue(c0, s_feat0, s_rec0);

        // ---- pixel colours (scaled) and coefficients of this label (log2
        // units): lane holds the tile's slots (rb, r) -> (2rb + (g>>1)) * 8 +
        // 4(g&1) + r, the rows 4g + r of the MFMA result blocks (on the tile
        // grid the pixel (x0 + 4(g&1) + r, y0 + 2rb + (g>>1))); both arrays
        // are tiled [tile][kTilePix] with the same slot order
        const float4 *pt = a.pix4 + (int64_t)tile * kTilePix;
        const float4 *cf = a.coef + (int64_t)lab * coef_label_stride + (int64_t)tile * kTilePix;
        float pr[RB][4], pg[RB][4], pb[RB][4];
        float nA[RB][4], nB[RB][4], nR[RB][4];  // location and texture factors, -reference
        bool anyvalid = false, weak = false;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int ti = (2 * rb + (g >> 1)) * 8 + 4 * (g & 1) + r;
                const bool v = slot_ok(rb, r);
                anyvalid |= v;
                const float4 c = pt[ti];
                pr[rb][r] = c.x;
                pg[rb][r] = c.y;
                pb[rb][r] = c.z;
                const float4 q = cf[ti];
                nA[rb][r] = q.x;
                nB[rb][r] = q.y;
                nR[rb][r] = q.z;
                // padding samples sit at Q ~ 2^100; a bandwidth wide enough to
                // reach them (or a non-finite one) goes to the exact kernel
                weak |= v && !(q.x < -1e-18f);
            }
        bool active = __ballot(anyvalid) != 0ull;  // wave-uniform
        const bool wave_valid = active;

        // ---- pixel rows of both MFMAs (built once per call by
        // k_pixel_operands): the FP6 texture operand into registers, the BF16
        // location operand straight into LDS (read at every step)
        i32x8 Aop[RB][KSTEPS];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            if constexpr (TEX) {
#pragma unroll
                for (int q = 0; q < KSTEPS; ++q) {
                    // six dwords (FP6) of the lane's 32-byte slot
                    const uint4 *src = reinterpret_cast<const uint4 *>(
                        a.aop + ((((int64_t)tile * RB + rb) * KSTEPS + q) * 64 + lane) * 8);
                    const uint4 lo4 = src[0];
                    const uint2 hi2 = *reinterpret_cast<const uint2 *>(src + 1);
                    Aop[rb][q] = i32x8{(int)lo4.x, (int)lo4.y, (int)lo4.z, (int)lo4.w, (int)hi2.x, (int)hi2.y, 0, 0};
                }
            }
            const uint8_t *bsrc = a.abf + (((int64_t)tile * RB + rb) * 64 + lane) * 16;
            __builtin_amdgcn_global_load_lds(bsrc, (lds_void *)&s_abf[wave][rb][0], 16, 0, 0);
        }
        bool item_bad = __ballot(weak) != 0ull;
        if (item_bad) active = false;
        bool ovf_wave = false;  // this wave's sums overflowed in the last pass
        s_nraise[wave][lane] = 0u;

        float S[RB][4];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int r = 0; r < 4; ++r) S[rb][r] = 0.0f;

        // One chunk computed from buffers (F, Rr) while the next one streams
        // into (Fn, Rn); the last chunk of the label stops after its last
        // 16-sample step that holds a real sample.
        auto process = [&](int c, const uint8_t *F, const float *Rr, uint8_t *Fn, float *Rn) {
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();  // chunk c resident in (F, Rr); the other pair is free
            if (c + 1 < c1) issue(c + 1, Fn, Rn);
            if (!active) return;
            const int nst = c + 1 == c1 ? last_steps : kChunkS / 16;
#pragma unroll
            for (int st = 0; st < kChunkS / 16; ++st) {
                if (st >= nst) break;
                // opaque lane index: the location operand is read from LDS here
                // at every step instead of being hoisted out of the loop into
                // registers
                int al = lane;
                __asm__ volatile("" : "+v"(al));
                const uint8_t *Fs = F + st * 16 * KP;
                const uint8_t *Rs = reinterpret_cast<const uint8_t *>(Rr) + st * 256;
                i32x8 Bop[KSTEPS];
                if constexpr (TEX) {
#pragma unroll
                    for (int q = 0; q < KSTEPS; ++q) {
                        const uint4 lo4 = *reinterpret_cast<const uint4 *>(Fs + foff[q][0]);
                        const uint2 hi2 = *reinterpret_cast<const uint2 *>(Fs + foff[q][1]);
                        Bop[q] = i32x8{(int)lo4.x, (int)lo4.y, (int)lo4.z, (int)lo4.w, (int)hi2.x, (int)hi2.y, 0, 0};
                    }
                }
                const s16x8 Bbf = *reinterpret_cast<const s16x8 *>(Rs + loff);
                const float4 col = *reinterpret_cast<const float4 *>(Rs + coff);
                f32x4 T[RB], Q[RB];
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    T[rb] = f32x4{0.f, 0.f, 0.f, 0.f};
                    if constexpr (TEX) {
#pragma unroll
                        for (int q = 0; q < KSTEPS; ++q)
                            // formats 2, 2: both operands FP6 E2M3; unit scales
                            T[rb] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(Aop[rb][q], Bop[q], T[rb],
                                                                                      2, 2, 0, 127, 0, 127);
                    }
                    Q[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, s_abf[wave][rb][al]),
                                                                    __builtin_bit_cast(bf16x8, Bbf),
                                                                    f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
                }
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const float dr = pr[rb][r] - col.x, dg = pg[rb][r] - col.y, db = pb[rb][r] - col.z;
                        float u = TEX ? fmaf(T[rb][r], nB[rb][r], nR[rb][r]) : nR[rb][r];
                        u = fmaf(Q[rb][r], nA[rb][r], u);
                        u = fmaf(-dr, dr, u);
                        u = fmaf(-dg, dg, u);
                        u = fmaf(-db, db, u);
                        S[rb][r] += __builtin_amdgcn_exp2f(u);
                    }
            }
            // A lane sum above 2^64 moves that pixel's reference up by a whole
            // power of two (exact rescale).  Entering a chunk the sums are at
            // most 2^64, so an overflowed sum means a term beyond 2^122 (64
            // terms per lane and chunk): the pass stops, and the item is
            // computed again with the reference of each such pixel raised (see
            // the retry below).
            // (the largest of the lane's sums: a NaN is passed over here and
            // marks the item bad at its end)
            float smax = S[0][0];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int r = 0; r < 4; ++r) smax = fmaxf(smax, S[rb][r]);
            if (__ballot(!(smax <= 0x1p64f))) {
                // the 16 lanes of a pixel (one sample column each) move
                // together, by the largest exponent among them, so that the
                // pixel keeps one reference
                ++n_rescale;
                bool over = false;
                uint32_t ob = 0;  // pixels (bit 4 rb + r) of this lane group that overflowed
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const float s = S[rb][r];
                        int e = 0;
                        if (!(s <= 0x1p64f)) {
                            if (s <= 3.0e38f) e = (int)((__float_as_uint(s) >> 23) & 0xFFu) - 127;
                            else e = 255;  // overflowed (or not a number)
                        }
#pragma unroll
                        for (int off = 1; off < 16; off <<= 1) e = max(e, __shfl_xor(e, off));
                        if (e == 255) {
                            over = true;
                            ob |= 1u << (4 * rb + r);
                        } else if (e > 0) {
                            S[rb][r] = ldexpf(s, -e);
                            nR[rb][r] -= (float)e;
                        }
                    }
                if (__ballot(over)) {
                    s_ovp[wave][lane] = (uint8_t)ob;
                    if (lane == 0) s_ovf = 1;
                    ovf_wave = true;
                    active = false;
                    ++n_overflow;
                }
            }
        };
        // Overflow retry.  A pixel whose sum overflowed has a term at least
        // 2^122 times its reference, so raising the reference by kRaise = 170
        // (log2 units) keeps every term of that size below 2^48 and loses only
        // terms below 2^-122 of it; the waves that overflowed compute the item
        // again (the others keep their sums and only help stream the chunks),
        // up to kRetries times before the item goes to the exact kernel.  Every
        // pixel of such a wave starts again from its own first reference less
        // kRaise per overflow of its own, so its result does not depend on the
        // pixels it shares the wave with.
        for (int attempt = 0;; ++attempt) {
            for (int c = c0; c < c1; c += 2) {
                process(c, s_feat0, s_rec0, s_feat1, s_rec1);
                if (c + 1 < c1) process(c + 1, s_feat1, s_rec1, s_feat0, s_rec0);
            }
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();  // every wave is past the pass; both buffer pairs are free
            const int again = s_ovf;
            __syncthreads();  // every wave has read the flag
            if (!again) break;
            if (tid == 0) s_ovf = 0;
            if (attempt == kRetries) {
                if (ovf_wave) item_bad = true;
                break;
            }
            active = ovf_wave;
            if (ovf_wave) {
                const uint32_t ob = s_ovp[wave][lane];
                // raise counts, four bits per pixel (at most kRetries)
                uint32_t nr = s_nraise[wave][lane];
                int al = lane;
                __asm__ volatile("" : "+v"(al));
                const float4 *cr = a.coef + (int64_t)lab * coef_label_stride + (int64_t)tile * kTilePix +
                                   (((al >> 5) * 8 + ((al >> 4) & 1) * 4));
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int j = 4 * rb + r;
                        nr += ((ob >> j) & 1u) << (4 * j);
                        S[rb][r] = 0.0f;
                        nR[rb][r] = cr[16 * rb + r].z - kRaise * (float)((nr >> (4 * j)) & 15u);
                    }
                s_nraise[wave][lane] = nr;
            }
            ovf_wave = false;
            issue(c0, s_feat0, s_rec0);
        }
        if (!wave_valid) continue;

        // ---- end of item: sum the 16 lanes sharing each pixel (one sample
        // column each, one reference); lane jl < 8 of each 16-lane group keeps
        // pixel (rb, r) = (jl >> 2, jl & 3) for the write
        bool bad = item_bad;
        float Rw = 0.0f, Sw = 1.0f;
        if (!bad) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float Rm = -nR[rb][r];
                    float sp = S[rb][r];
#pragma unroll
                    for (int off = 1; off < 16; off <<= 1) sp += __shfl_xor(sp, off);
                    if (slot_ok(rb, r) && !(sp <= 0x1p126f && sp > 0.0f)) bad = true;
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
            const int ti = (2 * rb + (g >> 1)) * 8 + 4 * (g & 1) + r;
            if (slot_ok(rb, r)) {
                const int64_t row = LIST ? (int64_t)tile * kTilePix + ti
                                         : (int64_t)(y0 + 2 * rb + (g >> 1)) * a.W + x0 + 4 * (g & 1) + r;
                const double K = (double)cf[ti].w;
                const double lg = kLn2F * ((double)Rw + (double)__builtin_amdgcn_logf(Sw)) + K;
                a.loglik[row * a.L + lab] = (float)lg;
            }
        }
    }
    if (lane == 0 && (n_rescale | n_overflow)) {
        if (n_rescale) atomicAdd(a.fix_count + 1, n_rescale);
        if (n_overflow) atomicAdd(a.fix_count + 2, n_overflow);
    }
}

// Colour levels, transposed 32 x 32 form.  The products run as
// v_mfma_scale_f32_32x32x64_f8f6f4 (texture, FP6) and
// v_mfma_f32_32x32x16_bf16 (location on K 0..15, colour on K 0..7) with the
// samples as rows (A) and the pixels as columns (B): lane l owns the tile
// slot l mod 32 (one pixel, its coefficients and its sum) and accumulates 16
// of every 32 samples, the lane l xor 32 the other 16.  Against the 16 x 16
// form the location and colour products use the whole K (14 and 8 of 16
// slots instead of 14 and 8 of 32), a quarter fewer matrix-core cycles per
// pair, and the per-pixel state is one register each.  The pair arithmetic
// is the same; the per-pixel reference, rescale and overflow retry work as
// in the 16 x 16 form (the two lanes of a pixel move together).  The pixel
// operands come from the arrays k_prep builds for the 16 x 16 form.
template <int KSTEPS, bool TEX, bool LIST>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
void k_parzen_mfma32(ParzenFastArgs a) {
    constexpr int RB = kParzenRB;
    constexpr int KP = 128 * KSTEPS;
    constexpr int NQ = 2 * KSTEPS;                   // 64-feature K steps
    constexpr int FEAT_B = TEX ? kChunkS * KP : 16;  // feature bytes per chunk
    __shared__ __align__(16) uint8_t s_feat0[FEAT_B];
    __shared__ __align__(16) uint8_t s_feat1[FEAT_B];
    __shared__ __align__(16) float s_rec0[kRecChunkF];
    __shared__ __align__(16) float s_rec1[kRecChunkF];
    __shared__ int s_item, s_queue;
    __shared__ int s_ovf;  // any wave of the workgroup overflowed in the last pass

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wave_u = __builtin_amdgcn_readfirstlane(wave);
    // h: K half of the lane's operands; j: its sample row (A) and its pixel,
    // tile slot j (B and the result column)
    const int h = lane >> 5, j = lane & 31;
    const int64_t coef_label_stride = (int64_t)a.ngroups * 4 * kTilePix;
    // LDS byte offsets of the lane's sample operands in step 0 of a chunk
    // buffer (step st adds 32 rows; the swizzle of rows j and 32 st + j is the
    // same): FP6 group 2 q + h of row j, location plane h, the colour plane
    int foff[NQ][2];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) foff[q][hh] = j * KP + 16 * swz(2 * (2 * q + h) + hh, j);
    const int loff = h * (16 * kChunkS) + 16 * j;
    const int coff = 32 * kChunkS + 16 * j;
    uint32_t n_rescale = 0;   // wave-chunks whose reference moved (wave-uniform)
    uint32_t n_overflow = 0;  // passes stopped by an overflow

    int queue = blockIdx.x % kParzenQueues, emptied = 0;
    if (tid == 0) s_ovf = 0;
    for (;;) {
        __syncthreads();  // the previous item's LDS reads are done
        if (tid == 0) {
            int it = -1;
            while (emptied < kParzenQueues) {
                const int nq = queue < a.ngroups ? (a.ngroups - 1 - queue) / kParzenQueues + 1 : 0;
                const int t = (int)atomicAdd(a.work_counter + queue * kQueueStride, 1u);
                if (t < nq * a.L) {
                    it = t;
                    break;
                }
                queue = queue + 1 == kParzenQueues ? 0 : queue + 1;
                ++emptied;
            }
            s_item = it;
            s_queue = queue;
        }
        __syncthreads();
        const int item = s_item;
        if (item < 0) break;
        // item -> (group, label): as in the 16 x 16 form
        const int qg = s_queue < a.ngroups ? (a.ngroups - 1 - s_queue) / kParzenQueues + 1 : 0;
        const int tg = qg < kTailGroups ? qg : kTailGroups;
        const int hg = qg - tg;
        const int head_items = hg * a.L;
        int gi, lrank;
        if (item < head_items) {
            const int nblk = (a.L + a.lblock - 1) / a.lblock;
            int b = item / (hg * a.lblock);
            if (b > nblk - 1) b = nblk - 1;
            const int bsz = b < nblk - 1 ? a.lblock : a.L - a.lblock * (nblk - 1);
            const int rr = item - hg * a.lblock * b;
            gi = rr / bsz;
            lrank = a.lblock * b + (rr - gi * bsz);
        } else {
            const int jj = item - head_items;
            lrank = jj / tg;
            gi = qg - tg + (jj - lrank * tg);
        }
        const int grp = s_queue + kParzenQueues * gi;
        const int lab = a.meta[a.L + 1 + lrank];
        const int c0 = a.meta[lab], c1 = a.meta[lab + 1];
        const int last_steps = a.meta[2 * a.L + 1 + lab];  // 16-sample steps of the last chunk
        const int tile = grp * 4 + wave;
        const bool tile_ok = tile < a.ntiles;
        const int ty_t = tile_ok ? tile / a.tiles_x : 0;
        const int x0 = (tile_ok ? tile - ty_t * a.tiles_x : 0) * 8, y0 = ty_t * 2 * RB;
        // this lane's pixel, slot j (fast_slot_row): on the grid (x0 + j mod 8,
        // y0 + j / 8), on a list entry 32 tile + j
        bool pv;
        if constexpr (LIST) {
            pv = (int64_t)tile * kTilePix + j < a.nlist;
        } else {
            pv = tile_ok && x0 + (j & 7) < a.W && y0 + (j >> 3) < a.H;
        }

        auto issue = [&](int c, uint8_t *sf, float *sr) {
            uint32_t off = (uint32_t)tid * 16u;
            __asm__ volatile("" : "+v"(off));
            if constexpr (TEX) {
                const uint8_t *fbase = a.feat + (int64_t)c * FEAT_B;
#pragma unroll
                for (int u = 0; u < FEAT_B / 4096; ++u)
                    __builtin_amdgcn_global_load_lds(fbase + u * 4096 + off,
                                                     (lds_void *)(sf + u * 4096 + wave_u * 1024), 16, 0, 0);
            }
            if (wave_u < 3) {
                const uint8_t *rbase = reinterpret_cast<const uint8_t *>(a.rec) + (int64_t)c * (kRecChunkF * 4);
                __builtin_amdgcn_global_load_lds(rbase + off, (lds_void *)(sr + wave_u * 256), 16, 0, 0);
            }
        };
        issue(c0, s_feat0, s_rec0);

        // coefficients of this label (log2 units): nA, nB, -reference, K
        const float4 *cf = a.coef + (int64_t)lab * coef_label_stride + (int64_t)tile * kTilePix;
        const float4 q4 = cf[j];
        const float nA = q4.x, nB = q4.y;
        float nR = q4.z;
        bool active = __ballot(pv) != 0ull;  // wave-uniform
        const bool wave_valid = active;
        // padding samples sit at Q ~ 2^100; a bandwidth wide enough to reach
        // them (or a non-finite one) goes to the exact kernel
        bool item_bad = __ballot(pv && !(q4.x < -1e-18f)) != 0ull;
        if (item_bad) active = false;

        // pixel operands (B): FP6 group 2 q + h of slot j, the BF16 location
        // pieces of K 8h .. 8h + 7 and (h = 0) the colour pieces, from the
        // arrays k_prep lays out for the 16 x 16 form (slot 16 rb + jl is row
        // jl of block rb there; group 4 qo + g is step qo, lane group g)
        const int rb = j >> 4, jl = j & 15;
        i32x8 Bop[NQ];
        if constexpr (TEX) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int g2 = 2 * q + h, qo = g2 >> 2, g = g2 & 3;
                const uint4 *src = reinterpret_cast<const uint4 *>(
                    a.aop + ((((int64_t)tile * RB + rb) * KSTEPS + qo) * 64 + g * 16 + jl) * 8);
                const uint4 lo4 = src[0];
                const uint2 hi2 = *reinterpret_cast<const uint2 *>(src + 1);
                Bop[q] = i32x8{(int)lo4.x, (int)lo4.y, (int)lo4.z, (int)lo4.w, (int)hi2.x, (int)hi2.y, 0, 0};
            }
        }
        const uint8_t *bb = a.abf + (((int64_t)tile * RB + rb) * 64 + jl) * 16;
        const s16x8 Bloc = *reinterpret_cast<const s16x8 *>(bb + h * 16 * 16);
        s16x8 Bcol = s16x8{0, 0, 0, 0, 0, 0, 0, 0};
        if (h == 0) Bcol = *reinterpret_cast<const s16x8 *>(bb + 2 * 16 * 16);

        float S = 0.0f;
        uint32_t nraise = 0;  // overflows of this pixel so far (reference raised by kRaise each)
        bool ovf_wave = false, ovf_pix = false;

        auto process = [&](int c, const uint8_t *F, const float *Rr, uint8_t *Fn, float *Rn) {
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();  // chunk c resident in (F, Rr); the other pair is free
            if (c + 1 < c1) issue(c + 1, Fn, Rn);
            if (!active) return;
            const int nst = c + 1 == c1 ? (last_steps + 1) / 2 : kChunkS / 32;
#pragma unroll
            for (int st = 0; st < kChunkS / 32; ++st) {
                if (st >= nst) break;
                const uint8_t *Fs = F + st * 32 * KP;
                const uint8_t *Rs = reinterpret_cast<const uint8_t *>(Rr) + st * 32 * 16;
                const s16x8 Aloc = *reinterpret_cast<const s16x8 *>(Rs + loff);
                const s16x8 Acol = *reinterpret_cast<const s16x8 *>(Rs + coff);
                f32x16 Z;
#pragma unroll
                for (int v = 0; v < 16; ++v) Z[v] = 0.0f;
                const f32x16 Q = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, Aloc),
                                                                         __builtin_bit_cast(bf16x8, Bloc), Z, 0, 0, 0);
                const f32x16 C = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, Acol),
                                                                         __builtin_bit_cast(bf16x8, Bcol), Z, 0, 0, 0);
                // location and colour first: their share of the exponent
                // overlaps this wave's chain of texture products
                f32x16 U;
#pragma unroll
                for (int v = 0; v < 16; ++v) U[v] = fmaf(C[v], a.kcol, fmaf(Q[v], nA, nR));
                f32x16 T;
#pragma unroll
                for (int v = 0; v < 16; ++v) T[v] = 0.0f;
                if constexpr (TEX) {
#pragma unroll
                    for (int q = 0; q < NQ; ++q) {
                        const uint4 lo4 = *reinterpret_cast<const uint4 *>(Fs + foff[q][0]);
                        const uint2 hi2 = *reinterpret_cast<const uint2 *>(Fs + foff[q][1]);
                        const i32x8 Aop =
                            i32x8{(int)lo4.x, (int)lo4.y, (int)lo4.z, (int)lo4.w, (int)hi2.x, (int)hi2.y, 0, 0};
                        // formats 2, 2: both operands FP6 E2M3; unit scales
                        T = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(Aop, Bop[q], T, 2, 2, 0, 127, 0, 127);
                    }
                }
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const float u = TEX ? fmaf(T[v], nB, U[v]) : U[v];
                    S += __builtin_amdgcn_exp2f(u);
                }
            }
            // A lane sum above 2^64 moves the pixel's reference up by a whole
            // power of two (the larger need of its two lanes; exact rescale).
            // An overflowed sum stops the wave's pass (retry below).
            if (__ballot(!(S <= 0x1p64f))) {
                ++n_rescale;
                int e = 0;
                if (!(S <= 0x1p64f)) {
                    if (S <= 3.0e38f) e = (int)((__float_as_uint(S) >> 23) & 0xFFu) - 127;
                    else e = 255;  // overflowed (or not a number)
                }
                e = max(e, __shfl_xor(e, 32));
                if (e == 255) {
                    ovf_pix = true;
                } else if (e > 0) {
                    S = ldexpf(S, -e);
                    nR -= (float)e;
                }
                if (__ballot(e == 255)) {
                    if (lane == 0) s_ovf = 1;
                    ovf_wave = true;
                    active = false;
                    ++n_overflow;
                }
            }
        };
        // Overflow retry, as in the 16 x 16 form: the waves that overflowed
        // compute the item again, each pixel from its own first reference less
        // kRaise per overflow of its own, up to kRetries times.
        for (int attempt = 0;; ++attempt) {
            for (int c = c0; c < c1; c += 2) {
                process(c, s_feat0, s_rec0, s_feat1, s_rec1);
                if (c + 1 < c1) process(c + 1, s_feat1, s_rec1, s_feat0, s_rec0);
            }
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();  // every wave is past the pass; both buffer pairs are free
            const int again = s_ovf;
            __syncthreads();  // every wave has read the flag
            if (!again) break;
            if (tid == 0) s_ovf = 0;
            if (attempt == kRetries) {
                if (ovf_wave) item_bad = true;
                break;
            }
            active = ovf_wave;
            if (ovf_wave) {
                nraise += ovf_pix ? 1u : 0u;
                S = 0.0f;
                int jo = j;
                __asm__ volatile("" : "+v"(jo));
                nR = cf[jo].z - kRaise * (float)nraise;
            }
            ovf_wave = false;
            ovf_pix = false;
            issue(c0, s_feat0, s_rec0);
        }
        if (!wave_valid) continue;

        // end of item: the two lanes of a pixel add their sums
        const float sp = S + __shfl_xor(S, 32);
        bool bad = item_bad || (pv && !(sp <= 0x1p126f && sp > 0.0f));
        if (__ballot(bad)) {
            if (lane == 0) {
                const unsigned int slot = atomicAdd(a.fix_count, 1u);
                if (slot < (unsigned int)a.fix_cap) a.fixlist[slot] = make_int2(lab, tile);
            }
            continue;
        }
        if (h == 0 && pv) {
            const int64_t row = LIST ? (int64_t)tile * kTilePix + j
                                     : (int64_t)(y0 + (j >> 3)) * a.W + x0 + (j & 7);
            const double K = (double)q4.w;
            const double lg = kLn2F * ((double)(-nR) + (double)__builtin_amdgcn_logf(sp)) + K;
            a.loglik[row * a.L + lab] = (float)lg;
        }
    }
    if (lane == 0 && (n_rescale | n_overflow)) {
        if (n_rescale) atomicAdd(a.fix_count + 1, n_rescale);
        if (n_overflow) atomicAdd(a.fix_count + 2, n_overflow);
    }
}

template <int KSTEPS, bool TEX, bool LIST>
static hipError_t launch_mfma32_k(const LaunchCtx &lc, const ParzenFastArgs &a) {
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_parzen_mfma32<KSTEPS, TEX, LIST>, 256, 0);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    int64_t blocks = (int64_t)lc.num_cu * per_cu;
    const int64_t items = (int64_t)a.ngroups * a.L;
    if (blocks > items) blocks = items;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL((k_parzen_mfma32<KSTEPS, TEX, LIST>), dim3((unsigned)blocks), dim3(256), 0, lc.stream, a);
    return hipGetLastError();
}

template <bool LIST>
static hipError_t launch_mfma32_list(const LaunchCtx &lc, const ParzenFastArgs &a) {
    if (!a.texture) return launch_mfma32_k<1, false, LIST>(lc, a);
    switch (a.ksteps) {
        case 1: return launch_mfma32_k<1, true, LIST>(lc, a);
        case 2: return launch_mfma32_k<2, true, LIST>(lc, a);
        default: return launch_mfma32_k<3, true, LIST>(lc, a);
    }
}

template <int KSTEPS, bool TEX, bool LIST>
static hipError_t launch_mfma_k(const LaunchCtx &lc, const ParzenFastArgs &a) {
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_parzen_mfma<KSTEPS, TEX, LIST>, 256, 0);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    int64_t blocks = (int64_t)lc.num_cu * per_cu;
    const int64_t items = (int64_t)a.ngroups * a.L;
    if (blocks > items) blocks = items;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL((k_parzen_mfma<KSTEPS, TEX, LIST>), dim3((unsigned)blocks), dim3(256), 0, lc.stream, a);
    return hipGetLastError();
}

template <bool LIST>
static hipError_t launch_mfma_list(const LaunchCtx &lc, const ParzenFastArgs &a) {
    if (!a.texture) return launch_mfma_k<1, false, LIST>(lc, a);
    switch (a.ksteps) {
        case 1: return launch_mfma_k<1, true, LIST>(lc, a);
        case 2: return launch_mfma_k<2, true, LIST>(lc, a);
        default: return launch_mfma_k<3, true, LIST>(lc, a);
    }
}

hipError_t launch_parzen_mfma(const LaunchCtx &lc, const ParzenFastArgs &a) {
    if (a.levels > 0) return a.list ? launch_mfma32_list<true>(lc, a) : launch_mfma32_list<false>(lc, a);
    return a.list ? launch_mfma_list<true>(lc, a) : launch_mfma_list<false>(lc, a);
}

}  // namespace cs
