// Learned surrogate of the data term on gfx950: a two-hidden-layer perceptron
// (GELU, 128 units) from a pixel's colour, normalised position and analysed
// vector (Sec. 2 a = O s of Sec. 3.1 patches) to its per-label
// log-likelihoods (the Sec. 3.1/3.2 data term), trained by Adam on exact
// targets.  Matrix products run on BF16 MFMA (v_mfma_f32_16x16x16_bf16 for
// training, 16x16x32 for inference) with FP32 accumulation; biases, GELU, the
// loss and Adam are FP32.
//
// Layout trick: every layer computes the TRANSPOSED product, units x rows.
// With A = weights (rows = units) and B = activations^T (columns = 16 batch
// rows), lane (g, j) of the result holds units 4g..4g+3 of batch row j, which
// is exactly the B-operand fragment (k = 4g..4g+3, column j) of the next
// layer.  So a 16-row tile flows through all layers in registers, and the
// backward pass reuses the same layout with the transposed weights as A.
//
// Weight gradients dW = delta^T act are reductions over the batch; the
// forward/backward kernel stores the BF16 activations and deltas feature-major
// ([unit][row]) so that the gradient kernel reads 4 consecutive rows per lane
// for both MFMA operands.  Partial sums over row chunks are added in a fixed
// order by the Adam kernel (deterministic).
#pragma clang fp contract(off)

#include "cs_internal.h"
#include "cs_device.h"

namespace cs {

typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr float kClipNats = 20.0f;
constexpr float kAdamB1 = 0.9f, kAdamB2 = 0.999f, kAdamEps = 1e-8f;

// erf by the rational approximation 7.1.26 of Abramowitz and Stegun
// (Handbook of Mathematical Functions), |error| <= 1.5e-7: a polynomial in
// t = 1 / (1 + p |x|) times exp(-x^2), branch-free.  GELU(z) = z Phi(z) with
// Phi(z) = (1 + erf(z / sqrt 2)) / 2.
__device__ __forceinline__ float erf_as(float x) {
    const float ax = fabsf(x);
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, ax, 1.0f));
    float poly = fmaf(1.061405429f, t, -1.453152027f);
    poly = fmaf(poly, t, 1.421413741f);
    poly = fmaf(poly, t, -0.284496736f);
    poly = fmaf(poly, t, 0.254829592f);
    poly *= t;
    const float e = __builtin_amdgcn_exp2f(-ax * ax * 1.4426950408889634f);
    const float r = fmaf(-poly, e, 1.0f);
    return copysignf(r, x);
}
__device__ __forceinline__ float gelu(float z) { return z * fmaf(0.5f, erf_as(z * 0.70710678118654752f), 0.5f); }
// FP32 -> BF16 bit pattern, round to nearest even (v_cvt_pk_bf16_f32).
__device__ __forceinline__ short to_bf16(float v) { return __builtin_bit_cast(short, (__bf16)v); }
__device__ __forceinline__ float gelu_grad(float z) {
    return 0.5f * (1.0f + erf_as(z * 0.70710678118654752f)) +
           z * __builtin_amdgcn_exp2f(-0.5f * 1.4426950408889634f * z * z) * 0.39894228040143268f;
}

__device__ __forceinline__ s16x4 ld4(const short *p) { return *reinterpret_cast<const s16x4 *>(p); }
__device__ __forceinline__ f32x4 mfma(s16x4 a, s16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// One 16-row tile through the three layers.  xb[ks]: the tile's inputs as
// B fragments (features 16ks + 4g .. +3 of row j).  W1 row stride ld1, W2 and
// W3 row stride ld2 (elements); the pointers may point to LDS or global.
template <bool KEEP>
__device__ __forceinline__ void mlp_tile_forward(const s16x4 (&xb)[kMlpMaxIn / 16], int nks, const short *W1,
                                                 int ld1, const short *W2, const short *W3, int ld2,
                                                 const float *b1, const float *b2, const float *b3, int out,
                                                 int g, int j, float (&z1)[8][4], float (&z2)[8][4],
                                                 s16x4 (&h2b)[8], f32x4 &y) {
    s16x4 h1b[8];
#pragma unroll
    for (int hb = 0; hb < 8; ++hb) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        const short *wr = W1 + (16 * hb + j) * ld1 + 4 * g;
        // weight fragments loaded unconditionally (clamped step), used below nks
        s16x4 wf[kMlpMaxIn / 16];
#pragma unroll
        for (int ks = 0; ks < kMlpMaxIn / 16; ++ks) wf[ks] = ld4(wr + 16 * (ks < nks ? ks : nks - 1));
#pragma unroll
        for (int ks = 0; ks < kMlpMaxIn / 16; ++ks)
            if (ks < nks) acc = mfma(wf[ks], xb[ks], acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float z = acc[r] + b1[16 * hb + 4 * g + r];
            if (KEEP) z1[hb][r] = z;
            h1b[hb][r] = to_bf16(gelu(z));
        }
    }
#pragma unroll
    for (int hb = 0; hb < 8; ++hb) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        const short *wr = W2 + (16 * hb + j) * ld2 + 4 * g;
#pragma unroll
        for (int kb = 0; kb < 8; ++kb) acc = mfma(ld4(wr + 16 * kb), h1b[kb], acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float z = acc[r] + b2[16 * hb + 4 * g + r];
            if (KEEP) z2[hb][r] = z;
            h2b[hb][r] = to_bf16(gelu(z));
        }
    }
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    const short *wr = W3 + j * ld2 + 4 * g;
#pragma unroll
    for (int kb = 0; kb < 8; ++kb) acc = mfma(ld4(wr + 16 * kb), h2b[kb], acc);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int o = 4 * g + r;
        y[r] = acc[r] + (o < out ? b3[o] : 0.0f);
    }
}

// ---- forward + backward of one batch (training and the gradient call) ----
// One workgroup per 16-row tile; wave w owns the hidden blocks 2w and 2w + 1
// (units 32w .. 32w + 31) of both hidden layers.  A layer's MFMA result
// fragments are the next layer's B operand for the same lane, so they pass
// between the waves through LDS as they are (lane l's fragment of block b at
// [b][l]).  The output layer and dY (16 outputs, one block) are computed by
// every wave alike; wave 0 writes them.
__global__ __launch_bounds__(256) void k_mlp_fwdbwd(MlpTrainArgs a) {
    __shared__ s16x4 sh_h1[8][64], sh_h2[8][64], sh_dz2[8][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, j = lane & 15;
    const int wt = blockIdx.x;  // tile
    const int b0 = wt * 16;
    if (b0 >= a.B) return;  // uniform over the workgroup
    const int rb = b0 + j;
    int64_t row = a.idx ? (int64_t)a.idx[rb] : (int64_t)rb;
    row = row < 0 ? 0 : (row >= a.n_rows ? a.n_rows - 1 : row);  // memory-safe on bad input
    const int nks = a.in_pad / 16;
    // inputs loaded unconditionally (clamped feature index: the loads are in
    // flight together), zero past in
    float xv[kMlpMaxIn / 16][4];
#pragma unroll
    for (int ks = 0; ks < kMlpMaxIn / 16; ++ks)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int f = 16 * ks + 4 * g + q;
            xv[ks][q] = a.x[row * a.in + (f < a.in ? f : a.in - 1)];
        }
    s16x4 xb[kMlpMaxIn / 16];
#pragma unroll
    for (int ks = 0; ks < kMlpMaxIn / 16; ++ks)
#pragma unroll
        for (int q = 0; q < 4; ++q) xb[ks][q] = to_bf16(16 * ks + 4 * g + q < a.in ? xv[ks][q] : 0.0f);
    // layer 1, own blocks
    float z1[2][4], z2[2][4];
    s16x4 h1b[2], h2b[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int hb = 2 * wave + h;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        const short *wr = a.W1b + (16 * hb + j) * a.in_pad + 4 * g;
        s16x4 wf[kMlpMaxIn / 16];
#pragma unroll
        for (int ks = 0; ks < kMlpMaxIn / 16; ++ks) wf[ks] = ld4(wr + 16 * (ks < nks ? ks : nks - 1));
#pragma unroll
        for (int ks = 0; ks < kMlpMaxIn / 16; ++ks)
            if (ks < nks) acc = mfma(wf[ks], xb[ks], acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            z1[h][r] = acc[r] + a.b1[16 * hb + 4 * g + r];
            h1b[h][r] = to_bf16(gelu(z1[h][r]));
        }
        sh_h1[hb][lane] = h1b[h];
    }
    __syncthreads();
    // layer 2, own blocks, from every block of layer 1
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int hb = 2 * wave + h;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        const short *wr = a.W2b + (16 * hb + j) * kMlpHid + 4 * g;
        s16x4 wf[8];
#pragma unroll
        for (int kb = 0; kb < 8; ++kb) wf[kb] = ld4(wr + 16 * kb);
#pragma unroll
        for (int kb = 0; kb < 8; ++kb) acc = mfma(wf[kb], sh_h1[kb][lane], acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            z2[h][r] = acc[r] + a.b2[16 * hb + 4 * g + r];
            h2b[h][r] = to_bf16(gelu(z2[h][r]));
        }
        sh_h2[hb][lane] = h2b[h];
    }
    __syncthreads();
    // output layer (every wave): y^T = W3 h2^T
    f32x4 y = {0.f, 0.f, 0.f, 0.f};
    {
        const short *wr = a.W3b + j * kMlpHid + 4 * g;
        s16x4 wf[8];
#pragma unroll
        for (int kb = 0; kb < 8; ++kb) wf[kb] = ld4(wr + 16 * kb);
#pragma unroll
        for (int kb = 0; kb < 8; ++kb) y = mfma(wf[kb], sh_h2[kb][lane], y);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int o = 4 * g + r;
            y[r] += o < a.out ? a.b3[o] : 0.0f;
        }
    }
    // clipped targets t = max(l, max_i l_i - 20); the row max over the four
    // lanes that share row j (lanes j, j+16, j+32, j+48)
    float ell[4], mx = -INFINITY;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int o = 4 * g + r;
        ell[r] = o < a.out ? a.ell[row * a.out + o] : -INFINITY;
        mx = fmaxf(mx, ell[r]);
    }
    mx = fmaxf(mx, __shfl_xor(mx, 16));
    mx = fmaxf(mx, __shfl_xor(mx, 32));
    const float scale = 2.0f / ((float)a.B * (float)a.out);
    float sq = 0.0f;
    float dy[4];
    s16x4 dyb;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int o = 4 * g + r;
        const float t = fmaxf(ell[r], mx - kClipNats);
        const float d = o < a.out ? y[r] - t : 0.0f;
        sq += d * d;
        dy[r] = scale * d;
        dyb[r] = to_bf16(dy[r]);
    }
    // dH2^T = W3^T dY^T (K = 16 outputs), dZ2 = dH2 * GELU'(z2), own blocks
    float dz2[2][4];
    s16x4 dz2b[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int hb = 2 * wave + h;
        const f32x4 acc = mfma(ld4(a.W3Tb + (16 * hb + j) * kMlpOutPad + 4 * g), dyb, f32x4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            dz2[h][r] = acc[r] * gelu_grad(z2[h][r]);
            dz2b[h][r] = to_bf16(dz2[h][r]);
        }
        sh_dz2[hb][lane] = dz2b[h];
    }
    __syncthreads();
    // dH1^T = W2^T dZ2^T, dZ1 = dH1 * GELU'(z1), own blocks
    float dz1[2][4];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int hb = 2 * wave + h;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        const short *wr = a.W2Tb + (16 * hb + j) * kMlpHid + 4 * g;
        s16x4 wf[8];
#pragma unroll
        for (int kb = 0; kb < 8; ++kb) wf[kb] = ld4(wr + 16 * kb);
#pragma unroll
        for (int kb = 0; kb < 8; ++kb) acc = mfma(wf[kb], sh_dz2[kb][lane], acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) dz1[h][r] = acc[r] * gelu_grad(z1[h][r]);
    }
    // feature-major BF16 stores for the weight-gradient products (the input
    // blocks split over the waves)
    const int B = a.B;
#pragma unroll
    for (int ks = 0; ks < kMlpMaxIn / 16; ++ks)
        if (ks < nks && (ks & 3) == wave)
#pragma unroll
            for (int q = 0; q < 4; ++q) a.Xt[(int64_t)(16 * ks + 4 * g + q) * B + rb] = xb[ks][q];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t u = (int64_t)(16 * (2 * wave + h) + 4 * g + r) * B + rb;
            a.H1t[u] = h1b[h][r];
            a.H2t[u] = h2b[h][r];
            a.DZ2t[u] = dz2b[h][r];
            a.DZ1t[u] = to_bf16(dz1[h][r]);
        }
    // bias gradients and squared error of the tile: sums over its 16 rows (FP32)
    float *bg = a.bgrad + (int64_t)wt * kMlpBiasStride;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float s1 = dz1[h][r], s2 = dz2[h][r];
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) {
                s1 += __shfl_xor(s1, off);
                s2 += __shfl_xor(s2, off);
            }
            const int u = 16 * (2 * wave + h) + 4 * g + r;
            if (j == 0) {
                bg[u] = s1;
                bg[kMlpHid + u] = s2;
            }
        }
    if (wave == 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) a.DYt[(int64_t)(4 * g + r) * B + rb] = dyb[r];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float s3 = dy[r];
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) s3 += __shfl_xor(s3, off);
            if (j == 0) bg[2 * kMlpHid + 4 * g + r] = s3;
        }
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) sq += __shfl_xor(sq, off);
        if (lane == 0) a.lossp[wt] = sq;
    }
}

// ---- weight gradients: one wave per (16x16 output tile, row chunk) ----
__global__ __launch_bounds__(256) void k_mlp_wgrad(MlpWgradArgs a) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, j = lane & 15;
    const int item = blockIdx.x * 4 + wave;
    const int nks = a.in_pad / 16;
    const int t1 = 8 * nks, t2 = t1 + 64, ntile = t2 + 8;
    if (item >= ntile * a.kc) return;
    const int tile = item % ntile, kc = item / ntile;
    const short *Am, *Bm;
    int hb, ib, ncols, nrows;
    int64_t off;
    if (tile < t1) {          // dW1 = dZ1^T X
        hb = tile / nks; ib = tile % nks; Am = a.DZ1t; Bm = a.Xt; off = a.off_W1; ncols = a.in; nrows = kMlpHid;
    } else if (tile < t2) {   // dW2 = dZ2^T H1
        hb = (tile - t1) / 8; ib = (tile - t1) % 8; Am = a.DZ2t; Bm = a.H1t; off = a.off_W2; ncols = kMlpHid;
        nrows = kMlpHid;
    } else {                  // dW3 = dY^T H2
        hb = 0; ib = tile - t2; Am = a.DYt; Bm = a.H2t; off = a.off_W3; ncols = kMlpHid; nrows = a.out;
    }
    const int B = a.B, chunk = B / a.kc, k0 = kc * chunk;
    const short *ar = Am + (int64_t)(16 * hb + j) * B + 4 * g;
    const short *br = Bm + (int64_t)(16 * ib + j) * B + 4 * g;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k = k0; k < k0 + chunk; k += 16) acc = mfma(ld4(ar + k), ld4(br + k), acc);
    float *gp = a.gpart + (int64_t)kc * a.P + off;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int rr = 16 * hb + 4 * g + r, cc = 16 * ib + j;
        if (rr < nrows && cc < ncols) gp[(int64_t)rr * ncols + cc] = acc[r];
    }
}

// ---- Adam (or gradient output) over the flat parameter vector ----
// Adam update of parameter p with gradient g, and its BF16 working copies.
__device__ void adam_update(const MlpAdamArgs &a, int64_t p, float gsum) {
    if (a.grad_out) {
        a.grad_out[p] = gsum;
        return;
    }
    const float m = kAdamB1 * a.m[p] + (1.0f - kAdamB1) * gsum;
    const float v = kAdamB2 * a.v[p] + (1.0f - kAdamB2) * gsum * gsum;
    a.m[p] = m;
    a.v[p] = v;
    const float mhat = m / a.bc1, vhat = v / a.bc2;
    const float w = a.params[p] - a.lr * mhat / (sqrtf(vhat) + kAdamEps);
    a.params[p] = w;
    const short wb = to_bf16(w);
    if (p < a.off_b1) {
        const int h = (int)(p / a.in), i = (int)(p % a.in);
        a.W1b[h * a.in_pad + i] = wb;
    } else if (p >= a.off_W2 && p < a.off_b2) {
        const int h = (int)((p - a.off_W2) / kMlpHid), k = (int)((p - a.off_W2) % kMlpHid);
        a.W2b[h * kMlpHid + k] = wb;
        a.W2Tb[k * kMlpHid + h] = wb;
    } else if (p >= a.off_W3 && p < a.off_b3) {
        const int o = (int)((p - a.off_W3) / kMlpHid), h = (int)((p - a.off_W3) % kMlpHid);
        a.W3b[o * kMlpHid + h] = wb;
        a.W3Tb[h * kMlpOutPad + o] = wb;
    }
}

// Sum over the lanes of a wave in a fixed order (butterfly), every lane gets it.
__device__ float wave_sum_f32(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// The first `wblocks` workgroups update the weights: thread p adds the kc
// row-chunk partials of its gradient (coalesced over p).  The others take one
// wave per bias unit (and one for the loss): each lane adds every 64th
// per-tile partial, in a fixed order, then the wave adds its lanes.
__global__ __launch_bounds__(256) void k_mlp_adam(MlpAdamArgs a, int wblocks) {
    if ((int)blockIdx.x < wblocks) {
        const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
        if (p >= a.P) return;
        const bool bias = (p >= a.off_b1 && p < a.off_W2) || (p >= a.off_b2 && p < a.off_W3) || p >= a.off_b3;
        if (bias) return;
        float gsum = 0.0f;
        for (int c = 0; c < a.kc; ++c) gsum += a.gpart[(int64_t)c * a.P + p];
        adam_update(a, p, gsum);
        return;
    }
    const int lane = threadIdx.x & 63;
    const int u = ((int)blockIdx.x - wblocks) * 4 + (threadIdx.x >> 6);  // bias unit, or the loss
    const int nbias = 2 * kMlpHid + a.out;
    if (u > nbias) return;
    if (u == nbias) {
        if (!a.loss_out) return;
        float s = 0.0f;
        for (int t = lane; t < a.ntiles; t += 64) s += a.lossp[t];
        s = wave_sum_f32(s);
        if (lane == 0) *a.loss_out = s / ((float)a.B * (float)a.out);
        return;
    }
    float s = 0.0f;
    for (int t = lane; t < a.ntiles; t += 64) s += a.bgrad[(int64_t)t * kMlpBiasStride + u];
    s = wave_sum_f32(s);
    if (lane != 0) return;
    const int64_t p = u < kMlpHid ? a.off_b1 + u : u < 2 * kMlpHid ? a.off_b2 + (u - kMlpHid) : a.off_b3 + (u - 2 * kMlpHid);
    adam_update(a, p, s);
}

// ---- exact fallback of the surrogate ----
// Pixels whose two largest surrogate outputs differ by less than `margin`
// nats are listed (list[*count ...]; *count is zero before): each thread
// tests kUncPer pixels, each wave compacts its flags by ballot, and one atomic
// per workgroup (not per wave: returning atomics on one address serialise
// across the chip) reserves the workgroup's slots.  The order of the list
// depends on the schedule; each listed pixel is recomputed on its own, so the
// results do not.
constexpr int kUncPer = 16;
__global__ __launch_bounds__(256) void k_mlp_uncertain(const float *y, int64_t n, int L, float margin,
                                                       int32_t *list, unsigned int *count) {
    __shared__ unsigned int s_wcnt[4], s_base;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t p0 = (int64_t)blockIdx.x * 256 * kUncPer + threadIdx.x;
    uint64_t ball[kUncPer];
    unsigned int wc = 0;
#pragma unroll
    for (int u = 0; u < kUncPer; ++u) {
        const int64_t i = p0 + (int64_t)u * 256;
        bool flag = false;
        if (i < n) {
            const float *r = y + i * L;
            float t1 = r[0], t2 = -INFINITY;
            for (int l = 1; l < L; ++l) {
                const float v = r[l];
                if (v > t1) {
                    t2 = t1;
                    t1 = v;
                } else if (v > t2) {
                    t2 = v;
                }
            }
            flag = L > 1 && !(t1 - t2 >= margin);  // NaN outputs are listed too
        }
        ball[u] = __ballot(flag);
        wc += (unsigned int)__popcll(ball[u]);
    }
    if (lane == 0) s_wcnt[wave] = wc;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned int tot = s_wcnt[0] + s_wcnt[1] + s_wcnt[2] + s_wcnt[3];
        s_base = tot ? atomicAdd(count, tot) : 0u;
    }
    __syncthreads();
    unsigned int off = s_base;
    for (int w = 0; w < wave; ++w) off += s_wcnt[w];
    const uint64_t lt = (1ull << lane) - 1ull;
#pragma unroll
    for (int u = 0; u < kUncPer; ++u) {
        if ((ball[u] >> lane) & 1ull) list[off + __popcll(ball[u] & lt)] = (int32_t)(p0 + (int64_t)u * 256);
        off += (unsigned int)__popcll(ball[u]);
    }
}

// out[list[i]][l] = ex[i][l] for the m listed rows of L values.
__global__ __launch_bounds__(256) void k_mlp_scatter_rows(const float *ex, const int32_t *list, int64_t m, int L,
                                                          float *out) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= m * L) return;
    const int64_t i = t / L;
    const int l = (int)(t - i * L);
    out[(int64_t)list[i] * L + l] = ex[t];
}

hipError_t launch_mlp_uncertain(const LaunchCtx &lc, const float *y, int64_t n, int L, float margin, int32_t *list,
                                unsigned int *count) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_uncertain, dim3((unsigned)((n + 256 * kUncPer - 1) / (256 * kUncPer))), dim3(256), 0,
                       lc.stream, y, n, L, margin, list, count);
    return hipGetLastError();
}

hipError_t launch_mlp_scatter_rows(const LaunchCtx &lc, const float *ex, const int32_t *list, int64_t m, int L,
                                   float *out) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_scatter_rows, dim3((unsigned)((m * L + 255) / 256)), dim3(256), 0, lc.stream, ex, list,
                       m, L, out);
    return hipGetLastError();
}

// BF16 working copies of the master FP32 parameters (padding stays zero).
__global__ __launch_bounds__(256) void k_mlp_convert(MlpAdamArgs a) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= a.P) return;
    const short wb = to_bf16(a.params[p]);
    if (p < a.off_b1) {
        const int h = (int)(p / a.in), i = (int)(p % a.in);
        a.W1b[h * a.in_pad + i] = wb;
    } else if (p >= a.off_W2 && p < a.off_b2) {
        const int h = (int)((p - a.off_W2) / kMlpHid), k = (int)((p - a.off_W2) % kMlpHid);
        a.W2b[h * kMlpHid + k] = wb;
        a.W2Tb[k * kMlpHid + h] = wb;
    } else if (p >= a.off_W3 && p < a.off_b3) {
        const int o = (int)((p - a.off_W3) / kMlpHid), h = (int)((p - a.off_W3) % kMlpHid);
        a.W3b[o * kMlpHid + h] = wb;
        a.W3Tb[h * kMlpOutPad + o] = wb;
    }
}

// ---- inference: persistent workgroups, BF16 weights staged once in LDS ----
// Uses v_mfma_f32_16x16x32_bf16 (K = 32 per instruction).  A layer's result
// holds units 4g..4g+3 of each 16-unit block in lane (g, j); the K = 32 step
// over blocks 2s and 2s+1 takes the B fragment [block 2s units 4g..4g+3,
// block 2s+1 units 4g..4g+3] and the matching weight columns in the same
// (permuted) order, so no data moves between lanes.
//
// The first layer's B fragment of lane (g, j) is features 32 ks + 8 g .. +7 of
// row j, read straight from global memory.  The kernel orders a surrogate
// input [r, g, b, col, row, a_0..a_{k-1}] as [a_0..a_{k-1}, 0 ..., r, g, b,
// col, row] (the five leading features in the last five of the 128 slots;
// the first layer's weight columns are permuted to match when they are staged
// in LDS), so a window below k is two 16-byte loads and the window that holds
// k takes clamped element loads.  Explicit rows x of more than five features
// take the same order, so both forms round alike; narrower rows keep theirs.
// Two 12-wave workgroups per CU (76 VGPRs, six waves per SIMD) hide the
// input loads without a prefetch; the hidden activations are evaluated as
// twice the GELU (gelu2x), 12 VALU instructions each, which is what bounds
// the kernel.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short s16x8 __attribute__((ext_vector_type(8)));
constexpr int kInfWaves = 12;          // waves per workgroup; two workgroups per CU (weights in LDS twice)
constexpr int kInfBlocksPerCu = 2;
constexpr int kInfNT = 1;              // 16-pixel tiles per wave and round (each weight fragment read feeds kInfNT products)
constexpr int kInfRows = 16 * kInfNT;  // pixels per wave and round
constexpr int kInfIn = 128;            // input features padded to whole K = 32 steps
constexpr int kInfKs = kInfIn / 32;
constexpr int kInfLd = kMlpHid + 8;    // LDS row stride (elements) of the weights

__device__ __forceinline__ f32x4 mfma32(s16x8 a, s16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
}
__device__ __forceinline__ s16x8 cat4(s16x4 lo, s16x4 hi) {
    return s16x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
}
// Twice the GELU with the erf approximation above: 2 GELU(z) = z + |z| erf(|z|
// / sqrt 2) = z + |z| (1 - P(t) e^{-z^2/2}), t = 1 / (1 + p |z| / sqrt 2) --
// 12 instructions.  The factor 2 is exact and is undone by halving the next
// layer's (BF16) weights, which is exact too.
__device__ __forceinline__ float gelu2x(float z) {
    const float az = fabsf(z);
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f * 0.70710678118654752f, az, 1.0f));
    float q = fmaf(1.061405429f, t, -1.453152027f);
    q = fmaf(q, t, 1.421413741f);
    q = fmaf(q, t, -0.284496736f);
    q = fmaf(q, t, 0.254829592f);
    const float e = __builtin_amdgcn_exp2f((z * z) * (-0.5f * 1.4426950408889634f));
    return fmaf(az, fmaf(-(q * t), e, 1.0f), z);
}
__device__ __forceinline__ short half_bf16(short w) {
    return to_bf16(0.5f * __builtin_bit_cast(float, (uint32_t)(uint16_t)w << 16));
}

__global__ __launch_bounds__(64 * kInfWaves) __attribute__((amdgpu_waves_per_eu(kInfWaves * kInfBlocksPerCu / 4))) void k_mlp_infer(MlpInferArgs a) {
    __shared__ __align__(16) short sW1[kMlpHid * kInfLd];
    __shared__ __align__(16) short sW2[kMlpHid * kInfLd];
    __shared__ __align__(16) short sW3[kMlpOutPad * kInfLd];
    __shared__ __align__(16) float sb[2 * kMlpHid + kMlpOutPad];
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int g = lane >> 4, j = lane & 15;
    // head: the five leading features go to slots kInfIn-5 .. kInfIn-1, the
    // w features after them to slots 0 .. w-1 (source rows of stride ld)
    const bool rows_x = a.x != nullptr;
    const bool head = !rows_x || a.in > 5;
    const int w = rows_x ? (head ? a.in - 5 : a.in) : a.k;
    const int ld = rows_x ? a.in : a.k;
    const float *src0 = rows_x ? a.x + (head ? 5 : 0) : a.alpha;
    for (int e = tid; e < kMlpHid * kInfIn; e += 64 * kInfWaves) {
        const int h = e / kInfIn, c = e - h * kInfIn;
        // network column of kernel feature c, or -1 for a zero slot
        const int nc = !head ? (c < a.in ? c : -1) : c < w ? 5 + c : c >= kInfIn - 5 ? c - (kInfIn - 5) : -1;
        sW1[h * kInfLd + c] = nc >= 0 ? a.W1b[h * a.in_pad + nc] : (short)0;
    }
    // the hidden layers hold twice their activations (gelu2x): halved weights
    for (int e = tid; e < kMlpHid * kMlpHid; e += 64 * kInfWaves)
        sW2[(e / kMlpHid) * kInfLd + e % kMlpHid] = half_bf16(a.W2b[e]);
    for (int e = tid; e < kMlpOutPad * kMlpHid; e += 64 * kInfWaves)
        sW3[(e / kMlpHid) * kInfLd + e % kMlpHid] = half_bf16(a.W3b[e]);
    for (int e = tid; e < 2 * kMlpHid + kMlpOutPad; e += 64 * kInfWaves)
        sb[e] = e < kMlpHid ? a.b1[e] : e < 2 * kMlpHid ? a.b2[e - kMlpHid] : (e - 2 * kMlpHid < a.out ? a.b3[e - 2 * kMlpHid] : 0.f);
    __syncthreads();
    const int ks1 = head ? kInfKs : (a.in + 31) / 32;
    const int64_t ngrp = (a.n + kInfRows - 1) / kInfRows;
    const int64_t N = (int64_t)a.H * a.W;
    const float sx = a.W > 1 ? 1.0f / (float)(a.W - 1) : 0.0f, sy = a.H > 1 ? 1.0f / (float)(a.H - 1) : 0.0f;
    // raw inputs of the round: features 32 ks + 8 g .. +7 of row 16 tt + j
    float raw[kInfNT][kInfKs][8];
    // Windows of the K steps below kf lie below w for every lane; the window
    // of step kf may cross w (its elements at or past w become zero).  The
    // source is read through a buffer resource that ends at the round's last
    // valid element, so rows past the end read zero.
    const int kf = w >> 5;
    const int voff = (j * ld + 8 * g) * 4;
    auto fetch = [&](int64_t t) {
        if (t >= ngrp) return;
        const int64_t p0 = t * kInfRows;
        const int rows = (int)(a.n - p0 < kInfRows ? a.n - p0 : kInfRows);
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(src0 + p0 * ld), (short)0, ((rows - 1) * ld + w) * 4, 0x00020000);
#pragma unroll
        for (int tt = 0; tt < kInfNT; ++tt) {
            const int vo = voff + 16 * tt * ld * 4;  // the range check covers the vector offset only
#pragma unroll
            for (int ks = 0; ks < kInfKs; ++ks) {
                if (ks < kf) {
                    const f32x4 lo = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, vo + 128 * ks, 0, 0));
                    const f32x4 hi = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, vo + 128 * ks + 16, 0, 0));
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        raw[tt][ks][c] = lo[c];
                        raw[tt][ks][4 + c] = hi[c];
                    }
                } else if (ks == kf) {
                    // opaque copies: keeps the compiler from hoisting 8 offsets
                    // and 8 lane masks per K step out of the loop
                    int o = vo + 128 * ks, nv = w - 32 * ks - 8 * g;
                    __asm__ volatile("" : "+v"(o), "+v"(nv));
#pragma unroll
                    for (int c = 0; c < 8; ++c) {
                        const float v = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, o + 4 * c, 0, 0));
                        raw[tt][ks][c] = c < nv ? v : 0.0f;
                    }
                } else {
#pragma unroll
                    for (int c = 0; c < 8; ++c) raw[tt][ks][c] = 0.0f;
                }
            }
            int64_t row = p0 + 16 * tt + j;
            if (row > a.n - 1) row = a.n - 1;  // rows past the end repeat the last (their outputs are not written)
            if (head) {
                float hv[5];
                if (rows_x) {
#pragma unroll
                    for (int c = 0; c < 5; ++c) hv[c] = a.x[row * a.in + c];
                } else {
                    const int pix = (int)row;  // images hold fewer than 2^31 pixels
                    const int prow = pix / a.W;
                    hv[0] = a.rgb[pix];
                    hv[1] = a.rgb[N + pix];
                    hv[2] = a.rgb[2 * N + pix];
                    hv[3] = (float)(pix - prow * a.W) * sx;
                    hv[4] = (float)prow * sy;
                }
#pragma unroll
                for (int c = 0; c < 5; ++c)
                    if (g == 3) raw[tt][kInfKs - 1][3 + c] = hv[c];
            }
        }
    };
    int64_t t = (int64_t)blockIdx.x * kInfWaves + wave;
    for (; t < ngrp; t += (int64_t)gridDim.x * kInfWaves) {
        const int64_t p0 = t * kInfRows;
        const int np = (int)(a.n - p0 < kInfRows ? a.n - p0 : kInfRows);
        fetch(t);
        s16x8 xb[kInfNT][kInfKs];
#pragma unroll
        for (int tt = 0; tt < kInfNT; ++tt)
#pragma unroll
            for (int ks = 0; ks < kInfKs; ++ks)
#pragma unroll
                for (int c = 0; c < 8; ++c) xb[tt][ks][c] = to_bf16(raw[tt][ks][c]);
        // layer 1 (kernel feature order, natural K: features 32 ks + 8 g .. +7)
        s16x4 h1b[kInfNT][8];
#pragma unroll
        for (int hb = 0; hb < 8; ++hb) {
            const f32x4 bias = *reinterpret_cast<const f32x4 *>(sb + 16 * hb + 4 * g);
            f32x4 acc[kInfNT];
#pragma unroll
            for (int tt = 0; tt < kInfNT; ++tt) acc[tt] = bias;
            const short *wr = sW1 + (16 * hb + j) * kInfLd + 8 * g;
#pragma unroll
            for (int ks = 0; ks < kInfKs; ++ks)
                if (ks < ks1) {
                    const s16x8 wf = *reinterpret_cast<const s16x8 *>(wr + 32 * ks);
#pragma unroll
                    for (int tt = 0; tt < kInfNT; ++tt) acc[tt] = mfma32(wf, xb[tt][ks], acc[tt]);
                }
#pragma unroll
            for (int tt = 0; tt < kInfNT; ++tt)
#pragma unroll
                for (int r = 0; r < 4; ++r) h1b[tt][hb][r] = to_bf16(gelu2x(acc[tt][r]));
            // every block: keeps the weight loads of later blocks from piling
            // up in VGPRs
            __builtin_amdgcn_sched_barrier(0);
        }
        // layer 2 (permuted K order over block pairs)
        s16x4 h2b[kInfNT][8];
#pragma unroll
        for (int hb = 0; hb < 8; ++hb) {
            const f32x4 bias = *reinterpret_cast<const f32x4 *>(sb + kMlpHid + 16 * hb + 4 * g);
            f32x4 acc[kInfNT];
#pragma unroll
            for (int tt = 0; tt < kInfNT; ++tt) acc[tt] = bias;
            const short *wr = sW2 + (16 * hb + j) * kInfLd + 4 * g;
#pragma unroll
            for (int s2 = 0; s2 < 4; ++s2) {
                const s16x8 wf = cat4(ld4(wr + 32 * s2), ld4(wr + 32 * s2 + 16));
#pragma unroll
                for (int tt = 0; tt < kInfNT; ++tt)
                    acc[tt] = mfma32(wf, cat4(h1b[tt][2 * s2], h1b[tt][2 * s2 + 1]), acc[tt]);
            }
#pragma unroll
            for (int tt = 0; tt < kInfNT; ++tt)
#pragma unroll
                for (int r = 0; r < 4; ++r) h2b[tt][hb][r] = to_bf16(gelu2x(acc[tt][r]));
            __builtin_amdgcn_sched_barrier(0);
        }
        const f32x4 bias3 = *reinterpret_cast<const f32x4 *>(sb + 2 * kMlpHid + 4 * g);
        f32x4 y[kInfNT];
#pragma unroll
        for (int tt = 0; tt < kInfNT; ++tt) y[tt] = bias3;
        {
            const short *wr = sW3 + j * kInfLd + 4 * g;
#pragma unroll
            for (int s2 = 0; s2 < 4; ++s2) {
                const s16x8 wf = cat4(ld4(wr + 32 * s2), ld4(wr + 32 * s2 + 16));
#pragma unroll
                for (int tt = 0; tt < kInfNT; ++tt)
                    y[tt] = mfma32(wf, cat4(h2b[tt][2 * s2], h2b[tt][2 * s2 + 1]), y[tt]);
            }
        }
#pragma unroll
        for (int tt = 0; tt < kInfNT; ++tt)
            if (16 * tt + j < np)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int o = 4 * g + r;
                    if (o < a.out) a.y[(p0 + 16 * tt + j) * a.out + o] = y[tt][r];
                }
    }
}

// Surrogate inputs of listed pixels: [r, g, b, col/(W-1), row/(H-1), a_0..a_{k-1}].
__global__ __launch_bounds__(256) void k_mlp_features(const float *rgb, int H, int W, const float *alpha, int k,
                                                       const int32_t *pix, int64_t n, float *x) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int in = 5 + k;
    if (e >= n * in) return;
    const int64_t r = e / in;
    const int f = (int)(e - r * in);
    const int64_t p = pix[r];
    const int64_t N = (int64_t)H * W;
    float v;
    if (f < 3) v = rgb[f * N + p];
    else if (f == 3) v = W > 1 ? (float)(p % W) * (1.0f / (float)(W - 1)) : 0.0f;
    else if (f == 4) v = H > 1 ? (float)(p / W) * (1.0f / (float)(H - 1)) : 0.0f;
    else v = alpha[p * k + (f - 5)];
    x[e] = v;
}

// Output bias b3_i = mean over the rows of the clipped target
// t_i = max(l_i, max_j l_j - 20); one workgroup per label, FP64 sum.
__global__ __launch_bounds__(256) void k_mlp_bias_mean(const float *ell, int64_t n, int out, float *b3) {
    __shared__ double red[256];
    const int lab = blockIdx.x;
    double s = 0.0;
    for (int64_t r = threadIdx.x; r < n; r += 256) {
        float mx = -INFINITY;
        for (int o = 0; o < out; ++o) mx = fmaxf(mx, ell[r * out + o]);
        s += (double)fmaxf(ell[r * out + lab], mx - kClipNats);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) b3[lab] = (float)(red[0] / (double)n);
}

hipError_t launch_mlp_bias_mean(const LaunchCtx &lc, const float *ell, int64_t n, int out, float *b3) {
    hipLaunchKernelGGL(k_mlp_bias_mean, dim3((unsigned)out), dim3(256), 0, lc.stream, ell, n, out, b3);
    return hipGetLastError();
}

hipError_t launch_mlp_fwdbwd(const LaunchCtx &lc, const MlpTrainArgs &a) {
    const int tiles = a.B / 16;  // one workgroup per 16-row tile
    hipLaunchKernelGGL(k_mlp_fwdbwd, dim3((unsigned)tiles), dim3(256), 0, lc.stream, a);
    return hipGetLastError();
}
hipError_t launch_mlp_wgrad(const LaunchCtx &lc, const MlpWgradArgs &a) {
    const int ntile = 8 * (a.in_pad / 16) + 64 + 8;
    const int items = ntile * a.kc;
    hipLaunchKernelGGL(k_mlp_wgrad, dim3((unsigned)((items + 3) / 4)), dim3(256), 0, lc.stream, a);
    return hipGetLastError();
}
hipError_t launch_mlp_adam(const LaunchCtx &lc, const MlpAdamArgs &a) {
    const int wblocks = (int)((a.P + 255) / 256);
    const int bblocks = (2 * kMlpHid + a.out + 1 + 3) / 4;  // one wave per bias unit and one for the loss
    hipLaunchKernelGGL(k_mlp_adam, dim3((unsigned)(wblocks + bblocks)), dim3(256), 0, lc.stream, a, wblocks);
    return hipGetLastError();
}
hipError_t launch_mlp_convert(const LaunchCtx &lc, const MlpAdamArgs &a) {
    hipLaunchKernelGGL(k_mlp_convert, dim3((unsigned)((a.P + 255) / 256)), dim3(256), 0, lc.stream, a);
    return hipGetLastError();
}
hipError_t launch_mlp_infer(const LaunchCtx &lc, const MlpInferArgs &a) {
    const int64_t ngrp = (a.n + kInfRows - 1) / kInfRows;
    int64_t blocks = (int64_t)lc.num_cu * kInfBlocksPerCu;
    if (blocks > (ngrp + kInfWaves - 1) / kInfWaves) blocks = (ngrp + kInfWaves - 1) / kInfWaves;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_mlp_infer, dim3((unsigned)blocks), dim3(64 * kInfWaves), 0, lc.stream, a);
    return hipGetLastError();
}
hipError_t launch_mlp_features(const LaunchCtx &lc, const float *rgb, int H, int W, const float *alpha, int k,
                               const int32_t *pix, int64_t n, float *x) {
    const int64_t total = n * (5 + k);
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_features, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, lc.stream, rgb, H, W,
                       alpha, k, pix, n, x);
    return hipGetLastError();
}

}  // namespace cs
