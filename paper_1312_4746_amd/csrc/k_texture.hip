// The paper's own texture factor (eq:joined, eq:post_text) on gfx950: each
// label's textural representative, then per pixel the texture posterior
// against the representatives, added in log form to the colour/location
// Parzen density that the Parzen kernels computed with the texture factor
// taken out of their sum.
//
// Representative (Sec. 2, the majority definition; Sec. 3.1 c_i).  Bit j of
// c_i is set when at least half of the label's m_i samples have j in their
// co-support (2 count_j >= m_i): for binary co-supports the component-wise
// median of eq:approx_cosupp, a tie counted in.  One workgroup per label;
// a wave takes 64 of the label's sorted sample records at a time and turns
// each co-support bit into a 64-lane ballot whose population count is that
// bit's vote over the 64 samples, so the votes cost one ballot per bit and
// sample group, no atomics.  The 16 waves' votes meet in LDS.
//
// Posterior (eq:post_text with beta_i = b rho_i, hard co-supports).  One
// thread per pixel: u_i = -TSM(m_x, c_i) / beta_i(x) for every label, a
// running log-sum-exp over the labels, then l_i += u_i - log sum_i' exp u_i'.
// rho_i(x) = alpha_rho sqrt(max(d2_i(x), r_f^2)) from the exact distance
// transform's d2, in FP64 as the coefficient kernel does.  Per pixel the
// kernel moves 12 L + 8 ceil(k/64) bytes (the row of L log-likelihoods read
// and written once, L distances, the mask): HBM-bound.

//
// Smooth co-supports (eq:map_tsm, the setting of the paper's experiments).
// iota(a)_j = exp(-a_j^2 / sigma); c_lj = the median of iota_j over the
// label's samples (eq:approx_cosupp), the element of rank floor(m/2) of the
// ascending values; u_i = -||c_i - iota(a_x)||_1 / beta_i(x) (eq:tsm).  The
// median is an exact radix selection on the FP32 bit patterns (non-negative
// values order as unsigned integers): one workgroup per (component, label),
// four 8-bit digit passes with an LDS histogram, the digit found by one
// wave's prefix scan.  The posterior kernel keeps the L distances of a pixel
// in registers while it streams the pixel's k analysed values once.

#include "cs_internal.h"

namespace cs {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kRepThreads = 1024;
constexpr int kRepWaves = kRepThreads / 64;
// Threads per workgroup of the posterior kernels (one thread per pixel).
constexpr int kPostThreads = 256;

__global__ __launch_bounds__(kRepThreads) void k_label_rep(TextureArgs a) {
    const int l = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int s0 = a.seg[l], m = a.seg[l + 1] - s0;
    const int nw = (a.k + 31) / 32;
    __shared__ uint32_t part[kRepWaves][256];
    uint32_t cnt[4] = {0u, 0u, 0u, 0u};  // votes of bits lane + 64 c
    for (int base = wave * 64; base < m; base += kRepThreads) {
        const int s = base + lane;
        const bool ok = s < m;
        // clamped record index (m >= 1): every lane loads, lanes past the
        // label's end vote with zero words
        const uint32_t *rw = a.recs[s0 + (ok ? s : 0)].w + 8;
        uint32_t mw[8];
#pragma unroll
        for (int w = 0; w < 8; ++w) {
            const uint32_t v = rw[w];  // a record always holds 8 co-support words
            mw[w] = (w < nw && ok) ? v : 0u;
        }
#pragma unroll
        for (int w = 0; w < 8; ++w) {
            if (w < nw) {
#pragma unroll
                for (int b = 0; b < 32; ++b) {
                    const uint32_t c = (uint32_t)__popcll(__ballot((mw[w] >> b) & 1u));
                    cnt[w >> 1] += lane == (w & 1) * 32 + b ? c : 0u;
                }
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) part[wave][lane + 64 * c] = cnt[c];
    __syncthreads();
    if (threadIdx.x < 256) {
        const int j = threadIdx.x;
        int64_t votes = 0;
#pragma unroll
        for (int w = 0; w < kRepWaves; ++w) votes += part[w][j];
        const bool in = j < a.k && 2 * votes >= (int64_t)m;
        const unsigned long long word = __ballot(in);
        if (lane == 0) a.rep[l * 4 + wave] = (uint64_t)word;
    }
}

__global__ __launch_bounds__(kPostThreads) void k_texture_post(TextureArgs a) {
    __shared__ uint64_t srep[kMaxLabels * 4];
    for (int t = threadIdx.x; t < a.L * 4; t += kPostThreads) srep[t] = a.rep[t];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kPostThreads + threadIdx.x;
    if (i >= a.npix) return;
    const int64_t pix = a.subset ? (int64_t)a.subset[i] : i;
    const int W64 = (a.k + 63) / 64;
    uint64_t mx[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) mx[w] = w < W64 ? a.masks[pix * W64 + w] : 0ull;
    // bits k.. of the last word are not part of the co-support
    const int tail = a.k - 64 * (W64 - 1);
    const uint64_t last = tail == 64 ? ~0ull : ((1ull << tail) - 1ull);
#pragma unroll
    for (int w = 0; w < 4; ++w)
        if (w == W64 - 1) mx[w] &= last;
    const double fl2 = a.rho_floor * a.rho_floor;
    auto u_of = [&](int l) -> float {
        int d = 0;
#pragma unroll
        for (int w = 0; w < 4; ++w) d += __popcll(mx[w] ^ srep[l * 4 + w]);
        const double d2 = (double)a.d2[(int64_t)l * a.N + pix];
        const double rho = a.alpha_rho * sqrt(d2 > fl2 ? d2 : fl2);
        return (float)(-(double)d / (a.beta_scale * rho));
    };
    float um = -INFINITY, s = 0.0f;
    for (int l = 0; l < a.L; ++l) {
        const float u = u_of(l);
        if (u > um) {
            s = s * expf(um - u) + 1.0f;
            um = u;
        } else {
            s += expf(u - um);
        }
    }
    const float lz = um + logf(s);
    float *row = a.loglik + i * a.L;
    for (int l = 0; l < a.L; ++l) row[l] += u_of(l) - lz;
}

__device__ __forceinline__ uint32_t soft_bits(const TextureArgs &a, int s, int j) {
    const uint32_t *rw = a.recs[s].w;
    const int64_t pix = (int64_t)__uint_as_float(rw[1]) * a.W + (int64_t)__uint_as_float(rw[0]);
    const float v = a.alpha[pix * a.k + j];
    return __float_as_uint(expf(-(v * v) * a.inv_sigma));
}

// Values a thread keeps in registers across the four digit passes (labels of
// up to 256 kRepCache samples; larger ones recompute them each pass).
constexpr int kRepCache = 8;

__global__ __launch_bounds__(256) void k_label_rep_soft(TextureArgs a) {
    const int j = blockIdx.x, l = blockIdx.y;
    const int s0 = a.seg[l], m = a.seg[l + 1] - s0;
    __shared__ uint32_t hist[256];
    __shared__ uint32_t s_prefix, s_rank;
    const bool cached = m <= 256 * kRepCache;
    uint32_t cache[kRepCache];
    if (cached) {
        // clamped indices (m >= 1): every load is in bounds and independent
#pragma unroll
        for (int q = 0; q < kRepCache; ++q) {
            const int s = (int)threadIdx.x + 256 * q;
            cache[q] = soft_bits(a, s0 + (s < m ? s : m - 1), j);
        }
    }
    uint32_t prefix = 0u, mask = 0u, rank = (uint32_t)(m / 2);
#pragma unroll 1
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 24 - 8 * pass;
        hist[threadIdx.x] = 0u;
        __syncthreads();
        if (cached) {
#pragma unroll
            for (int q = 0; q < kRepCache; ++q) {
                const int s = (int)threadIdx.x + 256 * q;
                const uint32_t v = cache[q];
                if (s < m && (v & mask) == prefix) atomicAdd(&hist[(v >> shift) & 255u], 1u);
            }
        } else {
            for (int s = threadIdx.x; s < m; s += 256) {
                const uint32_t v = soft_bits(a, s0 + s, j);
                if ((v & mask) == prefix) atomicAdd(&hist[(v >> shift) & 255u], 1u);
            }
        }
        __syncthreads();
        if (threadIdx.x < 64) {
            const int t = threadIdx.x;
            const uint32_t h0 = hist[4 * t], h1 = hist[4 * t + 1], h2 = hist[4 * t + 2], h3 = hist[4 * t + 3];
            const uint32_t c = h0 + h1 + h2 + h3;
            uint32_t incl = c;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t y = __shfl_up(incl, o);
                if (t >= o) incl += y;
            }
            const uint32_t excl = incl - c;
            // the values matching the prefix number at least rank + 1, so
            // exactly one lane holds the rank
            if (rank >= excl && rank < incl) {
                uint32_t rr = rank - excl;
                int d = 0;
                if (rr >= h0) { rr -= h0; d = 1;
                    if (rr >= h1) { rr -= h1; d = 2;
                        if (rr >= h2) { rr -= h2; d = 3; } } }
                s_prefix = prefix | ((uint32_t)(4 * t + d) << shift);
                s_rank = rr;
            }
        }
        __syncthreads();
        prefix = s_prefix;
        rank = s_rank;
        mask |= 255u << shift;
    }
    if (threadIdx.x == 0) a.crep[l * a.k + j] = __uint_as_float(prefix);
}

// LM: compile-time bound on the label count (registers for the distances).
// BUF: the analysed vectors are read with 16-byte buffer loads through one
// resource over the whole array (its size below 2^32 bytes), else with
// 4-byte global loads.
// The representatives sit in LDS with rows padded to a multiple of 8 values,
// so a chunk of 8 arrives with two 16-byte broadcast reads.
template <int LM, bool BUF>
__global__ __launch_bounds__(kPostThreads) void k_texture_post_soft(TextureArgs a) {
    extern __shared__ f32x4 screp4[];  // L x kp/4
    const int kp = (a.k + 7) & ~7;
    float *screp = reinterpret_cast<float *>(screp4);
    for (int t = threadIdx.x; t < a.L * kp; t += kPostThreads) {
        const int l = t / kp, j = t - l * kp;
        screp[t] = j < a.k ? a.crep[l * a.k + j] : 0.0f;
    }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kPostThreads + threadIdx.x;
    if (i >= a.npix) return;
    const int64_t pix = a.subset ? (int64_t)a.subset[i] : i;
    const float *ax = a.alpha + pix * a.k;
    float d[LM];
#pragma unroll
    for (int l = 0; l < LM; ++l) d[l] = 0.0f;
    auto add = [&](const float (&v)[8], int j0, int nv) {
        float io[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) io[c] = expf(-(v[c] * v[c]) * a.inv_sigma);
#pragma unroll
        for (int l = 0; l < LM; ++l) {
            if (l < a.L) {
                const f32x4 c0 = screp4[(l * kp + j0) / 4], c1 = screp4[(l * kp + j0) / 4 + 1];
                const float cr[8] = {c0[0], c0[1], c0[2], c0[3], c1[0], c1[1], c1[2], c1[3]};
#pragma unroll
                for (int c = 0; c < 8; ++c)
                    if (c < nv) d[l] += fabsf(cr[c] - io[c]);
            }
        }
    };
    if constexpr (BUF) {
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            (void *)a.alpha, (short)0, (int)((uint32_t)(a.N * a.k * 4)), 0x00020000);
        const int vo = (int)((uint32_t)(pix * a.k * 4));
        auto ld8 = [&](int j0, float (&v)[8]) {
            const f32x4 lo = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, vo + 4 * j0, 0, 0));
            const f32x4 hi = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, vo + 4 * j0 + 16, 0, 0));
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                v[c] = lo[c];
                v[4 + c] = hi[c];
            }
        };
        // whole chunks with 16-byte loads (inside the row, so inside the
        // resource), the tail with 4-byte loads clamped to the row
        const int k8 = a.k & ~7;
        float nxt[8];
        if (k8 > 0) ld8(0, nxt);
        for (int j0 = 0; j0 < k8; j0 += 8) {
            float cur[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) cur[c] = nxt[c];
            if (j0 + 8 < k8) ld8(j0 + 8, nxt);
            add(cur, j0, 8);
        }
        if (k8 < a.k) {
            const int nv = a.k - k8;
            float tl[8];
#pragma unroll
            for (int c = 0; c < 8; ++c)
                tl[c] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                                      rs, vo + 4 * (k8 + (c < nv ? c : 0)), 0, 0));
            add(tl, k8, nv);
        }
    } else {
        // the row streams in chunks of 8 values, the next chunk's loads in
        // flight while the current one is consumed
        const int k8 = a.k & ~7;
        float nxt[8];
        if (k8 > 0) {
#pragma unroll
            for (int c = 0; c < 8; ++c) nxt[c] = ax[c];
        }
        for (int j0 = 0; j0 < k8; j0 += 8) {
            float cur[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) cur[c] = nxt[c];
            if (j0 + 8 < k8) {
#pragma unroll
                for (int c = 0; c < 8; ++c) nxt[c] = ax[j0 + 8 + c];
            }
            add(cur, j0, 8);
        }
        if (k8 < a.k) {
            const int nv = a.k - k8;
            float tl[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) tl[c] = ax[k8 + (c < nv ? c : 0)];
            add(tl, k8, nv);
        }
    }
    const double fl2 = a.rho_floor * a.rho_floor;
    float um = -INFINITY;
#pragma unroll
    for (int l = 0; l < LM; ++l) {
        if (l < a.L) {
            const double d2 = (double)a.d2[(int64_t)l * a.N + pix];
            const double rho = a.alpha_rho * sqrt(d2 > fl2 ? d2 : fl2);
            d[l] = (float)(-(double)d[l] / (a.beta_scale * rho));
            um = fmaxf(um, d[l]);
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int l = 0; l < LM; ++l)
        if (l < a.L) s += expf(d[l] - um);
    const float lz = um + logf(s);
    float *row = a.loglik + i * a.L;
#pragma unroll
    for (int l = 0; l < LM; ++l)
        if (l < a.L) row[l] += d[l] - lz;
}

hipError_t launch_label_rep_soft(const LaunchCtx &lc, const TextureArgs &a) {
    hipLaunchKernelGGL(k_label_rep_soft, dim3((unsigned)a.k, (unsigned)a.L), dim3(256), 0, lc.stream, a);
    return hipGetLastError();
}

hipError_t launch_texture_post_soft(const LaunchCtx &lc, const TextureArgs &a) {
    if (!a.npix) return hipSuccess;
    const dim3 grid((unsigned)((a.npix + kPostThreads - 1) / kPostThreads));
    const size_t lds = sizeof(float) * (size_t)a.L * ((a.k + 7) & ~7);
    const bool buf = (uint64_t)a.N * (uint64_t)a.k * 4u < 0xFFFFFFF0ull;
    if (a.L <= 16) {
        if (buf) hipLaunchKernelGGL((k_texture_post_soft<16, true>), grid, dim3(kPostThreads), lds, lc.stream, a);
        else hipLaunchKernelGGL((k_texture_post_soft<16, false>), grid, dim3(kPostThreads), lds, lc.stream, a);
    } else {
        if (buf) hipLaunchKernelGGL((k_texture_post_soft<kMaxLabels, true>), grid, dim3(kPostThreads), lds, lc.stream, a);
        else hipLaunchKernelGGL((k_texture_post_soft<kMaxLabels, false>), grid, dim3(kPostThreads), lds, lc.stream, a);
    }
    return hipGetLastError();
}

hipError_t launch_label_rep(const LaunchCtx &lc, const TextureArgs &a) {
    hipLaunchKernelGGL(k_label_rep, dim3((unsigned)a.L), dim3(kRepThreads), 0, lc.stream, a);
    return hipGetLastError();
}

hipError_t launch_texture_post(const LaunchCtx &lc, const TextureArgs &a) {
    if (!a.npix) return hipSuccess;
    hipLaunchKernelGGL(k_texture_post, dim3((unsigned)((a.npix + kPostThreads - 1) / kPostThreads)),
                       dim3(kPostThreads), 0, lc.stream, a);
    return hipGetLastError();
}

}  // namespace cs
