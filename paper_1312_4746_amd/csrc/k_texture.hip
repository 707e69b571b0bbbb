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

#include "cs_internal.h"

namespace cs {

constexpr int kRepThreads = 1024;
constexpr int kRepWaves = kRepThreads / 64;

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

__global__ __launch_bounds__(256) void k_texture_post(TextureArgs a) {
    __shared__ uint64_t srep[kMaxLabels * 4];
    for (int t = threadIdx.x; t < a.L * 4; t += 256) srep[t] = a.rep[t];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
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

hipError_t launch_label_rep(const LaunchCtx &lc, const TextureArgs &a) {
    hipLaunchKernelGGL(k_label_rep, dim3((unsigned)a.L), dim3(kRepThreads), 0, lc.stream, a);
    return hipGetLastError();
}

hipError_t launch_texture_post(const LaunchCtx &lc, const TextureArgs &a) {
    if (!a.npix) return hipSuccess;
    hipLaunchKernelGGL(k_texture_post, dim3((unsigned)((a.npix + 255) / 256)), dim3(256), 0,
                       lc.stream, a);
    return hipGetLastError();
}

}  // namespace cs
