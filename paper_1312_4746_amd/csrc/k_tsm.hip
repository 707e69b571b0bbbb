// Texture similarity of co-supports (Sec. 2, TSM definition) on gfx950:
// TSM(a, b) = number of indices in exactly one of the two co-supports, i.e.
// the popcount of the XOR of the bit-packed masks.
//
// A 64 x 64 output tile per workgroup of 256 threads: the 64 A masks of the
// tile are staged in LDS, each lane keeps one B mask in registers and owns
// one output column, so a wave writes 64 consecutive int32 of an output row
// per step.  Bits at j >= k are cleared before counting.
#include "cs_internal.h"

namespace cs {

template <int NW>
__global__ __launch_bounds__(256) void k_tsm(const uint64_t *A, int64_t na, const uint64_t *B,
                                              int64_t nb, int k, int32_t *out) {
    __shared__ uint64_t sa[64][NW];
    const int64_t a0 = (int64_t)blockIdx.y * 64, b0 = (int64_t)blockIdx.x * 64;
    const int tid = threadIdx.x;
    const uint64_t lastmask = (k % 64) ? ((1ull << (k % 64)) - 1ull) : ~0ull;
    for (int idx = tid; idx < 64 * NW; idx += 256) {
        const int i = idx / NW, w = idx % NW;
        uint64_t v = 0;
        if (a0 + i < na) v = A[(a0 + i) * NW + w];
        if (w == NW - 1) v &= lastmask;
        sa[i][w] = v;
    }
    __syncthreads();
    const int bi = tid & 63;        // output column within the tile
    const int aq = (tid >> 6) * 16; // first of this wave's 16 A rows
    if (b0 + bi >= nb) return;
    uint64_t bm[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) bm[w] = B[(b0 + bi) * NW + w];
    bm[NW - 1] &= lastmask;
    for (int c = 0; c < 16; ++c) {
        const int ai = aq + c;
        if (a0 + ai >= na) break;
        int t = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) t += __popcll(bm[w] ^ sa[ai][w]);
        out[(a0 + ai) * nb + b0 + bi] = t;
    }
}

hipError_t launch_tsm(const LaunchCtx &lc, const uint64_t *A, int64_t na, const uint64_t *B,
                      int64_t nb, int k, int32_t *out) {
    if (na == 0 || nb == 0) return hipSuccess;
    const int64_t rows_per_launch = (int64_t)65535 * 64;
    for (int64_t a_off = 0; a_off < na; a_off += rows_per_launch) {
        const int64_t cnt = na - a_off < rows_per_launch ? na - a_off : rows_per_launch;
        const uint64_t *Aq = A + a_off * ((k + 63) / 64);
        int32_t *oq = out + a_off * nb;
        dim3 grid((unsigned)((nb + 63) / 64), (unsigned)((cnt + 63) / 64));
        switch ((k + 63) / 64) {
            case 1: hipLaunchKernelGGL(k_tsm<1>, grid, dim3(256), 0, lc.stream, Aq, cnt, B, nb, k, oq); break;
            case 2: hipLaunchKernelGGL(k_tsm<2>, grid, dim3(256), 0, lc.stream, Aq, cnt, B, nb, k, oq); break;
            case 3: hipLaunchKernelGGL(k_tsm<3>, grid, dim3(256), 0, lc.stream, Aq, cnt, B, nb, k, oq); break;
            default: hipLaunchKernelGGL(k_tsm<4>, grid, dim3(256), 0, lc.stream, Aq, cnt, B, nb, k, oq); break;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace cs
