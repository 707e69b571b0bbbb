// Exact squared Euclidean distance from every pixel to the nearest scribble
// sample of each label, with the identity of that sample, on gfx950.  This is
// the |x - x_{v_i}| that sets the spatial bandwidth rho_i(x) in Sec. 3.1.
//
// Separable two-pass transform on integer distances (exact):
//  1. columns: for every (label, column) a thread scans the column down and up
//     and keeps the row of the nearest seed in that column (coalesced: the
//     threads of a wave own adjacent columns);
//  2. rows: for every (label, row) a thread builds the lower envelope of the
//     parabolas (c - q)^2 + f(q) over the columns q that hold a seed, with
//     f(q) the squared column distance, and reads it off for every column.
//     Envelope breakpoints are compared by exact 64-bit cross-multiplication,
//     so no rounding enters; the stack of envelope sites lives in LDS.
#include "cs_internal.h"

namespace cs {

__global__ __launch_bounds__(256) void k_edt_cols(const uint8_t *seeds, int H, int W,
                                                   int32_t *colrow) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    const int l = blockIdx.y;
    if (c >= W) return;
    const int64_t N = (int64_t)H * W;
    const uint8_t *sd = seeds + (int64_t)l * N + c;
    int32_t *cr = colrow + (int64_t)l * N + c;
    int last = -1;
    for (int r = 0; r < H; ++r) {
        if (sd[(int64_t)r * W]) last = r;
        cr[(int64_t)r * W] = last;
    }
    int next = -1;
    for (int r = H - 1; r >= 0; --r) {
        if (sd[(int64_t)r * W]) next = r;
        const int cur = cr[(int64_t)r * W];
        if (next >= 0 && (cur < 0 || next - r < r - cur)) cr[(int64_t)r * W] = next;
    }
}

__device__ __forceinline__ int64_t env_F(int q, int fr) {  // f(q) + q^2
    return (int64_t)fr * fr + (int64_t)q * q;
}

__global__ void k_edt_rows(const int32_t *colrow, int H, int W, int L, int32_t *d2,
                           int32_t *nearest) {
    extern __shared__ int16_t stack_mem[];
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)H * L) return;
    const int l = (int)(gid / H), r = (int)(gid - (int64_t)(gid / H) * H);
    const int64_t N = (int64_t)H * W;
    const int32_t *cr = colrow + (int64_t)l * N + (int64_t)r * W;
    int16_t *v = stack_mem + (int64_t)threadIdx.x * W;
    // f(q) = (r - colrow[q])^2 ; F(q) = f(q) + q^2
    int top = -1;
    for (int q = 0; q < W; ++q) {
        const int rq = cr[q];
        if (rq < 0) continue;
        const int64_t Fq = env_F(q, r - rq);
        while (top >= 1) {
            const int a = v[top - 1], b = v[top];
            const int64_t Fa = env_F(a, r - cr[a]), Fb = env_F(b, r - cr[b]);
            // breakpoint(b, q) <= breakpoint(a, b)  ->  b is never the minimum
            if ((Fq - Fb) * (int64_t)(b - a) <= (Fb - Fa) * (int64_t)(q - b))
                --top;
            else
                break;
        }
        v[++top] = (int16_t)q;
    }
    int32_t *dd = d2 + (int64_t)l * N + (int64_t)r * W;
    int32_t *nn = nearest + (int64_t)l * N + (int64_t)r * W;
    if (top < 0) {  // no seed of this label anywhere (rejected before launch)
        for (int c = 0; c < W; ++c) {
            dd[c] = -1;
            nn[c] = -1;
        }
        return;
    }
    int kk = 0;
    for (int c = 0; c < W; ++c) {
        while (kk < top) {
            const int a = v[kk], b = v[kk + 1];
            const int64_t Fa = env_F(a, r - cr[a]), Fb = env_F(b, r - cr[b]);
            // breakpoint(a, b) = (Fb - Fa) / (2 (b - a)) <= c  ->  move to b
            if (Fb - Fa <= (int64_t)c * 2 * (b - a))
                ++kk;
            else
                break;
        }
        const int q = v[kk];
        const int dr = r - cr[q];
        dd[c] = (c - q) * (c - q) + dr * dr;
        nn[c] = cr[q] * W + q;
    }
}

hipError_t launch_edt(const LaunchCtx &lc, const uint8_t *seeds, int H, int W, int L,
                      int32_t *colrow, int32_t *d2, int32_t *nearest) {
    hipLaunchKernelGGL(k_edt_cols, dim3((W + 255) / 256, L), dim3(256), 0, lc.stream, seeds, H, W,
                       colrow);
    // Threads per workgroup bounded by a 64 KiB LDS stack budget.
    int tpb = (int)(65536 / (2 * (int64_t)W));
    if (tpb > 64) tpb = 64;
    if (tpb < 1) tpb = 1;
    const int64_t total = (int64_t)H * L;
    const size_t lds = (size_t)tpb * W * sizeof(int16_t);
    hipError_t e = hipFuncSetAttribute((const void *)k_edt_rows,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_edt_rows, dim3((unsigned)((total + tpb - 1) / tpb)), dim3(tpb), lds,
                       lc.stream, colrow, H, W, L, d2, nearest);
    return hipGetLastError();
}

}  // namespace cs
