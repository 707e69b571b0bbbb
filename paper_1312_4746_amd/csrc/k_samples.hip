// Scribble samples on gfx950 (the sets S_i of Sec. 3.1): validation, a
// stable counting sort by label into contiguous segments, and gathering of
// each sample's position, colour and co-support from its pixel into a 64-byte
// record that a wave reads with one scalar load.  Also marks the samples of
// each label in a per-label seed plane for the distance transform.
#include "cs_internal.h"

namespace cs {

constexpr int kChunk = 256;

// Per-chunk label counts (label-major: block_counts[l * nblocks + b]); a chunk
// with a bad label or pixel sets block_flags[b] = 1 (else 0).  Workgroups past
// nblocks clear the per-label seed plane (nseed16 16-byte words) instead.
__global__ __launch_bounds__(kChunk) void k_sample_count(const int32_t *label, const int32_t *pix,
                                                          int64_t M, int L, int64_t N,
                                                          int32_t *block_counts, int32_t *block_flags,
                                                          int nblocks, uint4 *seeds16, int64_t nseed16,
                                                          int nclear) {
    if ((int)blockIdx.x >= nblocks) {
        const int64_t stride = (int64_t)nclear * kChunk;
        for (int64_t i = (int64_t)(blockIdx.x - nblocks) * kChunk + threadIdx.x; i < nseed16; i += stride)
            seeds16[i] = make_uint4(0u, 0u, 0u, 0u);
        return;
    }
    __shared__ int cnt[kMaxLabels];
    __shared__ int bad;
    if (threadIdx.x < kMaxLabels) cnt[threadIdx.x] = 0;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    const int64_t idx = (int64_t)blockIdx.x * kChunk + threadIdx.x;
    if (idx < M) {
        const int l = label[idx];
        const int32_t px = pix[idx];
        if (l < 0 || l >= L || px < 0 || (int64_t)px >= N)
            bad = 1;
        else
            atomicAdd(&cnt[l], 1);
    }
    __syncthreads();
    if (threadIdx.x < L) block_counts[(int64_t)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
    if (threadIdx.x == 0) block_flags[blockIdx.x] = bad;
}

// Exclusive scan of block_counts in label-major order (in place), the label
// totals and the flags (bit 0: a bad sample, bit 1: a bad pixel of the list),
// one workgroup.  Also clears `nzero` words of counters for the kernels that
// follow, and hands totals and flags to the host: written to host memory
// (host_out[0..L]) and, after a system-scope fence, host_out[kHostTag] = tag.
__global__ __launch_bounds__(1024) void k_sample_scan(int32_t *block_counts, int L, int nblocks,
                                                       const int32_t *block_flags, const int32_t *pix_flags,
                                                       int npix_blocks, int32_t *totals_flags,
                                                       unsigned int *zero, int nzero,
                                                       volatile int32_t *host_out, int32_t tag) {
    __shared__ int32_t buf[1024];
    __shared__ int32_t carry, sflags;
    __shared__ int32_t tot[kMaxLabels];
    const int64_t total = (int64_t)L * nblocks;
    if (threadIdx.x == 0) {
        carry = 0;
        sflags = 0;
    }
    if (threadIdx.x < kMaxLabels) tot[threadIdx.x] = 0;
    for (int i = threadIdx.x; i < nzero; i += 1024) zero[i] = 0u;
    __syncthreads();
    int32_t f = 0;
    for (int i = threadIdx.x; i < nblocks; i += 1024) f |= block_flags[i] ? 1 : 0;
    for (int i = threadIdx.x; i < npix_blocks; i += 1024) f |= pix_flags[i] ? 2 : 0;
    if (f) atomicOr(&sflags, f);
    for (int64_t base = 0; base < total; base += 1024) {
        const int64_t i = base + threadIdx.x;
        const int32_t v = i < total ? block_counts[i] : 0;
        if (i < total) atomicAdd(&tot[i / nblocks], v);
        buf[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {  // Hillis-Steele inclusive scan
            int32_t t = threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
            __syncthreads();
            buf[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < total) block_counts[i] = carry + buf[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 1023) carry += buf[1023];
        __syncthreads();
    }
    if ((int)threadIdx.x <= L) {
        const int32_t v = (int)threadIdx.x < L ? tot[threadIdx.x] : sflags;
        totals_flags[threadIdx.x] = v;
        host_out[threadIdx.x] = v;
    }
    __threadfence_system();
    __syncthreads();
    if (threadIdx.x == 0) host_out[kHostTag] = tag;
}

hipError_t launch_sample_count(const LaunchCtx &lc, const int32_t *label, const int32_t *pix,
                               int64_t M, int L, int64_t N, int32_t *block_counts,
                               int32_t *block_flags, int nblocks, uint8_t *seeds, size_t seed_bytes) {
    // the seed plane is a multiple of 16 bytes (its caller pads it)
    const int64_t nseed16 = (int64_t)(seed_bytes / 16);
    int64_t nclear = (nseed16 + kChunk - 1) / kChunk;
    if (nclear > (int64_t)lc.num_cu * 4) nclear = (int64_t)lc.num_cu * 4;
    hipLaunchKernelGGL(k_sample_count, dim3((unsigned)(nblocks + nclear)), dim3(kChunk), 0, lc.stream, label, pix,
                       M, L, N, block_counts, block_flags, nblocks, reinterpret_cast<uint4 *>(seeds), nseed16,
                       (int)nclear);
    return hipGetLastError();
}

hipError_t launch_sample_scan(const LaunchCtx &lc, int32_t *block_counts, int L, int nblocks,
                              const int32_t *block_flags, const int32_t *pix_flags, int npix_blocks,
                              int32_t *totals_flags, unsigned int *zero, int nzero, int32_t *host_out,
                              int32_t tag) {
    hipLaunchKernelGGL(k_sample_scan, dim3(1), dim3(1024), 0, lc.stream, block_counts, L, nblocks, block_flags,
                       pix_flags, npix_blocks, totals_flags, zero, nzero, host_out, tag);
    return hipGetLastError();
}

// Stable scatter: a sample's slot is its chunk's offset for its label plus
// the number of earlier samples of the same label inside the chunk.
__global__ __launch_bounds__(kChunk) void k_sample_scatter(
    const int32_t *label, const int32_t *pix, int64_t M, int L, int H, int W, const float *rgb,
    const uint64_t *masks, int k, const int32_t *offsets, int nblocks, SampleRec *recs,
    uint8_t *seeds) {
    __shared__ int32_t lab[kChunk];
    const int64_t idx = (int64_t)blockIdx.x * kChunk + threadIdx.x;
    const int64_t N = (int64_t)H * W;
    int l = -1;
    int32_t px = 0;
    if (idx < M) {
        l = label[idx];
        px = pix[idx];
        if (l < 0 || l >= L || px < 0 || (int64_t)px >= N) l = -1;
    }
    lab[threadIdx.x] = l;
    __syncthreads();
    if (l < 0) return;
    int rank = 0;
    for (int i = 0; i < (int)threadIdx.x; ++i) rank += (lab[i] == l);
    const int64_t slot = (int64_t)offsets[(int64_t)l * nblocks + blockIdx.x] + rank;
    SampleRec r;
    r.w[0] = __float_as_uint((float)(px % W));
    r.w[1] = __float_as_uint((float)(px / W));
    r.w[2] = __float_as_uint(rgb[px]);
    r.w[3] = __float_as_uint(rgb[N + px]);
    r.w[4] = __float_as_uint(rgb[2 * N + px]);
    r.w[5] = r.w[6] = r.w[7] = 0;
    const int W64 = (k + 63) / 64;
    const uint64_t lastmask = (k % 64) ? ((1ull << (k % 64)) - 1ull) : ~0ull;
    for (int w = 0; w < 4; ++w) {
        uint64_t v = w < W64 ? masks[(int64_t)px * W64 + w] : 0ull;
        if (w == W64 - 1) v &= lastmask;
        r.w[8 + 2 * w] = (uint32_t)v;
        r.w[9 + 2 * w] = (uint32_t)(v >> 32);
    }
    recs[slot] = r;
    seeds[(int64_t)l * N + px] = 1;
}

hipError_t launch_sample_scatter(const LaunchCtx &lc, const int32_t *label, const int32_t *pix,
                                 int64_t M, int L, int H, int W, const float *rgb,
                                 const uint64_t *masks, int k, const int32_t *block_counts,
                                 int nblocks, SampleRec *recs, uint8_t *seeds) {
    hipLaunchKernelGGL(k_sample_scatter, dim3(nblocks), dim3(kChunk), 0, lc.stream, label, pix, M, L,
                       H, W, rgb, masks, k, block_counts, nblocks, recs, seeds);
    return hipGetLastError();
}

__global__ void k_fill_u32(unsigned int *p, size_t count, unsigned int v) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = v;
}

// 16 bytes per thread and step; the last count % 16 bytes by the first threads
__global__ void k_fill_u8x16(uint4 *p, size_t count16, unsigned int v4, int rem) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (size_t i = t; i < count16; i += stride) p[i] = make_uint4(v4, v4, v4, v4);
    if (t < (size_t)rem) reinterpret_cast<uint8_t *>(p + count16)[t] = (uint8_t)v4;
}

hipError_t launch_fill_u32(const LaunchCtx &lc, unsigned int *p, size_t count, unsigned int v) {
    if (!count) return hipSuccess;
    size_t blocks = (count + 255) / 256;
    if (blocks > (size_t)lc.num_cu * 8) blocks = (size_t)lc.num_cu * 8;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, lc.stream, p, count, v);
    return hipGetLastError();
}

// p must be 16-byte aligned (workspace allocations are).
hipError_t launch_fill_u8(const LaunchCtx &lc, uint8_t *p, size_t count, uint8_t v) {
    if (!count) return hipSuccess;
    const unsigned int v4 = 0x01010101u * v;
    const size_t c16 = count / 16;
    size_t blocks = (c16 + 255) / 256;
    if (blocks > (size_t)lc.num_cu * 8) blocks = (size_t)lc.num_cu * 8;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_fill_u8x16, dim3((unsigned)blocks), dim3(256), 0, lc.stream, reinterpret_cast<uint4 *>(p),
                       c16, v4, (int)(count - c16 * 16));
    return hipGetLastError();
}

}  // namespace cs

namespace cs {

// Range check of a caller-supplied pixel list: flags[b] = 1 where workgroup b
// saw a pixel out of range (else 0).
__global__ __launch_bounds__(256) void k_check_pix(const int32_t *pix, int64_t n, int64_t N, int32_t *flags) {
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int32_t v = pix[i];
        if (v < 0 || (int64_t)v >= N) bad = 1;
    }
    __syncthreads();
    if (threadIdx.x == 0) flags[blockIdx.x] = bad;
}

int check_pix_blocks(const LaunchCtx &lc, int64_t n) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > (int64_t)lc.num_cu * 8) blocks = (int64_t)lc.num_cu * 8;
    return (int)blocks;
}

hipError_t launch_check_pix(const LaunchCtx &lc, const int32_t *pix, int64_t n, int64_t N, int32_t *flags) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_check_pix, dim3((unsigned)check_pix_blocks(lc, n)), dim3(256), 0, lc.stream, pix, n, N,
                       flags);
    return hipGetLastError();
}

}  // namespace cs
