// Scribble samples on gfx950 (the sets S_i of Sec. 3.1): validation, a
// stable counting sort by label into contiguous segments, and gathering of
// each sample's position, colour and co-support from its pixel into a 64-byte
// record that a wave reads with one scalar load.  Also marks the samples of
// each label in a per-label seed plane for the distance transform.
#include "cs_internal.h"

namespace cs {

constexpr int kChunk = 256;

// Exclusive scan of block_counts in label-major order (in place), the label
// totals and the flags (bit 0: a bad sample, bit 1: a bad pixel of the list),
// by one workgroup (any power-of-two size up to 1024).  Also clears `nzero`
// words of counters for the kernels that follow, and hands totals and flags
// to the host: written to host memory (host_out[0..L]) and, after a
// system-scope fence, host_out[kHostTag] = tag.
__device__ void sample_scan(int32_t *block_counts, int L, int nblocks, const int32_t *block_flags,
                            const int32_t *pix_flags, int npix_blocks, int32_t *totals_flags, unsigned int *zero,
                            int nzero, unsigned int *zero2, int nzero2, volatile int32_t *host_out,
                            int32_t tag) {
    __shared__ int32_t buf[1024];
    __shared__ int32_t carry, sflags;
    __shared__ int32_t tot[kMaxLabels];
    const int B = blockDim.x, tid = threadIdx.x;
    const int64_t total = (int64_t)L * nblocks;
    if (tid == 0) {
        carry = 0;
        sflags = 0;
    }
    for (int i = tid; i < kMaxLabels; i += B) tot[i] = 0;
    for (int i = tid; i < nzero; i += B) zero[i] = 0u;
    for (int i = tid; i < nzero2; i += B) zero2[i] = 0u;
    __syncthreads();
    int32_t f = 0;
    for (int i = tid; i < nblocks; i += B) f |= block_flags[i] ? 1 : 0;
    for (int i = tid; i < npix_blocks; i += B) f |= pix_flags[i] ? 2 : 0;
    if (f) atomicOr(&sflags, f);
    for (int64_t base = 0; base < total; base += B) {
        const int64_t i = base + tid;
        const int32_t v = i < total ? block_counts[i] : 0;
        if (i < total) atomicAdd(&tot[i / nblocks], v);
        buf[tid] = v;
        __syncthreads();
        for (int off = 1; off < B; off <<= 1) {  // Hillis-Steele inclusive scan
            int32_t t = tid >= off ? buf[tid - off] : 0;
            __syncthreads();
            buf[tid] += t;
            __syncthreads();
        }
        if (i < total) block_counts[i] = carry + buf[tid] - v;
        __syncthreads();
        if (tid == B - 1) carry += buf[B - 1];
        __syncthreads();
    }
    for (int l = tid; l <= L; l += B) {
        const int32_t v = l < L ? tot[l] : sflags;
        totals_flags[l] = v;
        host_out[l] = v;
    }
    __threadfence_system();
    __syncthreads();
    if (tid == 0) host_out[kHostTag] = tag;
}

// Per-chunk label counts (label-major: block_counts[l * nblocks + b]); a chunk
// with a bad label or pixel sets block_flags[b] = 1 (else 0).  The last
// counting workgroup to finish (a device counter, zero between calls, reset
// by that workgroup) runs the scan.  Workgroups past nblocks clear the
// per-label seed plane (nseed16 16-byte words) instead.
__global__ __launch_bounds__(kChunk) void k_sample_count(SampleCountArgs a) {
    if ((int)blockIdx.x >= a.nblocks) {
        const int64_t stride = (int64_t)a.nclear * kChunk;
        for (int64_t i = (int64_t)(blockIdx.x - a.nblocks) * kChunk + threadIdx.x; i < a.nseed16; i += stride)
            a.seeds16[i] = make_uint4(0u, 0u, 0u, 0u);
        return;
    }
    __shared__ int cnt[kMaxLabels];
    __shared__ int bad, s_last;
    if (threadIdx.x < kMaxLabels) cnt[threadIdx.x] = 0;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    const int64_t idx = (int64_t)blockIdx.x * kChunk + threadIdx.x;
    if (idx < a.M) {
        const int l = a.label[idx];
        const int32_t px = a.pix[idx];
        if (l < 0 || l >= a.L || px < 0 || (int64_t)px >= a.N)
            bad = 1;
        else
            atomicAdd(&cnt[l], 1);
    }
    __syncthreads();
    if (threadIdx.x < a.L) a.block_counts[(int64_t)threadIdx.x * a.nblocks + blockIdx.x] = cnt[threadIdx.x];
    if (threadIdx.x == 0) a.block_flags[blockIdx.x] = bad;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();  // this workgroup's counts before its done count
        s_last = atomicAdd(a.done, 1u) == (unsigned int)a.nblocks - 1u;
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();  // every workgroup's counts
    if (threadIdx.x == 0) *a.done = 0u;
    sample_scan(a.block_counts, a.L, a.nblocks, a.block_flags, a.pix_flags, a.npix_blocks, a.totals_flags, a.zero,
                a.nzero, a.zero2, a.nzero2, a.host_out, a.tag);
}

hipError_t launch_sample_count(const LaunchCtx &lc, SampleCountArgs a, uint8_t *seeds, size_t seed_bytes) {
    // the seed plane is a multiple of 16 bytes (its caller pads it)
    a.seeds16 = reinterpret_cast<uint4 *>(seeds);
    a.nseed16 = (int64_t)(seed_bytes / 16);
    int64_t nclear = (a.nseed16 + kChunk - 1) / kChunk;
    if (nclear > (int64_t)lc.num_cu * 4) nclear = (int64_t)lc.num_cu * 4;
    a.nclear = (int)nclear;
    hipLaunchKernelGGL(k_sample_count, dim3((unsigned)(a.nblocks + nclear)), dim3(kChunk), 0, lc.stream, a);
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


hipError_t launch_fill_u32(const LaunchCtx &lc, unsigned int *p, size_t count, unsigned int v) {
    if (!count) return hipSuccess;
    size_t blocks = (count + 255) / 256;
    if (blocks > (size_t)lc.num_cu * 8) blocks = (size_t)lc.num_cu * 8;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, lc.stream, p, count, v);
    return hipGetLastError();
}


// Finite check of an input array: any NaN or infinity sets bit 0 of *flag;
// with levels n > 0 a finite value farther than 1e-4 / n from a multiple q / n
// with q in 0..255 sets bit 1.  Grid-stride loop, one float per thread and step.
__global__ __launch_bounds__(256) void k_check_finite(const float *p, int64_t n, int levels, unsigned int *flag) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    bool bad = false, off = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float v = p[i];
        const uint32_t b = __float_as_uint(v);
        const bool nf = (b & 0x7f800000u) == 0x7f800000u;  // exponent all ones: NaN or infinity
        bad |= nf;
        if (levels > 0 && !nf) {
            const float x = v * (float)levels, q = rintf(x);
            off |= !(q >= 0.0f && q <= 255.0f && fabsf(x - q) <= 1e-4f);
        }
    }
    const unsigned int f = (bad ? 1u : 0u) | (off ? 2u : 0u);
    if (f) atomicOr(flag, f);
}

hipError_t launch_check_finite(const LaunchCtx &lc, const float *p, int64_t n, int levels, unsigned int *flag) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > (int64_t)lc.num_cu * 8) blocks = (int64_t)lc.num_cu * 8;
    hipLaunchKernelGGL(k_check_finite, dim3((unsigned)blocks), dim3(256), 0, lc.stream, p, n, levels, flag);
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
