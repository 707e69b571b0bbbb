// Exact squared Euclidean distance from every pixel to the nearest scribble
// sample of each label, with the identity of that sample, on gfx950.  This is
// the |x - x_{v_i}| that sets the spatial bandwidth rho_i(x) in Sec. 3.1.
//
// Separable transform on integer distances (exact):
//  1. columns: the rows of every column are cut into short segments; a first
//     kernel records the first and last seed row of each segment, a second one
//     carries the nearest seed rows from the other segments in and scans its
//     own segment both ways (lanes own adjacent columns, so loads coalesce);
//  2. rows: one workgroup per (label, row) stages f(q) = squared column
//     distance of every column q in LDS, and the smallest f over blocks of 16
//     columns; each thread owns columns c and walks outward block by block,
//     keeping the best (c - q)^2 + f(q).  A block is scanned only when its
//     nearest column and its smallest f could still beat the best, and the walk
//     stops once the nearest column of the next blocks is at least that far.
#include "cs_internal.h"

namespace cs {

constexpr int kSegRows = 16;
constexpr int kNoSeed = -1;
constexpr int kRowBlk = 16;  // columns per block of the row pass
constexpr int32_t kInf = 0x3FFFFFFF;

// Per (label, segment, column): first and last seed row inside the segment.
__global__ __launch_bounds__(64) void k_edt_col_summary(const uint8_t *seeds, int H, int W,
                                                         int nseg, int32_t *first, int32_t *last) {
    const int c = blockIdx.x * 64 + threadIdx.x;
    const int seg = blockIdx.y, l = blockIdx.z;
    if (c >= W) return;
    const int64_t N = (int64_t)H * W;
    const uint8_t *sd = seeds + (int64_t)l * N + c;
    const int r0 = seg * kSegRows, r1 = min(H, r0 + kSegRows);
    int f = kNoSeed, la = kNoSeed;
#pragma unroll 4
    for (int r = r0; r < r1; ++r) {
        if (sd[(int64_t)r * W]) {
            if (f < 0) f = r;
            la = r;
        }
    }
    const int64_t o = ((int64_t)l * nseg + seg) * W + c;
    first[o] = f;
    last[o] = la;
}

// Nearest seed row in the column for every pixel of the segment.
__global__ __launch_bounds__(64) void k_edt_col_fill(const uint8_t *seeds, int H, int W, int nseg,
                                                      const int32_t *first, const int32_t *last,
                                                      int32_t *colrow) {
    const int c = blockIdx.x * 64 + threadIdx.x;
    const int seg = blockIdx.y, l = blockIdx.z;
    if (c >= W) return;
    const int64_t N = (int64_t)H * W;
    const int64_t sbase = (int64_t)l * nseg * W + c;
    int above = kNoSeed;  // last seed row in the segments above
    for (int s = seg - 1; s >= 0; --s) {
        const int v = last[sbase + (int64_t)s * W];
        if (v >= 0) {
            above = v;
            break;
        }
    }
    int below = kNoSeed;  // first seed row in the segments below
    for (int s = seg + 1; s < nseg; ++s) {
        const int v = first[sbase + (int64_t)s * W];
        if (v >= 0) {
            below = v;
            break;
        }
    }
    const uint8_t *sd = seeds + (int64_t)l * N + c;
    int32_t *cr = colrow + (int64_t)l * N + c;
    const int r0 = seg * kSegRows, r1 = min(H, r0 + kSegRows);
    // the segment's seed bytes, loaded unconditionally (rows clamped) so that
    // the loads are in flight together
    bool sv[kSegRows];
#pragma unroll
    for (int i = 0; i < kSegRows; ++i) sv[i] = sd[(int64_t)min(r0 + i, H - 1) * W] != 0;
    int up[kSegRows];
    int lastr = above;
#pragma unroll
    for (int i = 0; i < kSegRows; ++i) {
        const int r = r0 + i;
        if (r < r1 && sv[i]) lastr = r;
        up[i] = lastr;
    }
    int nextr = below;
#pragma unroll
    for (int i = kSegRows - 1; i >= 0; --i) {
        const int r = r0 + i;
        if (r >= r1) continue;
        if (sv[i]) nextr = r;
        const int a = up[i];
        int best = a;
        if (nextr >= 0 && (a < 0 || nextr - r < r - a)) best = nextr;
        cr[(int64_t)r * W] = best;
    }
}

__global__ __launch_bounds__(1024) void k_edt_rows(const int32_t *colrow, int H, int W,
                                                    int32_t *d2, int32_t *nearest) {
    extern __shared__ int32_t lds[];
    const int nb = (W + kRowBlk - 1) / kRowBlk;
    // f: squared column distance, kInf where the column has no seed, padded to
    // whole blocks with kInf (16-byte aligned: blocks are read as int4)
    int32_t *f = lds;
    int32_t *rowof = lds + nb * kRowBlk;      // nearest seed row of each column
    int32_t *fmin = lds + 2 * nb * kRowBlk;   // smallest f over each block
    const int r = blockIdx.x, l = blockIdx.y;
    const int64_t N = (int64_t)H * W;
    const int32_t *cr = colrow + (int64_t)l * N + (int64_t)r * W;
    for (int c = threadIdx.x; c < nb * kRowBlk; c += blockDim.x) {
        const int q = c < W ? cr[c] : -1;
        rowof[c] = q;
        f[c] = q < 0 ? kInf : (r - q) * (r - q);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        int m = kInf;
        for (int q = b * kRowBlk; q < b * kRowBlk + kRowBlk; ++q) m = min(m, f[q]);
        fmin[b] = m;
    }
    __syncthreads();
    int32_t *dd = d2 + (int64_t)l * N + (int64_t)r * W;
    int32_t *nn = nearest + (int64_t)l * N + (int64_t)r * W;
    for (int c = threadIdx.x; c < W; c += blockDim.x) {
        // The walk keeps only the smallest value and the block that first
        // reached it (strict improvement); the column is found afterwards in
        // that block, the first in ascending order with the smallest value.
        // Ties go as in a one-by-one scan: the own column first, then the
        // blocks in walk order, then ascending columns.
        int best = f[c], bb = -1;
        auto scan = [&](int b) {
            const int4 *f4 = reinterpret_cast<const int4 *>(f + b * kRowBlk);
            const int4 v0 = f4[0], v1 = f4[1], v2 = f4[2], v3 = f4[3];
            const int fv[16] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w,
                                v2.x, v2.y, v2.z, v2.w, v3.x, v3.y, v3.z, v3.w};
            int m = best;
#pragma unroll
            for (int i = 0; i < kRowBlk; ++i) {
                const int d = c - (b * kRowBlk + i);
                m = min(m, __mul24(d, d) + fv[i]);
            }
            if (m < best) {
                best = m;
                bb = b;
            }
        };
        const int cb = c / kRowBlk;
        scan(cb);  // own block, every column
        // blocks outward on both sides; a block is scanned only if its
        // nearest column and smallest f could beat the best so far, and the
        // walk stops once the nearest column of the next blocks is too far
        for (int db = 1;; ++db) {
            const int bl = cb - db, br = cb + db;
            const int gl = c - (bl * kRowBlk + kRowBlk - 1);  // distance to the left block's last column
            const int gr = br * kRowBlk - c;                     // distance to the right block's first column
            const bool lok = bl >= 0 && gl * gl < best;
            const bool rok = br < nb && gr * gr < best;
            if (!lok && !rok) break;
            if (lok && gl * gl + fmin[bl] < best) scan(bl);
            if (rok && gr * gr + fmin[br] < best) scan(br);
        }
        int bq = c;
        if (bb >= 0) {
            for (int i = kRowBlk - 1; i >= 0; --i) {
                const int q = bb * kRowBlk + i, d = c - q;
                if (__mul24(d, d) + f[q] == best) bq = q;
            }
        }
        if (best >= kInf) {  // no seed of this label anywhere (rejected before launch)
            dd[c] = -1;
            nn[c] = -1;
        } else {
            dd[c] = best;
            nn[c] = rowof[bq] * W + bq;
        }
    }
}

// Smallest f over each block of kRowBlk columns of every row and label (the
// block minima of k_edt_rows, for the listed form below): one thread per
// (row, block, label).
__global__ __launch_bounds__(256) void k_edt_block_min(const int32_t *colrow, int H, int W, int32_t *bmin) {
    const int nb = (W + kRowBlk - 1) / kRowBlk;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int l = blockIdx.y;
    if (i >= (int64_t)H * nb) return;
    const int r = (int)(i / nb), b = (int)(i - (int64_t)r * nb);
    const int32_t *cr = colrow + (int64_t)l * H * W + (int64_t)r * W;
    int fv[kRowBlk];
#pragma unroll
    for (int u = 0; u < kRowBlk; ++u) {
        const int q = b * kRowBlk + u;
        const int s = q < W ? cr[q] : -1;
        fv[u] = s < 0 ? kInf : (r - s) * (r - s);
    }
    int m = kInf;
#pragma unroll
    for (int u = 0; u < kRowBlk; ++u) m = min(m, fv[u]);
    bmin[(int64_t)l * H * nb + i] = m;
}

// The row pass for listed pixels only, one thread per (entry, label): the
// walk of k_edt_rows for the entry's column, reading f and the block minima
// from global memory instead of LDS (the same blocks are scanned in the same
// order, so the result and its ties are those of k_edt_rows).  Entries
// outside the image are skipped (the host rejects them after the launch).
__global__ __launch_bounds__(256) void k_edt_rows_list(const int32_t *colrow, const int32_t *bmin, int H,
                                                       int W, const int32_t *list, int64_t npix, int32_t *d2,
                                                       int32_t *nearest) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int l = blockIdx.y;
    if (e >= npix) return;
    const int64_t N = (int64_t)H * W;
    const int64_t pix = list[e];
    if (pix < 0 || pix >= N) return;
    const int r = (int)(pix / W), c = (int)(pix - (int64_t)r * W);
    const int nb = (W + kRowBlk - 1) / kRowBlk;
    const int32_t *cr = colrow + (int64_t)l * N + (int64_t)r * W;
    const int32_t *fm = bmin + ((int64_t)l * H + r) * nb;
    auto fval = [&](int q) {
        const int s = cr[q];
        return s < 0 ? kInf : (r - s) * (r - s);
    };
    int best = fval(c), bb = -1;
    auto scan = [&](int b) {
        int fv[kRowBlk];
#pragma unroll
        for (int i = 0; i < kRowBlk; ++i) {
            const int q = b * kRowBlk + i;
            fv[i] = q < W ? fval(q) : kInf;  // the full pass pads with kInf
        }
        int m = best;
#pragma unroll
        for (int i = 0; i < kRowBlk; ++i) {
            const int d = c - (b * kRowBlk + i);
            m = min(m, __mul24(d, d) + fv[i]);
        }
        if (m < best) {
            best = m;
            bb = b;
        }
    };
    const int cb = c / kRowBlk;
    scan(cb);
    for (int db = 1;; ++db) {
        const int bl = cb - db, br = cb + db;
        const int gl = c - (bl * kRowBlk + kRowBlk - 1);
        const int gr = br * kRowBlk - c;
        const bool lok = bl >= 0 && gl * gl < best;
        const bool rok = br < nb && gr * gr < best;
        if (!lok && !rok) break;
        const int ml = lok ? fm[bl] : kInf, mr = rok ? fm[br] : kInf;
        if (lok && gl * gl + ml < best) scan(bl);
        if (rok && gr * gr + mr < best) scan(br);
    }
    int bq = c;
    if (bb >= 0) {
        for (int i = kRowBlk - 1; i >= 0; --i) {
            const int q = bb * kRowBlk + i, d = c - q;
            if (q < W && __mul24(d, d) + fval(q) == best) bq = q;
        }
    }
    const int64_t o = (int64_t)l * N + pix;
    if (best >= kInf) {
        d2[o] = -1;
        nearest[o] = -1;
    } else {
        d2[o] = best;
        nearest[o] = cr[bq] * W + bq;
    }
}

// Scratch: first/last summaries, 2 * L * ceil(H/16) * W int32, then (listed
// form) the block minima, L * H * ceil(W/16) int32.
size_t edt_scratch_bytes(int H, int W, int L) {
    const int nseg = (H + kSegRows - 1) / kSegRows;
    const size_t nb = (size_t)(W + kRowBlk - 1) / kRowBlk;
    const size_t summaries = 2 * (size_t)L * nseg * W, minima = (size_t)L * H * nb;
    return sizeof(int32_t) * (summaries > minima ? summaries : minima);
}

hipError_t launch_edt(const LaunchCtx &lc, const uint8_t *seeds, int H, int W, int L,
                      int32_t *colrow, int32_t *d2, int32_t *nearest, int32_t *scratch,
                      const int32_t *list, int64_t npix) {
    const int nseg = (H + kSegRows - 1) / kSegRows;
    int32_t *first = scratch, *last = scratch + (size_t)L * nseg * W;
    dim3 g1((W + 63) / 64, nseg, L);
    hipLaunchKernelGGL(k_edt_col_summary, g1, dim3(64), 0, lc.stream, seeds, H, W, nseg, first, last);
    hipLaunchKernelGGL(k_edt_col_fill, g1, dim3(64), 0, lc.stream, seeds, H, W, nseg, first, last,
                       colrow);
    // a short list (at most an eighth of the pixels) takes the per-entry row
    // pass; longer ones the full pass, whose rows share their staging
    if (list && npix * 8 <= (int64_t)H * W) {
        if (npix == 0) return hipGetLastError();
        // block minima into the scratch (the column summaries are dead by now)
        const int64_t nbr = (int64_t)H * ((W + kRowBlk - 1) / kRowBlk);
        hipLaunchKernelGGL(k_edt_block_min, dim3((unsigned)((nbr + 255) / 256), L), dim3(256), 0, lc.stream,
                           colrow, H, W, scratch);
        hipLaunchKernelGGL(k_edt_rows_list, dim3((unsigned)((npix + 255) / 256), L), dim3(256), 0, lc.stream,
                           colrow, scratch, H, W, list, npix, d2, nearest);
        return hipGetLastError();
    }
    const size_t nbk = (size_t)(W + kRowBlk - 1) / kRowBlk;
    const size_t lds = sizeof(int32_t) * (2 * nbk * kRowBlk + nbk);
    hipError_t e = hipFuncSetAttribute((const void *)k_edt_rows,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    int threads = (W + 63) / 64 * 64;
    if (threads > 1024) threads = 1024;
    hipLaunchKernelGGL(k_edt_rows, dim3(H, L), dim3(threads), lds, lc.stream, colrow, H, W, d2, nearest);
    return hipGetLastError();
}

}  // namespace cs
