// Exact selection of the co-support threshold tau = frac * median|a| on
// gfx950.  The threshold stands in for the exact-zero test of the Sec. 2
// co-support definition; the median is the lower median over all N*k entries
// of the FP64 analysed vectors.
//
// 1. Radix select (11/11/10-bit digits, LDS-privatised histograms) finds the
//    float value v of the target rank among the rounded |a| (the |a| bit
//    patterns order like unsigned integers).
// 2. Every rounded |a| is within the proven margin m of its exact value, so
//    the exact median lies in [v - m, v + m]; entries whose rounded value lies
//    in [v - 2m, v + 2m] are gathered as candidates and the entries below that
//    window are counted.
// 3. The candidates are recomputed in FP64 (same operation order as the
//    oracle's patch and product) and a single-workgroup radix select over their
//    64-bit patterns picks the rank that remains after the count below.  The
//    whole chain runs without a host round trip; the host reads the result
//    once and retries with a larger candidate buffer if it overflowed.
#pragma clang fp contract(off)

#include "cs_internal.h"
#include "cs_device.h"

namespace cs {

// Clears the selection state and the histogram, and writes the largest
// per-row error bound (the half-width of the candidate window).
__global__ __launch_bounds__(256) void k_tau_init(TauState *st, unsigned long long rank0,
                                                   unsigned int *hist, const float *omega, int k, int n,
                                                   double coef, double *max_margin, double *margins) {
    __shared__ double red[256];
    red[threadIdx.x] = (int)threadIdx.x < k ? row_margin(omega, threadIdx.x, n, -1.0, coef) : 0.0;
    if (margins && (int)threadIdx.x < k) margins[threadIdx.x] = red[threadIdx.x];
    __syncthreads();
    for (int s2 = 128; s2 > 0; s2 >>= 1) {
        if ((int)threadIdx.x < s2) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s2]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *max_margin = red[0];
    if (threadIdx.x == 0) {
        st->rank0 = rank0;
        st->rank = rank0;
        st->prefix = 0;
        st->nparts = 0;
        st->ncand = 0;
        st->n_d = 0;
        st->n_r = 0;
        st->lo = st->hi = 0.0;
        st->median = 0.0;
        st->tau = 0.0;
    }
    for (int i = threadIdx.x; i < kHistBins; i += 256) hist[i] = 0;
}

// Histogram of one 11-bit digit of the |a| bit patterns that match the
// prefix selected so far.  SUB sub-histograms per workgroup (by lane % SUB)
// spread the LDS atomics of lanes that fall into the same few bins (first
// digit); later digits see few matching entries and use one.
// With pick_hist set the workgroup first picks digit pick_d (at pick_shift)
// from that complete histogram, from the state after digit pick_d - 1
// (workgroup 0 records the result for the next kernel).
template <int SUB>
__global__ __launch_bounds__(256) void k_tau_hist(const float *alpha, int64_t count, int shift,
                                                   unsigned int pmask, TauState *st,
                                                   unsigned int *hist, const unsigned int *pick_hist,
                                                   int pick_shift, int pick_d) {
    __shared__ unsigned int lh[SUB * kHistBins];
    unsigned int prefix = st->prefix;
    if (pick_hist) {
        unsigned long long rank;
        tau_pick_digit(pick_hist, pick_shift, st->pfx[pick_d - 1], st->rk[pick_d - 1], prefix, rank);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->pfx[pick_d] = prefix;
            st->rk[pick_d] = rank;
        }
    }
    for (int i = threadIdx.x; i < SUB * kHistBins; i += 256) lh[i] = 0;
    __syncthreads();
    const unsigned int pval = prefix & pmask;
    unsigned int *mine = lh + (threadIdx.x & (SUB - 1)) * kHistBins;
    auto add = [&](float x) {
        const unsigned int key = __float_as_uint(x) & 0x7FFFFFFFu;
        if ((key & pmask) == pval) atomicAdd(&mine[(key >> shift) & (kHistBins - 1)], 1u);
    };
    const int64_t n4 = count / 4;
    const float4 *a4 = reinterpret_cast<const float4 *>(alpha);
    const int64_t stride = (int64_t)gridDim.x * 256;
    int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    // four independent 16-byte loads in flight per thread
    for (; q + 3 * stride < n4; q += 4 * stride) {
        float4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = a4[q + u * stride];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            add(v[u].x);
            add(v[u].y);
            add(v[u].z);
            add(v[u].w);
        }
    }
    for (; q < n4; q += stride) {
        const float4 v = a4[q];
        add(v.x);
        add(v.y);
        add(v.z);
        add(v.w);
    }
    for (int64_t e = n4 * 4 + (int64_t)blockIdx.x * 256 + threadIdx.x; e < count; e += stride) add(alpha[e]);
    __syncthreads();
    for (int i = threadIdx.x; i < kHistBins; i += 256) {
        unsigned int t = 0;
#pragma unroll
        for (int c = 0; c < SUB; ++c) t += lh[c * kHistBins + i];
        if (t) atomicAdd(&hist[i], t);
    }
}

// Pick the digit holding the remaining rank (parallel prefix over the bins),
// then clear the histogram for the next pass.
__global__ __launch_bounds__(256) void k_tau_pick(unsigned int *hist, int shift, TauState *st) {
    constexpr int per = kHistBins / 256;
    __shared__ unsigned long long scan[256];
    const int t = threadIdx.x;
    unsigned int loc[per];
    unsigned long long sum = 0;
#pragma unroll
    for (int i = 0; i < per; ++i) {
        loc[i] = hist[t * per + i];
        sum += loc[i];
    }
    scan[t] = sum;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const unsigned long long v = t >= off ? scan[t - off] : 0ull;
        __syncthreads();
        scan[t] += v;
        __syncthreads();
    }
    const unsigned long long r = st->rank;
    const unsigned long long before = scan[t] - sum;
    __syncthreads();
    if (r >= before && r < scan[t]) {
        unsigned long long rr = r - before;
        for (int i = 0; i < per; ++i) {
            if (rr < loc[i]) {
                st->prefix |= (unsigned int)(t * per + i) << shift;
                st->rank = rr;
                break;
            }
            rr -= loc[i];
        }
    }
    for (int i = 0; i < per; ++i) hist[t * per + i] = 0;
}

hipError_t tau_pick(const LaunchCtx &lc, unsigned int *hist, int shift, TauState *st) {
    hipLaunchKernelGGL(k_tau_pick, dim3(1), dim3(256), 0, lc.stream, hist, shift, st);
    return hipGetLastError();
}

namespace {
unsigned hist_blocks(const LaunchCtx &lc, int64_t count, int per_cu) {
    int64_t b = (count / 4 + 255) / 256;
    const int64_t cap = (int64_t)lc.num_cu * per_cu;
    if (b > cap) b = cap;
    return (unsigned)(b < 1 ? 1 : b);
}
}  // namespace

hipError_t tau_first_digit(const LaunchCtx &lc, const float *alpha, int64_t count, unsigned int *hist,
                           TauState *st, const float *omega, int k, int n, double coef, double *max_margin,
                           double *margins) {
    hipLaunchKernelGGL(k_tau_init, dim3(1), dim3(256), 0, lc.stream, st,
                       (unsigned long long)((count - 1) / 2), hist, omega, k, n, coef, max_margin, margins);
    hipLaunchKernelGGL(k_tau_hist<8>, dim3(hist_blocks(lc, count, 2)), dim3(256), 0, lc.stream, alpha, count, 21,
                       0u, st, hist, nullptr, 0, 0);
    return tau_pick(lc, hist, 21, st);
}

hipError_t tau_select_float(const LaunchCtx &lc, const float *alpha, int64_t count,
                            unsigned int *hist, TauState *st, const float *omega, int k, int n,
                            double coef, double *max_margin, double *margins) {
    hipError_t e = tau_first_digit(lc, alpha, count, hist, st, omega, k, n, coef, max_margin, margins);
    if (e != hipSuccess) return e;
    const int shifts[2] = {10, 0};
    const unsigned int pmasks[2] = {0xFFE00000u, 0xFFFFFC00u};
    for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(k_tau_hist<1>, dim3(hist_blocks(lc, count, 1)), dim3(256), 0, lc.stream, alpha, count,
                           shifts[pass], pmasks[pass], st, hist, nullptr, 0, 0);
        if ((e = tau_pick(lc, hist, shifts[pass], st)) != hipSuccess) return e;
    }
    return hipGetLastError();
}

// The two digit passes of the fused co-support call (the gather that follows
// picks the second digit and gathers over its whole bin instead of a third
// digit pass).
hipError_t tau_digits_folded(const LaunchCtx &lc, const float *alpha, int64_t count, unsigned int *hist3,
                             TauState *st) {
    unsigned int *h1 = hist3, *h2 = hist3 + kHistBins;
    hipLaunchKernelGGL(k_tau_hist<8>, dim3(hist_blocks(lc, count, 2)), dim3(256), 0, lc.stream, alpha, count, 21,
                       0u, st, h1, nullptr, 0, 0);
    hipLaunchKernelGGL(k_tau_hist<1>, dim3(hist_blocks(lc, count, 1)), dim3(256), 0, lc.stream, alpha, count, 10,
                       0xFFE00000u, st, h2, h1, 21, 1);
    return hipGetLastError();
}

__global__ void k_tau_reset(TauState *st) {
    st->nparts = 0;
    st->ncand = 0;
}

hipError_t tau_reset_gather(const LaunchCtx &lc, TauState *st) {
    hipLaunchKernelGGL(k_tau_reset, dim3(1), dim3(1), 0, lc.stream, st);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_tau_gather(const float *alpha, int64_t count,
                                                     const double *max_margin, TauState *st,
                                                     int64_t *cand, int64_t cap, unsigned long long *parts) {
    __shared__ unsigned long long red[256];
    // The three digit passes left the selected float's bit pattern in prefix.
    const double v = (double)__uint_as_float(st->prefix);
    const double w = 2.0 * (*max_margin);
    const double lo = v - w, hi = v + w;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->lo = lo;
        st->hi = hi;
    }
    // The same tests on the float |a| bit patterns: x >= lo <=> x >= flo (the
    // smallest float >= lo), x <= hi <=> x <= fhi (the largest float <= hi);
    // non-negative floats order like their bit patterns.
    float flo = (float)lo, fhi = (float)hi;
    if ((double)flo < lo) flo = nextafterf(flo, INFINITY);
    if ((double)fhi > hi) fhi = nextafterf(fhi, -INFINITY);
    const unsigned int blo = lo <= 0.0 ? 0u : __float_as_uint(flo);
    const unsigned int bhi = __float_as_uint(fhi);
    unsigned long long below = 0;
    const int64_t stride = (int64_t)gridDim.x * 256;
    const int64_t n4 = count / 4;
    const float4 *a4 = reinterpret_cast<const float4 *>(alpha);
    // one atomic per wave: lanes with a candidate take consecutive slots
    auto visit = [&](float xv, bool live, int64_t e) {
        const unsigned int x = __float_as_uint(xv) & 0x7FFFFFFFu;
        below += (live && x < blo) ? 1ull : 0ull;
        const bool in = live && x >= blo && x <= bhi;
        const unsigned long long m = __ballot(in);
        if (m) {
            const int lane = threadIdx.x & 63;
            unsigned long long base = 0;
            if (lane == __ffsll((long long)m) - 1) base = atomicAdd(&st->ncand, (unsigned long long)__popcll(m));
            base = __shfl(base, __ffsll((long long)m) - 1);
            if (in) {
                const unsigned long long slot = base + __popcll(m & ((1ull << lane) - 1ull));
                if ((int64_t)slot < cap) cand[slot] = e;
            }
        }
    };
    int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    // four independent 16-byte loads in flight per thread (the trip count is
    // the same for all lanes of a wave up to the last round, which the
    // single-load loop below finishes)
    for (; q + 3 * stride < n4; q += 4 * stride) {
        float4 f[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) f[u] = a4[q + u * stride];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t e = (q + u * stride) * 4;
            visit(f[u].x, true, e);
            visit(f[u].y, true, e + 1);
            visit(f[u].z, true, e + 2);
            visit(f[u].w, true, e + 3);
        }
    }
    for (; q < n4 + 1; q += stride) {
        float vv[4] = {0.f, 0.f, 0.f, 0.f};
        int cnt = 4;
        if (q < n4) {
            const float4 f = a4[q];
            vv[0] = f.x; vv[1] = f.y; vv[2] = f.z; vv[3] = f.w;
        } else {
            cnt = (int)(count - n4 * 4);
            for (int u = 0; u < cnt; ++u) vv[u] = alpha[n4 * 4 + u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) visit(vv[u], u < cnt, q * 4 + u);
    }
    red[threadIdx.x] = below;
    __syncthreads();
    for (int s2 = 128; s2 > 0; s2 >>= 1) {
        if (threadIdx.x < s2) red[threadIdx.x] += red[threadIdx.x + s2];
        __syncthreads();
    }
    if (threadIdx.x == 0) parts[blockIdx.x] = red[0];
    if (blockIdx.x == 0 && threadIdx.x == 0) st->nparts = gridDim.x;
}

hipError_t tau_gather(const LaunchCtx &lc, const float *alpha, int64_t count,
                      const double *max_margin, TauState *st, int64_t *cand, int64_t cap,
                      unsigned long long *parts) {
    int64_t blocks = (count / 4 + 256) / 256;
    int64_t bcap = (int64_t)lc.num_cu * 4;
    if (bcap > kTauParts) bcap = kTauParts;
    if (blocks > bcap) blocks = bcap;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_tau_gather, dim3((unsigned)blocks), dim3(256), 0, lc.stream, alpha, count,
                       max_margin, st, cand, cap, parts);
    return hipGetLastError();
}

// FP64 recompute of each candidate entry e = pixel * k + j, one lane per
// candidate (exact_entry: every sum sequential in t, so the result is the
// bit pattern of the oracle's evaluation).  Persistent waves read the
// candidate count from the device state (no host round trip); counts beyond
// the capacity are left to the host's retry.
__global__ __launch_bounds__(64) void k_tau_recompute(const float *rgb, int H, int W, int p,
                                                       const double *wmask, const float *omega,
                                                       int k, const int64_t *cand, const TauState *st,
                                                       int64_t cap, double *vals, const double *pstats,
                                                       const unsigned int *ccnt, const unsigned long long *coff,
                                                       const int64_t *ccomp) {
    const int n = p * p;
    const int64_t stride = (int64_t)gridDim.x * 64;
    if (ccnt && (int64_t)st->ncand > kListCap) {
        // per-wave regions of the fused gather (a list too long to compact):
        // lane = region, its values written at the region's offset
        const int64_t nw = (int64_t)st->rg_waves, region = (int64_t)st->rg_size;
        for (int64_t r = (int64_t)blockIdx.x * 64 + threadIdx.x; r < nw; r += stride) {
            const unsigned int cnt = ccnt[r];
            const int64_t *src = cand + r * region;
            double *dst = vals + coff[r];
            for (unsigned int q = 0; q < cnt; ++q) {
                const int64_t e = src[q];
                const int64_t pix = e / k;
                const int j = (int)(e - pix * k);
                dst[q] = fabs(exact_entry(rgb, H, W, p, wmask, omega + (int64_t)j * n, pix, pstats));
            }
        }
        return;
    }
    // compact list: the fused gather's in ccomp (see k_list_compact), else cand
    const int64_t *lst = ccnt ? ccomp : cand;
    const unsigned long long nc = st->ncand;
    const int64_t ncand = (int64_t)nc < cap ? (int64_t)nc : cap;
    for (int64_t c = (int64_t)blockIdx.x * 64 + threadIdx.x; c < ncand; c += stride) {
        const int64_t e = lst[c];
        const int64_t pix = e / k;
        const int j = (int)(e - pix * k);
        vals[c] = fabs(exact_entry(rgb, H, W, p, wmask, omega + (int64_t)j * n, pix, pstats));
    }
}

// Offsets of the fused gather's per-wave regions in the compact lists
// (exclusive scans of their candidate and undecided-entry counts) and the two
// totals.  One workgroup per chunk of kScanChunk counts: it first adds up the
// counts of the chunks before its own (eight 16-byte loads per thread in
// flight, four of each count array),
// then scans its chunk through LDS (coalesced loads, each thread scanning 8
// consecutive counts); the last workgroup writes the totals.  (One workgroup
// walking every chunk in turn took 0.22 ms at 2048 x 2048.)
constexpr int kScanChunk = 8192;
__global__ __launch_bounds__(1024) void k_list_scan(const unsigned int *ccnt, const unsigned int *dcnt,
                                                    TauState *st, unsigned long long *coff,
                                                    unsigned long long *doff) {
    __shared__ unsigned int lc[kScanChunk], ld[kScanChunk];
    __shared__ unsigned long long s[2][1024];
    __shared__ unsigned long long s_carry[2];
    const int nw = (int)st->rg_waves;
    const int t = threadIdx.x;
    const int base = blockIdx.x * kScanChunk;
    if (base >= nw) return;  // workgroup-uniform
    // counts of the chunks before this one, four per 16-byte load (base is a
    // multiple of kScanChunk, the arrays 256-byte aligned)
    unsigned long long pc = 0, pd = 0;
    const uint4 *c4 = reinterpret_cast<const uint4 *>(ccnt), *d4 = reinterpret_cast<const uint4 *>(dcnt);
    for (int i0 = 0; i0 < base / 4; i0 += 4 * 1024) {
        uint4 vc[4], vd[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int r = i0 + u * 1024 + t;
            vc[u] = r < base / 4 ? c4[r] : make_uint4(0u, 0u, 0u, 0u);
            vd[u] = r < base / 4 ? d4[r] : make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            pc += (unsigned long long)vc[u].x + vc[u].y + vc[u].z + vc[u].w;
            pd += (unsigned long long)vd[u].x + vd[u].y + vd[u].z + vd[u].w;
        }
    }
    if (t == 0) s_carry[0] = s_carry[1] = 0ull;
    for (int i = t; i < kScanChunk; i += 1024) {
        const int r = base + i;
        lc[i] = r < nw ? ccnt[r] : 0u;
        ld[i] = r < nw ? dcnt[r] : 0u;
    }
    __syncthreads();
    if (pc) atomicAdd(&s_carry[0], pc);
    if (pd) atomicAdd(&s_carry[1], pd);
    unsigned long long sc = 0, sd = 0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        sc += lc[8 * t + u];
        sd += ld[8 * t + u];
    }
    s[0][t] = sc;
    s[1][t] = sd;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const unsigned long long vc = t >= off ? s[0][t - off] : 0ull, vd = t >= off ? s[1][t - off] : 0ull;
        __syncthreads();
        s[0][t] += vc;
        s[1][t] += vd;
        __syncthreads();
    }
    const unsigned long long carry_c = s_carry[0], carry_d = s_carry[1];
    unsigned long long bc = carry_c + s[0][t] - sc, bd = carry_d + s[1][t] - sd;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int r = base + 8 * t + u;
        if (r < nw) {
            coff[r] = bc;
            doff[r] = bd;
        }
        bc += lc[8 * t + u];
        bd += ld[8 * t + u];
    }
    if (t == 0 && base + kScanChunk >= nw) {
        st->ncand = carry_c + s[0][1023];
        st->n_d = carry_d + s[1][1023];
    }
}

// Both lists of the fused gather into compact form (lane = region), each only
// when its total fits kListCap; otherwise its consumer walks the regions.
__global__ __launch_bounds__(64) void k_list_compact(const int64_t *cand, const unsigned int *ccnt,
                                                     const unsigned long long *coff, const int64_t *didx,
                                                     const unsigned int *dcnt, const unsigned long long *doff,
                                                     const TauState *st, int64_t *ccomp, int64_t *dcomp) {
    const int64_t nw = (int64_t)st->rg_waves, region = (int64_t)st->rg_size;
    const bool cfit = (int64_t)st->ncand <= kListCap, dfit = (int64_t)st->n_d <= kListCap;
    for (int64_t r = (int64_t)blockIdx.x * 64 + threadIdx.x; r < nw; r += (int64_t)gridDim.x * 64) {
        if (cfit) {
            const unsigned int n = ccnt[r];
            const int64_t *src = cand + r * region;
            int64_t *dst = ccomp + coff[r];
            for (unsigned int q = 0; q < n; ++q) dst[q] = src[q];
        }
        if (dfit) {
            const unsigned int n = dcnt[r];
            const int64_t *src = didx + r * region;
            int64_t *dst = dcomp + doff[r];
            for (unsigned int q = 0; q < n; ++q) dst[q] = src[q];
        }
    }
}

// Short candidate lists (up to kRankMax): the rank of every candidate by
// comparison with all of them, one wave per candidate (lanes split the list),
// stored as (less, equal) for the selection below.  Longer lists are left to
// its radix select.
constexpr int kRankMax = kTauRank;
__global__ __launch_bounds__(64) void k_tau_rank(const double *vals, int64_t cap, const TauState *st,
                                                  unsigned long long *rk) {
    const unsigned long long nc = st->ncand;
    if (nc > (unsigned long long)kRankMax || nc > (unsigned long long)cap) return;
    const int64_t n = (int64_t)nc;
    const int lane = threadIdx.x;
    for (int64_t c = blockIdx.x; c < n; c += gridDim.x) {
        const unsigned long long key = (unsigned long long)__double_as_longlong(vals[c]);
        unsigned int less = 0, equal = 0;
        for (int64_t q = lane; q < n; q += 64) {
            const unsigned long long o = (unsigned long long)__double_as_longlong(vals[q]);
            less += o < key ? 1u : 0u;
            equal += o == key ? 1u : 0u;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            less += __shfl_xor(less, off);
            equal += __shfl_xor(equal, off);
        }
        if (lane == 0) rk[c] = (unsigned long long)less | ((unsigned long long)equal << 32);
    }
}

// Single-workgroup radix select of rank (rank0 - below) among the FP64
// candidate values (non-negative doubles order like their bit patterns).
// The digits above the highest bit in which the smallest and largest key
// differ are common to all candidates and skipped; the remaining digits are
// selected 8 bits at a time with an LDS histogram and a one-wave scan.
constexpr int kSelLds = 4096;  // candidates kept in LDS for the last digits
__global__ __launch_bounds__(1024) void k_tau_select(const double *vals, int64_t cap, double frac,
                                                      TauState *st, const unsigned long long *parts,
                                                      const unsigned long long *rk, double *tau_out) {
    __shared__ unsigned int hist[256];
    __shared__ unsigned long long s_min, s_max, s_prefix, s_rank, s_below;
    // the candidates left after a digit, once few enough: the later digits
    // read them here instead of passing over all candidates again
    __shared__ unsigned long long s_keys[kSelLds];
    __shared__ unsigned int s_left, s_nkeys;
    const int tid = threadIdx.x;
    // entries below the candidate window: the gather's per-workgroup counts
    if (tid == 0) s_below = 0;
    __syncthreads();
    unsigned long long pb = 0;
    const int np = (int)st->nparts;
    for (int i0 = 0; i0 < np; i0 += 8 * 1024) {
        unsigned long long pv8[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + u * 1024 + tid;
            pv8[u] = i < np ? parts[i] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) pb += pv8[u];
    }
    if (pb) atomicAdd(&s_below, pb);
    __syncthreads();
    const unsigned long long nc = st->ncand;
    const unsigned long long r0 = st->rank0, below = s_below;
    if (tid == 0) st->below = below;
    const bool ok = nc <= (unsigned long long)cap && r0 >= below && r0 - below < nc;
    if (!ok) {
        if (tid == 0) {
            st->median = __longlong_as_double(0x7FF8000000000000ll);  // NaN: retry or bound violated
            st->tau = st->median;
            if (tau_out) *tau_out = st->median;
        }
        return;
    }
    const int64_t ncand = (int64_t)nc;
    if (ncand <= kRankMax) {
        // ranked by k_tau_rank: the candidate whose rank range [less, less +
        // equal) holds the target (equal keys give the same value)
        const unsigned long long r = r0 - below;
        for (int64_t c = tid; c < ncand; c += 1024) {
            const unsigned long long v = rk[c];
            const unsigned long long less = v & 0xFFFFFFFFull, equal = v >> 32;
            if (r >= less && r < less + equal) {
                const double med = vals[c];
                st->median = med;
                st->tau = frac * med;
                if (tau_out) *tau_out = frac * med;
            }
        }
        return;
    }
    if (tid == 0) {
        s_min = ~0ull;
        s_max = 0ull;
        s_rank = r0 - below;
    }
    __syncthreads();
    // the candidate values are read eight per thread at a time (loads in flight
    // together): 8 x 1024 consecutive values per block of the loops below
    auto keys8 = [&](int64_t c0, unsigned long long (&kv)[8], bool (&ok)[8]) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t c = c0 + (int64_t)u * 1024 + tid;
            ok[u] = c < ncand;
            kv[u] = (unsigned long long)__double_as_longlong(vals[ok[u] ? c : 0]);
        }
    };
    unsigned long long mn = ~0ull, mx = 0ull;
    for (int64_t c0 = 0; c0 < ncand; c0 += 8 * 1024) {
        unsigned long long kv[8];
        bool ok[8];
        keys8(c0, kv, ok);
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (ok[u]) {
                mn = kv[u] < mn ? kv[u] : mn;
                mx = kv[u] > mx ? kv[u] : mx;
            }
    }
    atomicMin(&s_min, mn);
    atomicMax(&s_max, mx);
    __syncthreads();
    const unsigned long long diff = s_min ^ s_max;
    if (diff == 0ull) {
        if (tid == 0) {
            const double med = __longlong_as_double((long long)s_min);
            st->median = med;
            st->tau = frac * med;
            if (tau_out) *tau_out = frac * med;
        }
        return;
    }
    // digits of 8 bits from the highest bit in which the keys differ down
    // (the last one narrower), so that the first pass spreads the keys over
    // all 256 bins (a first digit of a few live bits would put every key into
    // a few bins, whose LDS atomics then serialise)
    const int top = 63 - __clzll((long long)diff);
    if (tid == 0) s_prefix = top + 1 >= 64 ? 0ull : (s_min & (~0ull << (top + 1)));
    __syncthreads();
    bool in_lds = false;  // the keys left are in s_keys (workgroup-uniform)
    for (int hi = top; hi >= 0;) {
        const int width = hi + 1 >= 8 ? 8 : hi + 1;
        const int shift = hi + 1 - width;
        if (tid < 256) hist[tid] = 0;
        __syncthreads();
        const unsigned long long hmask = shift + width >= 64 ? 0ull : (~0ull << (shift + width));
        const unsigned long long dmask = (1ull << width) - 1ull;
        const unsigned long long pv = s_prefix;
        if (in_lds) {
            const int nk = (int)s_nkeys;
            for (int i = tid; i < nk; i += 1024) {
                const unsigned long long kv = s_keys[i];
                if ((kv & hmask) == pv) atomicAdd(&hist[(kv >> shift) & dmask], 1u);
            }
        } else {
            for (int64_t c0 = 0; c0 < ncand; c0 += 8 * 1024) {
                unsigned long long kv[8];
                bool ok[8];
                keys8(c0, kv, ok);
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (ok[u] && (kv[u] & hmask) == pv) atomicAdd(&hist[(kv[u] >> shift) & dmask], 1u);
            }
        }
        __syncthreads();
        if (tid < 64) {
            // lane l owns bins 4l..4l+3; inclusive scan of the lane totals
            unsigned int b[4], tot = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                b[q] = hist[4 * tid + q];
                tot += b[q];
            }
            unsigned int incl = tot;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const unsigned int y = __shfl_up(incl, off);
                if (tid >= off) incl += y;
            }
            const unsigned long long r = s_rank;
            const unsigned int excl = incl - tot;
            if (r >= excl && r < incl) {
                unsigned long long rr = r - excl;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (rr < b[q]) {
                        s_prefix = pv | ((unsigned long long)(4 * tid + q) << shift);
                        s_rank = rr;
                        s_left = b[q];
                        break;
                    }
                    rr -= b[q];
                }
            }
        }
        __syncthreads();
        hi = shift - 1;
        if (!in_lds && hi >= 0 && s_left <= (unsigned int)kSelLds) {
            // one more pass over all candidates copies the keys that share the
            // prefix chosen so far (exactly s_left of them) into LDS
            if (tid == 0) s_nkeys = 0;
            __syncthreads();
            const unsigned long long nmask = ~0ull << shift;
            const unsigned long long np2 = s_prefix;
            for (int64_t c0 = 0; c0 < ncand; c0 += 8 * 1024) {
                unsigned long long kv[8];
                bool ok[8];
                keys8(c0, kv, ok);
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (ok[u] && (kv[u] & nmask) == np2) s_keys[atomicAdd(&s_nkeys, 1u)] = kv[u];
            }
            __syncthreads();
            in_lds = true;
        }
    }
    if (tid == 0) {
        const double med = __longlong_as_double((long long)s_prefix);
        st->median = med;
        st->tau = frac * med;
        if (tau_out) *tau_out = frac * med;
    }
}

hipError_t list_compact(const LaunchCtx &lc, int64_t nw, const int64_t *cand, const unsigned int *ccnt,
                        const int64_t *didx, const unsigned int *dcnt, TauState *st, FusedLists fl) {
    hipLaunchKernelGGL(k_list_scan, dim3((unsigned)((nw + kScanChunk - 1) / kScanChunk)), dim3(1024), 0, lc.stream,
                       ccnt, dcnt, st, fl.coff, fl.doff);
    hipLaunchKernelGGL(k_list_compact, dim3((unsigned)((nw + 63) / 64)), dim3(64), 0, lc.stream, cand, ccnt, fl.coff,
                       didx, dcnt, fl.doff, st, fl.ccomp, fl.dcomp);
    return hipGetLastError();
}

hipError_t tau_finish(const LaunchCtx &lc, const float *rgb, int H, int W, int p, int n,
                      const double *wmask, const float *omega, int k, const int64_t *cand,
                      int64_t cap, double *vals, double frac, TauState *st, unsigned long long *parts,
                      double *tau_out, const double *pstats, const unsigned int *ccnt, const FusedLists *fl) {
    (void)n;
    // one lane per entry of a compact list (or per region when the fused
    // gather's list was too long to compact: at most kMedianWavesMax of them)
    int64_t blocks = (int64_t)lc.num_cu * 8;
    if (!ccnt && blocks > (cap + 63) / 64) blocks = (cap + 63) / 64;
    if (ccnt && blocks < kMedianWavesMax / 64) blocks = kMedianWavesMax / 64;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_tau_recompute, dim3((unsigned)blocks), dim3(64), 0, lc.stream, rgb, H, W, p, wmask, omega,
                       k, cand, st, cap, vals, pstats, ccnt, fl ? fl->coff : nullptr, fl ? fl->ccomp : nullptr);
    unsigned long long *rk = parts + kTauParts;  // kRankMax (less, equal) pairs
    hipLaunchKernelGGL(k_tau_rank, dim3((unsigned)lc.num_cu * 4), dim3(64), 0, lc.stream, vals, cap, st, rk);
    hipLaunchKernelGGL(k_tau_select, dim3(1), dim3(1024), 0, lc.stream, vals, cap, frac, st, parts, rk, tau_out);
    return hipGetLastError();
}

}  // namespace cs
