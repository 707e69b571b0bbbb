// Host layer of the co-sparse data-term library: context, argument checks,
// device workspace, kernel-event timing and the order of launches behind each
// C-ABI call declared in include/cosparse.h.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/cosparse.h"
#include "cs_internal.h"

using namespace cs;

// Scratch memory of the allocation-free entry point (cs_cosupport_noalloc):
// one array per device, part of the library's code object, held until the
// process ends.  Host code must never use the array's name as an address:
// its device address on each device comes from hipGetSymbolAddress (see
// scratch_address), and every call on one device shares it.
constexpr size_t kScratchBytes = 8192;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct cs_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int num_cu = 0;
    std::string err;
    // growable device workspace (carved per call) and a separate candidate buffer
    char *ws = nullptr;
    size_t ws_bytes = 0;
    char *cand = nullptr;
    size_t cand_bytes = 0;
    // FP32 analysed vectors for the exact median of a BF16 analysis
    float *alpha32 = nullptr;
    size_t alpha32_bytes = 0;
    // pinned host staging for small device-to-host results
    char *pinned = nullptr;
    // coherent host memory that the sample scan writes the label counts and a
    // tag into (a log-likelihood call waits on the tag, not on the stream)
    int32_t *hcounts = nullptr, *hcounts_dev = nullptr;
    int32_t tag = 0;
    // device counters that are zero between calls (kCtr*)
    unsigned int *dctr = nullptr;
    // Gaussian patch mask of the last (p, sigma)
    double *wmask = nullptr;
    int wmask_p = 0;
    double wmask_sigma = 0.0;
    // kernel-event timing (of every span, or only of the spans named `only`)
    bool prof = false;
    std::string only;
    int prof_period = 1;                       // record one launch in prof_period per name
    std::map<std::string, int64_t> prof_seen;  // launches of each name seen while recording
    struct Span {
        std::string name;
        hipEvent_t a, b;
    };
    std::vector<Span> spans;
    std::vector<hipEvent_t> pool;
    std::map<std::string, std::pair<double, int64_t>> totals;
    // counters of the last full-image log-likelihood call (4 x u32, context-owned
    // device memory, cleared by that call's sample scan); valid when the last
    // log-likelihood call took the full-image path
    unsigned int *lstats = nullptr;
    bool lstats_valid = false;
    // optional finite check of rgb and omega before any launch
    bool check_finite = false;
    // the device's allocation-free scratch array (address on this device)
    char *scratch = nullptr;
    // the surrogate's exact fallback: pixel list, count and exact rows
    char *fb = nullptr;
    size_t fb_bytes = 0;
};

namespace {

constexpr size_t kPinnedBytes = 4096;

int fail(cs_ctx *c, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
    return code;
}

#define HIP_TRY(call)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(ctx, CS_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_));       \
    } while (0)

LaunchCtx lc_of(const cs_ctx *c) { return LaunchCtx{c->stream, c->num_cu}; }

// Device address of the scratch array on `device` (current), looked up once
// per device and kept for the life of the process.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_addr[kMaxDevices] = {};

hipError_t scratch_address(int device, char **out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[device]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_addr[device] = (char *)ptr;
    }
    *out = g_scratch_addr[device];
    return hipSuccess;
}

// Waits until the sample scan of this call has written `tag` into host memory
// (the label counts before it are then visible): spins, yields after 2 ms,
// and after 5 s waits for the stream and looks once more (a failed stream
// reports its error there).
int wait_host_tag(cs_ctx *ctx, int32_t tag) {
    volatile int32_t *t = ctx->hcounts + kHostTag;
    const auto t0 = std::chrono::steady_clock::now();
    for (int64_t it = 0; *t != tag; ++it) {
        if ((it & 1023) == 1023) {
            const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            if (sec > 5.0) {
                HIP_TRY(hipStreamSynchronize(ctx->stream));
                if (*t != tag) return fail(ctx, CS_ERR_HIP, "the label counts did not arrive from the device");
                break;
            }
            if (sec > 2e-3) std::this_thread::yield();
        }
        __builtin_ia32_pause();
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    return CS_OK;
}

struct Carve {
    size_t off = 0;
    size_t take(size_t bytes) {
        size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    }
};

// Work enqueued earlier may still read a buffer that is about to be freed, on
// this stream or on a stream used before cs_set_stream switched it: wait for
// the whole device before a workspace buffer is replaced.
int ensure_ws(cs_ctx *ctx, size_t bytes) {
    if (bytes <= ctx->ws_bytes) return CS_OK;
    const size_t want = std::max(bytes, ctx->ws_bytes + ctx->ws_bytes / 4);
    HIP_TRY(hipDeviceSynchronize());
    if (ctx->ws) HIP_TRY(hipFree(ctx->ws));
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
    if (hipMalloc((void **)&ctx->ws, want) != hipSuccess) {
        ctx->ws = nullptr;
        return fail(ctx, CS_ERR_NOMEM, "device workspace of %zu bytes could not be allocated", want);
    }
    ctx->ws_bytes = want;
    return CS_OK;
}

int ensure_fb(cs_ctx *ctx, size_t bytes) {
    if (bytes <= ctx->fb_bytes) return CS_OK;
    HIP_TRY(hipDeviceSynchronize());
    if (ctx->fb) HIP_TRY(hipFree(ctx->fb));
    ctx->fb = nullptr;
    ctx->fb_bytes = 0;
    if (hipMalloc((void **)&ctx->fb, bytes) != hipSuccess) {
        ctx->fb = nullptr;
        return fail(ctx, CS_ERR_NOMEM, "fallback buffer of %zu bytes could not be allocated", bytes);
    }
    ctx->fb_bytes = bytes;
    return CS_OK;
}

int ensure_cand(cs_ctx *ctx, size_t bytes) {
    if (bytes <= ctx->cand_bytes) return CS_OK;
    HIP_TRY(hipDeviceSynchronize());
    if (ctx->cand) HIP_TRY(hipFree(ctx->cand));
    ctx->cand = nullptr;
    ctx->cand_bytes = 0;
    if (hipMalloc((void **)&ctx->cand, bytes) != hipSuccess) {
        ctx->cand = nullptr;
        return fail(ctx, CS_ERR_NOMEM, "candidate buffer of %zu bytes could not be allocated", bytes);
    }
    ctx->cand_bytes = bytes;
    return CS_OK;
}

// HIP events around one launch when timing is on.
struct Timed {
    cs_ctx *c;
    const char *name;
    hipEvent_t a = nullptr, b = nullptr;
    Timed(cs_ctx *ctx, const char *nm) : c(ctx), name(nm) {
        if (!c->prof || (!c->only.empty() && c->only != nm)) return;
        if (c->prof_period > 1 && c->prof_seen[nm]++ % c->prof_period != 0) return;
        a = take();
        b = take();
        if (a) hipEventRecord(a, c->stream);
    }
    hipEvent_t take() {
        if (!c->pool.empty()) {
            hipEvent_t e = c->pool.back();
            c->pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    ~Timed() {
        if (!c->prof || !a || !b) return;
        hipEventRecord(b, c->stream);
        c->spans.push_back({name, a, b});
    }
};

// Gaussian mask w_t = exp(-(u^2+v^2) / (2 sigma^2)) of Sec. 3.1, host FP64,
// uploaded once per (p, sigma).
void mask_table(int p, double sigma, double *w) {
    const int h = (p - 1) / 2;
    for (int u = -h; u <= h; ++u)
        for (int v = -h; v <= h; ++v) {
            const double r2 = (double)(u * u + v * v);
            w[(u + h) * p + (v + h)] = std::exp(-r2 / (2.0 * sigma * sigma));
        }
}

int ensure_mask(cs_ctx *ctx, int p, double sigma) {
    if (ctx->wmask && ctx->wmask_p == p && ctx->wmask_sigma == sigma) return CS_OK;
    double w[15 * 15];
    mask_table(p, sigma, w);
    if (!ctx->wmask) HIP_TRY(hipMalloc((void **)&ctx->wmask, sizeof(double) * 15 * 15));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    HIP_TRY(hipMemcpy(ctx->wmask, w, sizeof(double) * p * p, hipMemcpyHostToDevice));
    ctx->wmask_p = p;
    ctx->wmask_sigma = sigma;
    return CS_OK;
}

int check_patch_args(cs_ctx *ctx, const float *rgb, int H, int W, int p, double mask_sigma,
                     const float *omega, int k, int precision) {
    if (!rgb || !omega) return fail(ctx, CS_ERR_ARG, "rgb and omega must be non-null");
    if (p < 3 || p > 15 || (p % 2) == 0) return fail(ctx, CS_ERR_ARG, "p must be odd in 3..15 (got %d)", p);
    const int h = (p - 1) / 2;
    if (H < h + 1 || W < h + 1)
        return fail(ctx, CS_ERR_ARG, "image %dx%d too small for %dx%d patches", W, H, p, p);
    if ((int64_t)H * W > ((int64_t)1 << 31) - 1)
        return fail(ctx, CS_ERR_ARG, "image of %lld pixels exceeds 2^31-1", (long long)H * W);
    if (H > 65535) return fail(ctx, CS_ERR_ARG, "H must be <= 65535");
    if (k < 1 || k > kMaxK) return fail(ctx, CS_ERR_ARG, "k must be in 1..%d (got %d)", kMaxK, k);
    if (!(mask_sigma > 0.0) || !std::isfinite(mask_sigma))
        return fail(ctx, CS_ERR_ARG, "mask_sigma must be positive and finite");
    if (precision != CS_FP32 && precision != CS_BF16)
        return fail(ctx, CS_ERR_ARG, "unknown precision %d", precision);
    return CS_OK;
}

// Optional finite check (cs_set_check_finite): the n0 floats at a and the n1
// floats at b (either may be null) are scanned on the device; the host reads
// the flag (this synchronises the stream) and fails with CS_ERR_NONFINITE
// before anything else is launched.  With colour levels n > 0 the values at a
// (colours) must also be multiples of 1/n in [0, 255/n] (else CS_ERR_ARG).
int check_inputs_finite(cs_ctx *ctx, const float *a, int64_t n0, const float *b, int64_t n1, int levels) {
    if (!ctx->check_finite) return CS_OK;
    unsigned int *flag = ctx->dctr + kCtrNonFinite;
    const LaunchCtx lc = lc_of(ctx);
    if (a) HIP_TRY(launch_check_finite(lc, a, n0, levels, flag));
    if (b) HIP_TRY(launch_check_finite(lc, b, n1, 0, flag));
    HIP_TRY(hipMemcpyAsync(ctx->pinned, flag, sizeof(unsigned int), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    unsigned int f;
    std::memcpy(&f, ctx->pinned, sizeof f);
    if (!f) return CS_OK;
    HIP_TRY(launch_fill_u32(lc, flag, 1, 0u));  // the counter is zero between calls
    if (f & 1u) return fail(ctx, CS_ERR_NONFINITE, "an input (rgb or omega) holds a NaN or an infinity");
    return fail(ctx, CS_ERR_ARG, "a colour is not a multiple of 1/%d in [0, 255/%d]", levels, levels);
}

int check_patch_inputs_finite(cs_ctx *ctx, const float *rgb, int H, int W, const float *omega, int k, int p) {
    return check_inputs_finite(ctx, rgb, 3 * (int64_t)H * W, omega, (int64_t)k * p * p, 0);
}

// Coefficient of the proven bound |a_rounded - a| <= coef * ||O_j||_2 (unit-norm patch):
// FP32: s and the accumulation each contribute at most (n + 2) unit roundoffs, doubled
// to allow round-toward-zero accumulation; BF16: both operands rounded to 8-bit
// significands (2^-8 each), the FP32 rounding of s, and the FP32 accumulation.
double margin_coef(int precision, int n) {
    const double u32 = std::ldexp(1.0, -24);
    if (precision == CS_BF16) return std::ldexp(1.0, -7) + std::ldexp(1.0, -15) + 2.0 * (n + 4) * u32;
    return 2.0 * (n + 4) * u32;
}

int n_pad_of(int n) { return (n + 15) / 16 * 16; }

}  // namespace

extern "C" {

int cs_create(cs_ctx **out, int device, void *hip_stream) {
    if (!out) return CS_ERR_ARG;
    *out = nullptr;
    cs_ctx *ctx = new (std::nothrow) cs_ctx();
    if (!ctx) return CS_ERR_NOMEM;
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    hipError_t e = hipSetDevice(device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ctx->num_cu, hipDeviceAttributeMultiprocessorCount, device);
    if (e == hipSuccess) e = hipHostMalloc((void **)&ctx->pinned, kPinnedBytes, hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&ctx->hcounts, sizeof(int32_t) * (kHostTag + 1),
                          hipHostMallocCoherent | hipHostMallocMapped);
    if (e == hipSuccess) e = hipHostGetDevicePointer((void **)&ctx->hcounts_dev, ctx->hcounts, 0);
    if (e == hipSuccess) e = hipMalloc((void **)&ctx->dctr, sizeof(unsigned int) * kCtrWords);
    if (e == hipSuccess) e = hipMalloc((void **)&ctx->lstats, sizeof(unsigned int) * 4);
    if (e == hipSuccess) e = launch_fill_u32(lc_of(ctx), ctx->dctr, kCtrWords, 0u);
    if (e == hipSuccess) e = launch_fill_u32(lc_of(ctx), ctx->lstats, 4, 0u);
    if (e == hipSuccess) e = scratch_address(device, &ctx->scratch);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        if (ctx->pinned) hipHostFree(ctx->pinned);
        if (ctx->hcounts) hipHostFree(ctx->hcounts);
        if (ctx->dctr) hipFree(ctx->dctr);
        if (ctx->lstats) hipFree(ctx->lstats);
        delete ctx;
        return CS_ERR_HIP;
    }
    std::memset(ctx->hcounts, 0, sizeof(int32_t) * (kHostTag + 1));
    *out = ctx;
    return CS_OK;
}

int cs_destroy(cs_ctx *ctx) {
    if (!ctx) return CS_ERR_ARG;
    hipStreamSynchronize(ctx->stream);
    for (auto &s : ctx->spans) {
        hipEventDestroy(s.a);
        hipEventDestroy(s.b);
    }
    for (auto e : ctx->pool) hipEventDestroy(e);
    if (ctx->ws) hipFree(ctx->ws);
    if (ctx->cand) hipFree(ctx->cand);
    if (ctx->fb) hipFree(ctx->fb);
    if (ctx->alpha32) hipFree(ctx->alpha32);
    if (ctx->wmask) hipFree(ctx->wmask);
    if (ctx->pinned) hipHostFree(ctx->pinned);
    if (ctx->hcounts) hipHostFree(ctx->hcounts);
    if (ctx->dctr) hipFree(ctx->dctr);
    if (ctx->lstats) hipFree(ctx->lstats);
    delete ctx;
    return CS_OK;
}

int cs_set_stream(cs_ctx *ctx, void *hip_stream) {
    if (!ctx) return CS_ERR_ARG;
    ctx->stream = (hipStream_t)hip_stream;
    return CS_OK;
}

const char *cs_last_error(const cs_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int cs_set_check_finite(cs_ctx *ctx, int on) {
    if (!ctx) return CS_ERR_ARG;
    ctx->check_finite = on != 0;
    return CS_OK;
}

}  // extern "C"

namespace {

// The analysis of cs_analyze_patches; pstats (N x 2, device) receives the
// exact patch statistics when non-null.
int analyze_stage(cs_ctx *ctx, const float *rgb, int H, int W, int p, double mask_sigma, const float *omega, int k,
                  int precision, float *alpha, double *pstats) {
    if (!ctx) return CS_ERR_ARG;
    int rc = check_patch_args(ctx, rgb, H, W, p, mask_sigma, omega, k, precision);
    if (rc) return rc;
    if (!alpha) return fail(ctx, CS_ERR_ARG, "alpha must be non-null");
    HIP_TRY(hipSetDevice(ctx->device));
    if ((rc = check_patch_inputs_finite(ctx, rgb, H, W, omega, k, p))) return rc;
    if ((rc = ensure_mask(ctx, p, mask_sigma))) return rc;
    AnalyzeArgs a{};
    a.rgb = rgb;
    a.H = H;
    a.W = W;
    a.p = p;
    a.n = p * p;
    a.n_pad = n_pad_of(a.n);
    a.k = k;
    a.wmask = ctx->wmask;
    a.omega = omega;
    a.alpha = alpha;
    a.pstats = pstats;
    Timed t(ctx, "analyze");
    HIP_TRY(launch_analyze(lc_of(ctx), a, precision));
    return CS_OK;
}

}  // namespace

extern "C" {

int cs_analyze_patches(cs_ctx *ctx, const float *rgb, int H, int W, int p, double mask_sigma,
                       const float *omega, int k, int precision, float *alpha) {
    return analyze_stage(ctx, rgb, H, W, p, mask_sigma, omega, k, precision, alpha, nullptr);
}

}  // extern "C"

namespace {

// Masks of Sec. 2 at tau (or at *tau_dev, read on the device, when non-null):
// per-row thresholds, then the decision from the stored analysed vectors or
// from a fused analysis.  Fills *cnt (device) with the recomputed-entry count
// and *mmax (device) with the largest margin.
int cosupport_stage(cs_ctx *ctx, const float *rgb, int H, int W, int p, const float *omega, int k,
                    int precision, const float *alpha, double tau, const double *tau_dev, double margin,
                    uint64_t *masks, unsigned long long *cnt, double *mmax, float *t_in, float *t_out,
                    double *marg, const double *pstats = nullptr) {
    const LaunchCtx lc = lc_of(ctx);
    const int n = p * p;
    {
        Timed t(ctx, "thresholds");
        HIP_TRY(launch_thresholds(lc, omega, k, n, tau, tau_dev, margin, margin_coef(precision, n), t_in, t_out,
                                  marg, mmax, cnt));
    }
    if (alpha) {
        Timed t(ctx, "cosupport");
        HIP_TRY(launch_mask_alpha(lc, alpha, (int64_t)H * W, k, t_in, t_out, tau, tau_dev, rgb, H, W, p,
                                  ctx->wmask, omega, masks, cnt, pstats));
    } else {
        AnalyzeArgs a{};
        a.rgb = rgb;
        a.H = H;
        a.W = W;
        a.p = p;
        a.n = n;
        a.n_pad = n_pad_of(n);
        a.k = k;
        a.wmask = ctx->wmask;
        a.omega = omega;
        a.masks = masks;
        a.t_in = t_in;
        a.t_out = t_out;
        a.tau = tau;
        a.recomputed = cnt;
        Timed t(ctx, "cosupport");
        HIP_TRY(launch_analyze(lc, a, precision));
    }
    return CS_OK;
}

// Workspace of cosupport_stage.
struct CosupportWs {
    size_t o_tin, o_tout, o_marg, o_max, o_cnt;
    void carve(Carve &cv, int k) {
        o_tin = cv.take(sizeof(float) * k);
        o_tout = cv.take(sizeof(float) * k);
        o_marg = cv.take(sizeof(double) * k);
        o_max = cv.take(sizeof(double));
        o_cnt = cv.take(sizeof(unsigned long long));
    }
};

// FP32 analysed vectors that define the exact median for a call at
// `precision`: alpha itself for FP32; for BF16 an internal FP32 analysis (the
// BF16 error bound would put a large share of all entries in the candidate
// window, the FP32 one a tiny share; the selected value is the same).
// The context's FP32 analysis buffer (the BF16 forms select tau on an FP32
// analysis), grown to `bytes` when needed.
int ensure_alpha32(cs_ctx *ctx, size_t bytes) {
    if (bytes <= ctx->alpha32_bytes) return CS_OK;
    HIP_TRY(hipDeviceSynchronize());
    if (ctx->alpha32) HIP_TRY(hipFree(ctx->alpha32));
    ctx->alpha32 = nullptr;
    ctx->alpha32_bytes = 0;
    if (hipMalloc((void **)&ctx->alpha32, bytes) != hipSuccess) {
        ctx->alpha32 = nullptr;
        return fail(ctx, CS_ERR_NOMEM, "FP32 analysis buffer of %zu bytes could not be allocated", bytes);
    }
    ctx->alpha32_bytes = bytes;
    return CS_OK;
}

int median_source(cs_ctx *ctx, const float *rgb, int H, int W, int p, double mask_sigma, const float *omega,
                  int k, int precision, const float *alpha, const float **src) {
    *src = alpha;
    if (precision != CS_BF16) return CS_OK;
    int rc = ensure_alpha32(ctx, sizeof(float) * (size_t)H * W * k);
    if (rc) return rc;
    rc = cs_analyze_patches(ctx, rgb, H, W, p, mask_sigma, omega, k, CS_FP32, ctx->alpha32);
    if (rc) return rc;
    *src = ctx->alpha32;
    return CS_OK;
}

// Exact tau = frac * median |a| (Sec. 2) of the FP32 vectors `a32` into st
// (device), with room for `cap` candidates.  With first = false only the
// gather and the exact stage run again (a retry with a larger cap).
int tau_stage(cs_ctx *ctx, const float *rgb, int H, int W, int p, const float *omega, int k, const float *a32,
              double frac, int64_t cap, bool first, unsigned int *hist, TauState *st, double *mmax,
              unsigned long long *parts, double *tau_out, const double *pstats = nullptr) {
    const LaunchCtx lc = lc_of(ctx);
    const int64_t count = (int64_t)H * W * k;
    const int n = p * p;
    int rc = ensure_cand(ctx, (size_t)cap * 16);
    if (rc) return rc;
    int64_t *cand = (int64_t *)ctx->cand;
    double *vals = (double *)(ctx->cand + (size_t)cap * 8);
    {
        Timed t(ctx, "tau_select");
        if (first) {
            HIP_TRY(tau_select_float(lc, a32, count, hist, st, omega, k, n, margin_coef(CS_FP32, n), mmax, nullptr));
        } else {
            HIP_TRY(tau_reset_gather(lc, st));
        }
        HIP_TRY(tau_gather(lc, a32, count, mmax, st, cand, cap, parts));
    }
    {
        Timed t(ctx, "tau_exact");
        HIP_TRY(tau_finish(lc, rgb, H, W, p, n, ctx->wmask, omega, k, cand, cap, vals, frac, st, parts, tau_out,
                           pstats));
    }
    return CS_OK;
}

struct TauWs {
    size_t o_hist, o_st, o_max, o_parts;
    void carve(Carve &cv) {
        o_hist = cv.take(sizeof(unsigned int) * 2048);
        o_st = cv.take(sizeof(TauState));
        o_max = cv.take(sizeof(double));
        o_parts = cv.take(sizeof(unsigned long long) * (kTauParts + kTauRank));
    }
};

}  // namespace

extern "C" {

int cs_cosupport(cs_ctx *ctx, const float *rgb, int H, int W, int p, double mask_sigma,
                 const float *omega, int k, int precision, const float *alpha, double tau,
                 double margin, uint64_t *masks, cs_cosupport_stats *stats) {
    if (!ctx) return CS_ERR_ARG;
    int rc = check_patch_args(ctx, rgb, H, W, p, mask_sigma, omega, k, precision);
    if (rc) return rc;
    if (!masks) return fail(ctx, CS_ERR_ARG, "masks must be non-null");
    if (!(tau >= 0.0) || !std::isfinite(tau)) return fail(ctx, CS_ERR_ARG, "tau must be finite and >= 0");
    if (std::isnan(margin) || std::isinf(margin)) return fail(ctx, CS_ERR_ARG, "margin must be finite");
    HIP_TRY(hipSetDevice(ctx->device));
    if ((rc = check_patch_inputs_finite(ctx, rgb, H, W, omega, k, p))) return rc;
    if ((rc = ensure_mask(ctx, p, mask_sigma))) return rc;
    Carve cv;
    CosupportWs cw;
    cw.carve(cv, k);
    if ((rc = ensure_ws(ctx, cv.off))) return rc;
    unsigned long long *cnt = (unsigned long long *)(ctx->ws + cw.o_cnt);
    double *mmax = (double *)(ctx->ws + cw.o_max);
    rc = cosupport_stage(ctx, rgb, H, W, p, omega, k, precision, alpha, tau, nullptr, margin, masks, cnt, mmax,
                         (float *)(ctx->ws + cw.o_tin), (float *)(ctx->ws + cw.o_tout),
                         (double *)(ctx->ws + cw.o_marg));
    if (rc) return rc;
    if (stats) {
        HIP_TRY(hipMemcpyAsync(ctx->pinned, cnt, sizeof(unsigned long long), hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(hipMemcpyAsync(ctx->pinned + 8, mmax, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(hipStreamSynchronize(ctx->stream));
        unsigned long long c;
        double m;
        std::memcpy(&c, ctx->pinned, 8);
        std::memcpy(&m, ctx->pinned + 8, 8);
        stats->recomputed = (int64_t)c;
        stats->max_margin = m;
    }
    return CS_OK;
}

int cs_cosupport_noalloc(cs_ctx *ctx, const float *rgb, int H, int W, int p, double mask_sigma,
                         const float *omega, int k, int precision, const float *alpha, double tau,
                         double margin, uint64_t *masks) {
    if (!ctx) return CS_ERR_ARG;
    int rc = check_patch_args(ctx, rgb, H, W, p, mask_sigma, omega, k, precision);
    if (rc) return rc;
    if (!masks) return fail(ctx, CS_ERR_ARG, "masks must be non-null");
    if (!(tau >= 0.0) || !std::isfinite(tau)) return fail(ctx, CS_ERR_ARG, "tau must be finite and >= 0");
    if (std::isnan(margin) || std::isinf(margin)) return fail(ctx, CS_ERR_ARG, "margin must be finite");
    // scratch layout: thresholds t_in, t_out (k floats each), per-row margins
    // (k doubles), the largest margin, the recompute counter, the mask table
    Carve cv;
    CosupportWs cw;
    cw.carve(cv, k);
    const size_t o_w = cv.take(sizeof(double) * p * p);
    if (cv.off > kScratchBytes)
        return fail(ctx, CS_ERR_ARG, "k = %d, p = %d need %zu bytes of scratch; the maximum is %zu", k, p, cv.off,
                    kScratchBytes);
    if (!ctx->scratch) return fail(ctx, CS_ERR_HIP, "the scratch array of device %d was not set up", ctx->device);
    HIP_TRY(hipSetDevice(ctx->device));
    const LaunchCtx lc = lc_of(ctx);
    char *sp = ctx->scratch;
    MaskTable tbl;
    mask_table(p, mask_sigma, tbl.w);
    double *wmask = (double *)(sp + o_w);
    HIP_TRY(launch_put_table(lc, wmask, tbl, p * p));
    float *t_in = (float *)(sp + cw.o_tin), *t_out = (float *)(sp + cw.o_tout);
    double *marg = (double *)(sp + cw.o_marg), *mmax = (double *)(sp + cw.o_max);
    unsigned long long *cnt = (unsigned long long *)(sp + cw.o_cnt);
    const int n = p * p;
    // the thresholds kernel also clears the recompute counter
    HIP_TRY(launch_thresholds(lc, omega, k, n, tau, nullptr, margin, margin_coef(precision, n), t_in, t_out, marg,
                              mmax, cnt));
    if (alpha) {
        HIP_TRY(launch_mask_alpha(lc, alpha, (int64_t)H * W, k, t_in, t_out, tau, nullptr, rgb, H, W, p, wmask,
                                  omega, masks, cnt, nullptr));
    } else {
        AnalyzeArgs a{};
        a.rgb = rgb;
        a.H = H;
        a.W = W;
        a.p = p;
        a.n = n;
        a.n_pad = n_pad_of(n);
        a.k = k;
        a.wmask = wmask;
        a.omega = omega;
        a.masks = masks;
        a.t_in = t_in;
        a.t_out = t_out;
        a.tau = tau;
        a.recomputed = cnt;
        HIP_TRY(launch_analyze(lc, a, precision));
    }
    return CS_OK;
}

int cs_tau_median(cs_ctx *ctx, const float *rgb, int H, int W, int p, double mask_sigma,
                  const float *omega, int k, int precision, const float *alpha, double frac,
                  double *tau_out) {
    if (!ctx) return CS_ERR_ARG;
    int rc = check_patch_args(ctx, rgb, H, W, p, mask_sigma, omega, k, precision);
    if (rc) return rc;
    if (!alpha || !tau_out) return fail(ctx, CS_ERR_ARG, "alpha and tau_out must be non-null");
    if (reinterpret_cast<uintptr_t>(alpha) % 16) return fail(ctx, CS_ERR_ARG, "alpha must be 16-byte aligned");
    if (!(frac >= 0.0) || !std::isfinite(frac)) return fail(ctx, CS_ERR_ARG, "frac must be finite and >= 0");
    HIP_TRY(hipSetDevice(ctx->device));
    if ((rc = check_patch_inputs_finite(ctx, rgb, H, W, omega, k, p))) return rc;
    if ((rc = ensure_mask(ctx, p, mask_sigma))) return rc;
    const int64_t count = (int64_t)H * W * k;
    const float *a32 = nullptr;
    if ((rc = median_source(ctx, rgb, H, W, p, mask_sigma, omega, k, precision, alpha, &a32))) return rc;
    Carve cv;
    TauWs tw;
    tw.carve(cv);
    if ((rc = ensure_ws(ctx, cv.off))) return rc;
    unsigned int *hist = (unsigned int *)(ctx->ws + tw.o_hist);
    TauState *st = (TauState *)(ctx->ws + tw.o_st);
    double *mmax = (double *)(ctx->ws + tw.o_max);
    int64_t cap = (int64_t)std::min<int64_t>(count, (int64_t)1 << 20);
    TauState hs;
    for (int attempt = 0;; ++attempt) {
        if ((rc = tau_stage(ctx, rgb, H, W, p, omega, k, a32, frac, cap, attempt == 0, hist, st, mmax,
                            (unsigned long long *)(ctx->ws + tw.o_parts), nullptr)))
            return rc;
        HIP_TRY(hipMemcpyAsync(ctx->pinned, st, sizeof(TauState), hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(hipStreamSynchronize(ctx->stream));
        std::memcpy(&hs, ctx->pinned, sizeof(TauState));
        if ((int64_t)hs.ncand <= cap) break;
        if (attempt > 0) return fail(ctx, CS_ERR_HIP, "candidate count changed between passes");
        cap = (int64_t)hs.ncand;  // one retry with room for every candidate
    }
    if (std::isnan(hs.median))
        return fail(ctx, CS_ERR_HIP, "exact median outside the candidate window (error bound violated)");
    *tau_out = hs.tau;
    return CS_OK;
}

int cs_cosupport_median(cs_ctx *ctx, const float *rgb, int H, int W, int p, double mask_sigma,
                        const float *omega, int k, int precision, double frac, double margin, float *alpha,
                        uint64_t *masks, double *tau_dev) {
    if (!ctx) return CS_ERR_ARG;
    int rc = check_patch_args(ctx, rgb, H, W, p, mask_sigma, omega, k, precision);
    if (rc) return rc;
    if (!alpha || !masks) return fail(ctx, CS_ERR_ARG, "alpha and masks must be non-null");
    if (reinterpret_cast<uintptr_t>(alpha) % 16) return fail(ctx, CS_ERR_ARG, "alpha must be 16-byte aligned");
    if (!(frac >= 0.0) || !std::isfinite(frac)) return fail(ctx, CS_ERR_ARG, "frac must be finite and >= 0");
    if (std::isnan(margin) || std::isinf(margin)) return fail(ctx, CS_ERR_ARG, "margin must be finite");
    HIP_TRY(hipSetDevice(ctx->device));
    if ((rc = check_patch_inputs_finite(ctx, rgb, H, W, omega, k, p))) return rc;
    if ((rc = ensure_mask(ctx, p, mask_sigma))) return rc;
    const int64_t count = (int64_t)H * W * k;
    if (margin < 0.0) {
        // the masks are decided in the candidate gather of the median: four
        // passes over alpha instead of five; the analysis kernel also sets up
        // the selection, and each digit is picked by the kernel after its
        // histogram.  For BF16 this runs on the FP32 analysis that the call
        // selects tau on anyway (its masks at the proven margin are the exact
        // masks, which the BF16 vectors at their proven margin give as well),
        // and the BF16 analysis then writes alpha.
        float *a32 = alpha;
        if (precision == CS_BF16) {
            if ((rc = ensure_alpha32(ctx, sizeof(float) * (size_t)count))) return rc;
            a32 = ctx->alpha32;
        }
        const int n = p * p;
        const LaunchCtx lc = lc_of(ctx);
        Carve cv;
        TauWs tw;
        tw.carve(cv);
        const size_t o_marg = cv.take(sizeof(double) * k);
        const size_t o_hist3 = cv.take(sizeof(unsigned int) * 3 * kHistBins);
        const size_t o_pst = cv.take(sizeof(double) * 2 * (size_t)H * W);
        // per-wave list counts of the gather and the candidate regions' offsets
        const size_t o_ccnt = cv.take(sizeof(unsigned int) * kMedianWavesMax);
        const size_t o_dcnt = cv.take(sizeof(unsigned int) * kMedianWavesMax);
        const size_t o_coff = cv.take(sizeof(unsigned long long) * kMedianWavesMax);
        const size_t o_doff = cv.take(sizeof(unsigned long long) * kMedianWavesMax);
        // compact lists (each up to kListCap entries, or count when smaller)
        const int64_t lcap = count < kListCap ? count : kListCap;
        const size_t o_ccomp = cv.take(sizeof(int64_t) * (size_t)lcap);
        const size_t o_dcomp = cv.take(sizeof(int64_t) * (size_t)lcap);
        if ((rc = ensure_ws(ctx, cv.off))) return rc;
        double *pst = (double *)(ctx->ws + o_pst);
        unsigned int *ccnt = (unsigned int *)(ctx->ws + o_ccnt), *dcnt = (unsigned int *)(ctx->ws + o_dcnt);
        FusedLists fl;
        fl.coff = (unsigned long long *)(ctx->ws + o_coff);
        fl.doff = (unsigned long long *)(ctx->ws + o_doff);
        fl.ccomp = (int64_t *)(ctx->ws + o_ccomp);
        fl.dcomp = (int64_t *)(ctx->ws + o_dcomp);
        // candidates, their FP64 values, listed mask entries (room for all)
        if ((rc = ensure_cand(ctx, (size_t)count * 24))) return rc;
        TauState *st = (TauState *)(ctx->ws + tw.o_st);
        double *mmax = (double *)(ctx->ws + tw.o_max);
        unsigned long long *parts = (unsigned long long *)(ctx->ws + tw.o_parts);
        double *marg = (double *)(ctx->ws + o_marg);
        int64_t *cand = (int64_t *)ctx->cand;
        double *vals = (double *)(ctx->cand + (size_t)count * 8);
        int64_t *didx = (int64_t *)(ctx->cand + (size_t)count * 16);
        unsigned int *hist3 = (unsigned int *)(ctx->ws + o_hist3);
        {
            AnalyzeArgs a{};
            a.rgb = rgb;
            a.H = H;
            a.W = W;
            a.p = p;
            a.n = n;
            a.n_pad = n_pad_of(n);
            a.k = k;
            a.wmask = ctx->wmask;
            a.omega = omega;
            a.alpha = a32;
            a.pstats = pst;
            a.tau_st = st;
            a.tau_hist3 = hist3;
            a.tau_margins = marg;
            a.tau_max_margin = mmax;
            a.tau_coef = margin_coef(CS_FP32, n);
            a.tau_rank0 = (unsigned long long)((count - 1) / 2);
            Timed t(ctx, "analyze");
            HIP_TRY(launch_analyze(lc, a, CS_FP32));
        }
        {
            Timed t(ctx, "tau_select");
            HIP_TRY(tau_digits_folded(lc, a32, count, hist3, st));
        }
        {
            Timed t(ctx, "cosupport");
            HIP_TRY(median_mask_gather(lc, a32, (int64_t)H * W, k, mmax, marg, frac, st, cand, ccnt, parts, didx,
                                       dcnt, masks, hist3));
            HIP_TRY(list_compact(lc, median_gather_waves((int64_t)H * W), cand, ccnt, didx, dcnt, st, fl));
        }
        {
            Timed t(ctx, "tau_exact");
            HIP_TRY(tau_finish(lc, rgb, H, W, p, n, ctx->wmask, omega, k, cand, count, vals, frac, st, parts,
                               tau_dev, pst, ccnt, &fl));
        }
        {
            Timed t(ctx, "cosupport_fix");
            HIP_TRY(median_mask_finish(lc, a32, rgb, H, W, p, ctx->wmask, omega, k, didx, dcnt, fl.dcomp, marg, st,
                                       masks, pst));
        }
        if (precision == CS_BF16) {
            AnalyzeArgs a{};
            a.rgb = rgb;
            a.H = H;
            a.W = W;
            a.p = p;
            a.n = n;
            a.n_pad = n_pad_of(n);
            a.k = k;
            a.wmask = ctx->wmask;
            a.omega = omega;
            a.alpha = alpha;
            Timed t(ctx, "analyze_bf16");
            HIP_TRY(launch_analyze(lc, a, CS_BF16));
        }
        return CS_OK;
    }
    Carve cv;
    TauWs tw;
    tw.carve(cv);
    CosupportWs cw;
    cw.carve(cv, k);
    const size_t o_pst = cv.take(sizeof(double) * 2 * (size_t)H * W);
    if ((rc = ensure_ws(ctx, cv.off))) return rc;
    double *pst = (double *)(ctx->ws + o_pst);
    if ((rc = analyze_stage(ctx, rgb, H, W, p, mask_sigma, omega, k, precision, alpha, pst))) return rc;
    const float *a32 = nullptr;
    if ((rc = median_source(ctx, rgb, H, W, p, mask_sigma, omega, k, precision, alpha, &a32))) return rc;
    TauState *st = (TauState *)(ctx->ws + tw.o_st);
    // room for every entry: the selection never needs the host
    rc = tau_stage(ctx, rgb, H, W, p, omega, k, a32, frac, count, true, (unsigned int *)(ctx->ws + tw.o_hist), st,
                   (double *)(ctx->ws + tw.o_max), (unsigned long long *)(ctx->ws + tw.o_parts), tau_dev, pst);
    if (rc) return rc;
    rc = cosupport_stage(ctx, rgb, H, W, p, omega, k, precision, alpha, 0.0, &st->tau, margin, masks,
                         (unsigned long long *)(ctx->ws + cw.o_cnt), (double *)(ctx->ws + cw.o_max),
                         (float *)(ctx->ws + cw.o_tin), (float *)(ctx->ws + cw.o_tout),
                         (double *)(ctx->ws + cw.o_marg), pst);
    return rc;
}

int cs_texture_similarity(cs_ctx *ctx, const uint64_t *A, int64_t na, const uint64_t *B,
                          int64_t nb, int k, int32_t *out) {
    if (!ctx) return CS_ERR_ARG;
    if (na < 0 || nb < 0) return fail(ctx, CS_ERR_ARG, "counts must be >= 0");
    if (k < 1 || k > kMaxK) return fail(ctx, CS_ERR_ARG, "k must be in 1..%d (got %d)", kMaxK, k);
    if ((na && !A) || (nb && !B) || (na && nb && !out))
        return fail(ctx, CS_ERR_ARG, "null pointer with nonzero count");
    HIP_TRY(hipSetDevice(ctx->device));
    Timed t(ctx, "tsm");
    HIP_TRY(launch_tsm(lc_of(ctx), A, na, B, nb, k, out));
    return CS_OK;
}

// mode 0: the texture factor exp(-TSM/beta) inside the Parzen sum, one per
// sample; mode 1: eq:joined, the Parzen sum without it times the texture
// posterior against the hard label representatives; mode 2: the same with
// smooth co-supports (alpha, sigma_iota) and median representatives.
static int label_loglik(cs_ctx *ctx, const float *rgb, int H, int W, const uint64_t *masks, int k,
                        const int32_t *sample_pix, const int32_t *sample_label, int64_t M, int L,
                        const cs_loglik_params *prm, const int32_t *pix_subset, int64_t n_subset,
                        float *loglik, int mode, const float *alpha = nullptr,
                        double sigma_iota = 0.0) {
    if (!ctx) return CS_ERR_ARG;
    if (!rgb || (mode == 2 ? !alpha : !masks) || !sample_pix || !sample_label || !prm)
        return fail(ctx, CS_ERR_ARG, "null pointer argument");
    if (mode == 2 && !(sigma_iota > 0.0 && std::isfinite(sigma_iota) && std::isfinite(1.0 / sigma_iota)))
        return fail(ctx, CS_ERR_ARG, "sigma_iota must be positive and finite");
    if (!loglik && !(pix_subset && n_subset == 0))
        return fail(ctx, CS_ERR_ARG, "loglik must be non-null unless the pixel subset is empty");
    if (H < 1 || W < 1 || H > 32767 || W > 16384)
        return fail(ctx, CS_ERR_ARG, "H must be in 1..32767 and W in 1..16384");
    if (k < 1 || k > kMaxK) return fail(ctx, CS_ERR_ARG, "k must be in 1..%d (got %d)", kMaxK, k);
    if (L < 1 || L > kMaxLabels) return fail(ctx, CS_ERR_ARG, "L must be in 1..%d (got %d)", kMaxLabels, L);
    if (M < 1 || M > (((int64_t)1 << 31) - 1)) return fail(ctx, CS_ERR_ARG, "M must be in 1..2^31-1");
    auto pos = [](double v) { return v > 0.0 && std::isfinite(v); };
    if (!pos(prm->alpha_rho) || !pos(prm->sigma_c) || !pos(prm->beta_scale) || !pos(prm->rho_floor_px))
        return fail(ctx, CS_ERR_ARG, "alpha_rho, sigma_c, beta_scale and rho_floor_px must be positive and finite");
    if (prm->colour_levels < 0 || prm->colour_levels > 255)
        return fail(ctx, CS_ERR_ARG, "colour_levels must be in 0..255 (got %d)", prm->colour_levels);
    const int64_t N = (int64_t)H * W;
    const int64_t npix = pix_subset ? n_subset : N;
    if (npix < 0) return fail(ctx, CS_ERR_ARG, "n_subset must be >= 0");
    const int64_t tiles = (npix + 63) / 64;
    if (tiles * L > (((int64_t)1 << 31) - 1)) return fail(ctx, CS_ERR_ARG, "too many pixels x labels");
    HIP_TRY(hipSetDevice(ctx->device));
    {
        int rcf = check_inputs_finite(ctx, rgb, 3 * (int64_t)H * W, nullptr, 0, prm->colour_levels);
        if (rcf) return rcf;
    }
    const int nblocks = (int)((M + 255) / 256);
    Carve cv;
    const size_t o_bc = cv.take(sizeof(int32_t) * (size_t)L * nblocks);
    const LaunchCtx lc0 = lc_of(ctx);
    const int npix_blocks = pix_subset && npix > 0 ? check_pix_blocks(lc0, npix) : 0;
    const size_t o_bflags = cv.take(sizeof(int32_t) * ((size_t)nblocks + npix_blocks));
    // label counts (L+1) and the exact kernel's two counters share one
    // region, cleared by the sample scan (the fast kernel's counters are the
    // context's own, cleared by the same scan, and outlive the call)
    const size_t o_tf = cv.take(sizeof(int32_t) * (L + 1 + 2));
    const size_t o_cnt = o_tf + sizeof(int32_t) * (L + 1);
    const size_t o_queue = cv.take(sizeof(unsigned int) * kParzenQueues * kQueueStride);  // right after o_tf
    const size_t o_rec = cv.take(sizeof(SampleRec) * (size_t)M);
    const size_t seed_bytes = ((size_t)L * N + 15) / 16 * 16;  // cleared in 16-byte words
    const size_t o_seed = cv.take(seed_bytes);
    const size_t o_col = cv.take(sizeof(int32_t) * (size_t)L * N);
    const size_t o_d2 = cv.take(sizeof(int32_t) * (size_t)L * N);
    const size_t o_nn = cv.take(sizeof(int32_t) * (size_t)L * N);
    const size_t o_edt = cv.take(edt_scratch_bytes(H, W, L));
    // matrix-core path (its exact integer location product needs positions
    // below 2048): FP6 sample features, records, fix-up queue.  The full image
    // goes in 8 x 4 pixel tiles; a pixel subset of at least kListFastMin
    // entries in tiles of kTilePix consecutive entries (below that the exact
    // kernel, whose set-up is lighter, takes it).
    const bool fast = W <= 2048 && H <= 2048 && (pix_subset == nullptr || npix >= kListFastMin);
    const bool listed = fast && pix_subset != nullptr;
    const int KP = 128 * tex_steps(k);  // bytes of a sample's feature row (32 per lane group and step)
    const int tiles_x = listed ? 1 : (W + 7) / 8;
    const int64_t ntiles = listed ? (npix + kTilePix - 1) / kTilePix
                                  : (int64_t)tiles_x * ((H + 2 * kParzenRB - 1) / (2 * kParzenRB));
    const int64_t ngroups = (ntiles + 3) / 4, ntiles_pad = ngroups * 4;
    const int64_t Mpad_max = M + (int64_t)(kStreamChunk - 1) * L;
    const size_t o_feat = fast ? cv.take((size_t)Mpad_max * KP) : 0;
    const size_t o_srec = fast ? cv.take(sizeof(float) * 12 * (size_t)Mpad_max) : 0;
    const size_t o_fix = fast ? cv.take(sizeof(int2) * (size_t)ntiles_pad * L) : 0;
    const size_t o_pix4 = fast ? cv.take(sizeof(float4) * (size_t)ntiles_pad * kTilePix) : 0;
    const size_t o_aop = fast ? cv.take((size_t)ntiles_pad * kParzenRB * (KP / 128) * 64 * 32) : 0;
    const size_t o_abf = fast ? cv.take((size_t)ntiles_pad * kParzenRB * 64 * 16) : 0;
    const size_t o_coef = cv.take(sizeof(float4) * (size_t)L *
                                  (size_t)(fast ? ntiles_pad * kTilePix : npix));
    const size_t o_rep = mode == 1 ? cv.take(sizeof(uint64_t) * 4 * (size_t)L) : 0;
    const size_t o_crep = mode == 2 ? cv.take(sizeof(float) * (size_t)L * k) : 0;
    // smooth mode: the Parzen stages run on all-zero masks (their texture
    // coefficient is 0, so the masks' values never reach a result)
    const size_t zwords = (size_t)N * ((k + 63) / 64) * 2;
    const size_t o_zmask = mode == 2 ? cv.take(sizeof(uint32_t) * zwords) : 0;
    int rc = ensure_ws(ctx, cv.off);
    if (rc) return rc;
    if (mode == 2) {
        masks = (const uint64_t *)(ctx->ws + o_zmask);
        HIP_TRY(launch_fill_u32(lc_of(ctx), (unsigned int *)(ctx->ws + o_zmask), zwords, 0u));
    }
    int32_t *bc = (int32_t *)(ctx->ws + o_bc), *tf = (int32_t *)(ctx->ws + o_tf);
    unsigned int *cnt = (unsigned int *)(ctx->ws + o_cnt);
    SampleRec *recs = (SampleRec *)(ctx->ws + o_rec);
    uint8_t *seeds = (uint8_t *)(ctx->ws + o_seed);
    int32_t *colrow = (int32_t *)(ctx->ws + o_col), *d2 = (int32_t *)(ctx->ws + o_d2),
            *nearest = (int32_t *)(ctx->ws + o_nn);
    const LaunchCtx lc = lc_of(ctx);

    int32_t *bflags = (int32_t *)(ctx->ws + o_bflags), *pflags = bflags + nblocks;
    const int32_t tag = ctx->tag = ctx->tag >= 0x3FFFFFFF ? 1 : ctx->tag + 1;
    {
        Timed t(ctx, "samples");
        if (pix_subset) HIP_TRY(launch_check_pix(lc, pix_subset, npix, N, pflags));
        // counts, their scan and the totals and flags to the host; the exact
        // kernel's and the fast kernel's counters and queues cleared for this
        // call; the seed plane cleared
        ctx->hcounts[kHostTag] = 0;
        SampleCountArgs sc{};
        sc.label = sample_label;
        sc.pix = sample_pix;
        sc.M = M;
        sc.N = N;
        sc.L = L;
        sc.nblocks = nblocks;
        sc.block_counts = bc;
        sc.block_flags = bflags;
        sc.pix_flags = pflags;
        sc.npix_blocks = npix_blocks;
        sc.totals_flags = tf;
        sc.zero = cnt;
        sc.nzero = (int)((o_queue - o_cnt) / sizeof(unsigned int)) + kParzenQueues * kQueueStride;
        sc.zero2 = ctx->lstats;
        sc.nzero2 = 4;
        sc.host_out = ctx->hcounts_dev;
        sc.tag = tag;
        sc.done = ctx->dctr + kCtrSampleCount;
        HIP_TRY(launch_sample_count(lc, sc, seeds, seed_bytes));
    }
    // The scatter and the distance transforms need no host decision (invalid
    // samples are skipped on the device): they run while the host waits for
    // the counts, which it needs for the segment layout and the constants.
    {
        Timed t(ctx, "samples");
        HIP_TRY(launch_sample_scatter(lc, sample_label, sample_pix, M, L, H, W, rgb, masks, k, bc,
                                      nblocks, recs, seeds));
    }
    if (npix > 0) {
        Timed t(ctx, "edt");
        HIP_TRY(launch_edt(lc, seeds, H, W, L, colrow, d2, nearest, (int32_t *)(ctx->ws + o_edt), pix_subset,
                           pix_subset ? npix : 0));
    }
    int rc_wait = wait_host_tag(ctx, tag);
    if (rc_wait) return rc_wait;
    int32_t counts[kMaxLabels + 1];
    for (int l = 0; l <= L; ++l) counts[l] = ((volatile int32_t *)ctx->hcounts)[l];
    if (counts[L] & 1) return fail(ctx, CS_ERR_ARG, "a sample label or pixel index is out of range");
    if (counts[L] & 2) return fail(ctx, CS_ERR_ARG, "a pixel index of pix_subset is out of range");
    for (int l = 0; l < L; ++l)
        if (counts[l] == 0) return fail(ctx, CS_ERR_EMPTY_LABEL, "label %d has no scribble sample", l);
    if (npix == 0) return CS_OK;

    StreamSegs segs{};
    for (int l = 0; l < L; ++l) {
        segs.seg[l + 1] = segs.seg[l] + counts[l];
        segs.pseg[l + 1] = segs.pseg[l] + (counts[l] + kStreamChunk - 1) / kStreamChunk * kStreamChunk;
    }
    if (fast) {
        Timed t(ctx, "stream");
        const float cscale = (float)std::sqrt(1.4426950408889634 / (2.0 * prm->sigma_c * prm->sigma_c));
        PrepArgs pr{};
        pr.recs = recs;
        pr.k = k;
        pr.KP = KP;
        pr.L = L;
        pr.segs = segs;
        pr.Mpad = segs.pseg[L];
        pr.cscale = cscale;
        pr.levels = prm->colour_levels;
        pr.feat = (uint8_t *)(ctx->ws + o_feat);
        pr.rec = (float *)(ctx->ws + o_srec);
        pr.rgb = rgb;
        pr.masks = masks;
        pr.H = H;
        pr.W = W;
        pr.tiles_x = tiles_x;
        pr.ntiles = (int)ntiles;
        pr.ksteps = KP / 128;
        pr.ntiles_pad = ntiles_pad;
        pr.list = listed ? pix_subset : nullptr;
        pr.nlist = listed ? npix : 0;
        pr.pix4 = (float4 *)(ctx->ws + o_pix4);
        pr.aop = (uint32_t *)(ctx->ws + o_aop);
        pr.abf = (uint4 *)(ctx->ws + o_abf);
        HIP_TRY(launch_prep(lc, pr));
    }
    unsigned int *fcnt = ctx->lstats;
    ParzenArgs pa{};
    pa.rgb = rgb;
    pa.masks = masks;
    pa.recs = recs;
    pa.d2 = d2;
    pa.nearest = nearest;
    pa.subset = pix_subset;
    pa.loglik = loglik;
    pa.work_counter = cnt;
    pa.fixups = cnt + 1;
    pa.H = H;
    pa.W = W;
    pa.L = L;
    pa.k = k;
    pa.nw32 = (k + 31) / 32;
    pa.npix = npix;
    pa.tiles = (int)tiles;
    pa.alpha_rho = prm->alpha_rho;
    pa.sigma_c = prm->sigma_c;
    pa.beta_scale = prm->beta_scale;
    pa.rho_floor = prm->rho_floor_px;
    const double pi = 3.14159265358979323846;
    pa.seg_off[0] = 0;
    for (int l = 0; l < L; ++l) {
        pa.seg_off[l + 1] = pa.seg_off[l] + counts[l];
        pa.kconst[l] = -std::log((double)counts[l]) - std::log(2.0 * pi) -
                       1.5 * std::log(2.0 * pi * prm->sigma_c * prm->sigma_c);
        pa.label_order[l] = l;
    }
    std::stable_sort(pa.label_order, pa.label_order + L,
                     [&](int x, int y) { return counts[x] > counts[y]; });
    pa.texture_in_sum = mode == 0 ? 1 : 0;
    TextureArgs tx{};
    if (mode != 0) {
        tx.recs = recs;
        tx.masks = masks;
        tx.d2 = d2;
        tx.subset = pix_subset;
        tx.rep = (uint64_t *)(ctx->ws + o_rep);
        tx.loglik = loglik;
        tx.N = N;
        tx.npix = npix;
        tx.k = k;
        tx.L = L;
        tx.alpha_rho = prm->alpha_rho;
        tx.beta_scale = prm->beta_scale;
        tx.rho_floor = prm->rho_floor_px;
        tx.W = W;
        tx.alpha = alpha;
        tx.crep = mode == 2 ? (float *)(ctx->ws + o_crep) : nullptr;
        tx.inv_sigma = (float)(1.0 / sigma_iota);
        for (int l = 0; l <= L; ++l) tx.seg[l] = pa.seg_off[l];
        Timed t(ctx, "texture_rep");
        HIP_TRY(mode == 2 ? launch_label_rep_soft(lc, tx) : launch_label_rep(lc, tx));
    }
    float4 *coef = (float4 *)(ctx->ws + o_coef);
    pa.coef = coef;
    pa.coef_tiled = fast ? 1 : 0;
    pa.tiles_x = tiles_x;
    pa.ntiles_real = (int)ntiles;
    pa.ntiles_pad = (int)ntiles_pad;
    {
        Timed t(ctx, "coef");
        HIP_TRY(launch_coef(lc, pa, coef));
    }
    if (fast) {
        ParzenFastArgs fa{};
        fa.rgb = rgb;
        fa.masks = masks;
        fa.feat = (const uint8_t *)(ctx->ws + o_feat);
        fa.rec = (const float *)(ctx->ws + o_srec);
        fa.coef = coef;
        fa.pix4 = (const float4 *)(ctx->ws + o_pix4);
        fa.aop = (const uint32_t *)(ctx->ws + o_aop);
        fa.abf = (const uint8_t *)(ctx->ws + o_abf);
        fa.loglik = loglik;
        fa.work_counter = (unsigned int *)(ctx->ws + o_queue);
        fa.fix_count = fcnt + 1;
        fa.fixlist = (int2 *)(ctx->ws + o_fix);
        fa.H = H;
        fa.W = W;
        fa.L = L;
        fa.k = k;
        fa.ksteps = KP / 128;
        fa.tiles_x = tiles_x;
        fa.ntiles = (int)ntiles;
        fa.ngroups = (int)ngroups;
        fa.fix_cap = (int)(ntiles_pad * L);
        fa.sigma_c = pa.sigma_c;
        fa.levels = prm->colour_levels;
        fa.kcol = prm->colour_levels > 0
                      ? (float)(-1.4426950408889634 / (2.0 * prm->sigma_c * prm->sigma_c *
                                                       (double)prm->colour_levels * prm->colour_levels))
                      : 0.0f;
        fa.texture = pa.texture_in_sum;
        fa.list = listed ? pix_subset : nullptr;
        fa.nlist = listed ? npix : 0;
        // labels per block of the work order: as many as keep their sample
        // streams (features and records of every chunk) within an XCD's 4 MiB
        // L2 together, counted from the largest labels (at least one).  Each
        // pixel group's operands are fetched once per block, and a block's
        // streams stay in L2 while the groups of a queue pass them.  At
        // 1024 x 1024, k = 242, 16 labels (blocks of two) the kernel fetches
        // 3.8 GB per launch; blocks of one label fetched 5.9 GB, of four 41 GB
        // (the streams no longer fit), and blocks cut to the budget one by
        // one (two to five labels) 5.1 GB
        {
            const size_t chunk_bytes = (size_t)(fa.texture ? kStreamChunk * KP : 0) + 12 * sizeof(float) * kStreamChunk;
            const size_t budget = (size_t)4 << 20;
            size_t used = 0;
            int lb = 0;
            while (lb < L) {
                const int l = pa.label_order[lb];  // decreasing sample count
                const size_t bytes = (size_t)((segs.pseg[l + 1] - segs.pseg[l]) / kStreamChunk) * chunk_bytes;
                if (lb > 0 && used + bytes > budget) break;
                used += bytes;
                ++lb;
            }
            fa.lblock = lb;
        }
        // per-label chunk ranges and the label order (kernel arguments: no copy)
        for (int l = 0; l <= L; ++l) fa.meta[l] = segs.pseg[l] / kStreamChunk;
        for (int l = 0; l < L; ++l) fa.meta[L + 1 + l] = pa.label_order[l];
        for (int l = 0; l < L; ++l) {
            const int in_last = counts[l] - (segs.pseg[l + 1] - segs.pseg[l] - kStreamChunk);
            fa.meta[2 * L + 1 + l] = (in_last + 15) / 16;
        }
        ctx->lstats_valid = true;
        {
            Timed t(ctx, "parzen");
            HIP_TRY(launch_parzen_mfma(lc, fa));
        }
        // exact two-pass kernel for the (label, tile) pairs the fast kernel queued
        pa.fixlist = fa.fixlist;
        pa.fix_count = fa.fix_count;
        pa.fix_cap = fa.fix_cap;
        pa.tiles = (int)ntiles_pad;
        {
            Timed t(ctx, "parzen_fixup");
            HIP_TRY(launch_parzen(lc, pa));
        }
    } else {
        ctx->lstats_valid = false;
        Timed t(ctx, "parzen");
        HIP_TRY(launch_parzen(lc, pa));
    }
    if (mode != 0) {
        Timed t(ctx, "texture");
        HIP_TRY(mode == 2 ? launch_texture_post_soft(lc, tx) : launch_texture_post(lc, tx));
    }
    if (prm->normalise) {
        Timed t(ctx, "normalise");
        HIP_TRY(launch_normalise(lc, loglik, npix, L));
    }
    return CS_OK;
}

int cs_label_loglik(cs_ctx *ctx, const float *rgb, int H, int W, const uint64_t *masks, int k,
                    const int32_t *sample_pix, const int32_t *sample_label, int64_t M, int L,
                    const cs_loglik_params *prm, const int32_t *pix_subset, int64_t n_subset,
                    float *loglik) {
    return label_loglik(ctx, rgb, H, W, masks, k, sample_pix, sample_label, M, L, prm, pix_subset,
                        n_subset, loglik, 0);
}

int cs_label_loglik_joint(cs_ctx *ctx, const float *rgb, int H, int W, const uint64_t *masks,
                          int k, const int32_t *sample_pix, const int32_t *sample_label, int64_t M,
                          int L, const cs_loglik_params *prm, const int32_t *pix_subset,
                          int64_t n_subset, float *loglik) {
    return label_loglik(ctx, rgb, H, W, masks, k, sample_pix, sample_label, M, L, prm, pix_subset,
                        n_subset, loglik, 1);
}

int cs_label_loglik_soft(cs_ctx *ctx, const float *rgb, int H, int W, const float *alpha, int k,
                         double sigma_iota, const int32_t *sample_pix, const int32_t *sample_label,
                         int64_t M, int L, const cs_loglik_params *prm, const int32_t *pix_subset,
                         int64_t n_subset, float *loglik) {
    return label_loglik(ctx, rgb, H, W, nullptr, k, sample_pix, sample_label, M, L, prm, pix_subset,
                        n_subset, loglik, 2, alpha, sigma_iota);
}

int cs_last_loglik_stats(cs_ctx *ctx, cs_loglik_stats *stats) {
    if (!ctx || !stats) return CS_ERR_ARG;
    stats->rescaled_chunks = stats->overflow_tiles = stats->exact_tiles = 0;
    if (!ctx->lstats_valid) return CS_OK;
    HIP_TRY(hipMemcpyAsync(ctx->pinned, ctx->lstats, 4 * sizeof(unsigned int),
                           hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    unsigned int c[4];
    std::memcpy(c, ctx->pinned, sizeof c);
    stats->exact_tiles = c[1];
    stats->rescaled_chunks = c[2];
    stats->overflow_tiles = c[3];
    return CS_OK;
}

int cs_profile_enable(cs_ctx *ctx, int on) {
    if (!ctx) return CS_ERR_ARG;
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    for (auto &s : ctx->spans) {
        ctx->pool.push_back(s.a);
        ctx->pool.push_back(s.b);
    }
    ctx->spans.clear();
    ctx->totals.clear();
    ctx->prof_seen.clear();
    ctx->prof = on != 0;
    return CS_OK;
}

int cs_profile_sample(cs_ctx *ctx, int period) {
    if (!ctx) return CS_ERR_ARG;
    if (period < 1) return fail(ctx, CS_ERR_ARG, "period must be >= 1");
    ctx->prof_period = period;
    ctx->prof_seen.clear();
    return CS_OK;
}

int cs_profile_only(cs_ctx *ctx, const char *name) {
    if (!ctx) return CS_ERR_ARG;
    ctx->only = name ? name : "";
    return CS_OK;
}

int cs_profile_read(cs_ctx *ctx, const char *name, double *total_ms, int64_t *launches) {
    if (!ctx || !name || !total_ms || !launches) return CS_ERR_ARG;
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    for (auto &s : ctx->spans) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, s.a, s.b));
        auto &t = ctx->totals[s.name];
        t.first += ms;
        t.second += 1;
        ctx->pool.push_back(s.a);
        ctx->pool.push_back(s.b);
    }
    ctx->spans.clear();
    auto it = ctx->totals.find(name);
    *total_ms = it == ctx->totals.end() ? 0.0 : it->second.first;
    *launches = it == ctx->totals.end() ? 0 : it->second.second;
    return CS_OK;
}

// ---- learned surrogate ----
}  // extern "C"

struct cs_mlp {
    int device = 0;
    int in = 0, in_pad = 0, out = 0;
    int64_t P = 0, off_b1 = 0, off_W2 = 0, off_b2 = 0, off_W3 = 0, off_b3 = 0;
    int64_t t = 0;  // Adam steps taken
    char *mem = nullptr;
    float *params = nullptr, *m = nullptr, *v = nullptr;
    short *W1b = nullptr, *W2b = nullptr, *W3b = nullptr, *W2Tb = nullptr, *W3Tb = nullptr;
};

namespace {

bool mlp_sizes_ok(int in, int hidden, int out) {
    return hidden == kMlpHid && in >= 1 && in <= kMlpMaxIn && out >= 1 && out <= kMlpOutPad;
}

MlpAdamArgs mlp_adam_args(cs_mlp *n) {
    MlpAdamArgs a{};
    a.params = n->params;
    a.m = n->m;
    a.v = n->v;
    a.P = n->P;
    a.off_b1 = n->off_b1;
    a.off_W2 = n->off_W2;
    a.off_b2 = n->off_b2;
    a.off_W3 = n->off_W3;
    a.off_b3 = n->off_b3;
    a.in = n->in;
    a.in_pad = n->in_pad;
    a.out = n->out;
    a.W1b = n->W1b;
    a.W2b = n->W2b;
    a.W3b = n->W3b;
    a.W2Tb = n->W2Tb;
    a.W3Tb = n->W3Tb;
    return a;
}

// Row chunks of the weight-gradient reduction: the largest kc <= 16 whose
// chunks are whole 16-row MFMA steps.
int mlp_kc(int B) {
    for (int kc = 16; kc > 1; --kc)
        if (B % (16 * kc) == 0) return kc;
    return 1;
}

// One forward/backward over B rows (idx or rows 0..B-1), then the weight
// gradients; scratch carved from the context workspace.
int mlp_backprop(cs_ctx *ctx, cs_mlp *n, const float *x, const float *ell, const int32_t *idx, int64_t n_rows,
                 int B, MlpAdamArgs &ad) {
    const int kc = mlp_kc(B);
    const int ntiles = B / 16;
    Carve cv;
    const size_t o_x = cv.take(sizeof(short) * (size_t)n->in_pad * B);
    const size_t o_h1 = cv.take(sizeof(short) * (size_t)kMlpHid * B);
    const size_t o_h2 = cv.take(sizeof(short) * (size_t)kMlpHid * B);
    const size_t o_dy = cv.take(sizeof(short) * (size_t)kMlpOutPad * B);
    const size_t o_dz2 = cv.take(sizeof(short) * (size_t)kMlpHid * B);
    const size_t o_dz1 = cv.take(sizeof(short) * (size_t)kMlpHid * B);
    const size_t o_bg = cv.take(sizeof(float) * (size_t)ntiles * kMlpBiasStride);
    const size_t o_lp = cv.take(sizeof(float) * (size_t)ntiles);
    const size_t o_gp = cv.take(sizeof(float) * (size_t)kc * n->P);
    int rc = ensure_ws(ctx, cv.off);
    if (rc) return rc;
    MlpTrainArgs t{};
    t.x = x;
    t.ell = ell;
    t.idx = idx;
    t.n_rows = n_rows;
    t.B = B;
    t.in = n->in;
    t.in_pad = n->in_pad;
    t.out = n->out;
    t.W1b = n->W1b;
    t.W2b = n->W2b;
    t.W3b = n->W3b;
    t.W2Tb = n->W2Tb;
    t.W3Tb = n->W3Tb;
    t.b1 = n->params + n->off_b1;
    t.b2 = n->params + n->off_b2;
    t.b3 = n->params + n->off_b3;
    t.Xt = (short *)(ctx->ws + o_x);
    t.H1t = (short *)(ctx->ws + o_h1);
    t.H2t = (short *)(ctx->ws + o_h2);
    t.DYt = (short *)(ctx->ws + o_dy);
    t.DZ2t = (short *)(ctx->ws + o_dz2);
    t.DZ1t = (short *)(ctx->ws + o_dz1);
    t.bgrad = (float *)(ctx->ws + o_bg);
    t.lossp = (float *)(ctx->ws + o_lp);
    MlpWgradArgs w{};
    w.Xt = t.Xt;
    w.H1t = t.H1t;
    w.H2t = t.H2t;
    w.DYt = t.DYt;
    w.DZ2t = t.DZ2t;
    w.DZ1t = t.DZ1t;
    w.B = B;
    w.in = n->in;
    w.in_pad = n->in_pad;
    w.out = n->out;
    w.kc = kc;
    w.P = n->P;
    w.off_W1 = 0;
    w.off_W2 = n->off_W2;
    w.off_W3 = n->off_W3;
    w.gpart = (float *)(ctx->ws + o_gp);
    const LaunchCtx lc = lc_of(ctx);
    {
        Timed tm(ctx, "mlp_fwdbwd");
        HIP_TRY(launch_mlp_fwdbwd(lc, t));
    }
    {
        Timed tm(ctx, "mlp_wgrad");
        HIP_TRY(launch_mlp_wgrad(lc, w));
    }
    ad.gpart = w.gpart;
    ad.bgrad = t.bgrad;
    ad.lossp = t.lossp;
    ad.kc = kc;
    ad.ntiles = ntiles;
    ad.B = B;
    return CS_OK;
}

}  // namespace

extern "C" {

int64_t cs_mlp_param_count(int in_dim, int hidden, int out_dim) {
    if (!mlp_sizes_ok(in_dim, hidden, out_dim)) return 0;
    return (int64_t)hidden * in_dim + hidden + (int64_t)hidden * hidden + hidden + (int64_t)out_dim * hidden +
           out_dim;
}

int cs_mlp_init(cs_ctx *ctx, cs_mlp **net, int in_dim, int hidden, int out_dim, const float *params) {
    if (!ctx) return CS_ERR_ARG;
    if (!net || !params) return fail(ctx, CS_ERR_ARG, "net and params must be non-null");
    *net = nullptr;
    if (!mlp_sizes_ok(in_dim, hidden, out_dim))
        return fail(ctx, CS_ERR_ARG, "unsupported network: hidden must be %d, in_dim 1..%d, out_dim 1..%d", kMlpHid,
                    kMlpMaxIn, kMlpOutPad);
    HIP_TRY(hipSetDevice(ctx->device));
    cs_mlp *n = new (std::nothrow) cs_mlp();
    if (!n) return fail(ctx, CS_ERR_NOMEM, "host allocation failed");
    n->device = ctx->device;
    n->in = in_dim;
    n->in_pad = (in_dim + 15) / 16 * 16;
    n->out = out_dim;
    n->off_b1 = (int64_t)kMlpHid * in_dim;
    n->off_W2 = n->off_b1 + kMlpHid;
    n->off_b2 = n->off_W2 + (int64_t)kMlpHid * kMlpHid;
    n->off_W3 = n->off_b2 + kMlpHid;
    n->off_b3 = n->off_W3 + (int64_t)out_dim * kMlpHid;
    n->P = n->off_b3 + out_dim;
    Carve cv;
    const size_t o_p = cv.take(sizeof(float) * n->P), o_m = cv.take(sizeof(float) * n->P),
                 o_v = cv.take(sizeof(float) * n->P);
    const size_t o_w1 = cv.take(sizeof(short) * kMlpHid * n->in_pad);
    const size_t o_w2 = cv.take(sizeof(short) * kMlpHid * kMlpHid);
    const size_t o_w2t = cv.take(sizeof(short) * kMlpHid * kMlpHid);
    const size_t o_w3 = cv.take(sizeof(short) * kMlpOutPad * kMlpHid);
    const size_t o_w3t = cv.take(sizeof(short) * kMlpHid * kMlpOutPad);
    if (hipMalloc((void **)&n->mem, cv.off) != hipSuccess) {
        delete n;
        return fail(ctx, CS_ERR_NOMEM, "network memory of %zu bytes could not be allocated", cv.off);
    }
    n->params = (float *)(n->mem + o_p);
    n->m = (float *)(n->mem + o_m);
    n->v = (float *)(n->mem + o_v);
    n->W1b = (short *)(n->mem + o_w1);
    n->W2b = (short *)(n->mem + o_w2);
    n->W2Tb = (short *)(n->mem + o_w2t);
    n->W3b = (short *)(n->mem + o_w3);
    n->W3Tb = (short *)(n->mem + o_w3t);
    const LaunchCtx lc = lc_of(ctx);
    int rc = CS_OK;
    auto chk = [&](hipError_t e) {
        if (e != hipSuccess && rc == CS_OK) rc = fail(ctx, CS_ERR_HIP, "network set-up: %s", hipGetErrorString(e));
    };
    chk(launch_fill_u32(lc, (unsigned int *)n->mem, cv.off / 4, 0u));  // zeros: moments and padding
    chk(hipMemcpyAsync(n->params, params, sizeof(float) * n->P, hipMemcpyDeviceToDevice, ctx->stream));
    MlpAdamArgs a = mlp_adam_args(n);
    chk(launch_mlp_convert(lc, a));
    if (rc) {
        hipFree(n->mem);
        delete n;
        return rc;
    }
    *net = n;
    return CS_OK;
}

int cs_mlp_free(cs_mlp *net) {
    if (!net) return CS_OK;
    hipSetDevice(net->device);
    hipDeviceSynchronize();
    if (net->mem) hipFree(net->mem);
    delete net;
    return CS_OK;
}

int cs_mlp_get_params(cs_ctx *ctx, const cs_mlp *net, float *params) {
    if (!ctx) return CS_ERR_ARG;
    if (!net || !params) return fail(ctx, CS_ERR_ARG, "net and params must be non-null");
    HIP_TRY(hipMemcpyAsync(params, net->params, sizeof(float) * net->P, hipMemcpyDeviceToDevice, ctx->stream));
    return CS_OK;
}

int cs_mlp_features(cs_ctx *ctx, const float *rgb, int H, int W, const float *alpha, int k, const int32_t *pix,
                    int64_t n, float *x) {
    if (!ctx) return CS_ERR_ARG;
    if (n < 0 || H < 1 || W < 1 || k < 1 || 5 + k > kMlpMaxIn)
        return fail(ctx, CS_ERR_ARG, "bad sizes (n >= 0, H, W >= 1, 1 <= k <= %d)", kMlpMaxIn - 5);
    if (n == 0) return CS_OK;
    if (!rgb || !alpha || !pix || !x) return fail(ctx, CS_ERR_ARG, "null pointer argument");
    HIP_TRY(hipSetDevice(ctx->device));
    Timed tm(ctx, "mlp_features");
    HIP_TRY(launch_mlp_features(lc_of(ctx), rgb, H, W, alpha, k, pix, n, x));
    return CS_OK;
}

int cs_mlp_grad(cs_ctx *ctx, cs_mlp *net, const float *x, const float *ell, int64_t n, float *grad, float *loss) {
    if (!ctx) return CS_ERR_ARG;
    if (!net || !x || !ell || !grad) return fail(ctx, CS_ERR_ARG, "null pointer argument");
    if (n < 16 || n > 8192 || n % 16) return fail(ctx, CS_ERR_ARG, "n must be a multiple of 16 in 16..8192");
    HIP_TRY(hipSetDevice(ctx->device));
    MlpAdamArgs a = mlp_adam_args(net);
    int rc = mlp_backprop(ctx, net, x, ell, nullptr, n, (int)n, a);
    if (rc) return rc;
    a.grad_out = grad;
    a.loss_out = loss;
    Timed tm(ctx, "mlp_adam");
    HIP_TRY(launch_mlp_adam(lc_of(ctx), a));
    return CS_OK;
}

int cs_mlp_train(cs_ctx *ctx, cs_mlp *net, const float *x, const float *ell, int64_t n_rows, const int32_t *order,
                 int64_t steps, int batch, double lr, float *loss_trace) {
    if (!ctx) return CS_ERR_ARG;
    if (!net || !x || !ell || !order) return fail(ctx, CS_ERR_ARG, "null pointer argument");
    if (batch < 16 || batch > 8192 || batch % 16) return fail(ctx, CS_ERR_ARG, "batch must be a multiple of 16 in 16..8192");
    if (steps < 0 || n_rows < 1) return fail(ctx, CS_ERR_ARG, "steps must be >= 0 and n_rows >= 1");
    if (!(lr > 0.0) || !std::isfinite(lr)) return fail(ctx, CS_ERR_ARG, "lr must be positive and finite");
    HIP_TRY(hipSetDevice(ctx->device));
    for (int64_t s = 0; s < steps; ++s) {
        MlpAdamArgs a = mlp_adam_args(net);
        int rc = mlp_backprop(ctx, net, x, ell, order + s * batch, n_rows, batch, a);
        if (rc) return rc;
        net->t += 1;
        a.lr = (float)lr;
        a.bc1 = (float)(1.0 - std::pow(0.9, (double)net->t));
        a.bc2 = (float)(1.0 - std::pow(0.999, (double)net->t));
        a.loss_out = loss_trace ? loss_trace + s : nullptr;
        Timed tm(ctx, "mlp_adam");
        HIP_TRY(launch_mlp_adam(lc_of(ctx), a));
    }
    return CS_OK;
}

int cs_mlp_fit_output_bias(cs_ctx *ctx, cs_mlp *net, const float *ell, int64_t n) {
    if (!ctx) return CS_ERR_ARG;
    if (!net || !ell || n < 1) return fail(ctx, CS_ERR_ARG, "null pointer or n < 1");
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(launch_mlp_bias_mean(lc_of(ctx), ell, n, net->out, net->params + net->off_b3));
    return CS_OK;
}

static int mlp_forward_impl(cs_ctx *ctx, const cs_mlp *net, const float *x, const float *rgb, int H, int W,
                            const float *alpha, int k, int64_t n, float *out) {
    HIP_TRY(hipSetDevice(ctx->device));
    MlpInferArgs a{};
    a.x = x;
    a.rgb = rgb;
    a.alpha = alpha;
    a.H = H;
    a.W = W;
    a.k = k;
    a.n = n;
    a.in = net->in;
    a.in_pad = net->in_pad;
    a.out = net->out;
    a.W1b = net->W1b;
    a.W2b = net->W2b;
    a.W3b = net->W3b;
    a.b1 = net->params + net->off_b1;
    a.b2 = net->params + net->off_b2;
    a.b3 = net->params + net->off_b3;
    a.y = out;
    Timed tm(ctx, "mlp_infer");
    HIP_TRY(launch_mlp_infer(lc_of(ctx), a));
    return CS_OK;
}

int cs_mlp_infer(cs_ctx *ctx, const cs_mlp *net, const float *rgb, int H, int W, const float *alpha, int k,
                 float *out) {
    if (!ctx) return CS_ERR_ARG;
    if (!net || !rgb || !alpha || !out) return fail(ctx, CS_ERR_ARG, "null pointer argument");
    if (H < 1 || W < 1 || (int64_t)H * W > ((int64_t)1 << 31) - 1) return fail(ctx, CS_ERR_ARG, "bad image size");
    if (net->in != 5 + k) return fail(ctx, CS_ERR_ARG, "in_dim %d does not match 5 + k = %d", net->in, 5 + k);
    return mlp_forward_impl(ctx, net, nullptr, rgb, H, W, alpha, k, (int64_t)H * W, out);
}

int cs_mlp_forward(cs_ctx *ctx, const cs_mlp *net, const float *x, int64_t n, float *out) {
    if (!ctx) return CS_ERR_ARG;
    if (!net || n < 0) return fail(ctx, CS_ERR_ARG, "bad arguments");
    if (n == 0) return CS_OK;
    if (!x || !out) return fail(ctx, CS_ERR_ARG, "null pointer argument");
    return mlp_forward_impl(ctx, net, x, nullptr, 1, 1, nullptr, 0, n, out);
}

int cs_mlp_infer_fallback(cs_ctx *ctx, const cs_mlp *net, const float *rgb, int H, int W, const float *alpha, int k,
                          const uint64_t *masks, int kmask, const int32_t *sample_pix, const int32_t *sample_label,
                          int64_t M, int L, const cs_loglik_params *prm, double margin, float *out,
                          int64_t *n_exact) {
    if (!ctx) return CS_ERR_ARG;
    if (!net || !rgb || !alpha || !out || !masks) return fail(ctx, CS_ERR_ARG, "null pointer argument");
    if (net->out != L) return fail(ctx, CS_ERR_ARG, "out_dim %d does not match L = %d", net->out, L);
    if (!(margin >= 0.0) || !std::isfinite(margin)) return fail(ctx, CS_ERR_ARG, "margin must be finite and >= 0");
    int rc = cs_mlp_infer(ctx, net, rgb, H, W, alpha, k, out);
    if (rc) return rc;
    const int64_t N = (int64_t)H * W;
    // list (N int32) then the count, then room for the exact rows of every
    // pixel (the count is known only after the list is made)
    const size_t o_cnt = ((size_t)N * 4 + 255) / 256 * 256;
    const size_t o_ex = o_cnt + 256;
    if ((rc = ensure_fb(ctx, o_ex + sizeof(float) * (size_t)N * L))) return rc;
    const LaunchCtx lc = lc_of(ctx);
    int32_t *list = (int32_t *)ctx->fb;
    unsigned int *cnt = (unsigned int *)(ctx->fb + o_cnt);
    HIP_TRY(launch_fill_u32(lc, cnt, 1, 0u));
    {
        Timed t(ctx, "mlp_uncertain");
        HIP_TRY(launch_mlp_uncertain(lc, out, N, L, (float)margin, list, cnt));
    }
    HIP_TRY(hipMemcpyAsync(ctx->pinned, cnt, sizeof(unsigned int), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    unsigned int m = 0;
    std::memcpy(&m, ctx->pinned, sizeof m);
    if (n_exact) *n_exact = (int64_t)m;
    if (m == 0) return CS_OK;
    float *ex = (float *)(ctx->fb + o_ex);
    rc = label_loglik(ctx, rgb, H, W, masks, kmask, sample_pix, sample_label, M, L, prm, list, (int64_t)m, ex, 0);
    if (rc) return rc;
    Timed t(ctx, "mlp_scatter");
    HIP_TRY(launch_mlp_scatter_rows(lc, ex, list, (int64_t)m, L, out));
    return CS_OK;
}

// ---- segmentation by convex relaxation ----
}  // extern "C"

namespace {

int check_segment_image(cs_ctx *ctx, const float *rgb, int H, int W) {
    if (!rgb) return fail(ctx, CS_ERR_ARG, "rgb must be non-null");
    if (H < 1 || W < 1 || (int64_t)H * W > ((int64_t)1 << 31) - 1)
        return fail(ctx, CS_ERR_ARG, "bad image size %dx%d", W, H);
    return CS_OK;
}

// Edge metric into g (working precision) and/or g32; returns the gamma used
// (read back on the host: a mean of zero, an image without gradient, leaves
// the metric undefined and is an argument error).
int edge_weight_stage(cs_ctx *ctx, const float *rgb, int H, int W, double gamma, int precision, void *g,
                      float *g32, double *mag, double *part, double *gamma_dev, double *gamma_used) {
    const LaunchCtx lc = lc_of(ctx);
    {
        Timed t(ctx, "edge_weight");
        HIP_TRY(launch_edge_weight(lc, rgb, H, W, gamma, mag, part, precision, g, g32, gamma_dev));
    }
    HIP_TRY(hipMemcpyAsync(ctx->pinned, gamma_dev, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    std::memcpy(gamma_used, ctx->pinned, sizeof(double));
    if (!(*gamma_used > 0.0) || !std::isfinite(*gamma_used))
        return fail(ctx, CS_ERR_ARG, "the edge metric needs gamma > 0 (the image has no gradient; pass gamma)");
    return CS_OK;
}

}  // namespace

extern "C" {

int cs_edge_weight(cs_ctx *ctx, const float *rgb, int H, int W, double gamma, float *g, double *gamma_out) {
    if (!ctx) return CS_ERR_ARG;
    int rc = check_segment_image(ctx, rgb, H, W);
    if (rc) return rc;
    if (!g) return fail(ctx, CS_ERR_ARG, "g must be non-null");
    if (std::isnan(gamma) || std::isinf(gamma)) return fail(ctx, CS_ERR_ARG, "gamma must be finite");
    HIP_TRY(hipSetDevice(ctx->device));
    if ((rc = check_inputs_finite(ctx, rgb, 3 * (int64_t)H * W, nullptr, 0, 0))) return rc;
    const int64_t N = (int64_t)H * W;
    Carve cv;
    const size_t o_mag = cv.take(sizeof(double) * (size_t)N);
    const size_t o_part = cv.take(sizeof(double) * (size_t)((N + 255) / 256));
    const size_t o_gam = cv.take(sizeof(double));
    if ((rc = ensure_ws(ctx, cv.off))) return rc;
    double used = 0.0;
    rc = edge_weight_stage(ctx, rgb, H, W, gamma, CS_FP32, nullptr, g, (double *)(ctx->ws + o_mag),
                           (double *)(ctx->ws + o_part), (double *)(ctx->ws + o_gam), &used);
    if (rc) return rc;
    if (gamma_out) *gamma_out = used;
    return CS_OK;
}

int cs_segment(cs_ctx *ctx, const float *rgb, int H, int W, const float *loglik, int L,
               const cs_segment_params *prm, int32_t *labels, float *u, cs_segment_stats *stats) {
    if (!ctx) return CS_ERR_ARG;
    int rc = check_segment_image(ctx, rgb, H, W);
    if (rc) return rc;
    if (!loglik || !prm || !labels) return fail(ctx, CS_ERR_ARG, "null pointer argument");
    if (L < 1 || L > kMaxLabels) return fail(ctx, CS_ERR_ARG, "L must be in 1..%d (got %d)", kMaxLabels, L);
    if (!(prm->lambda >= 0.0) || !std::isfinite(prm->lambda)) return fail(ctx, CS_ERR_ARG, "lambda must be finite and >= 0");
    if (!(prm->nu >= 0.0) || !std::isfinite(prm->nu)) return fail(ctx, CS_ERR_ARG, "nu must be finite and >= 0");
    if (std::isnan(prm->gamma) || std::isinf(prm->gamma)) return fail(ctx, CS_ERR_ARG, "gamma must be finite");
    if (prm->iterations < 0 || prm->iterations > 1000000)
        return fail(ctx, CS_ERR_ARG, "iterations must be in 0..1000000");
    if (prm->precision != CS_FP32 && prm->precision != CS_FP64)
        return fail(ctx, CS_ERR_ARG, "precision must be CS_FP32 or CS_FP64");
    HIP_TRY(hipSetDevice(ctx->device));
    if ((rc = check_inputs_finite(ctx, rgb, 3 * (int64_t)H * W, loglik, (int64_t)H * W * L, 0))) return rc;
    const int64_t N = (int64_t)H * W;
    const int64_t nb = (N + 255) / 256;
    const bool mdl = prm->nu > 0.0;
    const size_t es = prm->precision == CS_FP64 ? sizeof(double) : sizeof(float);
    const size_t plane = es * (size_t)N * L;
    Carve cv;
    const size_t o_mag = cv.take(sizeof(double) * (size_t)N);
    const size_t o_part = cv.take(sizeof(double) * (size_t)nb * (3 + L));
    const size_t o_small = cv.take(sizeof(double) * 8);  // gamma, energies, labels present
    const size_t o_g = cv.take(es * (size_t)N);
    const size_t o_f = cv.take(plane);
    size_t o_state[2][5];
    for (int b = 0; b < 2; ++b)
        for (int v = 0; v < 5; ++v) o_state[b][v] = (v < 4 || mdl) ? cv.take(plane) : 0;
    const size_t o_m = cv.take(sizeof(double) * (size_t)(prm->iterations + 1) * L);
    const size_t o_ms = cv.take(sizeof(double) * (size_t)(prm->iterations + 1) * L);
    if ((rc = ensure_ws(ctx, cv.off))) return rc;
    char *ws = ctx->ws;
    double *small = (double *)(ws + o_small);
    unsigned long long *used = (unsigned long long *)(small + 4);
    const LaunchCtx lc = lc_of(ctx);
    HIP_TRY(launch_fill_u32(lc, (unsigned int *)used, 2, 0u));
    double gamma = 0.0;
    rc = edge_weight_stage(ctx, rgb, H, W, prm->gamma, prm->precision, ws + o_g, nullptr, (double *)(ws + o_mag),
                           (double *)(ws + o_part), small, &gamma);
    if (rc) return rc;
    PdArgs a{};
    a.H = H;
    a.W = W;
    a.L = L;
    a.iters = prm->iterations;
    a.mdl = mdl ? 1 : 0;
    a.N = N;
    a.lambda = prm->lambda;
    a.nu = prm->nu;
    // diagonal preconditioning (alpha = 1) with the interior column sums
    a.sigma_xi = 0.5;
    a.sigma_mu = 0.5;
    a.tau_u = mdl ? 0.2 : 0.25;
    a.tau_m = 1.0 / (double)N;
    a.g = ws + o_g;
    a.f = ws + o_f;
    for (int b = 0; b < 2; ++b) {
        a.u[b] = ws + o_state[b][0];
        a.ub[b] = ws + o_state[b][1];
        a.px[b] = ws + o_state[b][2];
        a.py[b] = ws + o_state[b][3];
        a.mu[b] = mdl ? ws + o_state[b][4] : nullptr;
    }
    a.mval = (double *)(ws + o_m);
    a.msum = (double *)(ws + o_ms);
    {
        Timed t(ctx, "pd_init");
        HIP_TRY(launch_pd_init(lc, a, prm->precision, loglik));
    }
    for (int it = 0; it < prm->iterations; ++it) {
        Timed t(ctx, "pd_iter");
        HIP_TRY(launch_pd_iter(lc, a, prm->precision, it));
    }
    {
        Timed t(ctx, "pd_finish");
        HIP_TRY(launch_pd_finish(lc, a, prm->precision, labels, u, used, (double *)(ws + o_part),
                                 stats ? small + 1 : nullptr));
    }
    if (stats) {
        HIP_TRY(hipMemcpyAsync(ctx->pinned, small, sizeof(double) * 5, hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(hipStreamSynchronize(ctx->stream));
        double e[4];
        unsigned long long bits;
        std::memcpy(e, ctx->pinned, sizeof(double) * 4);
        std::memcpy(&bits, ctx->pinned + 4 * sizeof(double), sizeof bits);
        stats->gamma = gamma;
        stats->labels_used = __builtin_popcountll(bits);
        stats->primal = e[1];
        stats->binary = e[2] + prm->nu * (double)stats->labels_used;
        stats->dual = e[3];
    }
    return CS_OK;
}

int cs_unsupervised_loglik(cs_ctx *ctx, const float *rgb, int H, int W, const uint64_t *masks, int k,
                           const int32_t *init_colour, const int32_t *init_texture, const cs_unsup_params *prm,
                           float *loglik, double *colour_centroids, uint64_t *texture_centroids,
                           int32_t *colour_labels, int32_t *texture_labels) {
    if (!ctx) return CS_ERR_ARG;
    int rc = check_segment_image(ctx, rgb, H, W);
    if (rc) return rc;
    if (!masks || !init_colour || !init_texture || !prm || !loglik) return fail(ctx, CS_ERR_ARG, "null pointer argument");
    if (k < 1 || k > kMaxK) return fail(ctx, CS_ERR_ARG, "k must be in 1..%d (got %d)", kMaxK, k);
    const int Kc = prm->colour_classes, Kt = prm->texture_classes;
    if (Kc < 1 || Kc > kUnsupMaxClasses || Kt < 1 || Kt > kUnsupMaxClasses || Kc * Kt > kMaxLabels)
        return fail(ctx, CS_ERR_ARG, "colour and texture classes must be in 1..%d with a product of at most %d",
                    kUnsupMaxClasses, kMaxLabels);
    if (prm->iterations < 0 || prm->iterations > 100000) return fail(ctx, CS_ERR_ARG, "iterations must be in 0..100000");
    auto pos = [](double v) { return v > 0.0 && std::isfinite(v); };
    if (!pos(prm->sigma_c) || !pos(prm->beta)) return fail(ctx, CS_ERR_ARG, "sigma_c and beta must be positive and finite");
    const int64_t N = (int64_t)H * W;
    UnsupInit init{};
    for (int i = 0; i < Kc; ++i) init.pix[i] = init_colour[i];
    for (int i = 0; i < Kt; ++i) init.pix[Kc + i] = init_texture[i];
    for (int i = 0; i < Kc + Kt; ++i)
        if (init.pix[i] < 0 || init.pix[i] >= N) return fail(ctx, CS_ERR_ARG, "an initial pixel is out of range");
    HIP_TRY(hipSetDevice(ctx->device));
    if ((rc = check_inputs_finite(ctx, rgb, 3 * N, nullptr, 0, 0))) return rc;
    const int nw = (k + 63) / 64;
    const int64_t nb = (N + 255) / 256;
    Carve cv;
    const size_t o_cc = cv.take(sizeof(double) * Kc * 3);
    const size_t o_tc = cv.take(sizeof(uint64_t) * Kt * nw);
    const size_t o_cl = cv.take(sizeof(int32_t) * (size_t)N);
    const size_t o_tl = cv.take(sizeof(int32_t) * (size_t)N);
    const size_t o_cp = cv.take(sizeof(double) * (size_t)nb * Kc * 4);
    const size_t o_tn = cv.take(sizeof(unsigned int) * ((size_t)Kt * k + Kt));
    if ((rc = ensure_ws(ctx, cv.off))) return rc;
    UnsupArgs a{};
    a.rgb = rgb;
    a.masks = masks;
    a.N = N;
    a.H = H;
    a.W = W;
    a.k = k;
    a.nw = nw;
    a.Kc = Kc;
    a.Kt = Kt;
    a.sigma_c = prm->sigma_c;
    a.beta = prm->beta;
    a.ccent = colour_centroids ? colour_centroids : (double *)(ctx->ws + o_cc);
    a.tcent = texture_centroids ? texture_centroids : (uint64_t *)(ctx->ws + o_tc);
    a.clab = colour_labels ? colour_labels : (int32_t *)(ctx->ws + o_cl);
    a.tlab = texture_labels ? texture_labels : (int32_t *)(ctx->ws + o_tl);
    a.cpart = (double *)(ctx->ws + o_cp);
    a.tcount = (unsigned int *)(ctx->ws + o_tn);
    a.tsize = a.tcount + (size_t)Kt * k;
    const LaunchCtx lc = lc_of(ctx);
    HIP_TRY(launch_fill_u32(lc, a.tcount, (size_t)Kt * k + Kt, 0u));
    HIP_TRY(launch_unsup_init(lc, a, init));
    {
        Timed t(ctx, "kmeans");
        for (int it = 0; it < prm->iterations; ++it) HIP_TRY(launch_kmeans_step(lc, a, true));
        HIP_TRY(launch_kmeans_step(lc, a, false));
    }
    {
        Timed t(ctx, "kmedians");
        for (int it = 0; it < prm->iterations; ++it) HIP_TRY(launch_kmedians_step(lc, a, true));
        HIP_TRY(launch_kmedians_step(lc, a, false));
    }
    Timed t(ctx, "unsup_loglik");
    HIP_TRY(launch_unsup_loglik(lc, a, loglik));
    return CS_OK;
}

}  // extern "C"
