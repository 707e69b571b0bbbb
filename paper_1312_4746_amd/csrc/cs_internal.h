// Internal declarations shared by the host layer and the HIP kernels of the
// co-sparse data-term library (gfx950).  Not part of the C-ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

namespace cs {

// Pixels per analysis tile (one row segment of the image).
constexpr int kTilePx = 64;
// Words of a sample record (see SampleRec).
constexpr int kRecWords = 16;
// 16-pixel row blocks per wave in the MFMA Parzen kernel: a wave owns an
// 8 x (2 kParzenRB) pixel tile of kTilePix pixels.
constexpr int kParzenRB = 2;
// Work queues of the full-image Parzen kernel: one per XCD (workgroups are
// dispatched to the 8 XCDs round-robin), each counter on its own 128-byte line.
constexpr int kParzenQueues = 8;
constexpr int kQueueStride = 32;  // unsigned ints
constexpr int kTilePix = 8 * 2 * kParzenRB;
// Texture features of the matrix-core Parzen path (FP6 dot product of the
// TSM, see k_parzen_mfma.hip): the k mask bits, then tex_digits(k) + 1 slots
// for |A| and as many for |B|; 128 features per MFMA step.
__host__ __device__ constexpr int tex_digits(int k) { return (k / 7 + 6) / 7; }
__host__ __device__ constexpr int tex_features(int k) { return k + 2 * tex_digits(k) + 2; }
__host__ __device__ constexpr int tex_steps(int k) { return (tex_features(k) + 127) / 128; }
// Smallest pixel subset that the matrix-core Parzen path takes.
constexpr int64_t kListFastMin = 1024;

// Slot q (0 .. kTilePix-1) of tile t on the matrix-core Parzen path.  On the
// tile grid (list == nullptr) it is pixel (x0 + q % 8, y0 + q / 8) of the
// image, tiles_x tiles per band of 2 kParzenRB rows, and the output row is
// that pixel; with a pixel list the slot is list entry t kTilePix + q and the
// output row is that entry's index.  -1: outside the image or past the list.
__device__ __forceinline__ int64_t fast_slot_row(const int32_t *list, int64_t nlist, int H, int W, int tiles_x,
                                                 int ntiles, int t, int q) {
    if (list) {
        const int64_t s = (int64_t)t * kTilePix + q;
        return s < nlist ? s : -1;
    }
    const int ty = t / tiles_x;
    const int px = (t - ty * tiles_x) * 8 + (q & 7), py = ty * 2 * kParzenRB + (q >> 3);
    return t < ntiles && px < W && py < H ? (int64_t)py * W + px : -1;
}
// The pixel behind an output row of fast_slot_row (row >= 0).
__device__ __forceinline__ int64_t fast_row_pixel(const int32_t *list, int64_t row) {
    return list ? (int64_t)list[row] : row;
}
// Samples per chunk of the padded sample stream (label segments are rounded
// up to whole chunks).
constexpr int kStreamChunk = 64;
// Maximum label count and co-support length handled by the kernels.
constexpr int kMaxLabels = 64;
constexpr int kMaxK = 256;

// One scribble sample, gathered from its pixel, 64 bytes so that a wave
// fetches it with one scalar load: x (column), y (row), r, g, b as float32
// bit patterns, three unused words, then up to 8 32-bit co-support words.
struct SampleRec {
    uint32_t w[kRecWords];
};

struct LaunchCtx {
    hipStream_t stream;
    int num_cu;
};

// ---- analysis (k_analyze.hip) ----
struct AnalyzeArgs {
    const float *rgb;
    int H, W, p, n, n_pad, k;
    const double *wmask;  // n doubles, device
    const float *omega;   // k x n
    float *alpha;         // N x k or null
    uint64_t *masks;      // N x ceil(k/64) or null
    const float *t_in;    // k thresholds (|a| <= t_in: in)
    const float *t_out;   // k thresholds (|a| > t_out: out)
    double tau;
    unsigned long long *recomputed;  // device counter or null
    double *pstats;       // N x 2 exact patch statistics (mean, squared norm) out, or null
    // optional: the first workgroup also sets up the median selection that
    // follows (state, the three digit histograms, per-row margins); null st:
    // none
    struct TauState *tau_st;
    unsigned int *tau_hist3;       // 3 x kHistBins, cleared
    double *tau_margins;           // k per-row bounds
    double *tau_max_margin;        // their maximum
    double tau_coef;
    unsigned long long tau_rank0;  // target rank
};
hipError_t launch_analyze(const LaunchCtx &lc, const AnalyzeArgs &a, int precision);

// The Gaussian patch mask table written to device memory by a one-workgroup
// kernel that receives it by value as a kernel argument (no copy from host
// memory, no allocation).
struct MaskTable {
    double w[15 * 15];
};
hipError_t launch_put_table(const LaunchCtx &lc, double *dst, const MaskTable &t, int n);

// Masks from stored analysed vectors, same decisions as the analysis epilogue.
// A non-null tau_dev (device) replaces tau, read by the kernel.
hipError_t launch_mask_alpha(const LaunchCtx &lc, const float *alpha, int64_t N, int k, const float *t_in,
                             const float *t_out, double tau, const double *tau_dev, const float *rgb, int H,
                             int W, int p,
                             const double *wmask, const float *omega, uint64_t *masks,
                             unsigned long long *recomputed, const double *pstats);

// Per-row thresholds t_in/t_out = tau -/+ margin_j, rounded outward to float.
// margin < 0 selects the proven bound coef * ||O_j||_2 + tiny; writes the
// largest margin to *max_margin.  A non-null tau_dev (device) replaces tau;
// a non-null zero (device counter) is cleared.
hipError_t launch_thresholds(const LaunchCtx &lc, const float *omega, int k, int n, double tau,
                             const double *tau_dev, double margin, double coef, float *t_in, float *t_out,
                             double *margins, double *max_margin, unsigned long long *zero);

// ---- exact median of |alpha| (k_tau.hip) ----
constexpr int kHistBins = 2048;  // radix digit histogram bins
struct TauState {
    unsigned long long rank0;     // target rank floor((count-1)/2)
    unsigned long long rank;      // remaining rank inside the current prefix
    unsigned int prefix;          // float bits selected so far
    // folded selection: prefix and remaining rank after digit d (d = 0: none
    // yet), written by the kernel that picks digit d, read by the next
    unsigned int pfx[4];
    unsigned long long rk[4];
    unsigned int nparts;          // per-workgroup counts of entries below the window
    unsigned long long below;     // their sum (written by the selection)
    unsigned long long ncand;     // candidates found (may exceed capacity)
    double lo, hi;                // candidate window on |alpha| (float values)
    double median;                // exact FP64 median
    double tau;                   // frac * median
    unsigned long long n_d;       // deferred mask entries (fused co-support pass)
    unsigned long long n_r;       // deferred entries for the FP64 decision
    // fused co-support pass: its waves and the entries of each wave's region
    // of the candidate and deferred lists (wave w writes from w * rg_size on)
    unsigned int rg_waves;
    long long rg_size;
};
// Upper bound of the workgroups of a candidate gather (per-workgroup counts);
// the counts array is followed by kTauRank words for the ranks of short
// candidate lists.
constexpr int kTauParts = 1 << 16;
constexpr int kTauRank = 1 << 14;
// Radix select of the float |alpha| of the target rank; the first kernel also
// writes the largest per-row error bound (coef) of the rows of omega, and the
// per-row bounds to margins when non-null.
// The first two digits of the same selection, each picked at the start of
// the next kernel (every workgroup from the complete histogram): the state,
// the histograms (hist3, cleared) and the margins come from the analysis
// kernel before; the second digit is picked by the candidate gather, which
// gathers over the whole bin of the top 22 bits (no third digit pass).
hipError_t tau_digits_folded(const LaunchCtx &lc, const float *alpha, int64_t count, unsigned int *hist3,
                             TauState *st);
hipError_t tau_select_float(const LaunchCtx &lc, const float *alpha, int64_t count,
                            unsigned int *hist, TauState *st, const float *omega, int k, int n,
                            double coef, double *max_margin, double *margins);
hipError_t tau_reset_gather(const LaunchCtx &lc, TauState *st);
// The state reset, the row bounds and the first (11-bit) digit only.
hipError_t tau_first_digit(const LaunchCtx &lc, const float *alpha, int64_t count, unsigned int *hist,
                           TauState *st, const float *omega, int k, int n, double coef, double *max_margin,
                           double *margins);
// Pick the digit at `shift` holding the remaining rank; clears the histogram.
hipError_t tau_pick(const LaunchCtx &lc, unsigned int *hist, int shift, TauState *st);
// Candidates of the window around the selected float; parts (kTauParts
// entries) receives per-workgroup counts of the entries below the window.
hipError_t tau_gather(const LaunchCtx &lc, const float *alpha, int64_t count,
                      const double *max_margin, TauState *st, int64_t *cand, int64_t cap,
                      unsigned long long *parts);
// FP64 recompute of the candidates and the exact selection; the candidate
// count is read on the device (at most cap are used; more leaves NaN).  tau
// also goes to tau_out (device) when non-null.  parts holds kTauParts +
// kTauRank words.
// Compact forms of the fused co-support pass's per-wave lists: region
// offsets (kMedianWavesMax words each) and lists of up to kListCap entries.
constexpr int64_t kListCap = (int64_t)1 << 22;
struct FusedLists {
    unsigned long long *coff, *doff;
    int64_t *ccomp, *dcomp;
};
// Scan of the region counts (totals into st->ncand, st->n_d) and the copy of
// each list that fits kListCap into its compact array.
hipError_t list_compact(const LaunchCtx &lc, int64_t nw, const int64_t *cand, const unsigned int *ccnt,
                        const int64_t *didx, const unsigned int *dcnt, TauState *st, FusedLists fl);
// pstats: the exact patch statistics of every pixel (N x 2) or null.  With
// ccnt non-null the candidates come from the fused co-support pass (fl: its
// compact list, or its per-wave regions of cand when it did not fit).
hipError_t tau_finish(const LaunchCtx &lc, const float *rgb, int H, int W, int p, int n,
                      const double *wmask, const float *omega, int k, const int64_t *cand,
                      int64_t cap, double *vals, double frac, TauState *st, unsigned long long *parts,
                      double *tau_out, const double *pstats, const unsigned int *ccnt = nullptr,
                      const FusedLists *fl = nullptr);
// Device counters of a context that are zero between calls (each use resets
// its own): [kCtrSampleCount] the sample-count workgroups done,
// [kCtrNonFinite] the flag of the optional finite check of the inputs.
constexpr int kCtrSampleCount = 0, kCtrNonFinite = 1, kCtrWords = 64;
// Sets *flag (device, zero before) to 1 when any of the n floats at p is a NaN
// or an infinity.
hipError_t launch_check_finite(const LaunchCtx &lc, const float *p, int64_t n, int levels, unsigned int *flag);

// ---- co-support at frac * median|a| fused with the candidate gather
// (k_cosupport_median.hip) ----
// After the three digits: the candidate window and the masks of every entry
// whose rounded |a| is clear of the tau interval by more than its row margin.
// Each wave lists its candidates and the other undecided entries in its own
// region of cand and didx (both with room for N*k entries; counts in ccnt and
// dcnt, kMedianWavesMax words each), so the pass takes no global atomics.
constexpr int kMedianWavesMax = 4 * kTauParts;
hipError_t median_mask_gather(const LaunchCtx &lc, const float *alpha, int64_t N, int k,
                              const double *max_margin, const double *margins, double frac, TauState *st,
                              int64_t *cand, unsigned int *ccnt, unsigned long long *parts, int64_t *didx,
                              unsigned int *dcnt, uint64_t *masks, const unsigned int *hist3);
// After the exact tau: the listed entries, decided in one launch (the rounded
// value where it is clear of tau by the row margin, else in FP64).
hipError_t median_mask_finish(const LaunchCtx &lc, const float *alpha, const float *rgb, int H, int W, int p,
                              const double *wmask, const float *omega, int k, const int64_t *didx,
                              const unsigned int *dcnt, const int64_t *dcomp, const double *margins,
                              const TauState *st, uint64_t *masks, const double *pstats);
// The number of waves of median_mask_gather for N pixels.
int64_t median_gather_waves(int64_t N);

// ---- texture similarity (k_tsm.hip) ----
hipError_t launch_tsm(const LaunchCtx &lc, const uint64_t *A, int64_t na, const uint64_t *B,
                      int64_t nb, int k, int32_t *out);

// ---- samples, distance transform, Parzen sum (k_parzen.hip, k_edt.hip) ----
// Host-memory slot that k_sample_scan sets to its tag once totals and flags
// are visible to the host.
constexpr int kHostTag = 255;
// Label counts per chunk of samples, their scan and the hand-over of the
// label totals to the host (host_out, then the tag), and the per-label seed
// plane cleared (seed_bytes, a multiple of 16), in one launch.
struct SampleCountArgs {
    const int32_t *label, *pix;
    int64_t M, N;
    int L, nblocks;
    int32_t *block_counts, *block_flags;
    const int32_t *pix_flags;  // workgroup flags of the pixel-list check (npix_blocks)
    int npix_blocks;
    int32_t *totals_flags;     // device copy of the totals and flags (L + 1)
    unsigned int *zero;        // counters cleared for the kernels that follow
    int nzero;
    unsigned int *zero2;       // a second such region (context-owned counters) or null
    int nzero2;
    int32_t *host_out;         // coherent host memory (device address)
    int32_t tag;
    unsigned int *done;        // device counter, zero between calls
    // set by launch_sample_count
    uint4 *seeds16;
    int64_t nseed16;
    int nclear;
};
hipError_t launch_sample_count(const LaunchCtx &lc, SampleCountArgs a, uint8_t *seeds, size_t seed_bytes);
int check_pix_blocks(const LaunchCtx &lc, int64_t n);
hipError_t launch_sample_scatter(const LaunchCtx &lc, const int32_t *label, const int32_t *pix,
                                 int64_t M, int L, int H, int W, const float *rgb,
                                 const uint64_t *masks, int k, const int32_t *block_counts,
                                 int nblocks, SampleRec *recs, uint8_t *seeds);
hipError_t launch_check_pix(const LaunchCtx &lc, const int32_t *pix, int64_t n, int64_t N, int32_t *flags);
size_t edt_scratch_bytes(int H, int W, int L);
// list (or null: every pixel): with a list of npix entries the row pass runs
// for the listed pixels only (d2 and nearest of other pixels are left as they
// were); the listed entries equal those of the full pass bit for bit
hipError_t launch_edt(const LaunchCtx &lc, const uint8_t *seeds, int H, int W, int L,
                      int32_t *colrow, int32_t *d2, int32_t *nearest, int32_t *scratch,
                      const int32_t *list = nullptr, int64_t npix = 0);

struct ParzenArgs {
    const float *rgb;
    const uint64_t *masks;
    const SampleRec *recs;
    const int32_t *d2;       // L x N
    const int32_t *nearest;  // L x N
    const int32_t *subset;   // or null
    float *loglik;
    unsigned int *work_counter;
    unsigned int *fixups;
    // fix-up mode: items are (label, 8x8 tile) pairs queued by the MFMA kernel
    const int2 *fixlist;
    const unsigned int *fix_count;
    int fix_cap;
    int tiles_x;
    // coefficients {nA, nB, -R, K} (k_coef): [label][npix] for a pixel list, or
    // tiled [label][ntiles_pad][kTilePix] for the full image
    // (with coef_tiled and a subset, the slots of the tiles are the subset's
    // entries in order: see fast_slot_row)
    const float4 *coef;
    int coef_tiled, ntiles_real, ntiles_pad;
    int H, W, L, k, nw32;
    int64_t npix;
    int tiles;               // ceil(npix / 64)
    double alpha_rho, sigma_c, beta_scale, rho_floor;
    int texture_in_sum;      // 0: the texture factor leaves the Parzen sum
    int seg_off[kMaxLabels + 1];
    int label_order[kMaxLabels];
    double kconst[kMaxLabels];  // -log m_i - log(2 pi) - 1.5 log(2 pi sigma_c^2)
};
hipError_t launch_parzen(const LaunchCtx &lc, const ParzenArgs &a);

// ---- joint texture factor (k_texture.hip) ----
struct TextureArgs {
    const SampleRec *recs;   // samples sorted by label
    const uint64_t *masks;   // N x ceil(k/64)
    const int32_t *d2;       // L x N squared distances to the nearest sample
    const int32_t *subset;   // or null
    uint64_t *rep;           // L x 4 words, the label representatives
    float *loglik;           // npix x L, updated in place
    int64_t N, npix;
    int k, L, W;
    double alpha_rho, beta_scale, rho_floor;
    // smooth co-supports: analysed vectors N x k, representatives L x k
    const float *alpha;
    float *crep;
    float inv_sigma;         // 1 / sigma of the smooth map
    int seg[kMaxLabels + 1];
};
hipError_t launch_label_rep(const LaunchCtx &lc, const TextureArgs &a);
hipError_t launch_texture_post(const LaunchCtx &lc, const TextureArgs &a);
hipError_t launch_label_rep_soft(const LaunchCtx &lc, const TextureArgs &a);
hipError_t launch_texture_post_soft(const LaunchCtx &lc, const TextureArgs &a);
hipError_t launch_coef(const LaunchCtx &lc, const ParzenArgs &a, float4 *coef);

struct StreamSegs {
    int seg[kMaxLabels + 1];   // label segments of the sorted samples
    int pseg[kMaxLabels + 1];  // the same segments rounded up to whole chunks
};
struct ParzenFastArgs {
    const float *rgb;
    const uint64_t *masks;
    const uint8_t *feat;   // Mpad x 128*ksteps FP6 sample features (swizzled rows, 32 B per 32 features)
                           // (positions below 2048: the location product is exact)
    const float *rec;      // per chunk of 64 slots: BF16 location pieces (2 x 1 KiB), colours (1 KiB:
                           // scaled floats, or BF16 colour pieces with levels > 0)
    const float4 *coef;    // tiled: [label][group*4 + tile][kTilePix] {nA, nB, -R, K}
    const float4 *pix4;    // tiled: [group*4 + tile][kTilePix] {scaled r, g, b, |A|}
    const uint32_t *aop;   // [tile][row block][step][lane][8]: FP6 texture operands (6 of 8 dwords)
    const uint8_t *abf;    // [tile][row block][lane][16 B]: BF16 location (and colour) operands
    float *loglik;
    unsigned int *work_counter;  // kParzenQueues counters, kQueueStride apart, zero at launch
    unsigned int *fix_count;  // [0] queued (label, tile), [1] rescaled wave-chunks, [2] overflowed passes
    int2 *fixlist;
    int fix_cap;
    int H, W, L, k, ksteps;
    int tiles_x, ntiles, ngroups;
    int texture;           // 0: texture factor out of the sum (no FP6 products)
    int lblock;            // labels per block of the work order (1..L)
    const int32_t *list;   // pixel list (tile slots are its entries) or null (tile grid)
    int64_t nlist;
    double sigma_c;
    // colour levels n > 0: colours are the integers rint(c n) and the colour
    // term is kcol times their squared distance (kcol = -log2(e) / (2 sigma_c^2
    // n^2)), formed on the matrix cores; 0: scaled float colours on the VALU
    int levels;
    float kcol;
    // passed by value (kernel arguments): [0..L] first chunk of each label's
    // padded segment (chunk units), [L+1 .. 2L] the labels by decreasing
    // sample count, [2L+1 .. 3L] the 16-sample steps of each label's last
    // chunk that hold real samples
    int meta[3 * kMaxLabels + 1];
};
// The full-image path's per-call preparation (one launch): the sample stream
// (FP6 features and per-chunk records), the tiled pixel records and the pixel
// operands of both MFMAs.
struct PrepArgs {
    const SampleRec *recs;
    int k, KP, L;
    StreamSegs segs;
    int64_t Mpad;
    float cscale;
    int levels;            // colour levels n (0: float colours; see ParzenFastArgs::levels)
    uint8_t *feat;
    float *rec;
    const float *rgb;
    const uint64_t *masks;
    int H, W, tiles_x, ntiles, ksteps;
    int64_t ntiles_pad;
    const int32_t *list;   // pixel list (tile slots are its entries) or null (tile grid)
    int64_t nlist;
    float4 *pix4;
    uint32_t *aop;
    uint4 *abf;
    // set by launch_prep
    int64_t nslots, nthreads;
    int b_stream, b_tiles;
};
hipError_t launch_prep(const LaunchCtx &lc, PrepArgs a);
hipError_t launch_parzen_mfma(const LaunchCtx &lc, const ParzenFastArgs &a);
// Pixel records of the full-image path (nslots = padded tiles x kTilePix).
// MFMA pixel operands of the full-image path (ntiles_pad tiles).
hipError_t launch_normalise(const LaunchCtx &lc, float *loglik, int64_t npix, int L);

// ---- segmentation by convex relaxation (k_segment.hip) ----
// State of the primal-dual iteration: label-major planes of N values in the
// working precision (float or double), ping-pong pairs for the iterated fields.
struct PdArgs {
    int H, W, L, iters, mdl;
    int64_t N;
    double lambda, nu, sigma_xi, sigma_mu, tau_u, tau_m;
    const void *g;           // edge metric, N values
    void *f;                 // data term f_i = -l_i, L planes
    void *u[2], *ub[2], *px[2], *py[2], *mu[2];
    double *mval;            // (iters + 1) x L: m^t
    double *msum;            // (iters + 1) x L: sum_x mu^t (zero before)
};
// |grad I| into mag (N doubles), per-workgroup partial sums into part
// (ceil(N / 256) doubles), then g in the working precision (g, N values) and/or
// FP32 (g32), and the gamma used (gamma_out, device, nullable).
hipError_t launch_edge_weight(const LaunchCtx &lc, const float *rgb, int H, int W, double gamma, double *mag,
                              double *part, int precision, void *g, float *g32, double *gamma_out);
// Start state (and f = -loglik as planes), iteration t (reads buffer t & 1,
// writes the other), then the labels (and u pixel-major into u_out when
// non-null), the labels present (used, zero before) and, with energies
// non-null, {primal, binary without label cost, dual} (part: ceil(N / 256) x
// (3 + L) doubles of scratch).
hipError_t launch_pd_init(const LaunchCtx &lc, const PdArgs &a, int precision, const float *loglik);
hipError_t launch_pd_iter(const LaunchCtx &lc, const PdArgs &a, int precision, int t);
hipError_t launch_pd_finish(const LaunchCtx &lc, const PdArgs &a, int precision, int32_t *labels, float *u_out,
                            unsigned long long *used, double *part, double *energies);

// ---- unsupervised data term (k_unsup.hip) ----
constexpr int kUnsupMaxClasses = 16;  // colour or texture classes
struct UnsupArgs {
    const float *rgb;
    const uint64_t *masks;
    int64_t N;
    int H, W, k, nw, Kc, Kt;
    double sigma_c, beta;
    double *ccent;          // Kc x 3 colour centroids
    uint64_t *tcent;        // Kt x nw texture centroids
    int32_t *clab, *tlab;   // N colour and texture classes
    double *cpart;          // ceil(N / 256) x Kc x 4 partial sums
    unsigned int *tcount;   // Kt x k bit counts (zero before an assignment with counts)
    unsigned int *tsize;    // Kt class sizes (idem)
};
struct UnsupInit {
    int32_t pix[2 * kUnsupMaxClasses];  // pixels of the first centroids: Kc colour, then Kt texture
};
hipError_t launch_unsup_init(const LaunchCtx &lc, const UnsupArgs &a, const UnsupInit &init);
// One assignment (and, with update, the centroids moved to their classes).
hipError_t launch_kmeans_step(const LaunchCtx &lc, const UnsupArgs &a, bool update);
hipError_t launch_kmedians_step(const LaunchCtx &lc, const UnsupArgs &a, bool update);
hipError_t launch_unsup_loglik(const LaunchCtx &lc, const UnsupArgs &a, float *loglik);

// ---- learned surrogate (k_mlp.hip) ----
constexpr int kMlpHid = 128;                          // hidden units per layer
constexpr int kMlpMaxIn = 128;                        // input features (padded to 16)
constexpr int kMlpOutPad = 16;                        // outputs (labels), padded
constexpr int kMlpBiasStride = 2 * kMlpHid + kMlpOutPad;
struct MlpTrainArgs {
    const float *x;        // rows x in (FP32)
    const float *ell;      // rows x out raw log-likelihoods
    const int32_t *idx;    // B row indices, or null (row b)
    int64_t n_rows;        // rows of x and ell (indices are clamped to them)
    int B, in, in_pad, out;
    const short *W1b, *W2b, *W3b, *W2Tb, *W3Tb;  // BF16 working copies
    const float *b1, *b2, *b3;
    short *Xt, *H1t, *H2t, *DYt, *DZ2t, *DZ1t;   // feature-major [unit][B]
    float *bgrad;          // [B/16][kMlpBiasStride] per-tile bias-gradient sums
    float *lossp;          // [B/16] per-tile squared error
};
struct MlpWgradArgs {
    const short *Xt, *H1t, *H2t, *DYt, *DZ2t, *DZ1t;
    int B, in, in_pad, out, kc;
    int64_t P, off_W1, off_W2, off_W3;
    float *gpart;          // [kc][P]
};
struct MlpAdamArgs {
    float *params, *m, *v;
    const float *gpart, *bgrad, *lossp;
    float *grad_out;       // non-null: write the gradient, no update
    float *loss_out;       // non-null: mean loss of the batch
    int64_t P, off_b1, off_W2, off_b2, off_W3, off_b3;
    int kc, ntiles, B, in, in_pad, out;
    float lr, bc1, bc2;    // step size, 1 - beta1^t, 1 - beta2^t
    short *W1b, *W2b, *W3b, *W2Tb, *W3Tb;
};
struct MlpInferArgs {
    const float *x;        // explicit rows x in, or null: features from rgb/alpha
    const float *rgb, *alpha;
    int H, W, k;
    int64_t n;
    int in, in_pad, out;
    const short *W1b, *W2b, *W3b;
    const float *b1, *b2, *b3;
    float *y;              // n x out
};
hipError_t launch_mlp_fwdbwd(const LaunchCtx &lc, const MlpTrainArgs &a);
hipError_t launch_mlp_wgrad(const LaunchCtx &lc, const MlpWgradArgs &a);
hipError_t launch_mlp_adam(const LaunchCtx &lc, const MlpAdamArgs &a);
hipError_t launch_mlp_convert(const LaunchCtx &lc, const MlpAdamArgs &a);
hipError_t launch_mlp_infer(const LaunchCtx &lc, const MlpInferArgs &a);
hipError_t launch_mlp_bias_mean(const LaunchCtx &lc, const float *ell, int64_t n, int out, float *b3);
// Exact fallback of the surrogate: pixels whose top-two outputs differ by less
// than margin are listed (count zero before), and exact rows are put back.
hipError_t launch_mlp_uncertain(const LaunchCtx &lc, const float *y, int64_t n, int L, float margin, int32_t *list,
                                unsigned int *count);
hipError_t launch_mlp_scatter_rows(const LaunchCtx &lc, const float *ex, const int32_t *list, int64_t m, int L,
                                   float *out);
hipError_t launch_mlp_features(const LaunchCtx &lc, const float *rgb, int H, int W, const float *alpha, int k,
                               const int32_t *pix, int64_t n, float *x);
hipError_t launch_fill_u32(const LaunchCtx &lc, unsigned int *p, size_t count, unsigned int v);

}  // namespace cs
