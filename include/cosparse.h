/*
 * cosparse.h -- C-ABI of the MI355X (gfx950) co-sparse data-term library.
 *
 * Method: Nieuwenhuis, Hawe, Kleinsteuber, Cremers, "Co-Sparse Textural
 * Similarity for Image Segmentation" (arXiv 1312.4746).  The library computes,
 * for every pixel x and label i, the log-likelihood l_i(x) = -f_i(x) of the
 * supervised data term (Sec. 3.1, Sec. 3.2): every pixel's normalised gray
 * patch is analysed by the operator O (Sec. 2), the analysed vector is
 * thresholded into a co-support, co-supports are compared with the texture
 * similarity TSM (Sec. 2), and TSM is combined with colour and location
 * Gaussian kernels in the spatially varying Parzen sum over each label's
 * scribble samples (Sec. 3.1).
 *
 * Conventions shared by every call:
 *  - Images are three float32 planes R, G, B, each H*W, in DEVICE memory;
 *    pixel x = (col, row) has linear index row*W + col.  N = H*W.
 *  - Patches are p x p (p odd, 3..15), n = p*p, element t = (u+h)*p + (v+h)
 *    for row offset u and column offset v in [-h, h], h = (p-1)/2; borders
 *    use symmetric reflection that repeats the edge pixel.
 *  - The operator O is k x n float32 row-major in DEVICE memory, 1 <= k <= 256.
 *  - A co-support mask is ceil(k/64) uint64 words per pixel; index j is bit
 *    (j mod 64) of word j/64; bits at j >= k are 0.
 *  - Every pointer marked "device" is caller-owned device memory, "host" is
 *    caller-owned host memory.  The library never frees or keeps caller
 *    pointers beyond the work it enqueues; device buffers must stay alive until
 *    the context's stream has completed that work.
 *  - All calls enqueue asynchronously on the context's HIP stream and return,
 *    except where a call returns a host value (noted), which synchronises it.
 *  - Calls return CS_OK or an error code; they never abort or throw.  Argument
 *    errors are detected before anything is launched.  cs_last_error gives a
 *    message.  A context is used by one host thread at a time.
 */
#ifndef COSPARSE_H
#define COSPARSE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CS_OK 0
#define CS_ERR_ARG 1          /* invalid argument (null pointer, size or range) */
#define CS_ERR_EMPTY_LABEL 2  /* some label has no scribble sample (m_i = 0)     */
#define CS_ERR_HIP 3          /* a HIP runtime call failed                        */
#define CS_ERR_NOMEM 4        /* device workspace allocation failed               */
#define CS_ERR_NONFINITE 5    /* an input holds a NaN or an infinity (optional    */
                              /* check, see cs_set_check_finite)                  */

#define CS_FP32 0 /* O s on FP32 MFMA, FP32 accumulation                        */
#define CS_BF16 1 /* O s on BF16 MFMA (both operands rounded), FP32 accumulation */
#define CS_FP64 2 /* (segmentation only) the primal-dual iteration in FP64        */

typedef struct cs_ctx cs_ctx;

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the default stream).  The context owns a device
 * workspace that grows on demand and is freed by cs_destroy. */
int cs_create(cs_ctx **ctx, int device, void *hip_stream);
int cs_destroy(cs_ctx *ctx);
/* Switch the stream later calls enqueue on (the workspace is not copied). */
int cs_set_stream(cs_ctx *ctx, void *hip_stream);
/* Message of the last failed call on this context ("" if none). */
const char *cs_last_error(const cs_ctx *ctx);
/* Optional finite check of the inputs (default off).  When on, every call
 * that reads an image or an operator (cs_analyze_patches, cs_tau_median,
 * cs_cosupport, cs_cosupport_median: rgb and omega; the cs_label_loglik
 * forms: rgb) first scans them on the device, synchronises the stream and
 * returns CS_ERR_NONFINITE, launching nothing else, if any value is a NaN
 * or an infinity.  The method's arithmetic is only defined on finite
 * colours and operator entries (Sec. 2, Sec. 3.1).  Off, no call
 * synchronises for it and non-finite inputs give unspecified outputs. */
int cs_set_check_finite(cs_ctx *ctx, int on);

/*
 * Analysed vectors a = O s_x of every pixel (Sec. 2; the patch s_x of Sec. 3.1
 * is the gray patch, multiplied element-wise by the Gaussian mask
 * w_t = exp(-(u^2+v^2)/(2 mask_sigma^2)) and normalised to zero mean and unit
 * norm; a patch of zero norm gives s = 0).  The patch is formed in FP64; the
 * contraction runs on MFMA in `precision` with FP32 accumulation.
 *   rgb    device, 3*H*W float32         omega  device, k*n float32
 *   alpha  device out, N*k float32, pixel-major (alpha[x*k + j])
 * Errors: CS_ERR_ARG for null pointers, even p, p outside 3..15, H or W < h+1,
 * k outside 1..256, mask_sigma <= 0, unknown precision.
 */
int cs_analyze_patches(cs_ctx *ctx, const float *rgb, int H, int W, int p, double mask_sigma,
                       const float *omega, int k, int precision, float *alpha);

/*
 * Exact co-support threshold tau = frac * median{|a_j(x)|} over all N*k
 * entries, the median being the entry of rank floor((N*k-1)/2) in ascending
 * order of the exact (FP64) analysed vectors.  The threshold replaces the
 * exact-zero test of the Sec. 2 co-support definition.  `alpha` must be the
 * output of cs_analyze_patches for the same inputs and precision; entries whose
 * rounded value lies within the proven error bound of the selected median are
 * recomputed in FP64, so tau equals the FP64 value bit for bit.  With
 * precision CS_BF16 the selection runs on an FP32 analysis made inside the
 * call (its error bound, and so its candidate window, is far smaller); the
 * context keeps that N*k float buffer until it is destroyed.
 *   alpha   device, N*k float32, 16-byte aligned
 *   tau_out host out.  Synchronises the stream (returns a host value).
 * Errors: as cs_analyze_patches, plus CS_ERR_ARG for frac < 0 or NaN or a
 * misaligned alpha; CS_ERR_HIP if the exact median falls outside the
 * candidate window (the error bound would have been violated).
 */
int cs_tau_median(cs_ctx *ctx, const float *rgb, int H, int W, int p, double mask_sigma,
                  const float *omega, int k, int precision, const float *alpha, double frac,
                  double *tau_out);

typedef struct {
    int64_t recomputed; /* entries decided by the FP64 recompute          */
    double max_margin;  /* largest per-row margin used                      */
} cs_cosupport_stats;

/*
 * Co-support masks (Sec. 2 co-support definition with threshold tau):
 * bit j of pixel x is 1 iff |a_j(x)| <= tau for the exact (FP64) a.  The
 * rounded analysed vectors come from `alpha` (the output of
 * cs_analyze_patches for the same inputs and precision) or, when alpha is
 * NULL, are recomputed on MFMA in `precision` inside the call; every entry
 * whose rounded |a| lies within `margin` of tau is recomputed in FP64 (the
 * library's only FP64 contraction) and decided exactly.
 * margin < 0 selects the proven per-row error bound of the precision, which
 * makes the masks equal to the FP64 masks bit for bit; margin >= 0 is an
 * absolute margin (entries outside it are decided by the rounded value).
 *   alpha  device, N*k float32, or NULL
 *   masks  device out, N*ceil(k/64) uint64
 *   stats  host out or NULL; non-NULL synchronises the stream.
 * Errors: as cs_analyze_patches, plus CS_ERR_ARG for tau < 0 or NaN.
 */
int cs_cosupport(cs_ctx *ctx, const float *rgb, int H, int W, int p, double mask_sigma,
                 const float *omega, int k, int precision, const float *alpha, double tau,
                 double margin, uint64_t *masks, cs_cosupport_stats *stats);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the masks of
 * cs_cosupport, bit for bit, from a call that allocates nothing.  Its scratch
 * (per-row thresholds and margins, a counter and the patch mask table, at
 * most 8 KiB: k <= 256, p <= 15 always fit) lives in a static device array of
 * the library, one per device, set up by cs_create and held until the process
 * ends; the call only launches kernels on the context's stream (no copy, no
 * synchronisation, no allocation, no event).  Every call on one device shares
 * that array: calls that overlap on one device (other streams, other contexts,
 * other host threads) race and must be ordered by the caller.  No statistics
 * are returned and the optional finite check is not applied (both would
 * synchronise).
 * Arguments, layouts, ownership and errors: as cs_cosupport (without stats);
 * CS_ERR_ARG also when the scratch would exceed its maximum.
 */
int cs_cosupport_noalloc(cs_ctx *ctx, const float *rgb, int H, int W, int p, double mask_sigma,
                         const float *omega, int k, int precision, const float *alpha, double tau,
                         double margin, uint64_t *masks);

/*
 * The whole co-support step of Sec. 2 from pixels, with no host round trip:
 * analysed vectors (as cs_analyze_patches), tau = frac * median{|a|} selected
 * exactly on the device (as cs_tau_median), and the masks at that tau (as
 * cs_cosupport with alpha).  Results equal those of the three calls bit for
 * bit.  The call only enqueues work; tau stays on the device.  With the
 * proven margin (margin < 0) the masks are decided in the pass that gathers
 * the candidates of the exact median: an entry clear of the interval that
 * tau is known to lie in by then is decided at once, the few others once tau
 * is selected.  In BF16 that pass runs on the FP32 analysis that tau is
 * selected on (at the proven margin the masks are the exact masks either
 * way), and the BF16 analysis then writes alpha.  The context reserves device memory for lists that could
 * hold every entry (24 bytes per entry of N*k; 16 bytes in the other forms),
 * so that their lengths never need the host.
 *   alpha    device out, N*k float32, 16-byte aligned
 *   masks    device out, N*ceil(k/64) uint64
 *   tau_dev  device out (one double) or NULL: tau, written in stream order.
 *            NaN if the exact median fell outside the candidate window (the
 *            error bound would have been violated; the masks are then not
 *            meaningful).
 * Errors: as cs_analyze_patches, plus CS_ERR_ARG for frac < 0 or NaN, a
 * non-finite margin, null or misaligned alpha, null masks.
 */
int cs_cosupport_median(cs_ctx *ctx, const float *rgb, int H, int W, int p, double mask_sigma,
                        const float *omega, int k, int precision, double frac, double margin, float *alpha,
                        uint64_t *masks, double *tau_dev);

/*
 * Texture similarity (Sec. 2, TSM definition): out[a*nb + b] = number of
 * indices j < k in exactly one of the co-supports A[a] and B[b] (the Hamming
 * distance of the masks; bits at j >= k are ignored).
 *   A device, na*ceil(k/64) uint64; B device, nb*ceil(k/64); out device, na*nb int32.
 * Errors: CS_ERR_ARG for null pointers with nonzero counts, k outside 1..256,
 * negative counts.
 */
int cs_texture_similarity(cs_ctx *ctx, const uint64_t *A, int64_t na, const uint64_t *B,
                          int64_t nb, int k, int32_t *out);

typedef struct {
    double alpha_rho;    /* spatial bandwidth scale (Sec. 3.1 sets 1.3)               */
    double sigma_c;      /* colour kernel standard deviation, RGB units (0.05)        */
    double beta_scale;   /* b in beta_i(x) = b * rho_i(x) (beta proportional to rho)  */
    double rho_floor_px; /* rho_i(x) = alpha_rho * max(d_i(x), rho_floor_px)          */
    int normalise;       /* 1: subtract log sum_i exp l_i(x) (labels normalise)       */
    int colour_levels;   /* 0: colours are any floats; n in 1..255: every colour      */
                         /* value is a multiple of 1/n in [0, 255/n] (n = 255 for     */
                         /* 8-bit images), see below                                  */
} cs_loglik_params;

/*
 * Per-pixel, per-label log-likelihood of the supervised data term
 * (Sec. 3.1 Parzen sum; Sec. 3.2 data term f_i = -l_i):
 *   l_i(x) = log( 1/m_i * sum_{y in S_i} N2(x; y, rho_i(x)^2) * N3(I(x); I(y), sigma_c^2)
 *                                        * exp(-TSM(x, y) / beta_i(x)) )
 * where S_i are the samples with label i (m_i = |S_i|), rho_i(x) = alpha_rho *
 * max(d_i(x), rho_floor_px) with d_i(x) the exact Euclidean distance from x to
 * the nearest sample of label i, beta_i(x) = beta_scale * rho_i(x), N2/N3 are
 * normalised isotropic Gaussians, and each sample's colour, position and mask
 * are those of its pixel.  Computed in FP32 with log-sum-exp accumulation.
 *   rgb           device, 3*H*W float32
 *   masks         device, N*ceil(k/64) uint64 (co-supports of every pixel)
 *   sample_pix    device, M int32 linear pixel indices (0..N-1)
 *   sample_label  device, M int32 labels (0..L-1), 1 <= L <= 64
 *   prm           host
 *   pix_subset    device, n_subset int32 pixel indices, or NULL for all N pixels
 *   loglik        device out, (n_subset or N) * L float32, loglik[r*L + i]
 *                 (may be NULL when pix_subset is non-NULL and n_subset is 0)
 * Colour levels: with colour_levels = n > 0 the matrix-core kernel takes each
 * colour value c as the integer q = rint(c n) (clamped to 0..255), so that the
 * squared colour distance of two pixels is the integer sum over channels of
 * (q_x - q_y)^2, formed exactly on the matrix cores and scaled by 1/n^2; for a
 * value that is the FP32 rounding of a multiple of 1/n this differs from the
 * FP32 input by less than 2^-24 relative.  Values that are not such multiples
 * are rounded to the nearest one (the data term of the rounded image); with
 * the finite check on (cs_set_check_finite), such a value, or one outside
 * [0, 255/n], returns CS_ERR_ARG.  The exact per-pixel kernel and the
 * coefficients use the FP32 values either way.
 * Route: images up to 2048 x 2048 go to the matrix-core kernel, the full
 * image in 8 x 4 pixel tiles, a subset of 1024 or more entries in tiles of 32
 * consecutive entries (duplicates allowed); smaller subsets and larger images
 * to the exact per-pixel kernel.  Both give the same sums within FP32
 * rounding; on the matrix-core path a pixel's row does not depend on which
 * other pixels are computed with it.
 * Synchronises once after sorting the samples by label (to check labels).
 * Errors: CS_ERR_ARG (null pointers, H outside 1..32767, W outside 1..16384,
 * k outside 1..256, L outside 1..64, prm values <= 0 or not finite, sample
 * pixel, sample label or subset pixel out of range), CS_ERR_EMPTY_LABEL when
 * some label has no sample.
 */
int cs_label_loglik(cs_ctx *ctx, const float *rgb, int H, int W, const uint64_t *masks, int k,
                    const int32_t *sample_pix, const int32_t *sample_label, int64_t M, int L,
                    const cs_loglik_params *prm, const int32_t *pix_subset, int64_t n_subset,
                    float *loglik);

/*
 * The paper's own combination of the two factors (eq:joined): the colour and
 * location Parzen density of eq:color times the texture posterior of
 * eq:post_text,
 *   l_i(x) = log( 1/m_i * sum_{y in S_i} N2(x; y, rho_i(x)^2) * N3(I(x); I(y), sigma_c^2) )
 *            + u_i(x) - log sum_i' exp u_i'(x),   u_i(x) = -TSM(x, c_i) / beta_i(x),
 * where c_i is the textural representative of label i (Sec. 2, majority
 * definition; Sec. 3.1): bit j of c_i is set iff at least half of the
 * label's samples have j in their co-support (2 count_j >= m_i, the
 * component-wise median of eq:approx_cosupp for hard co-supports).  rho_i,
 * beta_i, the arguments, layouts, ownership, synchronisation and errors are
 * those of cs_label_loglik; prm->normalise is applied last.
 */
int cs_label_loglik_joint(cs_ctx *ctx, const float *rgb, int H, int W, const uint64_t *masks,
                          int k, const int32_t *sample_pix, const int32_t *sample_label, int64_t M,
                          int L, const cs_loglik_params *prm, const int32_t *pix_subset,
                          int64_t n_subset, float *loglik);

/*
 * The joint form with the smooth co-support of Sec. 2 (eq:map_tsm), the
 * setting of the paper's experiments: iota(a)_j = exp(-a_j^2 / sigma_iota)
 * (the paper uses sigma_iota = 0.01), the texture distance of eq:tsm and the
 * median representative of eq:approx_cosupp:
 *   l_i(x) = log( 1/m_i * sum_{y in S_i} N2(x; y, rho_i(x)^2) * N3(I(x); I(y), sigma_c^2) )
 *            + u_i(x) - log sum_i' exp u_i'(x),   u_i(x) = -||c_i - iota(a_x)||_1 / beta_i(x),
 * c_ij = the element of rank floor(m_i/2) of the ascending iota(a_y)_j over
 * the label's samples y (the upper median; for 0/1 values the majority of
 * cs_label_loglik_joint).
 *   alpha       device, N*k float32 analysed vectors of every pixel, row-major
 *               (as written by cs_analyze_patches)
 *   sigma_iota  > 0 and finite
 * The other arguments, layouts, ownership, synchronisation and errors are
 * those of cs_label_loglik (no masks are read); CS_ERR_ARG also for
 * sigma_iota.
 */
int cs_label_loglik_soft(cs_ctx *ctx, const float *rgb, int H, int W, const float *alpha, int k,
                         double sigma_iota, const int32_t *sample_pix, const int32_t *sample_label,
                         int64_t M, int L, const cs_loglik_params *prm, const int32_t *pix_subset,
                         int64_t n_subset, float *loglik);

typedef struct {
    int64_t rescaled_chunks;  /* wave-chunks whose log-sum-exp reference moved up   */
    int64_t overflow_tiles;   /* (label, tile) pairs whose fast sum overflowed       */
    int64_t exact_tiles;      /* (label, tile) pairs finished by the exact two-pass  */
                              /* kernel (overflow, non-finite or empty sums)         */
} cs_loglik_stats;

/* Counters of the last log-likelihood call (any of the three forms) on this
 * context that got past its argument checks: matrix-core path only (full
 * image, or a subset of 1024 or more pixels), zeros for a call that took the
 * exact kernel.  They live in context-owned device memory that no other call
 * touches.  Synchronises the stream. */
int cs_last_loglik_stats(cs_ctx *ctx, cs_loglik_stats *stats);

/* Kernel timing on the context stream (HIP events around each launch of the
 * named kernel).  cs_profile_enable(ctx, 1) starts recording and clears totals;
 * cs_profile_read synchronises and returns the summed milliseconds and launch
 * count of kernel `name` ("parzen", "analyze", "edt", ...). */
int cs_profile_enable(cs_ctx *ctx, int on);
/* Record only the kernel `name` (NULL: every kernel); each recorded launch
 * adds two events to the stream. */
int cs_profile_only(cs_ctx *ctx, const char *name);
/* Record one launch in `period` (>= 1, default 1) of each profiled kernel,
 * counted from the last cs_profile_enable; the others run without events.
 * Averages over the recorded launches then cost the stream fewer bubbles. */
int cs_profile_sample(cs_ctx *ctx, int period);
int cs_profile_read(cs_ctx *ctx, const char *name, double *total_ms, int64_t *launches);

/* ---- Segmentation by convex relaxation (Sec. 3.2 energy, Sec. 4) ----
 * The data term f_i = -l_i of every pixel and label, the boundary length of
 * each region weighted by the edge metric g (Sec. 3.2 prior) and, for
 * unsupervised use, a cost nu per label present (eq:mdl) make the energy of
 * eq:energy1.  Its convex relaxation (Sec. 4.1: indicator functions u_i
 * relaxed to [0, 1] with sum_i u_i = 1, the boundary length as the weighted
 * total variation sup over |xi_i(x)| <= lambda g(x) / 2 of -sum u_i div xi_i,
 * label variables m_i >= u_i(x) with multipliers mu <= 0) is solved by the
 * primal-dual iteration of Sec. 4.2, and the segmentation is
 * l(x) = argmax_i u_i(x) (ties to the lowest label).
 * Readings: forward differences with zero gradient across the last column
 * and row, the divergence as minus their adjoint, isotropic norms; |grad I|
 * the Euclidean norm over the three colour channels; steps by diagonal
 * preconditioning with the interior column sums (sigma_xi = sigma_mu = 1/2,
 * tau_u = 1/4, or 1/5 with label variables, tau_m = 1/N); start u = 1/L,
 * xi = 0, mu = 0, m = 1; nu = 0 leaves the label variables out. */

/* Edge metric of Sec. 3.2: g(x) = exp(-|grad I(x)| / gamma) / (2 gamma), with
 * gamma <= 0 selecting the mean of |grad I| over the image.
 *   rgb        device, 3*H*W float32
 *   g          device out, H*W float32
 *   gamma_out  host out or NULL: the gamma used
 * Synchronises (reads gamma back to validate it).
 * Errors: CS_ERR_ARG for null pointers, a non-finite gamma, or gamma <= 0 on
 * an image without gradient. */
int cs_edge_weight(cs_ctx *ctx, const float *rgb, int H, int W, double gamma, float *g, double *gamma_out);

typedef struct {
    double lambda;   /* weight of the boundary length, >= 0                        */
    double gamma;    /* edge metric scale; <= 0: the mean |grad I| of the image    */
    double nu;       /* cost per label present (eq:mdl), >= 0; 0 = supervised     */
    int iterations;  /* primal-dual iterations, 0..1000000                        */
    int precision;   /* CS_FP32 or CS_FP64: arithmetic of the iteration          */
} cs_segment_params;

typedef struct {
    double primal;   /* relaxed energy of u (the label cost as nu max_x u_i)       */
    double binary;   /* energy (eq:energy1) of the segmentation l = argmax u       */
    double dual;     /* dual energy at (xi, mu): a lower bound of the relaxed      */
                     /* optimum, so binary - dual bounds l's distance from it      */
    double gamma;    /* gamma used by the edge metric                              */
    int labels_used; /* labels present in l                                        */
} cs_segment_stats;

/* Segmentation of the image from its per-pixel, per-label log-likelihoods.
 *   rgb        device, 3*H*W float32 (for the edge metric)
 *   loglik     device, H*W*L float32, pixel-major (as cs_label_loglik writes
 *              it); the data term is f_i = -loglik_i
 *   labels     device out, H*W int32
 *   u          device out, H*W*L float32 pixel-major (the relaxed solution),
 *              or NULL
 *   stats      host out or NULL (energies; non-NULL adds a synchronisation)
 * The context's workspace holds the iteration's planes (about 9 L N values
 * of the working precision, 11 L N with a label cost).  Synchronises once to
 * read gamma back.
 * Errors: CS_ERR_ARG for null pointers, sizes, L outside 1..64, lambda or nu
 * negative or not finite, iterations outside 0..1000000, an unknown
 * precision, or an undefined edge metric (see cs_edge_weight). */
int cs_segment(cs_ctx *ctx, const float *rgb, int H, int W, const float *loglik, int L,
               const cs_segment_params *prm, int32_t *labels, float *u, cs_segment_stats *stats);

/* ---- Unsupervised data term (Sec. 3.1, unsupervised segmentation) ----
 * Without scribbles the segment classes come from clustering: k-means on the
 * pixels' colours (Lloyd: assign to the nearest centroid in squared Euclidean
 * distance, move each centroid to its pixels' mean) gives Kc colour classes,
 * k-medians on the co-support masks (assign by TSM, the Hamming distance;
 * move each centroid to the component-wise median, i.e. the majority of its
 * masks, a tie in) gives Kt texture classes, and every pair (a, b) is a
 * segment class i = a Kt + b represented by the two centroids.  Each pixel
 * gets a colour and a texture likelihood in the form of eq:post_text:
 *   loglik_i(x) = -d_c(x, a) - log sum_j exp(-d_c(x, a_j))
 *                 - d_t(x, b) - log sum_j exp(-d_t(x, b_j))   (sums over all Kc Kt classes)
 * with d_c = ||I(x) - mu_a||^2 / (2 sigma_c^2) and d_t = TSM(x, c_b) / beta
 * (no scribbles, so no location term and a constant beta).  cs_segment with a
 * label cost nu > 0 (eq:mdl) then removes unneeded classes.
 * Readings: the first centroids are the colours and masks of caller-given
 * pixels (random numbers of the method are inputs); a fixed iteration count;
 * distance ties to the lowest class; a class without pixels keeps its
 * centroid. */
typedef struct {
    int colour_classes;   /* Kc, 1..16                                           */
    int texture_classes;  /* Kt, 1..16, Kc * Kt <= 64                            */
    int iterations;       /* Lloyd iterations of each clustering, 0..100000     */
    double sigma_c;       /* colour kernel standard deviation, > 0              */
    double beta;          /* texture temperature, > 0                           */
} cs_unsup_params;

/* Clustering and class likelihoods of every pixel.
 *   rgb              device, 3*H*W float32
 *   masks, k         device, H*W*ceil(k/64) uint64 co-supports (as cs_cosupport)
 *   init_colour      host, Kc pixel indices (the first colour centroids)
 *   init_texture     host, Kt pixel indices (the first texture centroids)
 *   loglik           device out, H*W*(Kc*Kt) float32, pixel-major
 *   colour_centroids device out, Kc*3 float64, or NULL
 *   texture_centroids device out, Kt*ceil(k/64) uint64, or NULL
 *   colour_labels, texture_labels  device out, H*W int32 each, or NULL
 * Errors: CS_ERR_ARG for null pointers, sizes, class counts, iterations,
 * sigma_c or beta not positive, initial pixels out of range. */
int cs_unsupervised_loglik(cs_ctx *ctx, const float *rgb, int H, int W, const uint64_t *masks, int k,
                           const int32_t *init_colour, const int32_t *init_texture, const cs_unsup_params *prm,
                           float *loglik, double *colour_centroids, uint64_t *texture_centroids,
                           int32_t *colour_labels, int32_t *texture_labels);

/* ---- Learned surrogate of the data term ----
 * A two-hidden-layer perceptron maps a pixel's colour, normalised position
 * and analysed vector (Sec. 2 a = O s of the Sec. 3.1 patch) to its per-label
 * log-likelihoods (the Sec. 3.2 data term), trained per image on exact values
 * of cs_label_loglik at sampled pixels.  The paper has no surrogate; the
 * readings are: input x = [r, g, b, col/(W-1), row/(H-1), a_0..a_{k-1}]
 * (a zero coordinate when W or H is 1), z1 = W1 x + b1, h1 = GELU(z1),
 * z2 = W2 h1 + b2, h2 = GELU(z2), y = W3 h2 + b3 with the exact (erf) GELU;
 * loss = mean over rows and labels of (y - t)^2 with the clipped target
 * t_i = max(l_i, max_j l_j - 20); Adam (0.9, 0.999, 1e-8) with bias
 * correction.  Matrix products run in BF16 with FP32 accumulation; biases,
 * GELU, the loss and Adam in FP32 on FP32 master parameters.
 * Parameters are one flat FP32 vector: W1 (hidden x in_dim, row-major), b1,
 * W2 (hidden x hidden), b2, W3 (out_dim x hidden), b3.
 * Limits: hidden = 128, 1 <= in_dim <= 128, 1 <= out_dim <= 16.
 */
typedef struct cs_mlp cs_mlp;

/* Number of parameters of the network (0 for unsupported sizes). */
int64_t cs_mlp_param_count(int in_dim, int hidden, int out_dim);

/* Create a network on the context's device from initial parameters.
 *   params  device, cs_mlp_param_count(...) float32 (the initial values are
 *           the caller's: random numbers of the method are inputs)
 * Allocates the network's device memory (freed by cs_mlp_free).
 * Errors: CS_ERR_ARG (unsupported sizes, null pointers), CS_ERR_NOMEM. */
int cs_mlp_init(cs_ctx *ctx, cs_mlp **net, int in_dim, int hidden, int out_dim, const float *params);
int cs_mlp_free(cs_mlp *net);

/* Current master parameters into `params` (device, param_count float32). */
int cs_mlp_get_params(cs_ctx *ctx, const cs_mlp *net, float *params);

/* Surrogate inputs of listed pixels.
 *   rgb    device 3*H*W float32;  alpha  device H*W*k float32 (pixel-major)
 *   pix    device n int32 linear pixel indices
 *   x      device out, n*(5+k) float32, row-major
 * Errors: CS_ERR_ARG (null pointers, 5+k > 128, n < 0). */
int cs_mlp_features(cs_ctx *ctx, const float *rgb, int H, int W, const float *alpha, int k,
                    const int32_t *pix, int64_t n, float *x);

/* Gradient of the mean loss over all n rows (no update).
 *   x      device n*in_dim float32;  ell  device n*out_dim raw log-likelihoods
 *   grad   device out, param_count float32;  loss  device out, 1 float32 (nullable)
 * n must be a multiple of 16 in 16..8192.  Errors: CS_ERR_ARG. */
int cs_mlp_grad(cs_ctx *ctx, cs_mlp *net, const float *x, const float *ell, int64_t n, float *grad,
                float *loss);

/* Set the output bias b3 to the mean clipped target of each label over the
 * n rows of ell (device n*out_dim raw log-likelihoods): a data-dependent
 * start so that the optimiser does not spend its first steps moving the
 * outputs to the scale of the targets.  Errors: CS_ERR_ARG. */
int cs_mlp_fit_output_bias(cs_ctx *ctx, cs_mlp *net, const float *ell, int64_t n);

/* `steps` Adam steps; step s uses the rows order[s*batch .. s*batch+batch-1]
 * of (x, ell) (the data order is an input).
 *   order       device steps*batch int32 row indices in 0..n_rows-1 (indices
 *               outside are clamped into the range)
 *   loss_trace  device out, steps float32: loss of each batch before its update
 *               (nullable)
 * batch must be a multiple of 16 in 16..8192; lr > 0.  The Adam step count
 * continues across calls.  Errors: CS_ERR_ARG. */
int cs_mlp_train(cs_ctx *ctx, cs_mlp *net, const float *x, const float *ell, int64_t n_rows,
                 const int32_t *order, int64_t steps, int batch, double lr, float *loss_trace);

/* Surrogate log-likelihoods of every pixel, inputs assembled on the fly.
 *   rgb device 3*H*W; alpha device H*W*k (in_dim must equal 5+k)
 *   out device out, H*W*out_dim float32 (out[x*out_dim + i])
 * Errors: CS_ERR_ARG. */
int cs_mlp_infer(cs_ctx *ctx, const cs_mlp *net, const float *rgb, int H, int W, const float *alpha, int k,
                 float *out);

/* Surrogate log-likelihoods of every pixel with the exact data term as the
 * fallback: after cs_mlp_infer, every pixel whose two largest outputs differ
 * by less than `margin` nats (the surrogate is unsure of the label argmax) is
 * recomputed exactly, as cs_label_loglik computes it for a pixel list, and
 * its row of `out` replaced.
 *   net, rgb, H, W, alpha, k, out   as cs_mlp_infer (out_dim must equal L)
 *   masks, kmask, sample_pix, sample_label, M, L, prm   as cs_label_loglik
 *               (masks of k_mask entries; kmask may differ from the
 *               surrogate's k, e.g. a BF16 analysis feeding the network and
 *               exact FP64-decided masks feeding the fallback)
 *   margin      >= 0 and finite (0: no pixel is recomputed unless its two
 *               outputs tie or are not numbers)
 *   n_exact     host out or NULL: the number of pixels recomputed
 * Synchronises once (to read the count).  The context keeps a device buffer
 * of 4 N (L + 1) bytes for the list and the exact rows.
 * Errors: those of cs_mlp_infer and cs_label_loglik, CS_ERR_ARG for margin. */
int cs_mlp_infer_fallback(cs_ctx *ctx, const cs_mlp *net, const float *rgb, int H, int W, const float *alpha, int k,
                          const uint64_t *masks, int kmask, const int32_t *sample_pix, const int32_t *sample_label,
                          int64_t M, int L, const cs_loglik_params *prm, double margin, float *out,
                          int64_t *n_exact);

/* Surrogate outputs of explicit input rows x (device n*in_dim) into out
 * (device n*out_dim).  Errors: CS_ERR_ARG. */
int cs_mlp_forward(cs_ctx *ctx, const cs_mlp *net, const float *x, int64_t n, float *out);

#ifdef __cplusplus
}
#endif
#endif
