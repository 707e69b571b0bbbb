/*
 * FP64 CPU oracle of the co-sparse data term.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may build, load or call this library.  It
 * shares no code with the HIP library: it is written from the paper's
 * definitions, plainly and slowly, so that a reader can check each step
 * against the paper by eye.
 *
 * Paper: Nieuwenhuis, Hawe, Kleinsteuber, Cremers, "Co-Sparse Textural
 * Similarity for Image Segmentation" (arXiv 1312.4746).
 *
 * Steps (readings of points the paper leaves open are marked "reading"):
 *   gray value of the patch pixels ............ Sec. 3.1 (patch s_x); reading: BT.601 weights
 *   patch with symmetric border reflection .... Sec. 3.1; reading: edge pixel repeated
 *   Gaussian mask before normalisation ........ Sec. 3.1 (texture paragraph); reading: sigma = p/4
 *   zero-mean, unit-norm patch ................ Sec. 2 (bias and gain model)
 *   analysed vector a = O s ................... Sec. 2
 *   threshold tau = frac * median |a| .......... reading: lower median over all entries
 *   co-support Co(a) = {j : |a_j| <= tau} ..... Sec. 2, co-support definition (tau = 0: exact zeros)
 *   texture similarity TSM .................... Sec. 2, TSM definition (indicator form)
 *   adaptive spatial bandwidth rho_i(x) ....... Sec. 3.1, text after the Parzen colour density
 *   texture temperature beta_i = b * rho_i .... Sec. 3.1, text after the texture posterior
 *   Parzen colour/location/texture sum ........ Sec. 3.1, joint factorisation and Parzen density
 *   data term f_i = -log P .................... Sec. 3.2, energy and its data term
 *
 * Compile with -O2 -ffp-contract=off (no FMA contraction, no fast-math): every
 * floating-point operation below is an IEEE-754 double operation in the
 * order written.
 */
#include "cso_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int g_threads = 0; /* 0: OpenMP default */

void cso_set_threads(int n) { g_threads = n; }

int cso_get_threads(void) {
#ifdef _OPENMP
    return g_threads > 0 ? g_threads : omp_get_max_threads();
#else
    return 1;
#endif
}

#define NTHREADS() (cso_get_threads())

/* Gray value (reading: BT.601 luma weights), FP64, evaluated as
 * (0.299 R + 0.587 G) + 0.114 B from the float32 colour planes. */
static double gray_at(const float *rgb, int64_t N, int64_t idx) {
    double r = (double)rgb[idx];
    double g = (double)rgb[N + idx];
    double b = (double)rgb[2 * N + idx];
    return (0.299 * r + 0.587 * g) + 0.114 * b;
}

int cso_gray(const float *rgb, int H, int W, double *gray) {
    if (!rgb || !gray || H <= 0 || W <= 0) return CSO_ERR_ARG;
    int64_t N = (int64_t)H * W;
    for (int64_t i = 0; i < N; ++i) gray[i] = gray_at(rgb, N, i);
    return CSO_OK;
}

/* Symmetric border reflection that repeats the edge pixel:
 * -1 -> 0, -2 -> 1, W -> W-1, W+1 -> W-2 (reading; the paper is silent). */
static int reflect(int i, int n) {
    if (i < 0) return -i - 1;
    if (i >= n) return 2 * n - i - 1;
    return i;
}

/* Gaussian mask applied element-wise before normalisation (Sec. 3.1).
 * w_t = exp(-(u^2 + v^2) / (2 sigma^2)), t = (u+h)*p + (v+h), u the row
 * offset and v the column offset; peak value 1 (reading: sigma = p/4). */
int cso_mask_table(int p, double sigma, double *w) {
    if (!w || p < 1 || (p % 2) == 0 || !(sigma > 0.0)) return CSO_ERR_ARG;
    int h = (p - 1) / 2;
    for (int u = -h; u <= h; ++u)
        for (int v = -h; v <= h; ++v) {
            double r2 = (double)(u * u + v * v);
            w[(u + h) * p + (v + h)] = exp(-r2 / (2.0 * sigma * sigma));
        }
    return CSO_OK;
}

/* Normalised, masked gray patch s_x of one pixel (Sec. 2 and Sec. 3.1):
 * q_t = w_t g_t; mu = (sum_t q_t)/n; z_t = q_t - mu; nu2 = sum_t z_t^2;
 * s_t = z_t / sqrt(nu2), or s = 0 when nu2 = 0 (reading).  Sums run
 * sequentially in t. */
static void patch_s(const float *rgb, int H, int W, int p, const double *w, int64_t pix, double *s) {
    int64_t N = (int64_t)H * W;
    int h = (p - 1) / 2, n = p * p;
    int row = (int)(pix / W), col = (int)(pix % W);
    for (int u = -h; u <= h; ++u)
        for (int v = -h; v <= h; ++v) {
            int rr = reflect(row + u, H), cc = reflect(col + v, W);
            int t = (u + h) * p + (v + h);
            s[t] = w[t] * gray_at(rgb, N, (int64_t)rr * W + cc);
        }
    double sum = 0.0;
    for (int t = 0; t < n; ++t) sum = sum + s[t];
    double mu = sum / (double)n;
    for (int t = 0; t < n; ++t) s[t] = s[t] - mu;
    double nu2 = 0.0;
    for (int t = 0; t < n; ++t) nu2 = nu2 + s[t] * s[t];
    if (nu2 == 0.0) {
        for (int t = 0; t < n; ++t) s[t] = 0.0;
        return;
    }
    double nu = sqrt(nu2);
    for (int t = 0; t < n; ++t) s[t] = s[t] / nu;
}

/* 1 when every one of the n floats is finite (no NaN, no infinity): the
 * method is defined on finite colours and operator entries only. */
static int all_finite(const float *v, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

static int check_image(const float *rgb, int H, int W, int p) {
    if (!rgb || p < 1 || p > 15 || (p % 2) == 0) return 0;
    int h = (p - 1) / 2;
    if (H < h + 1 || W < h + 1) return 0;
    return 1;
}

int cso_patches(const float *rgb, int H, int W, int p, double mask_sigma,
                const int32_t *pix, int64_t npix, double *s_out) {
    if (!check_image(rgb, H, W, p) || !s_out || !(mask_sigma > 0.0)) return CSO_ERR_ARG;
    int64_t N = (int64_t)H * W;
    int64_t cnt = pix ? npix : N;
    int n = p * p;
    double w[15 * 15];
    cso_mask_table(p, mask_sigma, w);
    for (int64_t i = 0; i < cnt; ++i) {
        int64_t px = pix ? pix[i] : i;
        if (px < 0 || px >= N) return CSO_ERR_ARG;
        patch_s(rgb, H, W, p, w, px, s_out + i * n);
    }
    return CSO_OK;
}

/* Analysed vector a = O s (Sec. 2): a_j = sum_t O_jt s_t, sequential in t. */
int cso_analyze(const float *rgb, int H, int W, int p, double mask_sigma,
                const float *omega, int k, const int32_t *pix, int64_t npix, double *alpha) {
    if (!check_image(rgb, H, W, p) || !omega || !alpha || k < 1 || !(mask_sigma > 0.0))
        return CSO_ERR_ARG;
    int64_t N = (int64_t)H * W;
    int64_t cnt = pix ? npix : N;
    int n = p * p;
    if (!all_finite(rgb, 3 * N) || !all_finite(omega, (int64_t)k * n)) return CSO_ERR_NONFINITE;
    if (pix)
        for (int64_t i = 0; i < cnt; ++i)
            if (pix[i] < 0 || pix[i] >= N) return CSO_ERR_ARG;
    double w[15 * 15];
    cso_mask_table(p, mask_sigma, w);
#pragma omp parallel for schedule(static) num_threads(NTHREADS())
    for (int64_t i = 0; i < cnt; ++i) {
        double s[15 * 15];
        int64_t px = pix ? pix[i] : i;
        patch_s(rgb, H, W, p, w, px, s);
        for (int j = 0; j < k; ++j) {
            double a = 0.0;
            for (int t = 0; t < n; ++t) a = a + (double)omega[(int64_t)j * n + t] * s[t];
            alpha[i * k + j] = a;
        }
    }
    return CSO_OK;
}

static int cmp_double(const void *a, const void *b) {
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* tau = frac * median{|a_j(x)|}, lower median: rank floor((count-1)/2) of
 * the ascending order (reading).  Sorting is the library qsort. */
int cso_tau_median(const double *alpha, int64_t count, double frac, double *tau, double *median) {
    if (!alpha || count < 1 || !tau || !(frac >= 0.0)) return CSO_ERR_ARG;
    double *v = (double *)malloc((size_t)count * sizeof(double));
    if (!v) return CSO_ERR_NOMEM;
    for (int64_t i = 0; i < count; ++i) v[i] = fabs(alpha[i]);
    qsort(v, (size_t)count, sizeof(double), cmp_double);
    double med = v[(count - 1) / 2];
    free(v);
    if (median) *median = med;
    *tau = frac * med;
    return CSO_OK;
}

/* Co-support as a bit mask: bit j of pixel x is 1 iff |a_j(x)| <= tau
 * (Sec. 2, co-support definition; tau = 0 is its exact-zero form).  Bit j is bit
 * (j mod 64) of word j/64; padding bits are 0. */
int cso_cosupport(const double *alpha, int64_t npix, int k, double tau, uint64_t *masks) {
    if (!alpha || !masks || k < 1 || !(tau >= 0.0)) return CSO_ERR_ARG;
    int words = (k + 63) / 64;
    for (int64_t i = 0; i < npix; ++i) {
        for (int q = 0; q < words; ++q) masks[i * words + q] = 0;
        for (int j = 0; j < k; ++j)
            if (fabs(alpha[i * k + j]) <= tau)
                masks[i * words + j / 64] |= (uint64_t)1 << (j % 64);
    }
    return CSO_OK;
}

static int bit_of(const uint64_t *m, int j) { return (int)((m[j / 64] >> (j % 64)) & 1u); }

/* TSM(s1, s2) = sum_{j=1..k} |1_Co1(j) - 1_Co2(j)| (Sec. 2, TSM definition). */
static int tsm_pair(const uint64_t *a, const uint64_t *b, int k) {
    int t = 0;
    for (int j = 0; j < k; ++j) t += abs(bit_of(a, j) - bit_of(b, j));
    return t;
}

int cso_tsm(const uint64_t *A, int64_t na, const uint64_t *B, int64_t nb, int k, int32_t *out) {
    if ((!A && na) || (!B && nb) || !out || k < 1 || na < 0 || nb < 0) return CSO_ERR_ARG;
    int words = (k + 63) / 64;
#pragma omp parallel for schedule(static) num_threads(NTHREADS())
    for (int64_t i = 0; i < na; ++i)
        for (int64_t j = 0; j < nb; ++j)
            out[i * nb + j] = tsm_pair(A + i * words, B + j * words, k);
    return CSO_OK;
}

/* Squared distance from pixel x to the nearest scribble sample of label i
 * (the x_{v_i} of Sec. 3.1), by brute force in integer arithmetic. */
int cso_nearest_d2(int H, int W, const int32_t *sample_pix, const int32_t *sample_label,
                   int64_t M, int L, const int32_t *pix, int64_t npix, int64_t *d2) {
    if (H <= 0 || W <= 0 || !sample_pix || !sample_label || M < 1 || L < 1 || !d2) return CSO_ERR_ARG;
    int64_t N = (int64_t)H * W;
    int64_t cnt = pix ? npix : N;
    for (int64_t s = 0; s < M; ++s) {
        if (sample_label[s] < 0 || sample_label[s] >= L) return CSO_ERR_ARG;
        if (sample_pix[s] < 0 || sample_pix[s] >= N) return CSO_ERR_ARG;
    }
#pragma omp parallel for schedule(static) num_threads(NTHREADS())
    for (int64_t i = 0; i < cnt; ++i) {
        int64_t px = pix ? pix[i] : i;
        int64_t xr = px / W, xc = px % W;
        for (int l = 0; l < L; ++l) d2[i * L + l] = -1;
        for (int64_t s = 0; s < M; ++s) {
            int64_t yr = sample_pix[s] / W, yc = sample_pix[s] % W;
            int64_t dd = (xc - yc) * (xc - yc) + (xr - yr) * (xr - yr);
            int64_t *slot = &d2[i * L + sample_label[s]];
            if (*slot < 0 || dd < *slot) *slot = dd;
        }
    }
    return CSO_OK;
}

/*
 * Textural representative of each label (Sec. 2, the majority definition of a
 * representative's co-support; Sec. 3.1, c_i of the label's samples): bit j
 * of c_l is set iff at least half of the label's m_l samples have j in their
 * co-support, 2 * count_j >= m_l.  For binary vectors this is the
 * component-wise median of eq:approx_cosupp with a tie (even m_l, half the
 * votes) counted in.  rep: L x ceil(k/64) words, bits k.. zero.
 */
int cso_label_rep(const uint64_t *masks, int64_t N, int k, const int32_t *sample_pix,
                  const int32_t *sample_label, int64_t M, int L, uint64_t *rep) {
    if (!masks || N < 1 || k < 1 || !sample_pix || !sample_label || M < 1 || L < 1 || !rep)
        return CSO_ERR_ARG;
    int words = (k + 63) / 64;
    int64_t *votes = (int64_t *)calloc((size_t)L * k, sizeof(int64_t));
    int64_t *m = (int64_t *)calloc((size_t)L, sizeof(int64_t));
    if (!votes || !m) { free(votes); free(m); return CSO_ERR_NOMEM; }
    for (int64_t s = 0; s < M; ++s) {
        int l = sample_label[s];
        if (l < 0 || l >= L || sample_pix[s] < 0 || sample_pix[s] >= N) {
            free(votes); free(m); return CSO_ERR_ARG;
        }
        m[l]++;
        for (int j = 0; j < k; ++j) votes[(int64_t)l * k + j] += bit_of(masks + sample_pix[s] * words, j);
    }
    for (int l = 0; l < L; ++l) {
        if (m[l] == 0) { free(votes); free(m); return CSO_ERR_EMPTY_LABEL; }
        for (int w = 0; w < words; ++w) rep[(int64_t)l * words + w] = 0;
        for (int j = 0; j < k; ++j)
            if (2 * votes[(int64_t)l * k + j] >= m[l]) rep[(int64_t)l * words + j / 64] |= (uint64_t)1 << (j % 64);
    }
    free(votes);
    free(m);
    return CSO_OK;
}

/*
 * Smooth-co-support representative of each label (eq:approx_cosupp; c_i of
 * Sec. 3.1): c_lj = the median over the label's samples of
 * iota(a)_j = exp(-a_j^2 / sigma_iota) (eq:map_tsm), taken as the element of
 * 0-based rank floor(m_l/2) of the ascending values (the upper median: for
 * 0/1 values it is the majority with a tie counted in, as in cso_label_rep).
 * alpha: N x k, FP64.  rep: L x k.
 */
int cso_label_rep_soft(const double *alpha, int64_t N, int k, double sigma_iota,
                       const int32_t *sample_pix, const int32_t *sample_label, int64_t M, int L,
                       double *rep) {
    if (!alpha || N < 1 || k < 1 || !(sigma_iota > 0.0) || !sample_pix || !sample_label || M < 1 ||
        L < 1 || !rep)
        return CSO_ERR_ARG;
    double *v = (double *)malloc((size_t)M * sizeof(double));
    if (!v) return CSO_ERR_NOMEM;
    for (int64_t s = 0; s < M; ++s)
        if (sample_label[s] < 0 || sample_label[s] >= L || sample_pix[s] < 0 || sample_pix[s] >= N) {
            free(v); return CSO_ERR_ARG;
        }
    for (int l = 0; l < L; ++l) {
        for (int j = 0; j < k; ++j) {
            int64_t m = 0;
            for (int64_t s = 0; s < M; ++s) {
                if (sample_label[s] != l) continue;
                double a = alpha[(int64_t)sample_pix[s] * k + j];
                v[m++] = exp(-(a * a) / sigma_iota);
            }
            if (m == 0) { free(v); return CSO_ERR_EMPTY_LABEL; }
            qsort(v, (size_t)m, sizeof(double), cmp_double);
            rep[(int64_t)l * k + j] = v[m / 2];
        }
    }
    free(v);
    return CSO_OK;
}

/*
 * Per-pixel, per-label log-likelihood l_i(x) = -f_i(x) (Sec. 3.1, Sec. 3.2).
 *
 * For label i with samples S_i (m_i = |S_i| >= 1):
 *   d2_i(x)  = min_{y in S_i} |x - y|^2
 *   rho_i(x) = alpha_rho * sqrt(max(d2_i(x), r_f^2))      (Sec. 3.1; reading: floor r_f)
 *   beta_i(x)= b * rho_i(x)                                 (Sec. 3.1, beta proportional to rho)
 *   e(x,y)   = -|x-y|^2 / (2 rho^2) - |I(x)-I(y)|^2 / (2 sigma_c^2) - TSM(x,y) / beta
 *   l_i(x)   = log( (1/m_i) sum_y (2 pi rho^2)^-1 (2 pi sigma_c^2)^-3/2 exp(e(x,y)) )
 * evaluated as E + log sum_y exp(e - E) - log m_i - log(2 pi rho^2) - 1.5 log(2 pi sigma_c^2),
 * E = max_y e (two passes in sample-index order).  The texture factor
 * exp(-TSM/beta) sits inside the Parzen sum, one factor per sample.
 * With normalise != 0 the output is l_i - log sum_i' exp(l_i').
 * masks: co-support masks of every image pixel (N x ceil(k/64) words); each
 * sample's colour, position and mask are those of its pixel.
 */
/* joint: 0 texture factor per sample inside the sum (masks), 1 hard label
 * representatives (masks), 2 smooth co-supports and their median
 * representatives (alpha, sigma_iota). */
static int loglik(const float *rgb, int H, int W, const uint64_t *masks, const double *alpha,
                  double sigma_iota, int k, const int32_t *sample_pix, const int32_t *sample_label,
                  int64_t M, int L, double alpha_rho, double sigma_c, double beta_scale,
                  double rho_floor, int normalise, const int32_t *pix, int64_t npix, double *out,
                  int joint) {
    if (!rgb || H <= 0 || W <= 0 || k < 1 || !sample_pix || !sample_label || M < 1 ||
        L < 1 || !out || !(alpha_rho > 0.0) || !(sigma_c > 0.0) || !(beta_scale > 0.0) ||
        !(rho_floor > 0.0))
        return CSO_ERR_ARG;
    if (joint == 2 ? (!alpha || !(sigma_iota > 0.0)) : !masks) return CSO_ERR_ARG;
    int64_t N = (int64_t)H * W;
    int64_t cnt = pix ? npix : N;
    int words = (k + 63) / 64;
    if (!all_finite(rgb, 3 * N)) return CSO_ERR_NONFINITE;
    /* label segments in sample-index order */
    int64_t *count = (int64_t *)calloc((size_t)L, sizeof(int64_t));
    int64_t *start = (int64_t *)calloc((size_t)L + 1, sizeof(int64_t));
    int64_t *order = (int64_t *)malloc((size_t)M * sizeof(int64_t));
    if (!count || !start || !order) { free(count); free(start); free(order); return CSO_ERR_NOMEM; }
    for (int64_t s = 0; s < M; ++s) {
        if (sample_label[s] < 0 || sample_label[s] >= L || sample_pix[s] < 0 || sample_pix[s] >= N) {
            free(count); free(start); free(order); return CSO_ERR_ARG;
        }
        count[sample_label[s]]++;
    }
    int64_t maxm = 0;
    for (int l = 0; l < L; ++l) {
        if (count[l] == 0) { free(count); free(start); free(order); return CSO_ERR_EMPTY_LABEL; }
        start[l + 1] = start[l] + count[l];
        if (count[l] > maxm) maxm = count[l];
    }
    {
        int64_t *fill = (int64_t *)calloc((size_t)L, sizeof(int64_t));
        if (!fill) { free(count); free(start); free(order); return CSO_ERR_NOMEM; }
        for (int64_t s = 0; s < M; ++s) {
            int l = sample_label[s];
            order[start[l] + fill[l]++] = s;
        }
        free(fill);
    }
    uint64_t *rep = NULL;
    double *crep = NULL;
    if (joint == 1) {
        rep = (uint64_t *)malloc((size_t)L * words * sizeof(uint64_t));
        if (!rep) { free(count); free(start); free(order); return CSO_ERR_NOMEM; }
        int rc = cso_label_rep(masks, N, k, sample_pix, sample_label, M, L, rep);
        if (rc) { free(rep); free(count); free(start); free(order); return rc; }
    } else if (joint == 2) {
        crep = (double *)malloc((size_t)L * k * sizeof(double));
        if (!crep) { free(count); free(start); free(order); return CSO_ERR_NOMEM; }
        int rc = cso_label_rep_soft(alpha, N, k, sigma_iota, sample_pix, sample_label, M, L, crep);
        if (rc) { free(crep); free(count); free(start); free(order); return rc; }
    }
    const double pi = 3.14159265358979323846;
    double col_norm = 1.5 * log(2.0 * pi * sigma_c * sigma_c);
    int bad = 0;
#pragma omp parallel num_threads(NTHREADS())
    {
        double *e = (double *)malloc((size_t)maxm * sizeof(double));
        double *lab = (double *)malloc((size_t)L * sizeof(double));
        double *u = (double *)malloc((size_t)L * sizeof(double));
        if (!e || !lab || !u) {
#pragma omp atomic write
            bad = 1;
        }
#pragma omp for schedule(static)
        for (int64_t i = 0; i < cnt; ++i) {
            if (!e || !lab || !u) continue;
            int64_t px = pix ? pix[i] : i;
            int64_t xr = px / W, xc = px % W;
            double Ir = rgb[px], Ig = rgb[N + px], Ib = rgb[2 * N + px];
            const uint64_t *mx = masks ? masks + px * words : NULL;
            for (int l = 0; l < L; ++l) {
                int64_t m = count[l];
                int64_t d2 = -1;
                for (int64_t q = 0; q < m; ++q) {
                    int64_t y = sample_pix[order[start[l] + q]];
                    int64_t dd = (xc - y % W) * (xc - y % W) + (xr - y / W) * (xr - y / W);
                    if (d2 < 0 || dd < d2) d2 = dd;
                }
                double d2f = (double)d2;
                double fl2 = rho_floor * rho_floor;
                double rho = alpha_rho * sqrt(d2f > fl2 ? d2f : fl2);
                double rho2 = rho * rho;
                double beta = beta_scale * rho;
                double E = -INFINITY;
                for (int64_t q = 0; q < m; ++q) {
                    int64_t y = sample_pix[order[start[l] + q]];
                    double dxc = (double)(xc - y % W), dxr = (double)(xr - y / W);
                    double loc2 = dxc * dxc + dxr * dxr;
                    double dr = Ir - (double)rgb[y], dg = Ig - (double)rgb[N + y],
                           db = Ib - (double)rgb[2 * N + y];
                    double col2 = dr * dr + dg * dg + db * db;
                    double ev = -loc2 / (2.0 * rho2) - col2 / (2.0 * sigma_c * sigma_c);
                    if (!joint) ev = ev - (double)tsm_pair(mx, masks + y * words, k) / beta;
                    e[q] = ev;
                    if (ev > E) E = ev;
                }
                double sum = 0.0;
                for (int64_t q = 0; q < m; ++q) sum = sum + exp(e[q] - E);
                lab[l] = E + log(sum) - log((double)m) - log(2.0 * pi * rho2) - col_norm;
                /* texture exponent of eq:post_text against the label's representative */
                if (joint == 1) u[l] = -(double)tsm_pair(mx, rep + (int64_t)l * words, k) / beta;
                if (joint == 2) {
                    /* eq:tsm: l1 distance between the smooth co-supports */
                    double d = 0.0;
                    for (int j = 0; j < k; ++j) {
                        double a = alpha[px * k + j];
                        d = d + fabs(crep[(int64_t)l * k + j] - exp(-(a * a) / sigma_iota));
                    }
                    u[l] = -d / beta;
                }
            }
            if (joint) {
                /* log of the texture posterior: u_l - log sum_l' exp(u_l') */
                double U = -INFINITY;
                for (int l = 0; l < L; ++l)
                    if (u[l] > U) U = u[l];
                double usum = 0.0;
                for (int l = 0; l < L; ++l) usum = usum + exp(u[l] - U);
                double lz = U + log(usum);
                for (int l = 0; l < L; ++l) lab[l] = lab[l] + (u[l] - lz);
            }
            if (normalise) {
                double Lm = -INFINITY;
                for (int l = 0; l < L; ++l)
                    if (lab[l] > Lm) Lm = lab[l];
                double ssum = 0.0;
                for (int l = 0; l < L; ++l) ssum = ssum + exp(lab[l] - Lm);
                double lse = Lm + log(ssum);
                for (int l = 0; l < L; ++l) out[i * L + l] = lab[l] - lse;
            } else {
                for (int l = 0; l < L; ++l) out[i * L + l] = lab[l];
            }
        }
        free(e);
        free(lab);
        free(u);
    }
    free(rep);
    free(crep);
    free(count);
    free(start);
    free(order);
    return bad ? CSO_ERR_NOMEM : CSO_OK;
}

int cso_label_loglik(const float *rgb, int H, int W, const uint64_t *masks, int k,
                     const int32_t *sample_pix, const int32_t *sample_label, int64_t M, int L,
                     double alpha_rho, double sigma_c, double beta_scale, double rho_floor,
                     int normalise, const int32_t *pix, int64_t npix, double *out) {
    return loglik(rgb, H, W, masks, NULL, 0.0, k, sample_pix, sample_label, M, L, alpha_rho,
                  sigma_c, beta_scale, rho_floor, normalise, pix, npix, out, 0);
}

/*
 * The paper's own combination (eq:joined): the colour/location Parzen density
 * (eq:color) times the texture posterior (eq:post_text),
 *   l_i(x) = P_i(x) + u_i(x) - log sum_i' exp u_i'(x),
 *   P_i(x) = log( (1/m_i) sum_{y in S_i} (2 pi rho^2)^-1 (2 pi sigma_c^2)^-3/2
 *                 exp(-|x-y|^2 / (2 rho^2) - |I(x)-I(y)|^2 / (2 sigma_c^2)) ),
 *   u_i(x) = -TSM(m_x, c_i) / beta_i(x),
 * with c_i the label's textural representative (cso_label_rep) and rho, beta
 * as in cso_label_loglik.  Hard co-supports stand in for the smooth map of
 * Sec. 2 (its sigma -> 0 limit), so the median of eq:approx_cosupp is the
 * majority vote.  normalise as in cso_label_loglik, applied last.
 */
int cso_label_loglik_joint(const float *rgb, int H, int W, const uint64_t *masks, int k,
                           const int32_t *sample_pix, const int32_t *sample_label, int64_t M,
                           int L, double alpha_rho, double sigma_c, double beta_scale,
                           double rho_floor, int normalise, const int32_t *pix, int64_t npix,
                           double *out) {
    return loglik(rgb, H, W, masks, NULL, 0.0, k, sample_pix, sample_label, M, L, alpha_rho,
                  sigma_c, beta_scale, rho_floor, normalise, pix, npix, out, 1);
}

/*
 * The joint form with the smooth co-support of Sec. 2 (eq:map_tsm), as in
 * the paper's experiments: iota(a)_j = exp(-a_j^2 / sigma_iota), the texture
 * distance of eq:tsm (l1 norm of the difference of the smooth co-supports),
 * the representative c_i of eq:approx_cosupp (cso_label_rep_soft), and
 *   l_i(x) = P_i(x) + u_i(x) - log sum_i' exp u_i'(x),
 *   u_i(x) = -|| c_i - iota(a_x) ||_1 / beta_i(x),
 * with P_i the colour/location density of cso_label_loglik_joint.
 * alpha: N x k analysed vectors of every pixel (row-major, FP64).
 */
int cso_label_loglik_soft(const float *rgb, int H, int W, const double *alpha, int k,
                          double sigma_iota, const int32_t *sample_pix, const int32_t *sample_label,
                          int64_t M, int L, double alpha_rho, double sigma_c, double beta_scale,
                          double rho_floor, int normalise, const int32_t *pix, int64_t npix,
                          double *out) {
    return loglik(rgb, H, W, NULL, alpha, sigma_iota, k, sample_pix, sample_label, M, L, alpha_rho,
                  sigma_c, beta_scale, rho_floor, normalise, pix, npix, out, 2);
}
