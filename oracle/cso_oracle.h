/*
 * FP64 CPU oracle of the co-sparse data term -- TEST INFRASTRUCTURE ONLY.
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * use it.  It shares nothing with the HIP library or its header.
 *
 * All arrays are host memory owned by the caller.  Images are three float32
 * planes (R, G, B), each H*W, pixel x = (col, row) at linear index row*W+col.
 * Functions return CSO_OK or an error code; they never abort.
 */
#ifndef CSO_ORACLE_H
#define CSO_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CSO_OK 0
#define CSO_ERR_ARG 1
#define CSO_ERR_EMPTY_LABEL 2
#define CSO_ERR_NOMEM 4
#define CSO_ERR_NONFINITE 5 /* an input colour or operator entry is a NaN or an infinity */

void cso_set_threads(int n);
int cso_get_threads(void);

int cso_gray(const float *rgb, int H, int W, double *gray);
int cso_mask_table(int p, double sigma, double *w);
/* s_out: npix x p*p normalised patches (pix NULL: all N pixels) */
int cso_patches(const float *rgb, int H, int W, int p, double mask_sigma,
                const int32_t *pix, int64_t npix, double *s_out);
/* alpha: npix x k analysed vectors (pix NULL: all N pixels) */
int cso_analyze(const float *rgb, int H, int W, int p, double mask_sigma,
                const float *omega, int k, const int32_t *pix, int64_t npix, double *alpha);
int cso_tau_median(const double *alpha, int64_t count, double frac, double *tau, double *median);
int cso_cosupport(const double *alpha, int64_t npix, int k, double tau, uint64_t *masks);
int cso_tsm(const uint64_t *A, int64_t na, const uint64_t *B, int64_t nb, int k, int32_t *out);
int cso_nearest_d2(int H, int W, const int32_t *sample_pix, const int32_t *sample_label,
                   int64_t M, int L, const int32_t *pix, int64_t npix, int64_t *d2);
int cso_label_loglik(const float *rgb, int H, int W, const uint64_t *masks, int k,
                     const int32_t *sample_pix, const int32_t *sample_label, int64_t M, int L,
                     double alpha_rho, double sigma_c, double beta_scale, double rho_floor,
                     int normalise, const int32_t *pix, int64_t npix, double *out);
int cso_label_rep(const uint64_t *masks, int64_t N, int k, const int32_t *sample_pix,
                  const int32_t *sample_label, int64_t M, int L, uint64_t *rep);
int cso_label_rep_soft(const double *alpha, int64_t N, int k, double sigma_iota,
                       const int32_t *sample_pix, const int32_t *sample_label, int64_t M, int L,
                       double *rep);
int cso_label_loglik_soft(const float *rgb, int H, int W, const double *alpha, int k,
                          double sigma_iota, const int32_t *sample_pix, const int32_t *sample_label,
                          int64_t M, int L, double alpha_rho, double sigma_c, double beta_scale,
                          double rho_floor, int normalise, const int32_t *pix, int64_t npix,
                          double *out);
int cso_label_loglik_joint(const float *rgb, int H, int W, const uint64_t *masks, int k,
                           const int32_t *sample_pix, const int32_t *sample_label, int64_t M,
                           int L, double alpha_rho, double sigma_c, double beta_scale,
                           double rho_floor, int normalise, const int32_t *pix, int64_t npix,
                           double *out);

#ifdef __cplusplus
}
#endif
#endif
