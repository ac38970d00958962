/*
 * dppix_oracle.h — plain, slow CPU oracle for region-adaptive differentially
 * private pixelization (Liu, "A Parallel Region-Adaptive Differential Privacy
 * Framework for Image Pixelization", arXiv 2511.04261).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this code; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with the
 * HIP implementation.
 *
 * Every routine follows the paper's definitions literally, in fp64:
 *   - grid geometry and cell means             Sec. IV-A, Eq. (1)-(4)
 *   - Laplace mechanism, sigma = Delta/eps     Sec. IV-B, Eq. (8)-(9)
 *   - sensitivity Delta = 255 m / b^2          Sec. IV-D, Eq. (11)
 *   - mirror padding + grid reshape            Algorithm 2 (steps 3-5), Algorithm 3 (steps 1-4)
 *   - mask means, simple/complex split         Algorithm 3 (steps 5-6)
 *   - simple cells: mean, noise, clip, assign  Algorithm 3 (steps 7-11)
 *   - complex cells: subgrids s_b = b/n        Algorithm 3 (steps 12-19), Eq. (16)-(17)
 *   - un-grid and crop                         Algorithm 3 (steps 20-21)
 *   - compact store                            Table IV (Sec. VI-F)
 *   - reconstruction from the store            Sec. VI-F, last paragraphs
 * The adjoint (orc_backward) is not in the paper: it is the exact derivative
 * of the forward map above with the noise held fixed.
 *
 * Readings of points the paper leaves open (mirror mode, mask polarity and
 * threshold, per-region budgets, the noise generator, rounding) are listed in
 * the repository's design notes; the choices are fixed by the parameters below.
 */
#ifndef DPPIX_ORACLE_H
#define DPPIX_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Border handling.  SYMMETRIC / REFLECT: the frame is mirror-padded to whole
 * cells (Algorithm 2 step 4, Algorithm 3 step 3) and every mean divides by
 * the full cell area.  NONE: Algorithm 1 — a border cell (or subcell) holds
 * only its h x w real pixels and its mean divides by h*w; a subcell with no
 * real pixel releases nothing (value 0, no noise drawn). */
enum { ORC_PAD_SYMMETRIC = 0, ORC_PAD_REFLECT = 1, ORC_PAD_NONE = 2 };

typedef struct {
    int32_t  height, width, channels; /* M, N, C                                    */
    int32_t  b;                       /* grid size of simple regions (paper b)       */
    int32_t  sb;                      /* subgrid size of complex regions (paper s_b) */
    int32_t  m;                       /* max varying pixels (paper m)                */
    double   eps_simple;              /* budget of simple cells; +inf = no noise     */
    double   eps_complex;             /* budget of complex subcells; +inf = no noise */
    int32_t  tau;                     /* complex iff foreground count >= tau;
                                         0 selects ceil(area/2) with area = b*b
                                         (padded modes) or the cell's real pixel
                                         count (NONE): the paper's "simple iff
                                         simple-mask mean > 0.5" rule                */
    int32_t  pad_mode;                /* ORC_PAD_SYMMETRIC, _REFLECT or _NONE        */
    uint64_t seed;                    /* Philox key                                  */
    uint64_t frame_index;             /* Philox counter words 2..3                   */
} orc_params_t;

/* Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Noise counter layout: ctr = (id, ch | level<<8, frame_lo, frame_hi),
 * key = (seed_lo, seed_hi).  level 0 = simple coarse cell (id = r*G_C + c),
 * level 1 = complex subcell (id = global subgrid index). */
void orc_noise_words(uint64_t seed, uint64_t frame_index, uint32_t id, int32_t ch,
                     int32_t level, uint32_t out[4]);

/* Uniform on (0,1) from the first two Philox words: u = (2k+1) 2^-53, k = x>>12. */
double orc_uniform(uint32_t w0, uint32_t w1);

/* Laplace(0, sigma) by inverse CDF of u in (0,1). */
double orc_laplace(double u, double sigma);

/* sigma = Delta / eps with Delta = 255 m / b^2 (Eq. 11); 0 when eps is +inf. */
double orc_sigma(int32_t b, int32_t m, double eps);

/* Mirror index of padded coordinate x >= 0 into [0, L). */
int64_t orc_fold(int64_t x, int64_t L, int32_t mode);

/* Validate parameters; returns 0 when usable. */
int32_t orc_check(const orc_params_t* p);

/* Geometry: G_R, G_C, n = b/s_b; returns 0 on success. */
int32_t orc_geometry(const orc_params_t* p, int32_t* GR, int32_t* GC, int32_t* n);

/*
 * Forward pass of Algorithm 3 (Algorithm 2 when the mask is NULL: every cell
 * simple).  Inputs:
 *   img   : M*N*C doubles, HWC row-major (pixel values in [0,255])
 *   mask  : M*N bytes, nonzero = foreground/complex; NULL = all simple
 * Outputs (caller allocates; any may be NULL except flags/bg/fg/counts):
 *   flags      : G_R*G_C bytes, 1 = complex
 *   bg         : capacity G_R*G_C*C floats   (stats of simple cells, [k][C])
 *   fg         : capacity G_R*G_C*n*n*C      (stats of complex cells, [k][n*n][C])
 *   counts     : {n_bg, n_fg}
 *   recon_f32  : M*N*C floats, reconstruction (unrounded)
 *   recon_u8   : M*N*C bytes, reconstruction rounded half-to-even
 *   recon_f64  : M*N*C doubles, reconstruction before the fp32 rounding of the
 *                statistics (used for fp64 finite differences)
 *   coarse_sum : G_R*G_C*C doubles, padded b x b sums of every cell
 *   fine_sum   : (G_R*n)*(G_C*n)*C doubles, padded s_b x s_b sums of every subcell
 *   pass_bg/fg : per stat, 1 when 0 <= mean+noise <= 255 (same shape as bg/fg)
 * Returns 0 on success, nonzero on invalid parameters or allocation failure.
 */
int32_t orc_forward(const orc_params_t* p, const double* img, const uint8_t* mask,
                    uint8_t* flags, float* bg, float* fg, int64_t counts[2],
                    float* recon_f32, uint8_t* recon_u8, double* recon_f64,
                    double* coarse_sum, double* fine_sum,
                    uint8_t* pass_bg, uint8_t* pass_fg);

/*
 * Complexity label from the image itself (the paper's Sec. VI-A names the
 * Sobel operator as one way to obtain the mask).  S(i,j) = sum of the C
 * channels; Gx, Gy = 3x3 Sobel responses of S with neighbours past the border
 * mirrored (pad_mode; NONE mirrors like SYMMETRIC); a pixel is an edge pixel (mask byte 1) when
 * |Gx| + |Gy| >= threshold * C.  img: M*N*C doubles (HWC, integer-valued);
 * out: M*N bytes.
 */
int32_t orc_edge_mask(int32_t M, int32_t N, int32_t C, const double* img, int32_t threshold, int32_t pad_mode,
                      uint8_t* out);

/*
 * Utility metrics of the paper's runtime/utility study (Sec. VII-A): mean
 * squared error and SSIM (Wang, Bovik, Sheikh, Simoncelli 2004) between two
 * M x N x C images (HWC doubles, values 0..255).  SSIM uses 7 x 7 windows
 * with equal weights, sample (co)variances (divisor 48), K1 = 0.01,
 * K2 = 0.03, dynamic range 255; the SSIM map is averaged over the windows
 * that lie fully inside the frame and over channels.  Needs M, N >= 7.
 */
int32_t orc_metrics(int32_t M, int32_t N, int32_t C, const double* x, const double* y, double* mse, double* ssim);

/* Reconstruction from the compact store only (flags, bg, fg, b, s_b, M x N). */
int32_t orc_reconstruct(const orc_params_t* p, const uint8_t* flags, const float* bg,
                        const float* fg, float* recon_f32, uint8_t* recon_u8);

/*
 * Adjoint of the forward map y = reconstruct(clip(mean + noise)) with the noise
 * and the mask held fixed:  grad_in = J^T grad_out, fp64, HWC.
 */
int32_t orc_backward(const orc_params_t* p, const double* img, const uint8_t* mask,
                     const double* grad_out, double* grad_in);

#ifdef __cplusplus
}
#endif

#endif
