/*
 * dppix_oracle.c — plain CPU oracle (TEST INFRASTRUCTURE ONLY; see the header).
 *
 * Written for readability against the paper, not for speed: the padded image
 * and mask are materialised (Algorithm 3, step 3), cells are visited in
 * row-major order, and every mean is taken from scratch in fp64.
 */
#include "dppix_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon et al., SC'11, Sec. 5): a 4-word counter is mixed by
 * ten rounds; each round multiplies words 0 and 2 by two fixed constants,
 * splits the 64-bit products into high and low halves, xors the high halves
 * with words 1 and 3 and with the round key, and permutes.  The two key words
 * are incremented by two Weyl constants between rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t MUL_A = 0xD2511F53u, MUL_B = 0xCD9E8D57u;
    const uint32_t WEYL_A = 0x9E3779B9u, WEYL_B = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += WEYL_A;
            k1 += WEYL_B;
        }
        uint64_t pa = (uint64_t)MUL_A * (uint64_t)x0;
        uint64_t pb = (uint64_t)MUL_B * (uint64_t)x2;
        uint32_t pa_hi = (uint32_t)(pa >> 32), pa_lo = (uint32_t)pa;
        uint32_t pb_hi = (uint32_t)(pb >> 32), pb_lo = (uint32_t)pb;
        uint32_t y0 = pb_hi ^ x1 ^ k0;
        uint32_t y1 = pb_lo;
        uint32_t y2 = pa_hi ^ x3 ^ k1;
        uint32_t y3 = pa_lo;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

void orc_noise_words(uint64_t seed, uint64_t frame_index, uint32_t id, int32_t ch,
                     int32_t level, uint32_t out[4])
{
    uint32_t ctr[4], key[2];
    ctr[0] = id;
    ctr[1] = (uint32_t)ch | ((uint32_t)level << 8);
    ctr[2] = (uint32_t)(frame_index & 0xFFFFFFFFu);
    ctr[3] = (uint32_t)(frame_index >> 32);
    key[0] = (uint32_t)(seed & 0xFFFFFFFFu);
    key[1] = (uint32_t)(seed >> 32);
    orc_philox4x32_10(ctr, key, out);
}

double orc_uniform(uint32_t w0, uint32_t w1)
{
    uint64_t x = ((uint64_t)w1 << 32) | (uint64_t)w0;
    uint64_t k = x >> 12;                        /* 52 random bits */
    return ldexp((double)(2 * k + 1), -53);      /* exactly representable, in (0,1) */
}

/* Laplace(0, sigma): CDF F(x) = 1/2 exp(x/sigma) for x < 0 and
 * 1 - 1/2 exp(-x/sigma) for x >= 0, inverted piecewise (Eq. 9). */
double orc_laplace(double u, double sigma)
{
    if (u < 0.5)
        return sigma * log(2.0 * u);
    return -sigma * log(2.0 * (1.0 - u));
}

/* Eq. (11): Delta P_b = 255 m / b^2, and Eq. (8): sigma = Delta / eps. */
double orc_sigma(int32_t b, int32_t m, double eps)
{
    if (isinf(eps))
        return 0.0;
    double delta = 255.0 * (double)m / ((double)b * (double)b);
    return delta / eps;
}

/* Mirror padding (Algorithm 2 step 4 / Algorithm 3 step 3).  Symmetric mode
 * repeats the edge pixel (period 2L); reflect mode does not (period 2L-2).
 * Not defined for the unpadded mode, which never folds. */
int64_t orc_fold(int64_t x, int64_t L, int32_t mode)
{
    if (mode == ORC_PAD_SYMMETRIC) {
        int64_t y = x % (2 * L);
        return y < L ? y : 2 * L - 1 - y;
    }
    if (L == 1)
        return 0;
    int64_t y = x % (2 * L - 2);
    return y < L ? y : 2 * L - 2 - y;
}

int32_t orc_check(const orc_params_t* p)
{
    if (p->height < 1 || p->width < 1 || p->channels < 1 || p->channels > 4)
        return 1;
    if (p->b < 1 || p->sb < 1 || p->sb > p->b || p->b % p->sb != 0)
        return 1; /* Eq. (16): b = n * s_b */
    if (p->m < 1)
        return 1;
    if (!(p->eps_simple > 0.0) || !(p->eps_complex > 0.0))
        return 1;
    if (p->tau < 0 || (int64_t)p->tau > (int64_t)p->b * p->b)
        return 1;
    if (p->pad_mode != ORC_PAD_SYMMETRIC && p->pad_mode != ORC_PAD_REFLECT && p->pad_mode != ORC_PAD_NONE)
        return 1;
    return 0;
}

int32_t orc_geometry(const orc_params_t* p, int32_t* GR, int32_t* GC, int32_t* n)
{
    if (orc_check(p))
        return 1;
    *GR = (p->height + p->b - 1) / p->b; /* G_R = ceil(M/b) */
    *GC = (p->width + p->b - 1) / p->b;  /* G_C = ceil(N/b) */
    *n = p->b / p->sb;
    return 0;
}

/* Noise for one statistic; eps = +inf gives exactly zero. */
static double noise_for(const orc_params_t* p, uint32_t id, int32_t ch, int32_t level,
                        double sigma, double eps)
{
    if (isinf(eps))
        return 0.0;
    uint32_t w[4];
    orc_noise_words(p->seed, p->frame_index, id, ch, level, w);
    return orc_laplace(orc_uniform(w[0], w[1]), sigma);
}

static double clip255(double v)
{
    if (v < 0.0)
        return 0.0;
    if (v > 255.0)
        return 255.0;
    return v;
}

/*
 * Forward pass, following Algorithm 3 step by step.
 */
int32_t orc_forward(const orc_params_t* p, const double* img, const uint8_t* mask,
                    uint8_t* flags, float* bg, float* fg, int64_t counts[2],
                    float* recon_f32, uint8_t* recon_u8, double* recon_f64,
                    double* coarse_sum, double* fine_sum,
                    uint8_t* pass_bg, uint8_t* pass_fg)
{
    int32_t GR, GC, n;
    if (orc_geometry(p, &GR, &GC, &n))
        return 1;
    const int64_t M = p->height, N = p->width, C = p->channels;
    const int64_t b = p->b, sb = p->sb;
    /* Step 1-2: grid dimensions and padding sizes. */
    const int64_t HP = (int64_t)GR * b, WP = (int64_t)GC * b; /* M + P_R, N + P_C */

    /* Step 3: mirror-pad image and mask to (M+P_R, N+P_C).  In the unpadded
     * mode (Algorithm 1) positions outside the frame stay empty: Rpad marks
     * the real ones, and an empty position adds nothing to any sum or count. */
    const int unpadded = p->pad_mode == ORC_PAD_NONE;
    double* Ipad = (double*)malloc(sizeof(double) * HP * WP * C);
    uint8_t* Fpad = (uint8_t*)malloc((size_t)(HP * WP));
    uint8_t* Rpad = (uint8_t*)malloc((size_t)(HP * WP));
    double* Opad = (double*)malloc(sizeof(double) * HP * WP * C); /* I_grid after assignment */
    double* Dpad = (double*)malloc(sizeof(double) * HP * WP * C); /* same, before fp32 rounding */
    if (!Ipad || !Fpad || !Rpad || !Opad || !Dpad) {
        free(Ipad); free(Fpad); free(Rpad); free(Opad); free(Dpad);
        return 2;
    }
    for (int64_t i = 0; i < HP; ++i)
        for (int64_t j = 0; j < WP; ++j) {
            const int real = i < M && j < N;
            Rpad[i * WP + j] = (uint8_t)(unpadded ? real : 1);
            if (unpadded && !real) {
                for (int64_t ch = 0; ch < C; ++ch)
                    Ipad[(i * WP + j) * C + ch] = 0.0;
                Fpad[i * WP + j] = 0;
                continue;
            }
            int64_t si = unpadded ? i : orc_fold(i, M, p->pad_mode);
            int64_t sj = unpadded ? j : orc_fold(j, N, p->pad_mode);
            for (int64_t ch = 0; ch < C; ++ch)
                Ipad[(i * WP + j) * C + ch] = img[(si * N + sj) * C + ch];
            Fpad[i * WP + j] = mask ? (uint8_t)(mask[si * N + sj] != 0) : 0;
        }

    /* Steps 4-6: view as (G_R, G_C, b, b); mask statistic per grid; classify.
     * The mask here marks the foreground (the complement of the paper's simple
     * mask); a cell is complex when its foreground count reaches tau. */
    for (int64_t r = 0; r < GR; ++r)
        for (int64_t c = 0; c < GC; ++c) {
            int64_t cnt = 0, area = 0;
            for (int64_t di = 0; di < b; ++di)
                for (int64_t dj = 0; dj < b; ++dj) {
                    cnt += Fpad[(r * b + di) * WP + (c * b + dj)];
                    area += Rpad[(r * b + di) * WP + (c * b + dj)];
                }
            const int64_t tau = p->tau > 0 ? p->tau : (area + 1) / 2;
            flags[r * GC + c] = (uint8_t)(mask != NULL && cnt >= tau);
        }

    /* Optional diagnostics: padded sums of every coarse cell and every subcell,
     * each computed on its own from the padded image. */
    if (coarse_sum)
        for (int64_t r = 0; r < GR; ++r)
            for (int64_t c = 0; c < GC; ++c)
                for (int64_t ch = 0; ch < C; ++ch) {
                    double s = 0.0;
                    for (int64_t di = 0; di < b; ++di)
                        for (int64_t dj = 0; dj < b; ++dj)
                            s += Ipad[((r * b + di) * WP + (c * b + dj)) * C + ch];
                    coarse_sum[(r * GC + c) * C + ch] = s;
                }
    if (fine_sum) {
        const int64_t FR = (int64_t)GR * n, FC = (int64_t)GC * n;
        for (int64_t fr = 0; fr < FR; ++fr)
            for (int64_t fc = 0; fc < FC; ++fc)
                for (int64_t ch = 0; ch < C; ++ch) {
                    double s = 0.0;
                    for (int64_t di = 0; di < sb; ++di)
                        for (int64_t dj = 0; dj < sb; ++dj)
                            s += Ipad[((fr * sb + di) * WP + (fc * sb + dj)) * C + ch];
                    fine_sum[(fr * FC + fc) * C + ch] = s;
                }
    }

    /* Steps 7-11: simple cells — grid mean, Laplace noise with
     * sigma = 255 m / (b^2 eps), clip to [0,255], assign over the grid. */
    const double sigma_s = orc_sigma((int32_t)b, p->m, p->eps_simple);
    int64_t k = 0;
    for (int64_t r = 0; r < GR; ++r)
        for (int64_t c = 0; c < GC; ++c) {
            if (flags[r * GC + c])
                continue;
            for (int64_t ch = 0; ch < C; ++ch) {
                double s = 0.0, area = 0.0;
                for (int64_t di = 0; di < b; ++di)
                    for (int64_t dj = 0; dj < b; ++dj) {
                        s += Ipad[((r * b + di) * WP + (c * b + dj)) * C + ch];
                        area += Rpad[(r * b + di) * WP + (c * b + dj)];
                    }
                double mu = s / area;   /* b*b, or h*w real pixels (Algorithm 1) */
                double eta = noise_for(p, (uint32_t)(r * GC + c), (int32_t)ch, 0, sigma_s,
                                       p->eps_simple);
                double z = mu + eta;
                double v = clip255(z);
                bg[k * C + ch] = (float)v;
                if (pass_bg)
                    pass_bg[k * C + ch] = (uint8_t)(z >= 0.0 && z <= 255.0);
                for (int64_t di = 0; di < b; ++di)
                    for (int64_t dj = 0; dj < b; ++dj) {
                        Opad[((r * b + di) * WP + (c * b + dj)) * C + ch] = (double)(float)v;
                        Dpad[((r * b + di) * WP + (c * b + dj)) * C + ch] = v;
                    }
            }
            ++k;
        }
    const int64_t n_bg = k;

    /* Steps 12-19: complex cells — split into n x n subgrids of size s_b,
     * subgrid means, noise with sigma_s = 255 m / (s_b^2 eps), clip, assign. */
    const double sigma_c = orc_sigma((int32_t)sb, p->m, p->eps_complex);
    const int64_t nn = (int64_t)n * n;
    k = 0;
    for (int64_t r = 0; r < GR; ++r)
        for (int64_t c = 0; c < GC; ++c) {
            if (!flags[r * GC + c])
                continue;
            for (int64_t i = 0; i < n; ++i)
                for (int64_t j = 0; j < n; ++j) {
                    uint32_t id = (uint32_t)((r * n + i) * ((int64_t)GC * n) + (c * n + j));
                    for (int64_t ch = 0; ch < C; ++ch) {
                        double s = 0.0, area = 0.0;
                        for (int64_t di = 0; di < sb; ++di)
                            for (int64_t dj = 0; dj < sb; ++dj) {
                                s += Ipad[((r * b + i * sb + di) * WP + (c * b + j * sb + dj)) * C + ch];
                                area += Rpad[(r * b + i * sb + di) * WP + (c * b + j * sb + dj)];
                            }
                        int64_t at = (k * nn + i * n + j) * C + ch;
                        double v = 0.0, z = 0.0;
                        if (area > 0.0) {
                            double mu = s / area;
                            double eta = noise_for(p, id, (int32_t)ch, 1, sigma_c, p->eps_complex);
                            z = mu + eta;
                            v = clip255(z);
                        }
                        fg[at] = (float)v;
                        if (pass_fg)
                            pass_fg[at] = (uint8_t)(area > 0.0 && z >= 0.0 && z <= 255.0);
                        for (int64_t di = 0; di < sb; ++di)
                            for (int64_t dj = 0; dj < sb; ++dj) {
                                int64_t o = ((r * b + i * sb + di) * WP + (c * b + j * sb + dj)) * C + ch;
                                Opad[o] = (double)(float)v;
                                Dpad[o] = v;
                            }
                    }
                }
            ++k;
        }
    counts[0] = n_bg;
    counts[1] = k;

    /* Steps 20-21: back to image layout and crop to M x N. */
    for (int64_t i = 0; i < M; ++i)
        for (int64_t j = 0; j < N; ++j)
            for (int64_t ch = 0; ch < C; ++ch) {
                double v = Opad[(i * WP + j) * C + ch];
                if (recon_f32)
                    recon_f32[(i * N + j) * C + ch] = (float)v;
                if (recon_u8)
                    recon_u8[(i * N + j) * C + ch] = (uint8_t)nearbyint(v);
                if (recon_f64)
                    recon_f64[(i * N + j) * C + ch] = Dpad[(i * WP + j) * C + ch];
            }

    free(Ipad);
    free(Fpad);
    free(Rpad);
    free(Opad);
    free(Dpad);
    return 0;
}

/* Mirror index of a coordinate that may be -1 (one step before the start);
 * the unpadded mode mirrors like the symmetric one here. */
static int64_t edge_fold(int64_t x, int64_t L, int32_t mode)
{
    if (mode == ORC_PAD_NONE)
        mode = ORC_PAD_SYMMETRIC;
    if (x < 0) {
        if (mode == ORC_PAD_SYMMETRIC || L == 1)
            return 0;
        return 1;
    }
    return orc_fold(x, L, mode);
}

int32_t orc_edge_mask(int32_t M, int32_t N, int32_t C, const double* img, int32_t threshold, int32_t pad_mode,
                      uint8_t* out)
{
    if (M < 1 || N < 1 || C < 1 || threshold < 0)
        return 1;
    for (int64_t i = 0; i < M; ++i)
        for (int64_t j = 0; j < N; ++j) {
            double S[3][3];
            for (int di = -1; di <= 1; ++di)
                for (int dj = -1; dj <= 1; ++dj) {
                    int64_t y = edge_fold(i + di, M, pad_mode), x = edge_fold(j + dj, N, pad_mode);
                    double s = 0.0;
                    for (int64_t ch = 0; ch < C; ++ch)
                        s += img[(y * N + x) * C + ch];
                    S[di + 1][dj + 1] = s;
                }
            /* Sobel: derivative [-1 0 1] along one axis, smoothing [1 2 1] along the other */
            double gx = (S[0][2] + 2.0 * S[1][2] + S[2][2]) - (S[0][0] + 2.0 * S[1][0] + S[2][0]);
            double gy = (S[2][0] + 2.0 * S[2][1] + S[2][2]) - (S[0][0] + 2.0 * S[0][1] + S[0][2]);
            out[i * N + j] = (uint8_t)(fabs(gx) + fabs(gy) >= (double)threshold * (double)C);
        }
    return 0;
}

int32_t orc_metrics(int32_t M, int32_t N, int32_t C, const double* x, const double* y, double* mse, double* ssim)
{
    if (M < 7 || N < 7 || C < 1)
        return 1;
    const int64_t total = (int64_t)M * N * C;
    double se = 0.0;
    for (int64_t q = 0; q < total; ++q)
        se += (x[q] - y[q]) * (x[q] - y[q]);
    *mse = se / (double)total;

    const double R = 255.0, c1 = (0.01 * R) * (0.01 * R), c2 = (0.03 * R) * (0.03 * R);
    const double np = 49.0;
    double acc = 0.0;
    int64_t windows = 0;
    for (int64_t ch = 0; ch < C; ++ch)
        for (int64_t i = 3; i < M - 3; ++i)
            for (int64_t j = 3; j < N - 3; ++j) {
                double sx = 0, sy = 0, sxx = 0, syy = 0, sxy = 0;
                for (int64_t di = -3; di <= 3; ++di)
                    for (int64_t dj = -3; dj <= 3; ++dj) {
                        double a = x[((i + di) * N + (j + dj)) * C + ch];
                        double b = y[((i + di) * N + (j + dj)) * C + ch];
                        sx += a; sy += b; sxx += a * a; syy += b * b; sxy += a * b;
                    }
                double ux = sx / np, uy = sy / np;
                /* sample variances: divide the centred sums by np - 1 */
                double vx = (sxx / np - ux * ux) * np / (np - 1.0);
                double vy = (syy / np - uy * uy) * np / (np - 1.0);
                double vxy = (sxy / np - ux * uy) * np / (np - 1.0);
                double s = ((2.0 * ux * uy + c1) * (2.0 * vxy + c2)) / ((ux * ux + uy * uy + c1) * (vx + vy + c2));
                acc += s;
                ++windows;
            }
    /* every channel has the same number of windows: the mean over all windows
     * equals the mean of the per-channel means */
    *ssim = acc / (double)windows;
    return 0;
}

/* Restoration from the stored metadata: broadcast each stored scalar over its
 * grid or subgrid in the padded frame, then crop. */
int32_t orc_reconstruct(const orc_params_t* p, const uint8_t* flags, const float* bg,
                        const float* fg, float* recon_f32, uint8_t* recon_u8)
{
    int32_t GR, GC, n;
    if (orc_geometry(p, &GR, &GC, &n))
        return 1;
    const int64_t M = p->height, N = p->width, C = p->channels;
    const int64_t b = p->b, sb = p->sb, nn = (int64_t)n * n;
    /* store index of every cell, in row-major order within each class */
    int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * (size_t)GR * GC);
    if (!idx)
        return 2;
    int64_t kb = 0, kf = 0;
    for (int64_t q = 0; q < (int64_t)GR * GC; ++q)
        idx[q] = flags[q] ? kf++ : kb++;
    for (int64_t i = 0; i < M; ++i)
        for (int64_t j = 0; j < N; ++j) {
            int64_t r = i / b, c = j / b, cell = r * GC + c;
            for (int64_t ch = 0; ch < C; ++ch) {
                float v;
                if (!flags[cell]) {
                    v = bg[idx[cell] * C + ch];
                } else {
                    int64_t si = (i - r * b) / sb, sj = (j - c * b) / sb;
                    v = fg[(idx[cell] * nn + si * n + sj) * C + ch];
                }
                if (recon_f32)
                    recon_f32[(i * N + j) * C + ch] = v;
                if (recon_u8)
                    recon_u8[(i * N + j) * C + ch] = (uint8_t)nearbyint((double)v);
            }
        }
    free(idx);
    return 0;
}

/*
 * Adjoint.  With the noise and classification fixed, statistic k is
 * v_k = clip(mu_k + eta_k) with mu_k = (1/area_k) * sum over the padded cell of
 * I(fold(x)).  Output pixel (i,j) equals the v_k of the cell holding it, so
 * dL/dI(q) = sum_k [0 <= mu_k+eta_k <= 255] * G_k / area_k * #{x in cell k : fold(x) = q},
 * where G_k sums dL/dy over the real pixels of cell k.
 */
int32_t orc_backward(const orc_params_t* p, const double* img, const uint8_t* mask,
                     const double* grad_out, double* grad_in)
{
    int32_t GR, GC, n;
    if (orc_geometry(p, &GR, &GC, &n))
        return 1;
    const int64_t M = p->height, N = p->width, C = p->channels;
    const int64_t b = p->b, sb = p->sb, nn = (int64_t)n * n;
    const int64_t cells = (int64_t)GR * GC;

    uint8_t* flags = (uint8_t*)malloc((size_t)cells);
    float* bg = (float*)malloc(sizeof(float) * (size_t)(cells * C));
    float* fg = (float*)malloc(sizeof(float) * (size_t)(cells * nn * C));
    uint8_t* pass_bg = (uint8_t*)malloc((size_t)(cells * C));
    uint8_t* pass_fg = (uint8_t*)malloc((size_t)(cells * nn * C));
    int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * (size_t)cells);
    if (!flags || !bg || !fg || !pass_bg || !pass_fg || !idx) {
        free(flags); free(bg); free(fg); free(pass_bg); free(pass_fg); free(idx);
        return 2;
    }
    int64_t counts[2];
    int32_t rc = orc_forward(p, img, mask, flags, bg, fg, counts, NULL, NULL, NULL, NULL, NULL,
                             pass_bg, pass_fg);
    if (rc) {
        free(flags); free(bg); free(fg); free(pass_bg); free(pass_fg); free(idx);
        return rc;
    }
    int64_t kb = 0, kf = 0;
    for (int64_t q = 0; q < cells; ++q)
        idx[q] = flags[q] ? kf++ : kb++;

    for (int64_t q = 0; q < M * N * C; ++q)
        grad_in[q] = 0.0;

    for (int64_t r = 0; r < GR; ++r)
        for (int64_t c = 0; c < GC; ++c) {
            int64_t cell = r * GC + c;
            int64_t parts = flags[cell] ? n : 1;     /* subcells per side */
            int64_t side = flags[cell] ? sb : b;     /* side of one statistic */
            for (int64_t i = 0; i < parts; ++i)
                for (int64_t j = 0; j < parts; ++j)
                    for (int64_t ch = 0; ch < C; ++ch) {
                        int64_t i0 = r * b + i * side, j0 = c * b + j * side;
                        int64_t at = flags[cell] ? (idx[cell] * nn + i * n + j) * C + ch
                                                 : idx[cell] * C + ch;
                        uint8_t pass = flags[cell] ? pass_fg[at] : pass_bg[at];
                        /* G_k over the real pixels of this statistic */
                        double G = 0.0;
                        for (int64_t di = 0; di < side; ++di)
                            for (int64_t dj = 0; dj < side; ++dj) {
                                int64_t y = i0 + di, x = j0 + dj;
                                if (y < M && x < N)
                                    G += grad_out[(y * N + x) * C + ch];
                            }
                        /* area: the full side^2, or the real pixels (Algorithm 1) */
                        double area = (double)(side * side);
                        if (p->pad_mode == ORC_PAD_NONE) {
                            int64_t h = M - i0 < side ? M - i0 : side, w = N - j0 < side ? N - j0 : side;
                            area = (h > 0 && w > 0) ? (double)(h * w) : 0.0;
                        }
                        double g = (pass && area > 0.0) ? G / area : 0.0;
                        /* spread over every padded position, folded to its source
                         * (unpadded mode: only the real positions themselves) */
                        for (int64_t di = 0; di < side; ++di)
                            for (int64_t dj = 0; dj < side; ++dj) {
                                int64_t y = i0 + di, x = j0 + dj;
                                if (p->pad_mode == ORC_PAD_NONE) {
                                    if (y >= M || x >= N)
                                        continue;
                                } else {
                                    y = orc_fold(y, M, p->pad_mode);
                                    x = orc_fold(x, N, p->pad_mode);
                                }
                                grad_in[(y * N + x) * C + ch] += g;
                            }
                    }
        }

    free(flags); free(bg); free(fg); free(pass_bg); free(pass_fg); free(idx);
    return 0;
}
