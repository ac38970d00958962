/* Drives every oracle function over random small frames and the degenerate
 * cases (1 x 1 frames, b = 1, frames smaller than a cell, every pad mode,
 * empty and full masks, noise off), for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer: any invalid access or undefined operation
 * aborts the run.  Exit status 0 and "ok" on the last line otherwise. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "dppix_oracle.h"

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;

static uint32_t next_u32(void)
{
    /* xorshift64*: test input generation only */
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return (uint32_t)((rng_state * 0x2545F4914F6CDD1Dull) >> 32);
}

static int pick(int lo, int hi) { return lo + (int)(next_u32() % (uint32_t)(hi - lo + 1)); }

static int run_case(int M, int N, int C, int b, int sb, int pad, int tau, int mask_kind, int noise)
{
    orc_params_t p = {M, N, C, b, sb, 4, noise ? 0.7 : INFINITY, noise ? 0.3 : INFINITY, tau, pad, 11, 5};
    int32_t GR, GC, n;
    if (orc_check(&p) != 0 || orc_geometry(&p, &GR, &GC, &n) != 0)
        return -1;  /* invalid parameters are refused, nothing else to run */
    const size_t px = (size_t)M * N, cells = (size_t)GR * GC;
    double* img = malloc(sizeof(double) * px * C);
    uint8_t* mask = malloc(px);
    for (size_t i = 0; i < px * C; ++i)
        img[i] = (double)(next_u32() % 256u);
    for (size_t i = 0; i < px; ++i)
        mask[i] = mask_kind == 0 ? 0 : (mask_kind == 1 ? 1 : (uint8_t)(next_u32() % 3u == 0));
    uint8_t* flags = malloc(cells);
    float* bg = malloc(sizeof(float) * cells * C);
    float* fg = malloc(sizeof(float) * cells * n * n * C);
    int64_t counts[2];
    float* r32 = malloc(sizeof(float) * px * C);
    uint8_t* r8 = malloc(px * C);
    double* r64 = malloc(sizeof(double) * px * C);
    double* cs = malloc(sizeof(double) * cells * C);
    double* fs = malloc(sizeof(double) * cells * n * n * C);
    uint8_t* pb = malloc(cells * C);
    uint8_t* pf = malloc(cells * n * n * C);
    int err = orc_forward(&p, img, mask_kind < 0 ? NULL : mask, flags, bg, fg, counts, r32, r8, r64, cs, fs, pb, pf);
    float* q32 = malloc(sizeof(float) * px * C);
    uint8_t* q8 = malloc(px * C);
    err |= orc_reconstruct(&p, flags, bg, fg, q32, q8);
    double* go = malloc(sizeof(double) * px * C);
    double* gi = malloc(sizeof(double) * px * C);
    for (size_t i = 0; i < px * C; ++i)
        go[i] = (double)(int)(next_u32() % 200u) - 100.0;
    err |= orc_backward(&p, img, mask_kind < 0 ? NULL : mask, go, gi);
    uint8_t* em = malloc(px);
    err |= orc_edge_mask(M, N, C, img, pick(0, 300), pad, em);
    if (M >= 7 && N >= 7) {
        double mse, ssim;
        err |= orc_metrics(M, N, C, img, img, &mse, &ssim);
    }
    free(img); free(mask); free(flags); free(bg); free(fg); free(r32); free(r8); free(r64);
    free(cs); free(fs); free(pb); free(pf); free(q32); free(q8); free(go); free(gi); free(em);
    return err;
}

int main(void)
{
    int failures = 0, cases = 0, refused = 0, r;
    /* fixed degenerate cases */
    const int fixed[][7] = {{1, 1, 1, 1, 1, 0, 1}, {1, 1, 3, 8, 4, 1, 0}, {5, 3, 3, 8, 4, 2, 1},
                            {2, 17, 1, 16, 8, 0, 1}, {9, 9, 4, 3, 1, 2, 0}, {16, 16, 2, 16, 16, 1, 1},
                            {7, 31, 3, 32, 8, 0, 2}, {13, 29, 1, 8, 2, 2, 3}};
    for (size_t k = 0; k < sizeof fixed / sizeof fixed[0]; ++k)
        for (int mk = -1; mk <= 2; ++mk)
            for (int noise = 0; noise <= 1; ++noise) {
                const int* f = fixed[k];
                r = run_case(f[0], f[1], f[2], f[3], f[4], f[5], f[6], mk, noise);
                failures += r > 0;
                refused += r < 0;
                ++cases;
            }
    /* random cases */
    const int sbs[] = {1, 2, 3, 4, 8};
    for (int t = 0; t < 300; ++t) {
        const int sb = sbs[pick(0, 4)], n = pick(1, 4);
        r = run_case(pick(1, 40), pick(1, 40), pick(1, 4), sb * n, sb, pick(0, 2), pick(0, 6), pick(-1, 2), pick(0, 1));
        failures += r > 0;
        refused += r < 0;
        ++cases;
    }
    /* the scalar helpers over their whole argument ranges */
    for (int k = 0; k < 100000; ++k) {
        const uint32_t ctr[4] = {next_u32(), next_u32(), next_u32(), next_u32()}, key[2] = {next_u32(), next_u32()};
        uint32_t out[4];
        orc_philox4x32_10(ctr, key, out);
        const double u = orc_uniform(out[0], out[1]);
        if (!(u > 0.0 && u < 1.0) || !isfinite(orc_laplace(u, 3.0)))
            ++failures;
        (void)orc_fold((int64_t)(next_u32() % 1000u), (int64_t)(1 + next_u32() % 50u), (int32_t)(next_u32() % 3u));
    }
    printf("%d cases (%d refused as invalid), %d failures\n", cases, refused, failures);
    if (failures || refused > cases / 10)
        return 1;
    printf("ok\n");
    return 0;
}
