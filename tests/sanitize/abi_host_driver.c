/* Drives the host-only entry points of libdppix (descriptor validation,
 * plan layout, sizes, frame information, status strings, and the calls that
 * must refuse an unbound plan before touching a device) with valid and
 * invalid descriptors, for a build whose host code has AddressSanitizer and
 * UndefinedBehaviorSanitizer.  No GPU is needed.  Exit status 0 and "ok" on
 * the last line when every call behaved as the header says. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "dppix.h"

static uint64_t rng_state = 0xD1B54A32D192ED03ull;

static uint32_t next_u32(void)
{
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return (uint32_t)((rng_state * 0x2545F4914F6CDD1Dull) >> 32);
}

static int pick(int lo, int hi) { return lo + (int)(next_u32() % (uint32_t)(hi - lo + 1)); }

static int bad = 0;

/* count an unexpected result; print the first few */
static void expect(int ok, const char* what, int t)
{
    if (ok)
        return;
    if (++bad <= 10)
        printf("case %d: %s (%s)\n", t, what, dp_pix_last_error());
}

static dppix_frame_desc_t random_desc(int valid)
{
    dppix_frame_desc_t d;
    memset(&d, 0, sizeof d);
    const int sbs[] = {1, 2, 4, 8, 16};
    d.height = pick(1, 3000);
    d.width = pick(1, 3000);
    d.channels = pick(1, 4);
    d.layout = pick(0, 1);
    d.pitch = d.layout == DPPIX_U8_HWC ? (int64_t)d.width * d.channels + pick(0, 40) : d.width + pick(0, 10);
    d.pad_mode = pick(0, 2);
    d.b_fg = sbs[pick(0, 4)];
    d.b_bg = d.b_fg * pick(1, 8);
    d.m = pick(1, 64);
    d.eps_bg = pick(0, 9) == 0 ? INFINITY : 0.1 * pick(1, 30);
    d.eps_fg = pick(0, 9) == 0 ? INFINITY : 0.1 * pick(1, 30);
    d.fg_min_count = pick(0, d.b_bg * d.b_bg < 5 ? d.b_bg * d.b_bg : 5);
    d.tile_cells = pick(0, 3) == 0 ? pick(1, 64) : 0;
    d.seed = ((uint64_t)next_u32() << 32) | next_u32();
    d.frame_index = next_u32();
    if (!valid) {
        switch (pick(0, 9)) {
        case 0: d.height = -pick(0, 5); break;
        case 1: d.channels = pick(5, 9); break;
        case 2: d.pitch = (d.layout == DPPIX_U8_HWC ? d.width * (int64_t)d.channels : d.width) - 1; break;
        case 3: d.b_fg = 2 * pick(1, 8); d.b_bg = d.b_fg * pick(1, 4) + 1; break;
        case 4: d.b_fg = 0; break;
        case 5: d.m = 0; break;
        case 6: d.eps_bg = -1.0; break;
        case 7: d.layout = 7; break;
        case 8: d.pad_mode = 9; break;
        default: d.eps_fg = NAN; break;
        }
    }
    return d;
}

int main(void)
{
    for (int t = 0; t < 400; ++t) {
        const int valid = t % 4 != 3;
        dppix_frame_desc_t d[6];
        const int nf = pick(1, 6);
        for (int i = 0; i < nf; ++i)
            d[i] = random_desc(valid || i != nf - 1);
        dppix_sizes_t sz, sz2;
        const dppix_status_t s1 = dp_pix_plan_workspace_size(d, nf, &sz);
        dppix_plan_t p = NULL;
        const dppix_status_t s2 = dp_pix_plan_create(d, nf, &p);
        expect(s1 == s2, "workspace_size and create disagree", t);
        if (s2 != DPPIX_OK) {
            expect(p == NULL && dp_pix_last_error() != NULL && strlen(dp_pix_last_error()) > 0,
                   "refusal without a detail string", t);
            expect(!valid || s2 == DPPIX_ENOTSUP, "valid descriptors refused", t);
            continue;
        }
        expect(valid, "invalid descriptor accepted", t);
        expect(dp_pix_plan_sizes(p, &sz2) == DPPIX_OK && memcmp(&sz, &sz2, sizeof sz) == 0,
               "sizes differ from workspace_size", t);
        for (int i = 0; i < nf; ++i) {
            dppix_frame_info_t fi;
            expect(dp_pix_plan_frame_info(p, i, &fi) == DPPIX_OK, "frame_info of a frame refused", t);
        }
        dppix_frame_info_t fi;
        expect(dp_pix_plan_frame_info(p, nf, &fi) != DPPIX_OK, "frame_info past the batch accepted", t);
        /* calls on an unbound plan are refused on the host */
        dppix_store_t st;
        memset(&st, 0, sizeof st);
        expect(dp_pix_plan(p, NULL, &st, NULL) == DPPIX_EINVAL &&
                   dp_pix_forward(p, NULL, &st, NULL, NULL, NULL, NULL) == DPPIX_EINVAL &&
                   dp_pix_reconstruct(p, &st, NULL, NULL) == DPPIX_EINVAL &&
                   dp_pix_plan_labels(p, NULL, 10, &st, NULL) == DPPIX_EINVAL &&
                   dp_pix_backward_static(p, &st, NULL, NULL, NULL, NULL, NULL) == DPPIX_EINVAL,
               "a call on an unbound plan was not refused", t);
        (void)dp_pix_plan_set_launch(p, pick(0, 600), pick(0, 70));
        dp_pix_plan_destroy(p);
    }
    for (int s = 0; s <= 5; ++s)
        expect(dp_pix_status_string((dppix_status_t)s) != NULL, "status string missing", -1);
    expect(dp_pix_plan_create(NULL, 1, NULL) != DPPIX_OK && dp_pix_version() != NULL, "NULL descriptors accepted",
           -1);
    printf("%d unexpected results\n", bad);
    if (bad)
        return 1;
    printf("ok\n");
    return 0;
}
