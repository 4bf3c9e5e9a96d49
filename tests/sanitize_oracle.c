/* Host sanitizer run of the oracle (AddressSanitizer + UndefinedBehaviorSanitizer): one
 * translation unit with the oracle's source, driving its tree, matched filter, candidate and
 * front-end functions on a small ragged case in every mode.  Exits non-zero on a mismatch
 * between the shared-pattern tree and the per-DM recursion (and brute force in the linear
 * modes); the sanitizers abort on any memory or undefined-behaviour error. */
#include "../oracle/snd_oracle.c"

#include <stdio.h>

static uint32_t lcg(uint32_t *s) { *s = *s * 1664525u + 1013904223u; return *s >> 8; }

int main(void)
{
    enum { NCH = 13, NDM = 9, NT = 700 };
    double freq[NCH], dm[NDM];
    for (int c = 0; c < NCH; ++c) freq[c] = 416.0 - 0.8 * c;
    for (int k = 0; k < NDM; ++k) dm[k] = 6.0 * k;  /* the sweep at DM 48 is about 400 of the 700 samples */
    int32_t delays[NDM * NCH];
    if (orc_delays(NCH, freq, 0.138e-3, 0.0, NDM, dm, delays)) return 2;
    uint8_t x[NCH * NT];
    uint32_t s = 7;
    for (int i = 0; i < NCH * NT; ++i) x[i] = (uint8_t)(lcg(&s) % 100 < 12);
    int32_t maxd = 0;
    for (int i = 0; i < NDM * NCH; ++i) maxd = delays[i] > maxd ? delays[i] : maxd;
    const int64_t nout = NT - maxd;
    if (nout < 1) return 11;
    double *a = malloc(sizeof(double) * NDM * nout), *b = malloc(sizeof(double) * NDM * nout);
    double *c = malloc(sizeof(double) * NDM * nout);
    int64_t counts[2 * ORC_MAXLEV];
    for (int mode = 0; mode < 3; ++mode) {
        orc_params p = {mode, 3, 2, 2, 1, 3, 0};
        if (orc_snd_dedup(&p, NCH, freq, NT, x, ORC_IN_U8, NDM, delays, a, counts, ORC_MAXLEV) < 0 ||  /* level count */
            orc_snd_recursive(&p, NCH, freq, NT, x, ORC_IN_U8, NDM, delays, b))
            return 3;
        for (int64_t i = 0; i < NDM * nout; ++i)
            if (a[i] != b[i]) { fprintf(stderr, "mode %d: dedup != recursion at %lld\n", mode, (long long)i); return 4; }
        if (mode == ORC_FLOAT) {
            if (orc_bruteforce(mode, NCH, NT, x, ORC_IN_U8, NDM, delays, c)) return 5;
            for (int64_t i = 0; i < NDM * nout; ++i)
                if (a[i] != c[i]) { fprintf(stderr, "float: tree != brute force at %lld\n", (long long)i); return 6; }
        }
        int32_t w[3] = {1, 2, 4};
        double *snr = malloc(sizeof(double) * NDM * nout), mu[NDM], sg[NDM], sig_in[NDM];
        int32_t *widx = malloc(sizeof(int32_t) * NDM * nout);
        for (int k = 0; k < NDM; ++k) sig_in[k] = 0.5 + 0.1 * k;
        if (orc_matched_filter_sigma(mode != ORC_FLOAT, NDM, nout, a, 3, w, NULL, mode == 1 ? sig_in : NULL, 0.15, snr,
                                     widx, mu, sg))
            return 7;
        orc_cand cand[64];
        if (orc_candidates(NDM, nout, snr, widx, 2.0, 2, 1, cand, 64) < 0) return 8;
        free(snr);
        free(widx);
    }
    float z[NCH * 64];
    for (int i = 0; i < NCH * 64; ++i) z[i] = (float)((int)(lcg(&s) % 2001) - 1000) / 500.0f;
    for (int c2 = 0; c2 < NCH; ++c2) z[c2 * 64 + 9] += 6.0f;
    uint8_t flags[NCH * 3];
    double sig[NCH * 3];
    if (orc_flag_channels(NCH, 64, z, 25, 3.0, 1.4826022185056018, flags, sig)) return 9;
    if (orc_zero_dm(NCH, 64, z, 5.0) < 0) return 10;
    free(a);
    free(b);
    free(c);
    puts("sanitized oracle run ok");
    return 0;
}
