// Validation against injected pulses, host side (Methods, "Validation methodology"): the
// effective width of an injected pulse at its DM, and the greedy one-to-one matching of
// candidates to injections from which detection completeness is computed.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "snd_internal.h"

namespace {

snd_status fail(snd_status s, const char *msg)
{
    snd::set_error(msg);
    return s;
}

bool finite_all(int64_t n, const double *a)
{
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) return false;
    return true;
}

}  // namespace

extern "C" {

snd_status snd_effective_width(int32_t nchan, const double *freq_mhz, double tsamp_s, int64_t n, const double *dm,
                               const double *w_int_ms, double *h_weff_ms)
{
    if (nchan < 1 || !freq_mhz || n < 0 || (n > 0 && (!dm || !w_int_ms || !h_weff_ms)) || !(tsamp_s > 0.0) ||
        !std::isfinite(tsamp_s))
        return fail(SND_ERR_INVALID, "nchan >= 1, finite tsamp_s > 0, n >= 0 and non-null arrays needed");
    double fmax = freq_mhz[0], fmin = freq_mhz[0];
    for (int32_t c = 0; c < nchan; ++c) {
        if (!(freq_mhz[c] > 0.0) || !std::isfinite(freq_mhz[c])) return fail(SND_ERR_INVALID, "frequencies must be > 0");
        fmax = std::max(fmax, freq_mhz[c]);
        fmin = std::min(fmin, freq_mhz[c]);
    }
    // smearing inside one channel at the band centre, as in the multi-rate criterion
    const double fc = 0.5 * (fmax + fmin);
    const double df = nchan > 1 ? (fmax - fmin) / (double)(nchan - 1) : 0.0;
    const double dt = tsamp_s * 1e3;
    for (int64_t i = 0; i < n; ++i) {
        if (!(dm[i] >= 0.0) || !std::isfinite(dm[i])) return fail(SND_ERR_INVALID, "DMs must be finite and >= 0");
        if (!(w_int_ms[i] >= 0.0) || !std::isfinite(w_int_ms[i]))
            return fail(SND_ERR_INVALID, "intrinsic widths must be finite and >= 0");
    }
    for (int64_t i = 0; i < n; ++i) {
        const double tau = snd::kDM * dm[i] * df / (fc * fc * fc);
        h_weff_ms[i] = std::sqrt(w_int_ms[i] * w_int_ms[i] + tau * tau + dt * dt);
    }
    return SND_OK;
}

snd_status snd_match_injections(int64_t n_cand, const double *cand_dm, const double *cand_t_ms, const double *cand_snr,
                                int64_t n_inj, const double *inj_dm, const double *inj_t_ms, const double *inj_weff_ms,
                                double dm_tol, double t_frac, int32_t *h_match, int64_t *h_nmatched)
{
    if (n_cand < 0 || n_inj < 0 || !h_nmatched || (n_cand > 0 && (!cand_dm || !cand_t_ms || !cand_snr)) ||
        (n_inj > 0 && (!inj_dm || !inj_t_ms || !inj_weff_ms || !h_match)))
        return fail(SND_ERR_INVALID, "n_cand, n_inj >= 0 and non-null arrays needed");
    if (n_cand > 0x7fffffffLL) return fail(SND_ERR_INVALID, "at most 2^31 - 1 candidates");
    if (!(dm_tol >= 0.0) || !(t_frac >= 0.0) || !std::isfinite(dm_tol) || !std::isfinite(t_frac))
        return fail(SND_ERR_INVALID, "dm_tol and t_frac must be finite and >= 0");
    if (!finite_all(n_cand, cand_dm) || !finite_all(n_cand, cand_t_ms) || !finite_all(n_cand, cand_snr) ||
        !finite_all(n_inj, inj_dm) || !finite_all(n_inj, inj_t_ms) || !finite_all(n_inj, inj_weff_ms))
        return fail(SND_ERR_INVALID, "candidate and injection values must be finite");
    for (int64_t j = 0; j < n_inj; ++j) {
        if (inj_weff_ms[j] < 0.0) return fail(SND_ERR_INVALID, "effective widths must be >= 0");
        h_match[j] = -1;
    }
    // candidates in decreasing S/N; equal S/N keep their input order
    std::vector<int64_t> order((size_t)n_cand);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return cand_snr[a] > cand_snr[b]; });
    int64_t matched = 0;
    for (const int64_t i : order) {
        int64_t best = -1;
        double best_dt = 0.0, best_ddm = 0.0;
        for (int64_t j = 0; j < n_inj; ++j) {
            if (h_match[j] >= 0) continue;  // one to one
            const double ddm = std::fabs(cand_dm[i] - inj_dm[j]);
            const double dt = std::fabs(cand_t_ms[i] - inj_t_ms[j]);
            if (ddm > dm_tol || dt > t_frac * inj_weff_ms[j]) continue;
            // the admissible injection nearest in time, then in DM, then the lowest index
            if (best < 0 || dt < best_dt || (dt == best_dt && ddm < best_ddm)) {
                best = j;
                best_dt = dt;
                best_ddm = ddm;
            }
        }
        if (best >= 0) {
            h_match[best] = (int32_t)i;
            ++matched;
        }
    }
    *h_nmatched = matched;
    return SND_OK;
}

}  // extern "C"
