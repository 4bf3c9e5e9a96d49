// Multi-rate extension, host side (Methods, "Multi-rate extension"): scrunch factor per trial
// DM from the intra-channel smearing criterion, and the cross-band merge of candidates.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <string>
#include <vector>

#include "snd_internal.h"

namespace snd {
int launch_scrunch(const float *z, int64_t zp, int nchan, int64_t nout, int s, float r, float *out, int64_t op,
                   void *stream);
}

namespace {

snd_status fail(snd_status s, const char *msg)
{
    snd::set_error(msg);
    return s;
}

}  // namespace

extern "C" {

snd_status snd_scrunch_factors(int32_t nchan, const double *freq_mhz, double tsamp_s, int32_t ndm, const double *dm,
                               int32_t s_max, int32_t *h_factor)
{
    if (nchan < 1 || !freq_mhz || ndm < 0 || (ndm > 0 && (!dm || !h_factor)) || !(tsamp_s > 0.0) || s_max < 1 ||
        s_max > 1024)
        return fail(SND_ERR_INVALID, "nchan >= 1, tsamp_s > 0, 1 <= s_max <= 1024 and non-null arrays needed");
    double fmax = freq_mhz[0], fmin = freq_mhz[0];
    for (int32_t c = 0; c < nchan; ++c) {
        if (!(freq_mhz[c] > 0.0) || !std::isfinite(freq_mhz[c])) return fail(SND_ERR_INVALID, "frequencies must be > 0");
        fmax = std::max(fmax, freq_mhz[c]);
        fmin = std::min(fmin, freq_mhz[c]);
    }
    const double fc = 0.5 * (fmax + fmin);
    const double df = nchan > 1 ? (fmax - fmin) / (double)(nchan - 1) : 0.0;
    const double dt = tsamp_s * 1e3;
    for (int32_t k = 0; k < ndm; ++k) {
        if (!(dm[k] >= 0.0) || !std::isfinite(dm[k])) return fail(SND_ERR_INVALID, "trial DMs must be >= 0");
        const double tau = snd::kDM * dm[k] * df / (fc * fc * fc);
        int32_t s = 1;
        while (2 * s <= s_max && 2.0 * s * dt <= tau) s *= 2;
        h_factor[k] = s;
    }
    return SND_OK;
}

snd_status snd_scrunch(const float *d_z, int64_t z_pitch, int32_t nchan, int64_t nsamp, int32_t s, float *d_out,
                       int64_t out_pitch, void *stream)
{
    if (nchan < 1 || nchan > 65535 || nsamp < 1 || s < 1 || s > 1024) return fail(SND_ERR_INVALID, "bad nchan, nsamp or s");
    const int64_t nout = nsamp / s;
    if (nout == 0) return SND_OK;  // nothing to write (the output may be empty)
    if (!d_z || !d_out) return fail(SND_ERR_INVALID, "null pointer");
    if (z_pitch < nsamp || out_pitch < nout) return fail(SND_ERR_INVALID, "pitch too small");
    const float r = (float)(1.0 / std::sqrt((double)s));
    int e = snd::launch_scrunch(d_z, z_pitch, nchan, nout, s, r, d_out, out_pitch, stream);
    if (e) {
        snd::set_error(std::string("scrunch launch: ") + hipGetErrorString((hipError_t)e));
        return SND_ERR_HIP;
    }
    return SND_OK;
}

snd_status snd_merge_candidates(int64_t n, const snd_band_candidate *h_in, double dm_tol, double t_tol_ms,
                                snd_band_candidate *h_out, int64_t *h_count)
{
    if (n < 0 || (n > 0 && (!h_in || !h_out)) || !h_count || !(dm_tol >= 0.0) || !(t_tol_ms >= 0.0))
        return fail(SND_ERR_INVALID, "n >= 0, non-null arrays and non-negative tolerances needed");
    std::vector<int64_t> order((size_t)n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
        const snd_band_candidate &x = h_in[a], &y = h_in[b];
        if (x.snr != y.snr) return x.snr > y.snr;
        if (x.dm != y.dm) return x.dm < y.dm;
        return x.t_ms < y.t_ms;
    });
    std::vector<snd_band_candidate> kept;
    for (int64_t i : order) {
        const snd_band_candidate &c = h_in[i];
        bool absorbed = false;
        for (const snd_band_candidate &q : kept)
            if (std::fabs(c.dm - q.dm) <= dm_tol && std::fabs(c.t_ms - q.t_ms) <= t_tol_ms) {
                absorbed = true;
                break;
            }
        if (!absorbed) kept.push_back(c);
    }
    std::stable_sort(kept.begin(), kept.end(), [](const snd_band_candidate &x, const snd_band_candidate &y) {
        return x.t_ms != y.t_ms ? x.t_ms < y.t_ms : x.dm < y.dm;
    });
    for (size_t i = 0; i < kept.size(); ++i) h_out[i] = kept[i];
    *h_count = (int64_t)kept.size();
    return SND_OK;
}

}  // extern "C"
