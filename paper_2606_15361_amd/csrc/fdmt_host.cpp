// FDMT with the no-smear initialisation, host side (Methods, "Classical dedispersion
// algorithms": FDMT merges adjacent sub-bands iteratively, splitting each sub-band's delay by
// the f^-2 law; the no-smear initialisation takes every initial delay row of a channel to be
// the channel itself).  A comparison baseline for the SND tree on the same GPU.
//
// Channels are frequency intervals of width chan_bw around their centres, in descending order
// (channel 0 highest).  At iteration i sub-band s covers channels [s 2^i, (s + 1) 2^i); its
// reference is its upper edge, and its sweep span is r(S) = f_lo(S)^-2 - f_hi(S)^-2.  With
// D = the whole band's sweep at dm_max in samples, rounded up, sub-band S holds the delays
// delta = 0 .. n(S) - 1, n(S) = ceil(D r(S) / r(band)) + 1 (at most D + 1).  Merging S = U + L
// (U the upper half) gives, for each delta of S:
//   delta_U = round_half_even(delta * (f_mid^-2 - f_hi(S)^-2) / r(S)), clamped to n(U) - 1,
//   delta_L = min(delta - delta_U, n(L) - 1),
//   P_S[delta](t) = P_U[delta_U](t) + P_L[delta_L](t + delta_U),
// rows zero-extended past nsamp.  With the no-smear initialisation the channel rows P_c[delta]
// are all x_c, so the first merge reads the input directly.  The root rows are the output:
// row delta is the band sweep of delta samples, DM = delta * dm_per_delay.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "snd_internal.h"

namespace snd {
int launch_fdmt_merge(const float *src, int64_t src_pitch, float *dst, int64_t dst_pitch, const int32_t *tab,
                      int64_t rows, int64_t n, void *stream);
}

struct snd_fdmt_s {
    int32_t nchan = 0, iters = 0;
    int64_t nsamp = 0, n_delays = 0, max_rows = 0;
    double dm_per_delay = 0.0;
    std::vector<int64_t> rows;      // [iters]: rows of each iteration's output
    std::vector<int64_t> tab_off;   // [iters]: int32 offset of each iteration's table
    std::vector<int32_t> tables;    // per output row: source row U, source row L, delta_U, 0
    const int32_t *d_tables = nullptr;
};

namespace {

snd_status fail(snd_status s, const char *msg)
{
    snd::set_error(msg);
    return s;
}

double inv2(double f) { return 1.0 / (f * f); }

}  // namespace

extern "C" {

snd_status snd_fdmt_create(int32_t nchan, const double *freq_mhz, double chan_bw_mhz, double tsamp_s, double dm_max,
                           int64_t nsamp, snd_fdmt *out)
{
    if (!out || !freq_mhz) return fail(SND_ERR_INVALID, "null pointer");
    *out = nullptr;
    if (nchan < 2 || (nchan & (nchan - 1)) != 0 || nchan > (1 << 16))
        return fail(SND_ERR_INVALID, "nchan must be a power of two in 2..65536");
    if (!(chan_bw_mhz > 0.0) || !(tsamp_s > 0.0) || !(dm_max >= 0.0) || !std::isfinite(dm_max) || nsamp < 1 ||
        nsamp > 0x7fffffffLL)
        return fail(SND_ERR_INVALID, "chan_bw_mhz > 0, tsamp_s > 0, finite dm_max >= 0 and 1 <= nsamp < 2^31 needed");
    for (int32_t c = 0; c < nchan; ++c) {
        if (!(freq_mhz[c] - 0.5 * chan_bw_mhz > 0.0) || !std::isfinite(freq_mhz[c]))
            return fail(SND_ERR_INVALID, "channel lower edges must be > 0");
        if (c > 0 && !(freq_mhz[c] < freq_mhz[c - 1])) return fail(SND_ERR_INVALID, "frequencies must descend");
    }
    auto fhi = [&](int32_t c) { return freq_mhz[c] + 0.5 * chan_bw_mhz; };
    auto flo = [&](int32_t c) { return freq_mhz[c] - 0.5 * chan_bw_mhz; };
    const double r_band = inv2(flo(nchan - 1)) - inv2(fhi(0));
    const double dt_ms = tsamp_s * 1e3;
    const double dmax = std::ceil(snd::kDM * dm_max * r_band / dt_ms);
    if (dmax >= (double)nsamp) return fail(SND_ERR_INVALID, "the band sweep at dm_max does not fit nsamp");
    snd_fdmt_s *p = new (std::nothrow) snd_fdmt_s;
    if (!p) return fail(SND_ERR_NOMEM, "host allocation");
    p->nchan = nchan;
    p->nsamp = nsamp;
    const int64_t D = (int64_t)dmax;
    p->n_delays = D + 1;
    p->dm_per_delay = dt_ms / (snd::kDM * r_band);
    // delays held by sub-band [c0, c0 + w)
    auto nd = [&](int32_t c0, int32_t w) -> int64_t {
        const double r = inv2(flo(c0 + w - 1)) - inv2(fhi(c0));
        int64_t v = (int64_t)std::ceil((double)D * r / r_band) + 1;
        return v > D + 1 ? D + 1 : v;
    };
    // row index of (sub-band s, delta) within its iteration's rows: prefix sums of n(S)
    std::vector<int64_t> prev_base;  // iteration i - 1: first row of each sub-band
    std::vector<int64_t> prev_n;
    for (int32_t w = 2; w <= nchan; w *= 2) {
        const int32_t nsb = nchan / w, h = w / 2;
        std::vector<int64_t> base((size_t)nsb), cnt((size_t)nsb);
        int64_t rows = 0;
        for (int32_t s = 0; s < nsb; ++s) {
            base[(size_t)s] = rows;
            cnt[(size_t)s] = nd(s * w, w);
            rows += cnt[(size_t)s];
        }
        if (rows > 0x7fffffffLL) {
            delete p;
            return fail(SND_ERR_INVALID, "too many delay rows");
        }
        p->tab_off.push_back((int64_t)p->tables.size());
        p->rows.push_back(rows);
        p->max_rows = rows > p->max_rows ? rows : p->max_rows;
        for (int32_t s = 0; s < nsb; ++s) {
            const int32_t cu = s * w, cl = s * w + h;  // first channels of the upper and lower halves
            const double f_hi = fhi(cu), f_mid = flo(cu + h - 1), f_lo = flo(cl + h - 1);
            const double rs = inv2(f_lo) - inv2(f_hi), ru = inv2(f_mid) - inv2(f_hi);
            // delays held by the halves (single channels in the first merge: their own sweep)
            const int64_t nu = w == 2 ? nd(cu, 1) : prev_n[(size_t)(2 * s)];
            const int64_t nl = w == 2 ? nd(cl, 1) : prev_n[(size_t)(2 * s + 1)];
            for (int64_t d = 0; d < cnt[(size_t)s]; ++d) {
                int64_t du = (int64_t)std::nearbyint((double)d * ru / rs);
                if (du > nu - 1) du = nu - 1;
                int64_t dl = d - du;
                if (dl > nl - 1) dl = nl - 1;
                // first iteration: the sources are input channel rows (every delay row of a
                // channel is the channel itself); later ones: rows of the previous iteration
                const int64_t ru_row = w == 2 ? cu : prev_base[(size_t)(2 * s)] + du;
                const int64_t rl_row = w == 2 ? cl : prev_base[(size_t)(2 * s + 1)] + dl;
                p->tables.insert(p->tables.end(), {(int32_t)ru_row, (int32_t)rl_row, (int32_t)du, 0});
            }
        }
        prev_base = std::move(base);
        prev_n = std::move(cnt);
        ++p->iters;
    }
    *out = p;
    return SND_OK;
}

snd_status snd_fdmt_query(snd_fdmt p, int64_t *n_delays, int64_t *n_out, int64_t *table_bytes, int64_t *workspace_bytes,
                          double *dm_per_delay)
{
    if (!p) return fail(SND_ERR_INVALID, "null handle");
    if (n_delays) *n_delays = p->n_delays;
    if (n_out) *n_out = p->nsamp - (p->n_delays - 1);
    if (table_bytes) *table_bytes = (int64_t)(p->tables.size() * sizeof(int32_t));
    // two ping-pong buffers of the largest iteration (the last iteration writes the output)
    if (workspace_bytes) *workspace_bytes = 2 * p->max_rows * p->nsamp * (int64_t)sizeof(float);
    if (dm_per_delay) *dm_per_delay = p->dm_per_delay;
    return SND_OK;
}

snd_status snd_fdmt_upload(snd_fdmt p, void *d_tables, int64_t bytes, void *stream)
{
    if (!p || !d_tables) return fail(SND_ERR_INVALID, "null pointer");
    const int64_t need = (int64_t)(p->tables.size() * sizeof(int32_t));
    if (bytes < need) return fail(SND_ERR_NOMEM, "table buffer too small");
    if (hipMemcpyAsync(d_tables, p->tables.data(), (size_t)need, hipMemcpyHostToDevice, (hipStream_t)stream) != hipSuccess ||
        hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
        return fail(SND_ERR_HIP, "table upload");
    p->d_tables = static_cast<const int32_t *>(d_tables);
    return SND_OK;
}

snd_status snd_fdmt_execute(snd_fdmt p, const float *d_in, int64_t in_pitch, float *d_out, int64_t out_pitch,
                            void *d_ws, int64_t ws_bytes, void *stream)
{
    if (!p || !d_in || !d_out || !d_ws) return fail(SND_ERR_INVALID, "null pointer");
    if (!p->d_tables) return fail(SND_ERR_STATE, "tables not uploaded");
    if (in_pitch < p->nsamp || out_pitch < p->nsamp) return fail(SND_ERR_INVALID, "pitches must be >= nsamp");
    if (ws_bytes < 2 * p->max_rows * p->nsamp * (int64_t)sizeof(float)) return fail(SND_ERR_NOMEM, "workspace too small");
    float *buf[2] = {static_cast<float *>(d_ws), static_cast<float *>(d_ws) + p->max_rows * p->nsamp};
    const float *src = d_in;
    int64_t sp = in_pitch;
    for (int32_t i = 0; i < p->iters; ++i) {
        const bool last = i == p->iters - 1;
        float *dst = last ? d_out : buf[i & 1];
        const int64_t dp = last ? out_pitch : p->nsamp;
        int e = snd::launch_fdmt_merge(src, sp, dst, dp, p->d_tables + p->tab_off[(size_t)i], p->rows[(size_t)i],
                                       p->nsamp, stream);
        if (e) {
            snd::set_error("FDMT merge launch: " + std::string(hipGetErrorString((hipError_t)e)));
            return SND_ERR_HIP;
        }
        src = dst;
        sp = dp;
    }
    return SND_OK;
}

snd_status snd_fdmt_destroy(snd_fdmt p)
{
    delete p;
    return SND_OK;
}

}  // extern "C"
