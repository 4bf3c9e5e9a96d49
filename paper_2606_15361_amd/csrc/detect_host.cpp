// Matched-filter / candidate entry points: argument checks, kernel launches, and the host part
// of candidate detection (Methods, "Candidate detection"): binary closing and 8-connected
// labelling over the sparse set of thresholded cells returned by the device.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "snd_detect.h"
#include "snd_internal.h"

namespace snd {
void set_error(const std::string &msg);
}

namespace {

constexpr int64_t kHeader = 256;

int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

snd_status check_desc(const snd::PlanImpl &P, const snd_detect_desc *d)
{
    if (!d || !d->widths) { snd::set_error("null detect descriptor or widths"); return SND_ERR_INVALID; }
    if (d->nwidths < 1 || d->nwidths > SND_MAX_WIDTHS) { snd::set_error("nwidths must be 1..32"); return SND_ERR_INVALID; }
    for (int i = 0; i < d->nwidths; ++i) {
        if (d->widths[i] < 1 || d->widths[i] > SND_MAX_WIDTH || (i > 0 && d->widths[i] <= d->widths[i - 1])) {
            snd::set_error("widths must be strictly increasing in 1..1024");
            return SND_ERR_INVALID;
        }
    }
    if (!(d->threshold > 0.0) || !(d->sigma_min >= 0.0) || d->closing_radius < 0 || d->closing_radius > 64 ||
        d->n_min < 1 || d->max_pixels < 1) {
        snd::set_error("threshold must be > 0, sigma_min >= 0, 0 <= closing_radius <= 64, n_min >= 1, max_pixels >= 1");
        return SND_ERR_INVALID;
    }
    if (d->label_on_device != 0 && d->label_on_device != 1) {
        snd::set_error("label_on_device must be 0 or 1");
        return SND_ERR_INVALID;
    }
    if (d->label_on_device && d->max_pixels > 0x7fffffffLL) {
        snd::set_error("labelling on the device takes at most 2^31 - 1 cells");
        return SND_ERR_INVALID;
    }
    if (d->sigma_estimator != 0 && d->sigma_estimator != 1) {
        snd::set_error("sigma_estimator must be 0 (standard deviation) or 1 (median absolute deviation)");
        return SND_ERR_INVALID;
    }
    if (d->n_base_widths < 0 || d->n_base_widths > d->nwidths || !(d->width_alpha >= 0.0) ||
        !std::isfinite(d->width_alpha)) {
        snd::set_error("n_base_widths must be in 0..nwidths and width_alpha finite and >= 0");
        return SND_ERR_INVALID;
    }
    if (P.ndm > 65535) { snd::set_error("detect supports at most 65535 DM rows"); return SND_ERR_UNSUPPORTED; }
    if (P.n_out > 0x7fffffffLL) { snd::set_error("rows too long for detect"); return SND_ERR_UNSUPPORTED; }
    return SND_OK;
}

// Workspace: header (cell counter) | row statistics | thresholded cells | per-row width counts
int64_t pixels_offset(const snd::PlanImpl &P) { return kHeader + round_up((int64_t)P.ndm * 16, 256); }

int64_t row_nw_offset(const snd::PlanImpl &P, const snd_detect_desc *d)
{
    return round_up(pixels_offset(P) + d->max_pixels * (int64_t)sizeof(snd::Pixel), 256);
}

int64_t host_workspace_end(const snd::PlanImpl &P, const snd_detect_desc *d)
{
    return row_nw_offset(P, d) + round_up((int64_t)P.ndm * 4, 256);
}

// Labelling on the device: after the host part's regions, two bitmasks of the plane padded by
// 2r, then per-row and per-run tables (runs up to max_pixels), then the candidate list.
struct LabelLayout {
    int64_t rows = 0, wd = 0, mask_a = 0, mask_b = 0, nruns = 0, run_ptr = 0, rs = 0, re = 0, rk = 0, parent = 0,
            npix = 0, smax = 0, pkey = 0, pwidx = 0, ncand = 0, cand = 0, cand_npix = 0, end = 0;
};

LabelLayout label_layout(const snd::PlanImpl &P, const snd_detect_desc *d)
{
    LabelLayout L;
    const int64_t r = d->closing_radius, m = d->max_pixels;
    L.rows = P.ndm + 4 * r;
    L.wd = (P.n_out + 4 * r + 63) / 64;
    int64_t o = round_up(host_workspace_end(P, d), 256);
    auto take = [&](int64_t bytes) {
        const int64_t at = o;
        o = round_up(o + bytes, 256);
        return at;
    };
    L.mask_a = take(L.rows * L.wd * 8);
    L.mask_b = take(L.rows * L.wd * 8);
    L.nruns = take((int64_t)P.ndm * 4);
    L.run_ptr = take(((int64_t)P.ndm + 1) * 4);
    L.rs = take(m * 4);
    L.re = take(m * 4);
    L.rk = take(m * 4);
    L.parent = take(m * 4);
    L.npix = take(m * 8);
    L.smax = take(m * 8);
    L.pkey = take(m * 8);
    L.pwidx = take(m * 4);
    L.ncand = take(8);
    L.cand = take(m * (int64_t)sizeof(snd::Pixel));
    L.cand_npix = take(m * 8);
    L.end = o;
    return L;
}

int64_t workspace_bytes_for(const snd::PlanImpl &P, const snd_detect_desc *d)
{
    return d->label_on_device ? label_layout(P, d).end : host_workspace_end(P, d);
}

// DM-scaled width set: the number of leading widths each row uses (Methods, "Matched
// filtering", W(d_k)), from the unrounded sweep across the band at d_k.
void row_width_counts(const snd::PlanImpl &P, const snd_detect_desc *d, std::vector<int32_t> &nw)
{
    nw.assign((size_t)P.ndm, d->nwidths);
    if (d->n_base_widths <= 0) return;
    double fmin = P.freq[0];
    for (double f : P.freq) fmin = std::min(fmin, f);
    const double tms = P.desc.tsamp_s * 1e3;
    for (int k = 0; k < P.ndm; ++k) {
        double x = snd::kDM * P.dm[(size_t)k];
        x = x * (1.0 / (fmin * fmin) - 1.0 / (P.fref * P.fref));
        x = x / tms;
        const double lim = d->width_alpha * x;
        int32_t n = d->n_base_widths;
        for (int i = d->n_base_widths; i < d->nwidths; ++i)
            if ((double)d->widths[i] <= lim) n = i + 1;
        nw[(size_t)k] = n;
    }
}

// Per-row width counts into the workspace (only for a DM-scaled set); the pageable source is
// consumed when the copy call returns.
snd_status upload_row_nw(const snd::PlanImpl &P, const snd_detect_desc *d, uint8_t *ws, snd::SnrArgs &a,
                         hipStream_t st)
{
    a.row_nw = nullptr;
    if (d->n_base_widths <= 0) return SND_OK;
    std::vector<int32_t> nw;
    row_width_counts(P, d, nw);
    int32_t *dst = reinterpret_cast<int32_t *>(ws + row_nw_offset(P, d));
    hipError_t e = hipMemcpyAsync(dst, nw.data(), nw.size() * sizeof(int32_t), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) {
        snd::set_error(std::string("hipMemcpyAsync(row widths): ") + hipGetErrorString(e));
        return SND_ERR_HIP;
    }
    a.row_nw = dst;
    return SND_OK;
}

void fill_args(const snd_detect_desc *d, snd::SnrArgs &a)
{
    std::memset(&a, 0, sizeof(a));
    a.nw = d->nwidths;
    for (int i = 0; i < d->nwidths; ++i) {
        a.w[i] = d->widths[i];
        a.sqrtw[i] = std::sqrt((double)d->widths[i]);
    }
    a.threshold = d->threshold;
}

// ---- host closing + labelling on the sparse thresholded cells ----
// The thresholded cells are turned into runs of consecutive samples per DM row.  The square
// closing is separable: dilation along time (runs widened by r and merged), dilation along
// DM (union of the 2r+1 neighbouring rows), erosion along DM (intersection of the 2r+1
// neighbouring rows) and erosion along time (runs narrowed by r).  All of it works on runs, so
// the cost grows with the number of runs, not with the area of the islands.  Rows outside the
// plane are empty, which is the zero-extended plane.
struct Run {
    int64_t a, b;  // inclusive
};
using Rows = std::vector<std::vector<Run>>;

void merge_sorted(std::vector<Run> &v)
{
    if (v.empty()) return;
    size_t w = 0;
    for (size_t i = 1; i < v.size(); ++i) {
        if (v[i].a <= v[w].b + 1) v[w].b = std::max(v[w].b, v[i].b);
        else v[++w] = v[i];
    }
    v.resize(w + 1);
}

void intersect(const std::vector<Run> &x, const std::vector<Run> &y, std::vector<Run> &out)
{
    out.clear();
    size_t i = 0, j = 0;
    while (i < x.size() && j < y.size()) {
        const int64_t a = std::max(x[i].a, y[j].a), b = std::min(x[i].b, y[j].b);
        if (a <= b) out.push_back({a, b});
        if (x[i].b < y[j].b) ++i;
        else ++j;
    }
}

struct UF {
    std::vector<int32_t> p;
    explicit UF(size_t n) : p(n) { std::iota(p.begin(), p.end(), 0); }
    int32_t f(int32_t x)
    {
        while (p[x] != x) { p[x] = p[p[x]]; x = p[x]; }
        return x;
    }
    void u(int32_t a, int32_t b)
    {
        a = f(a); b = f(b);
        if (a != b) p[std::max(a, b)] = std::min(a, b);
    }
};

// Page-locked host memory for read-backs; null when it cannot be had (pageable copy then).
// The last buffer is deliberately kept until the process ends: freeing it from a thread-exit
// destructor could run after the HIP runtime has shut down.
struct PinnedBuffer {
    void *p = nullptr;
    size_t n = 0;
    void *get(size_t bytes)
    {
        if (bytes <= n) return p;
        const size_t want = std::max(bytes, n * 2);
        if (p) (void)hipHostFree(p);
        p = nullptr;
        n = 0;
        if (hipHostMalloc(&p, want, hipHostMallocDefault) != hipSuccess) {
            p = nullptr;
            return nullptr;
        }
        n = want;
        return p;
    }
};

snd_status candidates_from_pixels(std::vector<snd::Pixel> &px, const snd::PlanImpl &P, const snd_detect_desc *d,
                                  std::vector<snd_candidate> &out)
{
    out.clear();
    if (px.empty()) return SND_OK;
    {  // (k, t) order: a counting sort by row, then t within a row (each workgroup's cells arrive
       // as one segment of one row in increasing t, so rows are short runs of sorted segments)
        int32_t k0 = px[0].k, k1 = px[0].k;
        for (const snd::Pixel &q : px) { k0 = std::min(k0, q.k); k1 = std::max(k1, q.k); }
        std::vector<int64_t> at((size_t)(k1 - k0) + 2, 0);
        for (const snd::Pixel &q : px) ++at[(size_t)(q.k - k0) + 1];
        for (size_t i = 1; i < at.size(); ++i) at[i] += at[i - 1];
        std::vector<snd::Pixel> sorted(px.size());
        std::vector<int64_t> fill(at.begin(), at.end() - 1);
        for (const snd::Pixel &q : px) sorted[(size_t)fill[(size_t)(q.k - k0)]++] = q;
        auto by_t = [](const snd::Pixel &a, const snd::Pixel &b) { return a.t < b.t; };
        for (size_t r = 0; r + 1 < at.size(); ++r) {
            auto b = sorted.begin() + at[r], e = sorted.begin() + at[r + 1];
            if (!std::is_sorted(b, e, by_t)) std::sort(b, e, by_t);
        }
        px.swap(sorted);
    }
    const int64_t r = d->closing_radius;
    const int64_t kmin = px.front().k, kmax = px.back().k;
    // rows are indexed relative to K0 = kmin - 2r so every dilated/eroded row has a slot
    const int64_t K0 = kmin - 2 * r, NR = kmax - kmin + 4 * r + 1;
    Rows dt((size_t)NR);  // thresholded runs widened along time
    for (size_t i = 0; i < px.size();) {
        size_t j = i;
        const int64_t k = px[i].k;
        std::vector<Run> &row = dt[(size_t)(k - K0)];
        while (j < px.size() && px[j].k == k) {
            int64_t a = px[j].t, b = a;
            while (j + 1 < px.size() && px[j + 1].k == k && px[j + 1].t == b + 1) { ++j; ++b; }
            row.push_back({a - r, b + r});
            ++j;
        }
        merge_sorted(row);
        i = j;
    }
    Rows dil((size_t)NR);  // dilation along DM
    for (int64_t k = 0; k < NR; ++k) {
        std::vector<Run> &row = dil[(size_t)k];
        for (int64_t q = std::max<int64_t>(0, k - r); q <= std::min<int64_t>(NR - 1, k + r); ++q)
            row.insert(row.end(), dt[(size_t)q].begin(), dt[(size_t)q].end());
        std::sort(row.begin(), row.end(), [](const Run &x, const Run &y) { return x.a < y.a; });
        merge_sorted(row);
    }
    dt.clear();
    Rows cl((size_t)NR);  // erosion along DM, then along time
    std::vector<Run> tmp;
    for (int64_t k = 0; k < NR; ++k) {
        if (k - r < 0 || k + r >= NR) continue;  // a neighbouring row is outside the dilation: empty
        std::vector<Run> cur = dil[(size_t)(k - r)];
        for (int64_t q = k - r + 1; q <= k + r && !cur.empty(); ++q) {
            intersect(cur, dil[(size_t)q], tmp);
            cur.swap(tmp);
        }
        for (const Run &x : cur)
            if (x.a + r <= x.b - r) cl[(size_t)k].push_back({x.a + r, x.b - r});
    }
    dil.clear();
    // 8-connected labelling of the closed runs
    std::vector<int64_t> first((size_t)NR + 1, 0);
    for (int64_t k = 0; k < NR; ++k) first[(size_t)k + 1] = first[(size_t)k] + (int64_t)cl[(size_t)k].size();
    UF uf((size_t)first[(size_t)NR]);
    for (int64_t k = 0; k + 1 < NR; ++k) {
        const std::vector<Run> &x = cl[(size_t)k], &y = cl[(size_t)k + 1];
        size_t i = 0, j = 0;
        while (i < x.size() && j < y.size()) {
            if (y[j].a <= x[i].b + 1 && x[i].a <= y[j].b + 1)
                uf.u((int32_t)(first[(size_t)k] + (int64_t)i), (int32_t)(first[(size_t)k + 1] + (int64_t)j));
            if (x[i].b < y[j].b) ++i;
            else ++j;
        }
    }
    const size_t nruns = (size_t)first[(size_t)NR];
    std::vector<int64_t> npix(nruns, 0);
    std::vector<int32_t> peak(nruns, -1);
    for (int64_t k = 0; k < NR; ++k)
        for (size_t i = 0; i < cl[(size_t)k].size(); ++i) {
            const Run &x = cl[(size_t)k][i];
            npix[(size_t)uf.f((int32_t)(first[(size_t)k] + (int64_t)i))] += x.b - x.a + 1;
        }
    for (size_t pi = 0; pi < px.size(); ++pi) {  // thresholded cells in (k, t) order
        const snd::Pixel &q = px[pi];
        const std::vector<Run> &row = cl[(size_t)(q.k - K0)];
        auto it = std::upper_bound(row.begin(), row.end(), (int64_t)q.t, [](int64_t v, const Run &x) { return v < x.a; });
        if (it == row.begin()) continue;  // cannot happen: closing keeps every thresholded cell
        --it;
        if (q.t > it->b) continue;
        const int32_t c = uf.f((int32_t)(first[(size_t)(q.k - K0)] + (it - row.begin())));
        if (peak[(size_t)c] < 0) { peak[(size_t)c] = (int32_t)pi; continue; }
        const snd::Pixel &b = px[(size_t)peak[(size_t)c]];
        if (q.snr > b.snr) peak[(size_t)c] = (int32_t)pi;  // ties keep the earlier (k, t) cell
    }
    for (size_t c = 0; c < nruns; ++c) {
        if (uf.f((int32_t)c) != (int32_t)c || peak[c] < 0 || npix[c] < d->n_min) continue;
        const snd::Pixel &q = px[(size_t)peak[c]];
        snd_candidate cand{};
        cand.dm_index = q.k;
        cand.width = d->widths[q.widx];
        cand.t = q.t;
        cand.snr = q.snr;
        cand.dm = P.dm[q.k];
        cand.npix = npix[c];
        out.push_back(cand);
    }
    std::sort(out.begin(), out.end(), [](const snd_candidate &a, const snd_candidate &b) {
        return a.dm_index != b.dm_index ? a.dm_index < b.dm_index : a.t < b.t;
    });
    return SND_OK;
}

// Closing, labelling, island sizes and peaks on the device; only the candidates come back.
snd_status label_device(const snd::PlanImpl &P, const snd_detect_desc *d, uint8_t *ws, const snd::SnrArgs &sa,
                        snd_candidate *h_out, int64_t cap, int64_t *h_count, hipStream_t st)
{
    const LabelLayout L = label_layout(P, d);
    snd::LabelArgs a{};
    a.pixels = sa.pixels;
    a.count = sa.counter;
    a.max_pixels = d->max_pixels;
    a.ndm = P.ndm;
    a.n = P.n_out;
    a.r = d->closing_radius;
    a.rows = L.rows;
    a.wd = L.wd;
    a.mask_a = reinterpret_cast<uint64_t *>(ws + L.mask_a);
    a.mask_b = reinterpret_cast<uint64_t *>(ws + L.mask_b);
    a.nruns = reinterpret_cast<int32_t *>(ws + L.nruns);
    a.run_ptr = reinterpret_cast<int32_t *>(ws + L.run_ptr);
    a.rs = reinterpret_cast<int32_t *>(ws + L.rs);
    a.re = reinterpret_cast<int32_t *>(ws + L.re);
    a.rk = reinterpret_cast<int32_t *>(ws + L.rk);
    a.parent = reinterpret_cast<int32_t *>(ws + L.parent);
    a.npix = reinterpret_cast<unsigned long long *>(ws + L.npix);
    a.smax = reinterpret_cast<unsigned long long *>(ws + L.smax);
    a.pkey = reinterpret_cast<unsigned long long *>(ws + L.pkey);
    a.pwidx = reinterpret_cast<int32_t *>(ws + L.pwidx);
    a.max_runs = d->max_pixels;
    a.n_min = d->n_min;
    a.ncand = reinterpret_cast<unsigned int *>(ws + L.ncand);
    a.cand = reinterpret_cast<snd::Pixel *>(ws + L.cand);
    a.cand_npix = reinterpret_cast<int64_t *>(ws + L.cand_npix);
    *h_count = 0;
    auto hip_fail = [](hipError_t e, const char *what) {
        snd::set_error(std::string(what) + ": " + hipGetErrorString(e));
        return SND_ERR_HIP;
    };
    int e = snd::launch_label(a, st);
    if (e) return hip_fail((hipError_t)e, "labelling launch");
    int32_t total = 0;
    hipError_t he = hipMemcpyAsync(&total, a.run_ptr + P.ndm, sizeof(total), hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    if (he != hipSuccess) return hip_fail(he, "labelling read-back");
    if ((int64_t)total > a.max_runs) {  // the tables below hold max_pixels runs
        snd::set_error("the closed mask has more runs than max_pixels");
        return SND_ERR_CAPACITY;
    }
    e = snd::launch_label_finish(a, st);
    if (e) return hip_fail((hipError_t)e, "labelling launch");
    unsigned int nc = 0;
    he = hipMemcpyAsync(&nc, a.ncand, sizeof(nc), hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    if (he != hipSuccess) return hip_fail(he, "labelling read-back");
    std::vector<snd::Pixel> c(nc);
    std::vector<int64_t> np(nc);
    if (nc) {
        he = hipMemcpyAsync(c.data(), a.cand, sizeof(snd::Pixel) * nc, hipMemcpyDeviceToHost, st);
        if (he == hipSuccess) he = hipMemcpyAsync(np.data(), a.cand_npix, sizeof(int64_t) * nc, hipMemcpyDeviceToHost, st);
        if (he == hipSuccess) he = hipStreamSynchronize(st);
        if (he != hipSuccess) return hip_fail(he, "labelling read-back");
    }
    std::vector<snd_candidate> out(nc);
    for (unsigned int i = 0; i < nc; ++i) {
        snd_candidate &x = out[i];
        x = snd_candidate{};
        x.dm_index = c[i].k;
        x.width = d->widths[c[i].widx];
        x.t = c[i].t;
        x.snr = c[i].snr;
        x.dm = P.dm[(size_t)c[i].k];
        x.npix = np[i];
    }
    std::sort(out.begin(), out.end(), [](const snd_candidate &x, const snd_candidate &y) {
        return x.dm_index != y.dm_index ? x.dm_index < y.dm_index : x.t < y.t;
    });
    *h_count = (int64_t)out.size();
    for (int64_t i = 0; i < cap && i < (int64_t)out.size(); ++i) h_out[i] = out[(size_t)i];
    return SND_OK;
}

}  // namespace

extern "C" {

snd_status snd_detect_workspace(snd_plan plan, const snd_detect_desc *desc, int64_t *bytes)
{
    if (!plan || !bytes) { snd::set_error("null plan or output"); return SND_ERR_INVALID; }
    snd_status s = check_desc(plan->impl, desc);
    if (s != SND_OK) return s;
    *bytes = workspace_bytes_for(plan->impl, desc);
    return SND_OK;
}

snd_status snd_snr_plane(snd_plan plan, const void *d_plane, int64_t plane_pitch, const snd_detect_desc *desc,
                         float *d_snr, int64_t snr_pitch, int8_t *d_widx, int64_t widx_pitch, void *d_workspace,
                         int64_t workspace_bytes, void *stream)
{
    if (!plan || !d_plane || !d_snr || !d_widx || !d_workspace) { snd::set_error("null argument"); return SND_ERR_INVALID; }
    const auto &P = plan->impl;
    snd_status s = check_desc(P, desc);
    if (s != SND_OK) return s;
    if (workspace_bytes < workspace_bytes_for(P, desc) || ((uintptr_t)d_workspace & 255u)) {
        snd::set_error("detect workspace too small or not 256-byte aligned");
        return SND_ERR_NOMEM;
    }
    if (plane_pitch < P.n_out || snr_pitch < P.n_out || widx_pitch < P.n_out) { snd::set_error("pitch smaller than n_out"); return SND_ERR_INVALID; }
    snd::SnrArgs a;
    fill_args(desc, a);
    a.snr = d_snr;
    a.snr_pitch = snr_pitch;
    a.widx = d_widx;
    a.widx_pitch = widx_pitch;
    double *stats = reinterpret_cast<double *>(static_cast<uint8_t *>(d_workspace) + kHeader);
    s = upload_row_nw(P, desc, static_cast<uint8_t *>(d_workspace), a, (hipStream_t)stream);
    if (s != SND_OK) return s;
    int e = snd::launch_detect(P.out_dtype, d_plane, plane_pitch, P.ndm, P.n_out, desc->sigma_min, desc->sigma_estimator,
                                 stats, a, stream);
    if (e) { snd::set_error(std::string("detect launch: ") + hipGetErrorString((hipError_t)e)); return SND_ERR_HIP; }
    return SND_OK;
}

snd_status snd_detect_launch(snd_plan plan, const void *d_plane, int64_t plane_pitch, const snd_detect_desc *desc,
                             void *d_workspace, int64_t workspace_bytes, void *h_stage, int64_t stage_bytes,
                             void *stream)
{
    static_assert(sizeof(snd::Pixel) == 24, "staged cell size");
    if (!plan || !d_plane || !d_workspace || !h_stage) { snd::set_error("null argument"); return SND_ERR_INVALID; }
    if (stage_bytes < SND_DETECT_STAGE_HEADER) { snd::set_error("stage buffer smaller than its header"); return SND_ERR_INVALID; }
    const auto &P = plan->impl;
    snd_status s = check_desc(P, desc);
    if (s != SND_OK) return s;
    if (workspace_bytes < workspace_bytes_for(P, desc) || ((uintptr_t)d_workspace & 255u)) {
        snd::set_error("detect workspace too small or not 256-byte aligned");
        return SND_ERR_NOMEM;
    }
    if (plane_pitch < P.n_out) { snd::set_error("plane pitch smaller than n_out"); return SND_ERR_INVALID; }
    uint8_t *ws = static_cast<uint8_t *>(d_workspace);
    snd::SnrArgs a;
    fill_args(desc, a);
    a.counter = reinterpret_cast<unsigned int *>(ws);
    a.pixels = reinterpret_cast<snd::Pixel *>(ws + pixels_offset(P));
    a.max_pixels = desc->max_pixels;
    double *stats = reinterpret_cast<double *>(ws + kHeader);
    hipStream_t st = (hipStream_t)stream;
    s = upload_row_nw(P, desc, ws, a, st);
    if (s != SND_OK) return s;
    int e = snd::launch_detect(P.out_dtype, d_plane, plane_pitch, P.ndm, P.n_out, desc->sigma_min, desc->sigma_estimator,
                                 stats, a, stream);
    if (e) { snd::set_error(std::string("detect launch: ") + hipGetErrorString((hipError_t)e)); return SND_ERR_HIP; }
    uint8_t *hs = static_cast<uint8_t *>(h_stage);
    hipError_t he = hipMemcpyAsync(hs, a.counter, sizeof(unsigned int), hipMemcpyDeviceToHost, st);
    const int64_t ncells = std::min<int64_t>(SND_DETECT_STAGE_CELLS(stage_bytes), desc->max_pixels);
    if (he == hipSuccess && ncells > 0)
        he = hipMemcpyAsync(hs + SND_DETECT_STAGE_HEADER, a.pixels, (size_t)ncells * sizeof(snd::Pixel),
                            hipMemcpyDeviceToHost, st);
    if (he != hipSuccess) { snd::set_error(std::string("detect read-back: ") + hipGetErrorString(he)); return SND_ERR_HIP; }
    return SND_OK;
}

snd_status snd_detect_collect(snd_plan plan, const snd_detect_desc *desc, const void *h_stage, int64_t stage_bytes,
                              snd_candidate *h_out, int64_t cap, int64_t *h_count, int64_t *h_npixels)
{
    if (!plan || !h_stage || !h_count || (cap > 0 && !h_out)) { snd::set_error("null argument"); return SND_ERR_INVALID; }
    if (stage_bytes < SND_DETECT_STAGE_HEADER) { snd::set_error("stage buffer smaller than its header"); return SND_ERR_INVALID; }
    const auto &P = plan->impl;
    snd_status s = check_desc(P, desc);
    if (s != SND_OK) return s;
    const uint8_t *hs = static_cast<const uint8_t *>(h_stage);
    unsigned int count = 0;
    std::memcpy(&count, hs, sizeof(count));
    if (h_npixels) *h_npixels = count;
    *h_count = 0;
    const int64_t ncells = std::min<int64_t>(SND_DETECT_STAGE_CELLS(stage_bytes), desc->max_pixels);
    if ((int64_t)count > desc->max_pixels || (int64_t)count > ncells) {
        snd::set_error("more thresholded cells than max_pixels or than the stage buffer holds");
        return SND_ERR_CAPACITY;
    }
    std::vector<snd::Pixel> px(count);
    if (count) std::memcpy(px.data(), hs + SND_DETECT_STAGE_HEADER, sizeof(snd::Pixel) * count);
    std::vector<snd_candidate> cands;
    s = candidates_from_pixels(px, P, desc, cands);
    if (s != SND_OK) return s;
    *h_count = (int64_t)cands.size();
    for (int64_t i = 0; i < cap && i < (int64_t)cands.size(); ++i) h_out[i] = cands[i];
    return SND_OK;
}

// ---- batched detection ----
// Beams in batch-row order: grouped by plane dtype (u8, u16, f32), the caller's order within a
// group; each group is one launch of each kernel.  Workspace: header (cell counter) | row
// statistics of every batch row | cells | per-row width counts | the beams' table.
struct BatchLayout {
    std::vector<int32_t> order;     // beam indices in batch-row order
    std::vector<int32_t> row_base;  // per beam (caller's index)
    int64_t rows = 0;
    int64_t stats = 0, pixels = 0, row_nw = 0, table = 0, end = 0;
};

static snd_status batch_layout(int32_t n, const snd_plan *plans, const snd_detect_desc *desc, BatchLayout &L)
{
    if (n < 1 || !plans) { snd::set_error("no beams"); return SND_ERR_INVALID; }
    for (int32_t i = 0; i < n; ++i) {
        if (!plans[i]) { snd::set_error("null plan"); return SND_ERR_INVALID; }
        const snd_status s = check_desc(plans[i]->impl, desc);
        if (s != SND_OK) return s;
    }
    if (desc->sigma_estimator != 0 || desc->label_on_device != 0) {
        snd::set_error("batched detection takes the standard-deviation sigma and host labelling");
        return SND_ERR_UNSUPPORTED;
    }
    L.row_base.assign((size_t)n, 0);
    L.order.clear();
    for (int dt : {SND_DT_U8, SND_DT_U16, SND_DT_F32})
        for (int32_t i = 0; i < n; ++i)
            if (plans[i]->impl.out_dtype == dt) {
                L.order.push_back(i);
                L.row_base[(size_t)i] = (int32_t)L.rows;
                L.rows += plans[i]->impl.ndm;
                if (L.rows > 0x7fffffffLL) { snd::set_error("too many rows in one batch"); return SND_ERR_UNSUPPORTED; }
            }
    if ((int32_t)L.order.size() != n) { snd::set_error("unsupported plane dtype"); return SND_ERR_UNSUPPORTED; }
    L.stats = kHeader;
    L.pixels = round_up(L.stats + L.rows * 16, 256);
    L.row_nw = round_up(L.pixels + desc->max_pixels * (int64_t)sizeof(snd::Pixel), 256);
    L.table = round_up(L.row_nw + L.rows * 4, 256);
    L.end = round_up(L.table + (int64_t)n * (int64_t)sizeof(snd::DetBeam), 256);
    return SND_OK;
}

extern "C" {

snd_status snd_detect_batch_workspace(int32_t n, const snd_plan *plans, const snd_detect_desc *desc, int64_t *bytes)
{
    if (!bytes) { snd::set_error("null argument"); return SND_ERR_INVALID; }
    BatchLayout L;
    const snd_status s = batch_layout(n, plans, desc, L);
    if (s != SND_OK) return s;
    *bytes = L.end;
    return SND_OK;
}

snd_status snd_detect_batch_launch(int32_t n, const snd_plan *plans, const void *const *d_planes, const int64_t *pitches,
                                   const snd_detect_desc *desc, void *d_workspace, int64_t workspace_bytes,
                                   void *h_stage, int64_t stage_bytes, void *stream)
{
    if (!d_planes || !pitches || !d_workspace || !h_stage) { snd::set_error("null argument"); return SND_ERR_INVALID; }
    if (stage_bytes < SND_DETECT_STAGE_HEADER) { snd::set_error("stage buffer smaller than its header"); return SND_ERR_INVALID; }
    BatchLayout L;
    snd_status s = batch_layout(n, plans, desc, L);
    if (s != SND_OK) return s;
    if (workspace_bytes < L.end || ((uintptr_t)d_workspace & 255u)) {
        snd::set_error("batched detect workspace too small or not 256-byte aligned");
        return SND_ERR_NOMEM;
    }
    for (int32_t i = 0; i < n; ++i)
        if (!d_planes[i] || pitches[i] < plans[i]->impl.n_out) {
            snd::set_error("null plane or plane pitch smaller than n_out");
            return SND_ERR_INVALID;
        }
    uint8_t *ws = static_cast<uint8_t *>(d_workspace);
    hipStream_t st = (hipStream_t)stream;
    // per-row width counts (DM-scaled set) and the beams' table, one copy each (the pageable
    // sources are consumed when the copy calls return)
    std::vector<int32_t> nw_all;
    std::vector<snd::DetBeam> table((size_t)n);
    const bool scaled = desc->n_base_widths > 0;
    if (scaled) nw_all.resize((size_t)L.rows);
    for (size_t j = 0; j < L.order.size(); ++j) {
        const int32_t i = L.order[j];
        const auto &P = plans[i]->impl;
        const int32_t base = L.row_base[(size_t)i];
        if (scaled) {
            std::vector<int32_t> nw;
            row_width_counts(P, desc, nw);
            std::copy(nw.begin(), nw.end(), nw_all.begin() + base);
        }
        snd::DetBeam &b = table[j];
        b.plane = d_planes[i];
        b.pitch = pitches[i];
        b.n = P.n_out;
        b.row_nw = scaled ? reinterpret_cast<const int32_t *>(ws + L.row_nw) + base : nullptr;
        b.row_base = base;
        b.ndm = P.ndm;
    }
    hipError_t he = hipSuccess;
    if (scaled) he = hipMemcpyAsync(ws + L.row_nw, nw_all.data(), nw_all.size() * 4, hipMemcpyHostToDevice, st);
    if (he == hipSuccess)
        he = hipMemcpyAsync(ws + L.table, table.data(), table.size() * sizeof(snd::DetBeam), hipMemcpyHostToDevice, st);
    if (he != hipSuccess) { snd::set_error(std::string("batched detect tables: ") + hipGetErrorString(he)); return SND_ERR_HIP; }
    snd::SnrArgs a;
    fill_args(desc, a);
    a.counter = reinterpret_cast<unsigned int *>(ws);
    a.pixels = reinterpret_cast<snd::Pixel *>(ws + L.pixels);
    a.max_pixels = desc->max_pixels;
    double *stats = reinterpret_cast<double *>(ws + L.stats);
    int e = snd::launch_zero_counter(a.counter, stream);
    // one launch per plane dtype over that group's rows
    for (size_t j0 = 0; j0 < L.order.size() && !e;) {
        const int dt = plans[L.order[j0]]->impl.out_dtype;
        size_t j1 = j0;
        int64_t nrows = 0, n_max = 0;
        while (j1 < L.order.size() && plans[L.order[j1]]->impl.out_dtype == dt) {
            nrows += plans[L.order[j1]]->impl.ndm;
            n_max = std::max<int64_t>(n_max, plans[L.order[j1]]->impl.n_out);
            ++j1;
        }
        a.beams = reinterpret_cast<const snd::DetBeam *>(ws + L.table) + j0;
        a.nbeams = (int32_t)(j1 - j0);
        a.row0 = table[j0].row_base;
        e = snd::launch_detect_batch(dt, (int)nrows, n_max, desc->sigma_min, stats, a, stream);
        j0 = j1;
    }
    if (e) { snd::set_error(std::string("batched detect launch: ") + hipGetErrorString((hipError_t)e)); return SND_ERR_HIP; }
    uint8_t *hs = static_cast<uint8_t *>(h_stage);
    he = hipMemcpyAsync(hs, a.counter, sizeof(unsigned int), hipMemcpyDeviceToHost, st);
    const int64_t ncells = std::min<int64_t>(SND_DETECT_STAGE_CELLS(stage_bytes), desc->max_pixels);
    if (he == hipSuccess && ncells > 0)
        he = hipMemcpyAsync(hs + SND_DETECT_STAGE_HEADER, a.pixels, (size_t)ncells * sizeof(snd::Pixel),
                            hipMemcpyDeviceToHost, st);
    if (he != hipSuccess) { snd::set_error(std::string("batched detect read-back: ") + hipGetErrorString(he)); return SND_ERR_HIP; }
    return SND_OK;
}

snd_status snd_detect_batch_collect(int32_t n, const snd_plan *plans, const snd_detect_desc *desc, const void *h_stage,
                                    int64_t stage_bytes, snd_candidate *h_out, int64_t cap_per_beam, int64_t *h_counts,
                                    int64_t *h_npixels)
{
    if (!h_stage || !h_counts || !h_npixels || cap_per_beam < 0 || (cap_per_beam > 0 && !h_out)) {
        snd::set_error("null argument");
        return SND_ERR_INVALID;
    }
    if (stage_bytes < SND_DETECT_STAGE_HEADER) { snd::set_error("stage buffer smaller than its header"); return SND_ERR_INVALID; }
    BatchLayout L;
    snd_status s = batch_layout(n, plans, desc, L);
    if (s != SND_OK) return s;
    for (int32_t i = 0; i < n; ++i) h_counts[i] = h_npixels[i] = 0;
    const uint8_t *hs = static_cast<const uint8_t *>(h_stage);
    unsigned int count = 0;
    std::memcpy(&count, hs, sizeof(count));
    const int64_t ncells = std::min<int64_t>(SND_DETECT_STAGE_CELLS(stage_bytes), desc->max_pixels);
    if ((int64_t)count > desc->max_pixels || (int64_t)count > ncells) {
        snd::set_error("more thresholded cells than max_pixels or than the stage buffer holds");
        return SND_ERR_CAPACITY;
    }
    // cells by beam (batch row -> beam through the row ranges), rows back to each plan's own
    std::vector<std::vector<snd::Pixel>> px((size_t)n);
    for (unsigned int c = 0; c < count; ++c) {
        snd::Pixel q;
        std::memcpy(&q, hs + SND_DETECT_STAGE_HEADER + (size_t)c * sizeof(snd::Pixel), sizeof(q));
        size_t lo = 0, hi = L.order.size();  // last beam (batch-row order) whose base <= q.k
        while (hi - lo > 1) {
            const size_t mid = (lo + hi) / 2;
            if (L.row_base[(size_t)L.order[mid]] <= q.k) lo = mid;
            else hi = mid;
        }
        const int32_t i = L.order[lo];
        q.k -= L.row_base[(size_t)i];
        if (q.k < 0 || q.k >= plans[i]->impl.ndm) { snd::set_error("staged cell outside the batch"); return SND_ERR_INVALID; }
        px[(size_t)i].push_back(q);
    }
    std::vector<snd_candidate> cands;
    for (int32_t i = 0; i < n; ++i) {
        h_npixels[i] = (int64_t)px[(size_t)i].size();
        s = candidates_from_pixels(px[(size_t)i], plans[i]->impl, desc, cands);
        if (s != SND_OK) return s;
        h_counts[i] = (int64_t)cands.size();
        for (int64_t c = 0; c < cap_per_beam && c < (int64_t)cands.size(); ++c) h_out[i * cap_per_beam + c] = cands[(size_t)c];
    }
    return SND_OK;
}

}  // extern "C"

static snd_status detect_impl(snd_plan plan, const void *d_plane, int64_t plane_pitch, const snd_detect_desc *desc,
                       void *d_workspace, int64_t workspace_bytes, snd_candidate *h_out, int64_t cap, int64_t *h_count,
                       int64_t *h_npixels, void *stream);

snd_status snd_detect(snd_plan plan, const void *d_plane, int64_t plane_pitch, const snd_detect_desc *desc,
                      void *d_workspace, int64_t workspace_bytes, snd_candidate *h_out, int64_t cap, int64_t *h_count,
                      int64_t *h_npixels, void *stream)
{
    roctxRangePushA("snd detect");  // host timeline marker (rocprofv3 --marker-trace)
    const snd_status s = detect_impl(plan, d_plane, plane_pitch, desc, d_workspace, workspace_bytes, h_out, cap,
                                     h_count, h_npixels, stream);
    roctxRangePop();
    return s;
}

}  // extern "C"

// the body of snd_detect (internal linkage: not part of the exported C API)
static snd_status detect_impl(snd_plan plan, const void *d_plane, int64_t plane_pitch, const snd_detect_desc *desc,
                       void *d_workspace, int64_t workspace_bytes, snd_candidate *h_out, int64_t cap, int64_t *h_count,
                       int64_t *h_npixels, void *stream)
{
    if (!plan || !d_plane || !d_workspace || !h_count || (cap > 0 && !h_out)) { snd::set_error("null argument"); return SND_ERR_INVALID; }
    const auto &P = plan->impl;
    snd_status s = check_desc(P, desc);
    if (s != SND_OK) return s;
    if (workspace_bytes < workspace_bytes_for(P, desc) || ((uintptr_t)d_workspace & 255u)) {
        snd::set_error("detect workspace too small or not 256-byte aligned");
        return SND_ERR_NOMEM;
    }
    if (plane_pitch < P.n_out) { snd::set_error("plane pitch smaller than n_out"); return SND_ERR_INVALID; }
    uint8_t *ws = static_cast<uint8_t *>(d_workspace);
    snd::SnrArgs a;
    fill_args(desc, a);
    a.counter = reinterpret_cast<unsigned int *>(ws);
    a.pixels = reinterpret_cast<snd::Pixel *>(ws + pixels_offset(P));
    a.max_pixels = desc->max_pixels;
    double *stats = reinterpret_cast<double *>(ws + kHeader);
    hipStream_t st = (hipStream_t)stream;
    s = upload_row_nw(P, desc, ws, a, st);
    if (s != SND_OK) return s;
    int e = snd::launch_detect(P.out_dtype, d_plane, plane_pitch, P.ndm, P.n_out, desc->sigma_min, desc->sigma_estimator,
                                 stats, a, stream);
    if (e) { snd::set_error(std::string("detect launch: ") + hipGetErrorString((hipError_t)e)); return SND_ERR_HIP; }
    unsigned int count = 0;
    hipError_t he = hipMemcpyAsync(&count, a.counter, sizeof(count), hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    if (he != hipSuccess) { snd::set_error(std::string("detect readback: ") + hipGetErrorString(he)); return SND_ERR_HIP; }
    if (h_npixels) *h_npixels = count;
    if ((int64_t)count > desc->max_pixels) {
        *h_count = 0;
        snd::set_error("more thresholded cells than max_pixels");
        return SND_ERR_CAPACITY;
    }
    if (desc->label_on_device) return label_device(P, desc, ws, a, h_out, cap, h_count, st);
    std::vector<snd::Pixel> px(count);
    if (count) {
        // through a pinned staging buffer of this thread (grown on demand, kept until exit):
        // a pageable read-back of ~10^5 cells costs more than the labelling that follows
        thread_local PinnedBuffer stage;
        const size_t nb = sizeof(snd::Pixel) * count;
        void *h = stage.get(nb);
        he = hipMemcpyAsync(h ? h : px.data(), a.pixels, nb, hipMemcpyDeviceToHost, st);
        if (he == hipSuccess) he = hipStreamSynchronize(st);
        if (he != hipSuccess) { snd::set_error(std::string("detect readback: ") + hipGetErrorString(he)); return SND_ERR_HIP; }
        if (h) std::memcpy(px.data(), h, nb);
    }
    std::vector<snd_candidate> cands;
    s = candidates_from_pixels(px, P, desc, cands);
    if (s != SND_OK) return s;
    *h_count = (int64_t)cands.size();
    for (int64_t i = 0; i < cap && i < (int64_t)cands.size(); ++i) h_out[i] = cands[i];
    return SND_OK;
}
