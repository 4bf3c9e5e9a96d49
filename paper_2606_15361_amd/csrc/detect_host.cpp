// Matched-filter / candidate entry points: argument checks, kernel launches, and the host part
// of candidate detection (Methods, "Candidate detection"): binary closing and 8-connected
// labelling over the sparse set of thresholded cells returned by the device.
#include <hip/hip_runtime.h>

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
        d->n_min < 1 || d->max_pixels < 1 || d->reserved != 0) {
        snd::set_error("threshold must be > 0, sigma_min >= 0, 0 <= closing_radius <= 64, n_min >= 1, max_pixels >= 1");
        return SND_ERR_INVALID;
    }
    if (P.ndm > 65535) { snd::set_error("detect supports at most 65535 DM rows"); return SND_ERR_UNSUPPORTED; }
    if (P.n_out > 0x7fffffffLL) { snd::set_error("rows too long for detect"); return SND_ERR_UNSUPPORTED; }
    return SND_OK;
}

int64_t workspace_bytes_for(const snd::PlanImpl &P, const snd_detect_desc *d)
{
    return kHeader + round_up((int64_t)P.ndm * 16, 256) + d->max_pixels * (int64_t)sizeof(snd::Pixel);
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

snd_status candidates_from_pixels(std::vector<snd::Pixel> &px, const snd::PlanImpl &P, const snd_detect_desc *d,
                                  std::vector<snd_candidate> &out)
{
    out.clear();
    if (px.empty()) return SND_OK;
    std::sort(px.begin(), px.end(), [](const snd::Pixel &a, const snd::Pixel &b) {
        return a.k != b.k ? a.k < b.k : a.t < b.t;
    });
    const int64_t r = d->closing_radius;
    const int64_t reach = 2 * r + 1;  // two dilation squares touch (8-connected) within this distance
    const size_t n = px.size();
    // row starts in the sorted list
    UF uf(n);
    size_t rs = 0;
    std::vector<std::pair<int32_t, size_t>> rows;  // (k, first index)
    for (size_t i = 0; i < n; ++i)
        if (i == 0 || px[i].k != px[i - 1].k) rows.push_back({px[i].k, i});
    rows.push_back({INT32_MAX, n});
    for (size_t ri = 0; ri + 1 < rows.size(); ++ri) {
        const int32_t k = rows[ri].first;
        for (size_t rj = ri; rj + 1 < rows.size() && rows[rj].first <= k + reach; ++rj) {
            size_t b0 = rows[rj].second, b1 = rows[rj + 1].second;
            for (size_t i = rows[ri].second; i < rows[ri + 1].second; ++i) {
                const int64_t t = px[i].t;
                auto lo = std::lower_bound(px.begin() + b0, px.begin() + b1, t - reach,
                                           [](const snd::Pixel &a, int64_t v) { return a.t < v; });
                for (auto it = lo; it != px.begin() + b1 && it->t <= t + reach; ++it) uf.u((int32_t)i, (int32_t)(it - px.begin()));
            }
        }
    }
    (void)rs;
    // group pixels by component
    std::vector<int32_t> comp(n);
    for (size_t i = 0; i < n; ++i) comp[i] = uf.f((int32_t)i);
    std::vector<int32_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return comp[a] < comp[b]; });
    std::vector<uint8_t> A, Bm;
    std::vector<int32_t> lab;
    std::vector<int64_t> stack;
    for (size_t s = 0; s < n;) {
        size_t e = s;
        while (e < n && comp[order[e]] == comp[order[s]]) ++e;
        int64_t kmin = INT64_MAX, kmax = INT64_MIN, tmin = INT64_MAX, tmax = INT64_MIN;
        for (size_t i = s; i < e; ++i) {
            const snd::Pixel &q = px[order[i]];
            kmin = std::min<int64_t>(kmin, q.k); kmax = std::max<int64_t>(kmax, q.k);
            tmin = std::min<int64_t>(tmin, q.t); tmax = std::max<int64_t>(tmax, q.t);
        }
        const int64_t k0 = kmin - 2 * r, t0 = tmin - 2 * r;
        const int64_t H = kmax - kmin + 4 * r + 1, W = tmax - tmin + 4 * r + 1;
        if (H * W > (int64_t)1 << 31) { snd::set_error("candidate island too large for host labelling"); return SND_ERR_CAPACITY; }
        A.assign((size_t)(H * W), 0);
        Bm.assign((size_t)(H * W), 0);
        for (size_t i = s; i < e; ++i) {
            const snd::Pixel &q = px[order[i]];
            A[(size_t)((q.k - k0) * W + (q.t - t0))] = 1;
        }
        // dilation (square): along t, then along k, with running counts
        for (int64_t i = 0; i < H; ++i) {
            const uint8_t *a = &A[(size_t)(i * W)];
            uint8_t *b = &Bm[(size_t)(i * W)];
            int64_t cnt = 0;
            for (int64_t j = 0; j < std::min<int64_t>(r, W); ++j) cnt += a[j];
            for (int64_t j = 0; j < W; ++j) {
                if (j + r < W) cnt += a[j + r];
                if (j - r - 1 >= 0) cnt -= a[j - r - 1];
                b[j] = cnt > 0;
            }
        }
        for (int64_t j = 0; j < W; ++j) {
            int64_t cnt = 0;
            for (int64_t i = 0; i < std::min<int64_t>(r, H); ++i) cnt += Bm[(size_t)(i * W + j)];
            for (int64_t i = 0; i < H; ++i) {
                if (i + r < H) cnt += Bm[(size_t)((i + r) * W + j)];
                if (i - r - 1 >= 0) cnt -= Bm[(size_t)((i - r - 1) * W + j)];
                A[(size_t)(i * W + j)] = cnt > 0;
            }
        }
        // erosion (square); cells outside the grid are empty (the grid spans the dilation + r)
        const int64_t full = 2 * r + 1;
        for (int64_t i = 0; i < H; ++i) {
            const uint8_t *a = &A[(size_t)(i * W)];
            uint8_t *b = &Bm[(size_t)(i * W)];
            int64_t cnt = 0;
            for (int64_t j = 0; j < std::min<int64_t>(r, W); ++j) cnt += a[j];
            for (int64_t j = 0; j < W; ++j) {
                if (j + r < W) cnt += a[j + r];
                if (j - r - 1 >= 0) cnt -= a[j - r - 1];
                b[j] = (j - r >= 0 && j + r < W && cnt == full);
            }
        }
        for (int64_t j = 0; j < W; ++j) {
            int64_t cnt = 0;
            for (int64_t i = 0; i < std::min<int64_t>(r, H); ++i) cnt += Bm[(size_t)(i * W + j)];
            for (int64_t i = 0; i < H; ++i) {
                if (i + r < H) cnt += Bm[(size_t)((i + r) * W + j)];
                if (i - r - 1 >= 0) cnt -= Bm[(size_t)((i - r - 1) * W + j)];
                A[(size_t)(i * W + j)] = (i - r >= 0 && i + r < H && cnt == full);
            }
        }
        // the closed set lies inside the bounding box of the thresholded cells, hence inside
        // the plane; label it with 8-connectivity
        lab.assign((size_t)(H * W), -1);
        int32_t nlab = 0;
        std::vector<int64_t> npix;
        for (int64_t i = 0; i < H; ++i)
            for (int64_t j = 0; j < W; ++j) {
                const size_t c = (size_t)(i * W + j);
                if (!A[c] || lab[c] >= 0) continue;
                int64_t cntp = 0;
                stack.clear();
                stack.push_back((int64_t)c);
                lab[c] = nlab;
                while (!stack.empty()) {
                    const int64_t q = stack.back();
                    stack.pop_back();
                    ++cntp;
                    const int64_t qi = q / W, qj = q % W;
                    for (int64_t di = -1; di <= 1; ++di)
                        for (int64_t dj = -1; dj <= 1; ++dj) {
                            const int64_t ni = qi + di, nj = qj + dj;
                            if (ni < 0 || ni >= H || nj < 0 || nj >= W) continue;
                            const size_t nc = (size_t)(ni * W + nj);
                            if (A[nc] && lab[nc] < 0) { lab[nc] = nlab; stack.push_back((int64_t)nc); }
                        }
                }
                npix.push_back(cntp);
                ++nlab;
            }
        std::vector<int32_t> peak(nlab, -1);
        for (size_t i = s; i < e; ++i) {  // thresholded cells, visited in (k, t) order
            const int32_t pi = order[i];
            const snd::Pixel &q = px[pi];
            const int32_t l = lab[(size_t)((q.k - k0) * W + (q.t - t0))];
            if (l < 0) continue;  // cannot happen: closing keeps every original cell
            if (peak[l] < 0) { peak[l] = pi; continue; }
            const snd::Pixel &b = px[peak[l]];
            if (q.snr > b.snr || (q.snr == b.snr && (q.k < b.k || (q.k == b.k && q.t < b.t)))) peak[l] = pi;
        }
        for (int32_t l = 0; l < nlab; ++l) {
            if (npix[l] < d->n_min || peak[l] < 0) continue;
            const snd::Pixel &q = px[peak[l]];
            snd_candidate c{};
            c.dm_index = q.k;
            c.width = d->widths[q.widx];
            c.t = q.t;
            c.snr = q.snr;
            c.dm = P.dm[q.k];
            c.npix = npix[l];
            out.push_back(c);
        }
        s = e;
    }
    std::sort(out.begin(), out.end(), [](const snd_candidate &a, const snd_candidate &b) {
        return a.dm_index != b.dm_index ? a.dm_index < b.dm_index : a.t < b.t;
    });
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
    int e = snd::launch_detect(P.out_dtype, d_plane, plane_pitch, P.ndm, P.n_out, desc->sigma_min, stats, a, stream);
    if (e) { snd::set_error(std::string("detect launch: ") + hipGetErrorString((hipError_t)e)); return SND_ERR_HIP; }
    return SND_OK;
}

snd_status snd_detect(snd_plan plan, const void *d_plane, int64_t plane_pitch, const snd_detect_desc *desc,
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
    a.pixels = reinterpret_cast<snd::Pixel *>(ws + kHeader + round_up((int64_t)P.ndm * 16, 256));
    a.max_pixels = desc->max_pixels;
    double *stats = reinterpret_cast<double *>(ws + kHeader);
    hipStream_t st = (hipStream_t)stream;
    int e = snd::launch_detect(P.out_dtype, d_plane, plane_pitch, P.ndm, P.n_out, desc->sigma_min, stats, a, stream);
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
    std::vector<snd::Pixel> px(count);
    if (count) {
        he = hipMemcpyAsync(px.data(), a.pixels, sizeof(snd::Pixel) * count, hipMemcpyDeviceToHost, st);
        if (he == hipSuccess) he = hipStreamSynchronize(st);
        if (he != hipSuccess) { snd::set_error(std::string("detect readback: ") + hipGetErrorString(he)); return SND_ERR_HIP; }
    }
    std::vector<snd_candidate> cands;
    s = candidates_from_pixels(px, P, desc, cands);
    if (s != SND_OK) return s;
    *h_count = (int64_t)cands.size();
    for (int64_t i = 0; i < cap && i < (int64_t)cands.size(); ++i) h_out[i] = cands[i];
    return SND_OK;
}

}  // extern "C"
