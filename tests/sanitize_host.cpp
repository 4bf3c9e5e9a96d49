// Host sanitizer run of libsnd's host code (AddressSanitizer + UndefinedBehaviorSanitizer):
// the plan builder on the 1024-channel x 4096-DM shape in every mode and storage type and on
// ragged and degenerate trees, the host part of detection (closing and labelling of staged
// cells), the cross-band merge, streaming admission and checkpoint validation, batch record
// sizing, FDMT tables and the validation helpers.  Nothing here touches a GPU; the sanitizers
// abort on any memory error or undefined behaviour.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "snd.h"

#define CHECK(x)                                                                                          \
    do {                                                                                                  \
        const snd_status s_ = (x);                                                                        \
        if (s_ != SND_OK) {                                                                               \
            std::fprintf(stderr, "%s:%d %s -> %d (%s)\n", __FILE__, __LINE__, #x, (int)s_, snd_last_error()); \
            std::exit(1);                                                                                 \
        }                                                                                                 \
    } while (0)
#define EXPECT(x, want)                                                                                   \
    do {                                                                                                  \
        const snd_status s_ = (x);                                                                        \
        if (s_ != (want)) {                                                                               \
            std::fprintf(stderr, "%s:%d %s -> %d, expected %d\n", __FILE__, __LINE__, #x, (int)s_, (int)(want)); \
            std::exit(1);                                                                                 \
        }                                                                                                 \
    } while (0)

static std::vector<double> band(int nchan)
{
    std::vector<double> f(nchan);
    for (int c = 0; c < nchan; ++c) f[c] = 416.0 - (c + 0.5) * 16.0 / nchan;
    return f;
}

static std::vector<double> grid(int n, double hi)
{
    std::vector<double> d(n);
    for (int i = 0; i < n; ++i) d[i] = n > 1 ? hi * i / (n - 1) : hi;
    return d;
}

struct Shape {
    int nchan, ndm;
    double dm_hi;
    int64_t nsamp;
    int mode, branching, cluster, cap, in_dt, node_dt;
    uint32_t stage_levels;
    int generic, chunk, root_norm;
};

static snd_status make(const Shape &s, const std::vector<double> &f, const std::vector<double> &dm, snd_plan *p)
{
    snd_plan_desc d;
    std::memset(&d, 0, sizeof d);
    d.nchan = s.nchan;
    d.freq_mhz = f.data();
    d.tsamp_s = 0.138e-3;
    d.ndm = s.ndm;
    d.dm = dm.data();
    d.branching = s.branching;
    d.cluster = s.cluster;
    d.mode = s.mode;
    d.k_leaf = 2;
    d.k_int = 1;
    d.cap = s.cap;
    d.in_dtype = s.in_dt;
    d.node_dtype = s.node_dt;
    d.root_norm = s.root_norm;
    d.nsamp = s.nsamp;
    d.stage_levels = s.stage_levels;
    d.generic_kernels = s.generic;
    d.chunk = s.chunk;
    return snd_plan_create(&d, p);
}

static void plans()
{
    const int F = SND_MODE_FLOAT, G = SND_MODE_GRADED, B = SND_MODE_BINARY;
    const Shape shapes[] = {
        {1024, 4096, 2000.0, 1 << 17, F, 4, 4, 255, SND_DT_F32, SND_DT_F32, 0, 0, 0, 0},
        {1024, 4096, 2000.0, 1 << 17, F, 4, 4, 255, SND_DT_BF16, SND_DT_BF16, 0, 0, 0, 1},
        {1024, 4096, 2000.0, 1 << 17, F, 8, 4, 255, SND_DT_F32, SND_DT_F16, 0, 0, 0, 0},
        {1024, 4096, 2000.0, 1 << 17, G, 4, 4, 255, SND_DT_U8, SND_DT_U8, 0, 0, 0, 0},
        {1024, 4096, 2000.0, 1 << 17, G, 8, 4, 255, SND_DT_U8, SND_DT_U8, 0, 0, 0, 0},
        {1024, 4096, 2000.0, 1 << 17, G, 4, 4, 4095, SND_DT_U8, SND_DT_U16, 0, 0, 0, 0},
        {1024, 4096, 2000.0, 1 << 17, B, 4, 4, 255, SND_DT_BITS, SND_DT_BITS, 0, 0, 0, 0},
        {1024, 4096, 2000.0, 1 << 17, B, 8, 4, 255, SND_DT_U8, SND_DT_U8, 0, 0, 0, 0},
        {1024, 4096, 2000.0, 0, G, 4, 4, 255, SND_DT_U8, SND_DT_U8, 0, 0, 8192, 0},   // streaming plan
        {1000, 512, 500.0, 20000, G, 4, 4, 255, SND_DT_U8, SND_DT_U8, 0, 0, 0, 0},    // ragged tree
        {1000, 512, 500.0, 20000, F, 4, 4, 255, SND_DT_F32, SND_DT_F32, 0, 0, 0, 0},
        {37, 33, 40.0, 3000, G, 3, 3, 7, SND_DT_U8, SND_DT_U8, 0x3, 0, 0, 0},          // levels written
        {37, 33, 40.0, 3000, F, 3, 5, 255, SND_DT_F32, SND_DT_F32, SND_STAGE_NONE, 0, 0, 0},
        {64, 50, 60.0, 4000, B, 2, 4, 255, SND_DT_U8, SND_DT_U8, 0, 1, 0, 0},         // generic kernels
        {64, 50, 60.0, 4000, F, 4, 4, 255, SND_DT_F32, SND_DT_F32, 0x3, 0, 0, 0},
        {1, 1, 100.0, 70, F, 2, 1, 255, SND_DT_F32, SND_DT_F32, 0, 0, 0, 0},          // one channel
        {3, 4, 0.0, 300, G, 2, 4, 6, SND_DT_U8, SND_DT_U8, 0, 0, 0, 0},              // zero DMs
    };
    for (const Shape &s : shapes) {
        const std::vector<double> f = band(s.nchan), dm = grid(s.ndm, s.dm_hi);
        snd_plan p = nullptr;
        CHECK(make(s, f, dm, &p));
        snd_plan_info info;
        CHECK(snd_plan_query(p, &info));
        std::vector<int32_t> dl((size_t)s.ndm * s.nchan);
        CHECK(snd_plan_delays(p, dl.data(), (int64_t)dl.size()));
        if (info.n_out <= 0 || info.max_delay != *std::max_element(dl.begin(), dl.end())) {
            std::fprintf(stderr, "plan %d x %d: n_out %lld max_delay %lld\n", s.nchan, s.ndm, (long long)info.n_out,
                         (long long)info.max_delay);
            std::exit(1);
        }
        EXPECT(snd_plan_delays(p, dl.data(), (int64_t)dl.size() - 1), SND_ERR_NOMEM);  // buffer too small
        CHECK(snd_plan_destroy(p));
    }
    // malformed descriptors are refused without touching anything
    Shape bad = shapes[0];
    bad.branching = 1;
    const std::vector<double> f = band(1024), dm = grid(4096, 2000.0);
    snd_plan p = nullptr;
    EXPECT(make(bad, f, dm, &p), SND_ERR_INVALID);
    bad = shapes[0];
    bad.nsamp = 100;  // shorter than the largest delay
    EXPECT(make(bad, f, dm, &p), SND_ERR_INVALID);
}

// Staged cells (as snd_detect_launch leaves them in host memory) turned into candidates.
struct Cell {
    int32_t k, t;
    double snr;
    int32_t widx, pad;
};
static_assert(sizeof(Cell) == 24, "staged cell layout");

static void detection()
{
    const Shape s{64, 40, 60.0, 5000, SND_MODE_FLOAT, 4, 4, 255, SND_DT_F32, SND_DT_F32, 0, 0, 0, 0};
    const std::vector<double> f = band(s.nchan), dm = grid(s.ndm, s.dm_hi);
    snd_plan p = nullptr;
    CHECK(make(s, f, dm, &p));
    snd_plan_info info;
    CHECK(snd_plan_query(p, &info));
    const int32_t widths[4] = {1, 2, 4, 8};
    snd_detect_desc d;
    std::memset(&d, 0, sizeof d);
    d.widths = widths;
    d.nwidths = 4;
    d.closing_radius = 4;
    d.threshold = 6.0;
    d.sigma_min = 0.0;
    d.n_min = 3;
    d.max_pixels = 1 << 16;
    int64_t ws = 0;
    CHECK(snd_detect_workspace(p, &d, &ws));
    // islands of cells plus scattered single cells, each row's cells in increasing t
    std::mt19937 rng(7);
    std::vector<std::vector<Cell>> rows(s.ndm);
    for (int isl = 0; isl < 6; ++isl) {
        const int k0 = (int)(rng() % (s.ndm - 4)), t0 = (int)(rng() % (info.n_out - 10));
        for (int k = k0; k < k0 + 3; ++k)
            for (int t = t0; t < t0 + 7; ++t) rows[k].push_back({k, t, 6.0 + (rng() % 1000) * 1e-3, (int)(rng() % 4), 0});
    }
    for (int i = 0; i < 40; ++i) {
        const int k = (int)(rng() % s.ndm), t = (int)(rng() % info.n_out);
        rows[k].push_back({k, t, 6.5, 0, 0});
    }
    std::vector<Cell> cells;
    for (auto &r : rows) {
        std::sort(r.begin(), r.end(), [](const Cell &a, const Cell &b) { return a.t < b.t; });
        r.erase(std::unique(r.begin(), r.end(), [](const Cell &a, const Cell &b) { return a.t == b.t; }), r.end());
        cells.insert(cells.end(), r.begin(), r.end());
    }
    const int64_t bytes = SND_DETECT_STAGE_HEADER + (int64_t)sizeof(Cell) * (int64_t)cells.size();
    std::vector<unsigned char> stage((size_t)bytes, 0);
    const uint32_t count = (uint32_t)cells.size();
    std::memcpy(stage.data(), &count, 4);
    std::memcpy(stage.data() + SND_DETECT_STAGE_HEADER, cells.data(), cells.size() * sizeof(Cell));
    std::vector<snd_candidate> out(256);
    int64_t nc = 0, npx = 0;
    CHECK(snd_detect_collect(p, &d, stage.data(), bytes, out.data(), (int64_t)out.size(), &nc, &npx));
    const int64_t nc_single = nc;
    if (nc < 1 || npx != (int64_t)cells.size()) {
        std::fprintf(stderr, "collect: %lld candidates from %lld cells\n", (long long)nc, (long long)npx);
        std::exit(1);
    }
    // more cells counted than staged: capacity, no candidates
    const uint32_t over = count + 1;
    std::memcpy(stage.data(), &over, 4);
    EXPECT(snd_detect_collect(p, &d, stage.data(), bytes, out.data(), (int64_t)out.size(), &nc, &npx),
           SND_ERR_CAPACITY);

    // batched: the same cells as the first beam's (the float plan's), whose rows follow the
    // graded plan's in batch-row order (u8 planes first); nothing in the graded beam
    const Shape g{48, 30, 50.0, 4000, SND_MODE_GRADED, 4, 4, 255, SND_DT_U8, SND_DT_U8, 0, 0, 0, 0};
    const std::vector<double> fg = band(g.nchan), dg = grid(g.ndm, g.dm_hi);
    snd_plan pg = nullptr;
    CHECK(make(g, fg, dg, &pg));
    const snd_plan both[2] = {p, pg};
    int64_t wsb = 0;
    CHECK(snd_detect_batch_workspace(2, both, &d, &wsb));
    std::vector<Cell> shifted = cells;
    for (Cell &c : shifted) c.k += g.ndm;
    std::memcpy(stage.data(), &count, 4);
    std::memcpy(stage.data() + SND_DETECT_STAGE_HEADER, shifted.data(), shifted.size() * sizeof(Cell));
    std::vector<snd_candidate> bout(2 * 128);
    int64_t cnts[2], npxs[2];
    CHECK(snd_detect_batch_collect(2, both, &d, stage.data(), bytes, bout.data(), 128, cnts, npxs));
    if (cnts[1] != 0 || npxs[1] != 0 || cnts[0] != nc_single || npxs[0] != (int64_t)cells.size()) {
        std::fprintf(stderr, "batched collect: %lld/%lld candidates\n", (long long)cnts[0], (long long)cnts[1]);
        std::exit(1);
    }
    d.sigma_estimator = 1;  // the median-absolute-deviation sigma is single-plane only
    EXPECT(snd_detect_batch_workspace(2, both, &d, &wsb), SND_ERR_UNSUPPORTED);
    CHECK(snd_plan_destroy(pg));
    CHECK(snd_plan_destroy(p));
}

static void merge_and_validation()
{
    std::mt19937 rng(11);
    std::vector<snd_band_candidate> in(300), out(300);
    for (size_t i = 0; i < in.size(); ++i) {
        snd_band_candidate &c = in[i];
        std::memset(&c, 0, sizeof c);
        c.dm = (rng() % 2000) * 1.0;
        c.t_ms = (rng() % 18000) * 1.0;
        c.snr = 7.0 + (rng() % 100) * 0.1;
        c.band = (int32_t)(rng() % 4);
        c.dm_index = (int32_t)i;
        c.width = 1 << (rng() % 6);
        c.t = (int64_t)(rng() % 100000);
        c.npix = 10 + (int64_t)(rng() % 100);
    }
    int64_t kept = 0;
    CHECK(snd_merge_candidates((int64_t)in.size(), in.data(), 20.0, 200.0, out.data(), &kept));
    if (kept < 1 || kept > (int64_t)in.size()) std::exit(1);

    const std::vector<double> f = band(1024), dm = grid(4096, 2000.0);
    std::vector<int32_t> fac(dm.size());
    CHECK(snd_scrunch_factors(1024, f.data(), 0.138e-3, (int32_t)dm.size(), dm.data(), 16, fac.data()));
    std::vector<double> w(16, 2.0), we(16), idm(16), it(16);
    for (int i = 0; i < 16; ++i) {
        idm[i] = 100.0 * i;
        it[i] = 1000.0 * i;
    }
    CHECK(snd_effective_width(1024, f.data(), 0.138e-3, 16, idm.data(), w.data(), we.data()));
    std::vector<double> cdm(40), ct(40), cs(40);
    for (int i = 0; i < 40; ++i) {
        cdm[i] = idm[i % 16] + (double)(rng() % 5);
        ct[i] = it[i % 16] + (double)(rng() % 3) * 0.1;
        cs[i] = 7.0 + i;
    }
    std::vector<int32_t> match(16);
    int64_t nm = 0;
    CHECK(snd_match_injections(40, cdm.data(), ct.data(), cs.data(), 16, idm.data(), it.data(), we.data(), 10.0, 0.5,
                               match.data(), &nm));

    snd_fdmt fd = nullptr;
    std::vector<double> fdesc(1024);
    for (int c = 0; c < 1024; ++c) fdesc[c] = 416.0 - (c + 0.5) * 16.0 / 1024;
    CHECK(snd_fdmt_create(1024, fdesc.data(), 16.0 / 1024, 0.138e-3, 500.0, 1 << 15, &fd));
    int64_t nd = 0, no = 0, tb = 0, wb = 0;
    double step = 0;
    CHECK(snd_fdmt_query(fd, &nd, &no, &tb, &wb, &step));
    CHECK(snd_fdmt_destroy(fd));
    EXPECT(snd_fdmt_create(1000, fdesc.data(), 16.0 / 1024, 0.138e-3, 500.0, 1 << 15, &fd), SND_ERR_INVALID);
}

static void streaming_and_batching()
{
    const Shape sg{1024, 4096, 2000.0, 0, SND_MODE_GRADED, 4, 4, 255, SND_DT_U8, SND_DT_U8, 0, 0, 8192, 0};
    const Shape sf{1024, 4096, 2000.0, 0, SND_MODE_FLOAT, 4, 4, 255, SND_DT_BF16, SND_DT_BF16, 0, 0, 8192, 0};
    const std::vector<double> f = band(1024), dm = grid(4096, 2000.0);
    snd_plan pg = nullptr, pf = nullptr;
    CHECK(make(sg, f, dm, &pg));
    CHECK(make(sf, f, dm, &pf));
    int64_t hist = 0, adm = 0, adm_f = 0;
    CHECK(snd_stream_history_bytes(pg, &hist));
    CHECK(snd_stream_admission_bytes(pg, &adm));
    CHECK(snd_stream_admission_bytes(pf, &adm_f));
    snd_stream st = nullptr;
    CHECK(snd_stream_create(5 * adm + adm_f, &st));
    // admission touches no device memory: the history buffers here are placeholders
    void *fake = reinterpret_cast<void *>((uintptr_t)1 << 40);
    int admitted = 0;
    for (int b = 0; b < 8; ++b) {
        const snd_status r = snd_stream_admit(st, b, b % 2 ? pf : pg, fake, 1ll << 32);
        if (r == SND_OK) ++admitted;
        else if (r != SND_ERR_CAPACITY) std::exit(1);
    }
    EXPECT(snd_stream_admit(st, 0, pg, fake, 1ll << 32), SND_ERR_INVALID);  // already admitted
    int64_t budget = 0, used = 0;
    int32_t nb = 0;
    CHECK(snd_stream_usage(st, &budget, &used, &nb));
    if (nb != admitted || used > budget) std::exit(1);
    int64_t rec = 0, wsb = 0, rcv = 0, nxt = 0, emi = 0;
    std::vector<int32_t> ids;
    for (int b = 0; b < nb; ++b) ids.push_back(b);
    CHECK(snd_stream_batch_bytes(st, nb, ids.data(), &wsb, &rec));
    CHECK(snd_stream_beam_state(st, 0, &rcv, &nxt, &emi));
    int64_t xb = 0;
    CHECK(snd_stream_export_bytes(st, 0, &xb));
    std::vector<unsigned char> ck((size_t)xb, 0);  // a zeroed header: another ring shape
    EXPECT(snd_stream_import(st, 0, ck.data(), xb, nullptr), SND_ERR_INVALID);
    EXPECT(snd_stream_import(st, 0, ck.data(), 10, nullptr), SND_ERR_INVALID);
    CHECK(snd_stream_evict(st, 0));
    EXPECT(snd_stream_evict(st, 0), SND_ERR_STATE);
    CHECK(snd_stream_destroy(st));

    snd_plan plans[2] = {pg, pf};
    int64_t rb = 0;
    int32_t nl = 0;
    CHECK(snd_batch_records_bytes(2, plans, &rb, &nl));
    if (rb <= 0 || nl < 2) std::exit(1);
    CHECK(snd_plan_destroy(pg));
    CHECK(snd_plan_destroy(pf));
}

int main()
{
    plans();
    detection();
    merge_and_validation();
    streaming_and_batching();
    std::puts("sanitized host run ok");
    return 0;
}
