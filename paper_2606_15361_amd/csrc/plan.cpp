// Host-side SND plan builder (Methods, "The Spiking Neural Dedispersion algorithm").
//
// 1. Integer channel delays for every trial DM (Methods, "Incoherent dedispersion").
// 2. Tree shape: leaf clusters of C consecutive channels, B-ary levels above (last group of a
//    level may be smaller), reference channel = highest frequency of the node.
// 3. Shared patterns: at each node the DMs with the same delay pattern -- at a leaf the channel
//    delays relative to the node reference, above it the (child neuron, child shift) tuple --
//    share one neuron (one row of partial sums).
// 4. Stages: the levels flagged in stage_levels are written to device memory; every stage
//    evaluates the sub-tree between two such levels in registers, so each output row is a list
//    of (source row, time offset, closing depth) entries.
//
// Each neuron row is anchored at the smallest reference delay `lo` of the DMs it serves: row
// index i holds the node value at reference time lo + i for i < n_out + hi - lo.  A parent
// therefore reads its children at small relative offsets, and the output of the final stage is
// y_k(t), t in [0, n_out).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>

#include "snd_internal.h"

namespace snd {

int dtype_size(int dt)
{
    switch (dt) {
    case SND_DT_U8: return 1;
    case SND_DT_U16: return 2;
    case SND_DT_F32: return 4;
    case SND_DT_BF16: return 2;
    case SND_DT_F16: return 2;
    default: return 0;
    }
}

namespace {

// Open-addressing map from an int32 key of fixed length to a dense id (first-seen order).
class PatternMap {
public:
    PatternMap(int keylen, int expected) : keylen_(keylen)
    {
        size_t cap = 16;
        while (cap < (size_t)expected * 2) cap <<= 1;
        slots_.assign(cap, -1);
        mask_ = cap - 1;
        keys_.reserve((size_t)expected * keylen);
    }
    int32_t find_or_insert(const int32_t *key, bool *inserted)
    {
        uint64_t h = 0x9E3779B97F4A7C15ull;
        for (int i = 0; i < keylen_; ++i) {
            h ^= (uint64_t)(uint32_t)key[i] + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
        }
        h ^= h >> 31;
        h *= 0xBF58476D1CE4E5B9ull;
        h ^= h >> 29;
        size_t s = (size_t)h & mask_;
        for (;;) {
            int32_t id = slots_[s];
            if (id < 0) break;
            if (std::memcmp(&keys_[(size_t)id * keylen_], key, sizeof(int32_t) * keylen_) == 0) {
                *inserted = false;
                return id;
            }
            s = (s + 1) & mask_;
        }
        int32_t id = (int32_t)(keys_.size() / keylen_);
        keys_.insert(keys_.end(), key, key + keylen_);
        slots_[s] = id;
        *inserted = true;
        return id;
    }

private:
    int keylen_;
    size_t mask_;
    std::vector<int32_t> slots_;
    std::vector<int32_t> keys_;
};

int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

bool valid_dtype_pair(int mode, int in_dt, int node_dt, int cap)
{
    if (mode == SND_MODE_BINARY) return in_dt == SND_DT_U8 && node_dt == SND_DT_U8;
    if (mode == SND_MODE_GRADED)
        return in_dt == SND_DT_U8 && (node_dt == SND_DT_U16 || (node_dt == SND_DT_U8 && cap <= 255));
    if (mode == SND_MODE_FLOAT) {
        auto f = [](int d) { return d == SND_DT_F32 || d == SND_DT_BF16 || d == SND_DT_F16; };
        return f(in_dt) && f(node_dt);
    }
    return false;
}

}  // namespace

snd_status build_plan(const snd_plan_desc &d, PlanImpl &p, std::string &err)
{
    auto t_start = std::chrono::steady_clock::now();
    // ---------------- validation ----------------
    if (d.nchan < 1 || !d.freq_mhz || d.ndm < 1 || !d.dm || !(d.tsamp_s > 0.0) || d.nsamp < 1) {
        err = "nchan, ndm, nsamp must be >= 1, tsamp_s > 0 and freq/dm non-null";
        return SND_ERR_INVALID;
    }
    for (int i = 0; i < 8; ++i)
        if (d.reserved[i]) { err = "reserved descriptor fields must be zero"; return SND_ERR_INVALID; }
    if (d.branching < 2 || d.cluster < 1) { err = "branching must be >= 2 and cluster >= 1"; return SND_ERR_INVALID; }
    if (d.mode < SND_MODE_BINARY || d.mode > SND_MODE_FLOAT) { err = "unknown mode"; return SND_ERR_INVALID; }
    if (d.mode == SND_MODE_BINARY && (d.k_leaf < 1 || d.k_int < 1)) {
        err = "binary quorum thresholds must be >= 1";
        return SND_ERR_INVALID;
    }
    if (d.mode == SND_MODE_GRADED && (d.cap < 1 || d.cap > 65535)) { err = "graded cap must be in 1..65535"; return SND_ERR_INVALID; }
    if (!valid_dtype_pair(d.mode, d.in_dtype, d.node_dtype, d.cap)) {
        err = "unsupported input/node dtype for this mode";
        return SND_ERR_UNSUPPORTED;
    }
    p.desc = d;
    p.nchan = d.nchan;
    p.ndm = d.ndm;
    p.nsamp = d.nsamp;
    p.freq.assign(d.freq_mhz, d.freq_mhz + d.nchan);
    p.dm.assign(d.dm, d.dm + d.ndm);
    double fmax = 0.0;
    for (double f : p.freq) {
        if (!(f > 0.0) || !std::isfinite(f)) { err = "channel frequencies must be finite and > 0"; return SND_ERR_INVALID; }
        fmax = std::max(fmax, f);
    }
    for (double v : p.dm)
        if (!(v >= 0.0) || !std::isfinite(v)) { err = "trial DMs must be finite and >= 0"; return SND_ERR_INVALID; }
    p.fref = d.fref_mhz > 0.0 ? d.fref_mhz : fmax;
    if (p.fref < fmax) { err = "reference frequency below the highest channel frequency"; return SND_ERR_INVALID; }

    // ---------------- delays ----------------
    const int nc = p.nchan, nd = p.ndm;
    const double tms = d.tsamp_s * 1e3;
    p.delay.resize((size_t)nd * nc);
    int64_t dmax = 0;
    for (int k = 0; k < nd; ++k) {
        for (int c = 0; c < nc; ++c) {
            double x = kDM * p.dm[k];
            x = x * (1.0 / (p.freq[c] * p.freq[c]) - 1.0 / (p.fref * p.fref));
            x = x / tms;
            if (!(x < 2.0e9)) { err = "delay exceeds 2^31 samples"; return SND_ERR_INVALID; }
            int32_t v = (int32_t)std::nearbyint(x);
            p.delay[(size_t)k * nc + c] = v;
            dmax = std::max<int64_t>(dmax, v);
        }
    }
    p.max_delay = dmax;
    p.n_out = p.nsamp - dmax;
    if (p.n_out < 1) { err = "nsamp does not exceed the largest delay: no valid output samples"; return SND_ERR_INVALID; }

    // ---------------- tree shape ----------------
    p.lev.clear();
    {
        int n = (nc + d.cluster - 1) / d.cluster;
        for (int l = 0;; ++l) {
            if (l >= SND_MAX_LEVELS) { err = "tree deeper than SND_MAX_LEVELS"; return SND_ERR_INVALID; }
            Level L;
            L.nnodes = n;
            L.chlo.resize(n); L.chhi.resize(n); L.kidlo.resize(n); L.kidhi.resize(n); L.ref.resize(n);
            for (int i = 0; i < n; ++i) {
                if (l == 0) {
                    L.kidlo[i] = L.kidhi[i] = 0;
                    L.chlo[i] = i * d.cluster;
                    L.chhi[i] = std::min(nc, (i + 1) * d.cluster);
                } else {
                    const Level &P = p.lev[l - 1];
                    int a = i * d.branching, b = std::min(P.nnodes, (i + 1) * d.branching);
                    L.kidlo[i] = a; L.kidhi[i] = b;
                    L.chlo[i] = P.chlo[a];
                    L.chhi[i] = P.chhi[b - 1];
                }
                int r = L.chlo[i];
                for (int c = L.chlo[i] + 1; c < L.chhi[i]; ++c)
                    if (p.freq[c] > p.freq[r]) r = c;
                L.ref[i] = r;
            }
            p.lev.push_back(std::move(L));
            if (n == 1) break;
            n = (n + d.branching - 1) / d.branching;
        }
    }
    const int nlev = (int)p.lev.size();
    const int top = nlev - 1;

    // ---------------- shared patterns ----------------
    std::vector<int32_t> order(nd);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return p.dm[a] < p.dm[b]; });
    std::vector<int32_t> key;
    for (int l = 0; l < nlev; ++l) {
        Level &L = p.lev[l];
        L.nid.assign((size_t)L.nnodes * nd, -1);
        L.nneu.assign(L.nnodes, 0);
        L.row_base.assign(L.nnodes, 0);
        std::vector<std::vector<int32_t>> reps(L.nnodes);
        for (int q = 0; q < L.nnodes; ++q) {
            int fan = l == 0 ? L.chhi[q] - L.chlo[q] : L.kidhi[q] - L.kidlo[q];
            int keylen = l == 0 ? fan : 2 * fan;
            PatternMap map(keylen, std::min(nd, 1 << 16));
            key.resize(keylen);
            int32_t r = L.ref[q];
            for (int oi = 0; oi < nd; ++oi) {
                int k = order[oi];
                const int32_t *dk = &p.delay[(size_t)k * nc];
                if (l == 0) {
                    for (int i = 0; i < fan; ++i) key[i] = dk[L.chlo[q] + i] - dk[r];
                } else {
                    const Level &P = p.lev[l - 1];
                    for (int i = 0; i < fan; ++i) {
                        int ch = L.kidlo[q] + i;
                        key[2 * i] = P.nid[(size_t)ch * nd + k];
                        key[2 * i + 1] = dk[P.ref[ch]] - dk[r];
                    }
                }
                bool ins = false;
                int32_t id = map.find_or_insert(key.data(), &ins);
                if (ins) reps[q].push_back(k);
                L.nid[(size_t)q * nd + k] = id;
            }
            L.nneu[q] = (int32_t)reps[q].size();
        }
        int64_t rows = 0;
        for (int q = 0; q < L.nnodes; ++q) { L.row_base[q] = rows; rows += L.nneu[q]; }
        L.rows = rows;
        L.rep.resize(rows); L.lo.assign(rows, INT32_MAX); L.hi.assign(rows, INT32_MIN); L.node_of.resize(rows);
        L.synapses = 0;
        for (int q = 0; q < L.nnodes; ++q) {
            int fan = l == 0 ? L.chhi[q] - L.chlo[q] : L.kidhi[q] - L.kidlo[q];
            L.synapses += (int64_t)fan * L.nneu[q];
            for (int u = 0; u < L.nneu[q]; ++u) {
                L.rep[L.row_base[q] + u] = reps[q][u];
                L.node_of[L.row_base[q] + u] = q;
            }
            for (int k = 0; k < nd; ++k) {
                int64_t row = L.row_base[q] + L.nid[(size_t)q * nd + k];
                int32_t dr = p.delay[(size_t)k * nc + L.ref[q]];
                L.lo[row] = std::min(L.lo[row], dr);
                L.hi[row] = std::max(L.hi[row], dr);
            }
        }
    }

    // ---------------- stages ----------------
    uint32_t mask;
    if (d.stage_levels == SND_STAGE_NONE) {
        mask = 0;
    } else {
        if (top < 32 && (d.stage_levels >> top)) { err = "stage_levels flags a level at or above the root"; return SND_ERR_INVALID; }
        mask = d.stage_levels ? d.stage_levels : (top > 0 ? 1u : 0u);
    }
    std::vector<int> cuts;
    for (int l = 0; l < top; ++l)
        if (mask & (1u << l)) cuts.push_back(l);
    p.out_dtype = d.mode == SND_MODE_FLOAT ? SND_DT_F32 : (d.mode == SND_MODE_BINARY || d.cap <= 255 ? SND_DT_U8 : SND_DT_U16);

    p.stages.clear();
    int src = -1;
    std::vector<int> dsts = cuts;
    dsts.push_back(top);
    for (size_t si = 0; si < dsts.size(); ++si) {
        Stage S;
        S.src_level = src;
        S.dst_level = dsts[si];
        S.depth = S.dst_level - src;
        S.final_stage = si + 1 == dsts.size();
        if (S.depth > kMaxDepth) { err = "a stage spans more tree levels than supported (16); add stage_levels"; return SND_ERR_UNSUPPORTED; }
        S.src_dtype = src < 0 ? d.in_dtype : d.node_dtype;
        S.dst_dtype = S.final_stage ? p.out_dtype : d.node_dtype;
        S.src_rows = src < 0 ? nc : p.lev[src].rows;
        const Level &D = p.lev[S.dst_level];
        S.rows = S.final_stage ? nd : D.rows;
        if (S.src_rows > (int64_t)kRowMask) { err = "too many source rows for one stage"; return SND_ERR_UNSUPPORTED; }
        S.row_ptr.resize(S.rows + 1);
        S.row_len.resize(S.rows);
        S.ent.clear();
        const Level *SL = src >= 0 ? &p.lev[src] : nullptr;
        // depth-first walk of node q (at level m) down to the source level for DM k
        std::vector<int> closes_stack;
        for (int64_t row = 0; row < S.rows; ++row) {
            int k, qtop;
            int64_t base;  // time offset of the output row relative to node reference time
            if (S.final_stage) {
                k = (int)row;
                qtop = 0;
                base = p.delay[(size_t)k * nc + D.ref[0]];
                S.row_len[row] = (int32_t)p.n_out;
            } else {
                k = D.rep[row];
                qtop = D.node_of[row];
                base = D.lo[row];
                S.row_len[row] = (int32_t)(p.n_out + D.hi[row] - D.lo[row]);
            }
            S.row_ptr[row] = (uint32_t)S.ent.size();
            const int32_t *dk = &p.delay[(size_t)k * nc];
            const int64_t anchor = base - dk[D.ref[qtop]];
            // iterative DFS with an explicit stack of (level, node, next child)
            struct Fr { int l, q, next; };
            std::vector<Fr> st;
            st.push_back({S.dst_level, qtop, 0});
            while (!st.empty()) {
                Fr &f = st.back();
                const Level &L = p.lev[f.l];
                if (f.l == src + 1) {
                    if (src < 0) {
                        for (int c = L.chlo[f.q]; c < L.chhi[f.q]; ++c)
                            S.ent.push_back({(uint32_t)c, (int32_t)(anchor + dk[c])});
                    } else {
                        for (int ch = L.kidlo[f.q]; ch < L.kidhi[f.q]; ++ch) {
                            int64_t srow = SL->row_base[ch] + SL->nid[(size_t)ch * nd + k];
                            int64_t off = anchor + dk[SL->ref[ch]] - SL->lo[srow];
                            S.ent.push_back({(uint32_t)srow, (int32_t)off});
                        }
                    }
                    S.ent.back().rowc += 1u << 24;
                    st.pop_back();
                    continue;
                }
                int nk = L.kidhi[f.q] - L.kidlo[f.q];
                if (f.next < nk) {
                    int child = L.kidlo[f.q] + f.next;
                    ++f.next;
                    st.push_back({f.l - 1, child, 0});
                } else {
                    S.ent.back().rowc += 1u << 24;
                    st.pop_back();
                }
            }
        }
        S.row_ptr[S.rows] = (uint32_t)S.ent.size();
        if (S.ent.size() >= (size_t)UINT32_MAX) { err = "stage table too large"; return SND_ERR_UNSUPPORTED; }
        // bounds proof: every read index lies inside its source row
        for (int64_t row = 0; row < S.rows; ++row) {
            int64_t len = S.row_len[row];
            S.max_len = std::max(S.max_len, len);
            for (uint32_t e = S.row_ptr[row]; e < S.row_ptr[row + 1]; ++e) {
                const Entry &en = S.ent[e];
                int64_t srow = en.rowc & kRowMask;
                int64_t slen = src < 0 ? p.nsamp : (int64_t)(p.n_out + SL->hi[srow] - SL->lo[srow]);
                if (en.off < 0 || en.off + len > slen || srow >= S.src_rows || (int)(en.rowc >> 24) > S.depth) {
                    err = "internal error: stage table reads outside a source row";
                    return SND_ERR_INVALID;
                }
            }
        }
        S.pitch = S.final_stage ? 0 : round_up(S.max_len, 64);
        p.stages.push_back(std::move(S));
        src = dsts[si];
    }

    // ---------------- table image and workspace layout ----------------
    int64_t off = 0;
    for (Stage &S : p.stages) {
        S.off_row_ptr = off; off = round_up(off + (int64_t)S.row_ptr.size() * 4, 256);
        S.off_row_len = off; off = round_up(off + (int64_t)S.row_len.size() * 4, 256);
        S.off_ent = off; off = round_up(off + (int64_t)S.ent.size() * 8, 256);
    }
    p.table.assign((size_t)off, 0);
    for (Stage &S : p.stages) {
        std::memcpy(&p.table[S.off_row_ptr], S.row_ptr.data(), S.row_ptr.size() * 4);
        std::memcpy(&p.table[S.off_row_len], S.row_len.data(), S.row_len.size() * 4);
        std::memcpy(&p.table[S.off_ent], S.ent.data(), S.ent.size() * 8);
    }
    int64_t ws = 0;
    for (Stage &S : p.stages) {
        if (S.final_stage) continue;
        S.ws_off = ws;
        ws = round_up(ws + S.rows * S.pitch * dtype_size(S.dst_dtype), 256);
    }
    p.workspace_bytes = ws;

    // ---------------- info ----------------
    snd_plan_info &I = p.info;
    std::memset(&I, 0, sizeof(I));
    I.n_out = p.n_out;
    I.max_delay = p.max_delay;
    I.n_levels = nlev;
    I.n_stages = (int32_t)p.stages.size();
    I.out_dtype = p.out_dtype;
    for (int l = 0; l < nlev; ++l) {
        I.neurons_per_level[l] = p.lev[l].rows;
        I.synapses_per_level[l] = p.lev[l].synapses;
        I.nodes_per_level[l] = p.lev[l].nnodes;
        I.n_neurons += p.lev[l].rows;
        I.n_synapses += p.lev[l].synapses;
    }
    I.table_bytes = (int64_t)p.table.size();
    I.workspace_bytes = p.workspace_bytes;
    int64_t alg = 0;
    for (size_t si = 0; si < p.stages.size(); ++si) {
        Stage &S = p.stages[si];
        int64_t in_bytes;
        if (S.src_level < 0) {
            in_bytes = (int64_t)nc * p.nsamp * dtype_size(S.src_dtype);
        } else {
            const Level &SL = p.lev[S.src_level];
            in_bytes = 0;
            for (int64_t r = 0; r < SL.rows; ++r) in_bytes += (p.n_out + SL.hi[r] - SL.lo[r]);
            in_bytes *= dtype_size(S.src_dtype);
        }
        int64_t out_bytes = 0;
        for (int64_t r = 0; r < S.rows; ++r) out_bytes += S.row_len[r];
        out_bytes *= dtype_size(S.dst_dtype);
        S.alg_bytes = in_bytes + out_bytes;
        alg += S.alg_bytes;
        I.stage_alg_bytes[si] = S.alg_bytes;
        I.stage_rows[si] = S.rows;
        I.stage_entries[si] = (int64_t)S.ent.size();
    }
    I.alg_bytes = alg;
    I.build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    return SND_OK;
}

}  // namespace snd
