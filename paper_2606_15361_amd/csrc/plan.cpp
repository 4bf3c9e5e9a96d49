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
    default: return 0;  // SND_DT_BITS: less than a byte per element
    }
}

int64_t dtype_bytes(int dt, int64_t elems) { return dt == SND_DT_BITS ? (elems + 7) / 8 : elems * dtype_size(dt); }

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
    if (mode == SND_MODE_BINARY)
        return (in_dt == SND_DT_U8 && (node_dt == SND_DT_U8 || node_dt == SND_DT_BITS)) ||
               (in_dt == SND_DT_BITS && node_dt == SND_DT_BITS);
    if (mode == SND_MODE_GRADED)
        return in_dt == SND_DT_U8 && (node_dt == SND_DT_U16 || (node_dt == SND_DT_U8 && cap <= 255));
    if (mode == SND_MODE_FLOAT) {
        auto f = [](int d) { return d == SND_DT_F32 || d == SND_DT_BF16 || d == SND_DT_F16; };
        return f(in_dt) && f(node_dt);
    }
    return false;
}

// Final stage in LDS groups: kGroupRows rows (DMs adjacent in value) per workgroup share one
// staged window per distinct source row of each entry.  Every row of the final stage walks the
// same tree, so all rows have the same entry count and closing pattern.  Returns false (and
// leaves the stage on the generic kernel) when one entry alone does not fit the LDS budget.
// Variants: kGroupGeneric (any tree), kGroupFast (regular level-1 nodes, compile-time depth),
// kGroupLin (float mode: every row is one sum over its inputs, with no activation in between),
// kGroupPack (graded mode on u8 rows with regular level-1 nodes of 4 or 8 inputs: the linear
// kernel's staging, levels formed on pairs of 16-bit counts).
enum { kGroupGeneric = 0, kGroupFast = 1, kGroupLin = 2, kGroupPack = 3 };
bool build_group_lds(const PlanImpl &p, Stage &S, int variant)
{
    const bool allow_fast = variant == kGroupFast || variant == kGroupPack;
    const bool lin = variant == kGroupLin;
    const bool pack = variant == kGroupPack;
    const bool tab = lin || pack;  // kernels that copy by chunk tables and read offset words from LDS
    // these kernels read a materialised plane of f32, bf16 or f16 rows (linear) or u8 rows
    // (packed), whose pitch their copy table holds; the packed kernel's 16-bit counts hold any
    // level sum (fan-in x cap < 2^16)
    int64_t src_pitch = 0;
    if (tab) {
        const bool ok_src = S.src_dtype == SND_DT_F32 || S.src_dtype == SND_DT_BF16 || S.src_dtype == SND_DT_F16;
        if (lin && !(p.desc.mode == SND_MODE_FLOAT && ok_src && S.dst_dtype == SND_DT_F32)) return false;
        if (pack && !(p.desc.mode == SND_MODE_GRADED && S.src_dtype == SND_DT_U8 && S.dst_dtype == SND_DT_U8 &&
                      p.desc.cap <= 255 && (int64_t)p.desc.branching * p.desc.cap < 65536))
            return false;
        if (S.src_level < 0) return false;
        for (const Stage &Q : p.stages)
            if (!Q.final_stage && Q.dst_level == S.src_level) src_pitch = Q.pitch;
        const int64_t epu = 16 / dtype_size(S.src_dtype);  // elements per 16-byte unit
        if (src_pitch <= 0 || src_pitch % epu != 0 || (S.src_rows * src_pitch) / epu >= (int64_t(1) << 32))
            return false;
    }
    const int64_t rows = S.rows;
    if (rows < 1) return false;
    const int32_t ne = (int32_t)(S.row_ptr[1] - S.row_ptr[0]);
    for (int64_t r = 0; r < rows; ++r) {
        if ((int32_t)(S.row_ptr[r + 1] - S.row_ptr[r]) != ne || S.row_len[r] != S.row_len[0]) return false;
        for (int32_t e = 0; e < ne; ++e)
            if ((S.ent[S.row_ptr[r] + e].rowc >> 24) != (S.ent[e].rowc >> 24)) return false;
    }
    // Regular level-1 nodes (every f1-th input closes a node, nothing else does) allow the
    // specialised kernel, which sums each level-1 node's inputs directly.
    int32_t f1 = 0;
    {
        int32_t first = -1;
        for (int32_t e = 0; e < ne && first < 0; ++e)
            if ((S.ent[e].rowc >> 24) >= 1) first = e;
        f1 = first + 1;
        bool reg = f1 > 0 && ne % f1 == 0;
        for (int32_t e = 0; e < ne && reg; ++e)
            if (((S.ent[e].rowc >> 24) >= 1) != ((e + 1) % f1 == 0)) reg = false;
        if (!allow_fast || !reg || !group_fast_supported(f1, S.depth) ||
            !group_fast_types(p.desc.mode, S.src_dtype, S.dst_dtype))
            f1 = 0;
    }
    if (lin) f1 = 0;
    if (pack && !((f1 == 4 && S.depth <= 5) || (f1 == 8 && S.depth <= 4))) return false;
    const bool bits = S.src_dtype == SND_DT_BITS;
    if (bits && !f1) return false;  // bit rows: specialised kernel only
    // samples a window holds beyond its span (its tile, plus one unit for the linear kernel on
    // 16-bit rows), and the tile step in time
    const int tile = lin    ? lin_cover(S.src_dtype)
                     : pack ? pack_tile(f1, S.depth) + 16
                     : bits ? kGroupTileBits
                     : f1   ? kGroupTileFast
                            : kGroupTile;
    const int tile_step = lin ? lin_tile(S.src_dtype) : pack ? pack_tile(f1, S.depth) : tile;
    const int rpw = lin ? lin_rows(S.src_dtype) : pack ? pack_rows(f1, S.depth) : f1 ? kFastRows : 1;  // rows per wave
    const int max_entries = lin ? lin_max_batch_entries(S.src_dtype) : kPackMaxBatchEntries;  // table kernels
    const int n_words = lin ? kLinWords : kPackWords;
    const int n_smem = lin ? kLinSmemWords : kPackSmemWords;
    const int gr = kGroupRows * rpw;     // rows per group
    const int unit = f1 ? f1 : 1;  // batches end on level-1 node boundaries
    const int eb = bits ? 1 : 8 * dtype_size(S.src_dtype);  // bits per element
    // LDS bytes per batch buffer, less the share the caller's tune word gives up
    const int64_t full_budget = lin ? kLinLdsBytes : pack ? kPackLdsBytes : f1 ? kGroupFastLdsBytes : kGroupLdsBytes;
    const int64_t budget = full_budget * (4 - (int64_t)((p.desc.tune >> 8) & 15u)) / 4 * 8 / eb;
    const int32_t epd = 128 / eb;  // elements per 16-byte copy unit
    // LDS elements of one window: its span plus one tile, from a 16-byte boundary, whole units
    // (bit rows: one more unit, since a lane reads the word after its 32 samples too)
    auto slot_elems = [&](int32_t lo, int32_t span) {
        return (int64_t)round_up((int64_t)(lo % epd) + span + tile, epd) + (bits ? epd : 0);
    };
    std::vector<int32_t> order(rows);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return p.dm[a] < p.dm[b]; });
    const int64_t ng = (rows + gr - 1) / gr;
    std::vector<int32_t> grp_rows((size_t)(ng * gr), -1);
    for (int64_t i = 0; i < rows; ++i) grp_rows[(size_t)i] = order[(size_t)i];
    std::vector<int32_t> batch_ptr(1, 0), batches, slots;
    std::vector<uint32_t> ldsb((size_t)(ng * gr * ne), 0);
    // row w of group g (wave w / rpw, row w % rpw of that wave) at entry e
    auto ldsb_at = [&](int64_t g, int w, int32_t e) -> uint32_t & {
        return ldsb[(size_t)((((g * kGroupRows + w / rpw) * ne) + e) * rpw + w % rpw)];
    };
    int64_t max_elems = 0;
    const int32_t max_slots = kGroupRows * kGroupSlotsPerWave;
    // windows of one entry: the group's (source row, offset) reads, clustered per source row
    // so that each window spans at most kGroupMaxSpan offsets
    struct Rd { uint32_t row; int32_t off; int w; };
    struct Src { uint32_t row; int32_t lo, hi; };
    std::vector<Rd> rd;
    std::vector<Src> srcs;
    std::vector<int32_t> slot_of(gr);
    std::vector<Src> unit_srcs;
    std::vector<int32_t> unit_nsrc;
    // table kernels: copy chunks of the open batch
    int32_t batch_chunks = 0;
    auto lin_chunks = [&](const Src &s) {  // 64-unit copies of one window in a full tile
        const int64_t units = ((int64_t)(s.lo % epd) + (s.hi - s.lo) + tile + epd - 1) / epd;
        return (int32_t)((units + 63) / 64);
    };
    for (int64_t g = 0; g < ng; ++g) {
        int32_t e0 = 0, s0 = (int32_t)(slots.size() / 4);
        int64_t elems = 0;
        batch_chunks = 0;
        for (int32_t eu = 0; eu < ne; eu += unit) {
        // windows of every input of this unit, then one decision where the batch ends
        unit_srcs.clear();
        unit_nsrc.clear();
        std::vector<std::vector<int32_t>> unit_slot_of;
        for (int32_t e = eu; e < eu + unit; ++e) {
            rd.clear();
            for (int w = 0; w < gr; ++w) {
                const int32_t r = grp_rows[(size_t)(g * gr + w)];
                if (r < 0) continue;
                const Entry &en = S.ent[S.row_ptr[r] + e];
                rd.push_back({en.rowc & kRowMask, en.off, w});
            }
            std::sort(rd.begin(), rd.end(), [](const Rd &a, const Rd &b) {
                return a.row != b.row ? a.row < b.row : a.off < b.off;
            });
            srcs.clear();
            for (const Rd &x : rd) {
                if (srcs.empty() || srcs.back().row != x.row || x.off - srcs.back().lo > kGroupMaxSpan)
                    srcs.push_back({x.row, x.off, x.off});
                srcs.back().hi = x.off;
                slot_of[x.w] = (int32_t)srcs.size() - 1;
            }
            unit_nsrc.push_back((int32_t)srcs.size());
            unit_srcs.insert(unit_srcs.end(), srcs.begin(), srcs.end());
            unit_slot_of.push_back(slot_of);
        }
        int64_t need = 0;
        for (const Src &s : unit_srcs) need += slot_elems(s.lo, s.hi - s.lo);
        if (need > budget || (int32_t)unit_srcs.size() > max_slots) return false;
        const int32_t nslot_batch = (int32_t)(slots.size() / 4) - s0;
        bool lin_full = false;
        int32_t unit_chunks = 0;
        if (tab) {  // the batch's entries or the waves' copy chunks would overflow
            for (const Src &s : unit_srcs) unit_chunks += lin_chunks(s);
            if (unit_chunks > kGroupRows * kLinMaxChunks) return false;
            lin_full = batch_chunks + unit_chunks > kGroupRows * kLinMaxChunks || eu - e0 + unit > max_entries;
        }
        if (elems + need > budget || nslot_batch + (int32_t)unit_srcs.size() > max_slots || lin_full) {
            // close the batch
            batches.insert(batches.end(), {e0, eu, s0, (int32_t)(slots.size() / 4)});
            max_elems = std::max(max_elems, elems);
            e0 = eu;
            s0 = (int32_t)(slots.size() / 4);
            elems = 0;
            batch_chunks = 0;
        }
        batch_chunks += unit_chunks;
        size_t si0 = 0;
        for (int32_t e = eu; e < eu + unit; ++e) {
            const int32_t ns = unit_nsrc[(size_t)(e - eu)];
            std::vector<int32_t> slot_lds((size_t)ns);
            for (int32_t i = 0; i < ns; ++i) {
                const Src &sr = unit_srcs[si0 + (size_t)i];
                // 16-byte aligned footprint; the window starts `head` elements into it so that
                // the kernel can copy whole 16-byte units from the (16-byte aligned) source row
                const int32_t head = sr.lo % epd;
                slot_lds[(size_t)i] = (int32_t)elems + head;
                slots.insert(slots.end(), {(int32_t)sr.row, sr.lo, sr.hi - sr.lo, slot_lds[(size_t)i]});
                elems += slot_elems(sr.lo, sr.hi - sr.lo);
            }
            const std::vector<int32_t> &so = unit_slot_of[(size_t)(e - eu)];
            const uint32_t closes = S.ent[e].rowc & ~kRowMask;  // identical for every row
            for (int w = 0; w < gr; ++w) {
                const int32_t r = grp_rows[(size_t)(g * gr + w)];
                if (r < 0) {
                    ldsb_at(g, w, e) = closes;  // padding rows read offset 0 of the buffer; never stored
                    continue;
                }
                const Entry &en = S.ent[S.row_ptr[r] + e];
                const Src &sr = unit_srcs[si0 + (size_t)so[(size_t)w]];
                const uint32_t base = (uint32_t)(slot_lds[(size_t)so[(size_t)w]] + (en.off - sr.lo));
                ldsb_at(g, w, e) = base | closes;
            }
            si0 += (size_t)ns;
        }
        }
        batches.insert(batches.end(), {e0, ne, s0, (int32_t)(slots.size() / 4)});
        max_elems = std::max(max_elems, elems);
        batch_ptr.push_back((int32_t)(batches.size() / 4));
    }
    if (max_elems > budget || max_elems >= (1 << 24)) return false;
    // Copy descriptors of the staged windows, in the batches' slot order: (source row, element
    // offset of the window's 16-byte aligned footprint, LDS byte offset of the footprint,
    // elements from the footprint start to the window end without the tile, i.e. head + span).
    std::vector<int32_t> instrs;
    instrs.reserve(slots.size());
    for (size_t si = 0; si < slots.size(); si += 4) {
        const int32_t srow = slots[si], lo = slots[si + 1], span = slots[si + 2], lofs = slots[si + 3];
        if (lo < 0) return false;
        const int32_t head = lo % epd;
        instrs.insert(instrs.end(), {srow, lo - head, (int32_t)((int64_t)(lofs - head) * eb / 8), head + span});
    }
    std::vector<uint32_t> lin_tab, lin_smem;
    static_assert(lin_max_batch_entries(SND_DT_F32) <= 15 && lin_max_batch_entries(SND_DT_BF16) <= 15 &&
                      lin_rows(SND_DT_BF16) * 4 <= 32,
                  "per-row input counts are packed in 4 bits, one word per wave");
    static_assert(kPackMaxBatchEntries / 4 <= 16 && kPackRowsMax <= 4, "packed kernel: two closes words, 16-byte words");
    if (tab) {
        // per (batch, wave) the offset words of the wave's rows, and its copy chunks as scalar words
        const int64_t nb_all = (int64_t)(batches.size() / 4);
        lin_tab.assign((size_t)(nb_all * kGroupRows * n_words), 0u);
        lin_smem.assign((size_t)(nb_all * kGroupRows * n_smem), 0u);
        for (int64_t g = 0; g < ng; ++g) {
            for (int32_t b = batch_ptr[(size_t)g]; b < batch_ptr[(size_t)g + 1]; ++b) {
                const int32_t ex = batches[4 * (size_t)b], ey = batches[4 * (size_t)b + 1];
                const int32_t bz = batches[4 * (size_t)b + 2], bw = batches[4 * (size_t)b + 3];
                const int32_t n = ey - ex;
                if (n > max_entries) return false;
                for (int w = 0; w < kGroupRows; ++w) {
                    uint32_t *words = &lin_tab[(size_t)((b * kGroupRows + w) * n_words)];
                    uint32_t *sm = &lin_smem[(size_t)((b * kGroupRows + w) * n_smem)];
                    if (pack) {  // lane i, component q: input i of row q; then each node's closes
                        for (int q = 0; q < rpw; ++q) {
                            const int32_t r = grp_rows[(size_t)(g * gr + w * rpw + q)];
                            for (int32_t e = ex; e < ey && r >= 0; ++e)
                                words[4 * (e - ex) + q] = ldsb_at(g, w * rpw + q, e) & kRowMask;
                        }
                        for (int32_t k = 0; k < n / f1; ++k) {
                            const uint32_t c = S.ent[ex + k * f1 + f1 - 1].rowc >> 24;
                            if (c > 15) return false;
                            sm[22 + k / 8] |= c << (4 * (k % 8));
                        }
                        sm[n_smem - 1] = (uint32_t)n;
                        continue;
                    }
                    uint32_t even = 0;  // 16-bit rows: inputs starting a dword first, counts per row
                    for (int q = 0; q < rpw; ++q) {
                        const int32_t r = grp_rows[(size_t)(g * gr + w * rpw + q)];
                        int k = 0;
                        for (int ph = 0; ph < (eb == 16 ? 2 : 1); ++ph) {
                            for (int32_t e = ex; e < ey && r >= 0; ++e) {
                                const uint32_t o = (ldsb_at(g, w * rpw + q, e) & kRowMask) * (uint32_t)(eb / 8);
                                if (eb == 16 && (int)((o >> 1) & 1u) != ph) continue;
                                words[q * n + k++] = o;
                            }
                            if (ph == 0) even |= (uint32_t)k << (4 * q);
                        }
                    }
                    sm[n_smem - 2] = even;
                    sm[n_smem - 1] = (uint32_t)n;
                }
                // copy chunks of the batch's windows for a full tile, dealt to the waves in turn
                int32_t j = 0;
                for (int32_t si = bz; si < bw; ++si) {
                    const int32_t srow = slots[4 * (size_t)si], lo = slots[4 * (size_t)si + 1];
                    const int32_t span = slots[4 * (size_t)si + 2], lofs = slots[4 * (size_t)si + 3];
                    const int32_t head = lo % epd;
                    const int64_t units = ((int64_t)head + span + tile + epd - 1) / epd;
                    const int64_t unit0 = ((int64_t)srow * src_pitch + lo - head) / epd;
                    const int64_t lds0 = (int64_t)(lofs - head) * (eb / 8);
                    for (int64_t u0 = 0; u0 < units; u0 += 64, ++j) {
                        const int w = j % kGroupRows, c = j / kGroupRows;
                        if (c >= kLinMaxChunks) return false;
                        const int64_t nu = std::min<int64_t>(64, units - u0);
                        uint32_t *sm = &lin_smem[(size_t)((b * kGroupRows + w) * n_smem)];
                        sm[0] = (uint32_t)(c + 1);
                        sm[1 + c] = (uint32_t)(unit0 + u0);
                        sm[1 + kLinMaxChunks + c] = (uint32_t)(lds0 + 16 * u0);
                        sm[1 + 2 * kLinMaxChunks + c] = (uint32_t)nu;
                    }
                }
            }
        }
    }
    S.kernel = kKernelGroupLds;
    S.ngroups = ng;
    {  // workgroups dealt per XCD and time tile: an eighth of the groups, or the tune word's
        const uint32_t x = (p.desc.tune >> 4) & 15u;
        S.xcd_chunk = x ? (1 << (x - 1)) : (ng >= 8 ? (int32_t)(ng / 8) : 1);
    }
    S.n_entries = ne;
    S.group_f1 = f1;
    S.group_tile = tile_step;
    S.group_rpw = rpw;
    S.group_lin = lin;
    S.group_pack = pack;
    const int64_t buf_bytes = round_up(max_elems * eb / 8, 16);
    S.lds_buf_elems = (int32_t)(buf_bytes * 8 / eb);
    // general kernel: batches b+1, b+2 land while b is read; the others: b+1
    S.lds_bytes = (int32_t)(lin    ? kLinBuffers * (buf_bytes + kLinWordBytes)
                            : pack ? 2 * (buf_bytes + kPackWordBytes)
                                   : (f1 ? kFastBuffers : kGroupBuffers) * buf_bytes);
    S.grp_rows = std::move(grp_rows);
    S.batch_ptr = std::move(batch_ptr);
    S.batches = std::move(batches);
    S.slots = std::move(slots);
    S.instrs = std::move(instrs);
    if (f1) {
        // specialised kernel: LDS byte offsets without the closing counts, which are the same for
        // every row and kept once per level-1 node
        // (bit rows: byte offset of the word holding the first sample | bit offset << 27)
        for (uint32_t &w : ldsb) {
            const uint32_t o = w & kRowMask;
            w = bits ? ((o >> 5) << 2) | ((o & 31u) << 27) : o * (uint32_t)(eb / 8);
        }
        S.node_closes.resize((size_t)(ne / f1));
        for (int32_t k = 0; k < ne / f1; ++k) S.node_closes[(size_t)k] = (int32_t)(S.ent[k * f1 + f1 - 1].rowc >> 24);
    }
    if (tab) ldsb.clear();  // the table kernels read their own tables
    S.ldsb = std::move(ldsb);
    S.lin = std::move(lin_tab);
    S.lin_smem = std::move(lin_smem);
    return true;
}

// First stage anchored on the input: one workgroup per (node, window of reference samples)
// stages the node's channels once and produces the overlapping segment of every neuron row of
// that node.  Needs all entries of a node's rows to read that node's channels and the node's
// staged window to fit the LDS budget.  The window is the largest of 2048, 1024 or 512 samples
// whose staging keeps four workgroups on a CU (512 only needs the hard LDS limit).
bool build_anchored(const PlanImpl &p, Stage &S)
{
    const Level &D = p.lev[S.dst_level];
    const int es = dtype_size(S.src_dtype);
    const bool bits = S.src_dtype == SND_DT_BITS;
    if (S.depth > (bits ? 1 : 8)) return false;
    struct NodeSpan { int64_t r0, r1; int32_t c0, c1, rho_max; int64_t tlo, thi; };
    std::vector<NodeSpan> ns;
    int64_t worst = 0;  // largest (channels, rho_max) LDS footprint beyond the window itself
    int64_t chan_max = 0;
    for (int q = 0; q < D.nnodes; ++q) {
        NodeSpan n{D.row_base[q], D.row_base[q] + D.nneu[q], D.chlo[q], D.chhi[q], 0, INT64_MAX, INT64_MIN};
        for (int64_t r = n.r0; r < n.r1; ++r) {
            for (uint32_t e = S.row_ptr[r]; e < S.row_ptr[r + 1]; ++e) {
                const int32_t c = (int32_t)(S.ent[e].rowc & kRowMask);
                const int32_t rho = S.ent[e].off - D.lo[r];
                if (c < n.c0 || c >= n.c1 || rho < 0) return false;
                n.rho_max = std::max(n.rho_max, rho);
            }
            n.tlo = std::min<int64_t>(n.tlo, D.lo[r]);
            n.thi = std::max<int64_t>(n.thi, D.lo[r] + S.row_len[r]);
        }
        if (bits && n.tlo % 64 != 0) return false;
        worst = std::max<int64_t>(worst, (int64_t)(n.c1 - n.c0) * n.rho_max);
        chan_max = std::max<int64_t>(chan_max, n.c1 - n.c0);
        ns.push_back(n);
    }
    // bit input: leaf level only, tiles of kAnchorTileBits from 64-aligned row anchors
    int tile = bits ? kAnchorTileBits : kAnchorTile;
    const int forced = (int)(p.desc.tune & 15u);  // a window chosen by the caller (tuning)
    if (!bits && forced) {
        tile = kAnchorTile << (forced - 1);
    } else if (!bits) {
        for (int t = kAnchorMaxTile; t > kAnchorTile; t /= 2)
            if ((chan_max * t + worst) * es <= kAnchorLdsTarget) { tile = t; break; }
    }
    std::vector<int32_t> nodes, tiles;
    int64_t lds_max = 0;
    for (const NodeSpan &n : ns) {
        const int64_t lds = bits ? (int64_t)(n.c1 - n.c0) * anchor_bits_words(n.rho_max) * 4
                                 : (int64_t)(n.c1 - n.c0) * (tile + n.rho_max) * es;
        if (lds > kAnchorLdsBytes) return false;
        lds_max = std::max(lds_max, lds);
        const int32_t ni = (int32_t)(nodes.size() / 6);
        // last field: how far the node's rows reach past n_out, so that a run with fewer output
        // samples can skip the tiles it does not need
        nodes.insert(nodes.end(), {(int32_t)n.r0, (int32_t)n.r1, n.c0, n.c1, n.rho_max, (int32_t)(n.thi - p.n_out)});
        for (int64_t t = n.tlo; t < n.thi; t += tile) tiles.insert(tiles.end(), {ni, (int32_t)t});
    }
    S.anchor_tile = tile;
    S.kernel = kKernelAnchored;
    S.lds_bytes = (int32_t)round_up(lds_max, 16);
    S.nodes = std::move(nodes);
    S.ntiles = (int64_t)(tiles.size() / 2);
    S.tiles = std::move(tiles);
    S.row_lo.assign(D.lo.begin(), D.lo.end());
    return true;
}

}  // namespace

snd_status build_plan(const snd_plan_desc &d, PlanImpl &p, std::string &err)
{
    auto t_start = std::chrono::steady_clock::now();
    // ---------------- validation ----------------
    if (d.nchan < 1 || !d.freq_mhz || d.ndm < 1 || !d.dm || !(d.tsamp_s > 0.0) || (d.chunk <= 0 && d.nsamp < 1) ||
        d.chunk < 0) {
        err = "nchan, ndm, nsamp (or chunk) must be >= 1, tsamp_s > 0 and freq/dm non-null";
        return SND_ERR_INVALID;
    }
    for (int i = 0; i < 5; ++i)
        if (d.reserved[i]) { err = "reserved descriptor fields must be zero"; return SND_ERR_INVALID; }
    if ((d.tune & ~0xfffu) || (d.tune & 15u) > 4 || ((d.tune >> 4) & 15u) > 7 || ((d.tune >> 8) & 15u) > 3) {
        err = "unknown tune bits";
        return SND_ERR_INVALID;
    }
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
    if (d.in_dtype == SND_DT_BITS && d.cluster > 15) {
        err = "bit input needs cluster <= 15";
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
    if (d.chunk > 0) p.nsamp = p.desc.nsamp = dmax + d.chunk;
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

    // Every leaf row (below a root) starts on a 64-sample boundary (its anchor moves down by at
    // most 63 samples): the leaf stage's stores of a row are then whole 256-byte (f32) or
    // 128-byte (16-bit) lines, and bit rows are written in whole words.
    const bool bits = d.node_dtype == SND_DT_BITS;
    if (bits && (top < 1 || d.generic_kernels || (d.stage_levels != 0 && d.stage_levels != 1u))) {
        err = "bit rows need the default schedule (leaf level materialised) and the staged kernels";
        return SND_ERR_UNSUPPORTED;
    }
    if (top >= 1)
        for (int32_t &v : p.lev[0].lo) v -= v % 64;

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
        // row pitch in elements: 64, or 128 bits (16 bytes) for bit rows
        S.pitch = S.final_stage ? 0 : round_up(S.max_len, S.dst_dtype == SND_DT_BITS ? 128 : 64);
        p.stages.push_back(std::move(S));
        src = dsts[si];
    }

    // ---------------- kernel choice per stage ----------------
    for (Stage &S : p.stages) {
        S.kernel = kKernelGeneric;
        if (d.generic_kernels) continue;
        if (S.final_stage && (build_group_lds(p, S, kGroupLin) || build_group_lds(p, S, kGroupPack) ||
                              build_group_lds(p, S, kGroupFast) || (!bits && build_group_lds(p, S, kGroupGeneric))))
            continue;
        if (!S.final_stage && S.src_level < 0 && !build_anchored(p, S) && (d.tune & 15u)) {
            err = "the requested leaf-stage window does not fit the LDS";
            return SND_ERR_UNSUPPORTED;
        }
    }
    if (bits && (p.stages.size() != 2 || p.stages[0].kernel != kKernelAnchored ||
                 p.stages[1].kernel != kKernelGroupLds)) {
        err = "bit rows need level-1 nodes of equal fan-in (2, 4 or 8) and a leaf stage that fits the staged kernels";
        return SND_ERR_UNSUPPORTED;
    }

    // ---------------- table image and workspace layout ----------------
    int64_t off = 0;
    auto reserve = [&](int64_t bytes) {
        int64_t o = off;
        off = round_up(off + bytes, 256);
        return o;
    };
    for (Stage &S : p.stages) {
        S.off_row_ptr = reserve((int64_t)S.row_ptr.size() * 4);
        S.off_row_len = reserve((int64_t)S.row_len.size() * 4);
        S.off_ent = reserve((int64_t)S.ent.size() * 8);
        S.off_grp_rows = reserve((int64_t)S.grp_rows.size() * 4);
        S.off_batch_ptr = reserve((int64_t)S.batch_ptr.size() * 4);
        S.off_batches = reserve((int64_t)S.batches.size() * 4);
        S.off_instrs = reserve((int64_t)S.instrs.size() * 4);
        S.off_ldsb = reserve((int64_t)S.ldsb.size() * 4);
        S.off_node_closes = reserve((int64_t)S.node_closes.size() * 4);
        S.off_lin = reserve((int64_t)S.lin.size() * 4);
        S.off_lin_smem = reserve((int64_t)S.lin_smem.size() * 4);
        S.off_nodes = reserve((int64_t)S.nodes.size() * 4);
        S.off_tiles = reserve((int64_t)S.tiles.size() * 4);
        S.off_row_lo = reserve((int64_t)S.row_lo.size() * 4);
    }
    p.table.assign((size_t)off, 0);
    auto put = [&](int64_t o, const void *src, size_t bytes) {
        if (bytes) std::memcpy(&p.table[(size_t)o], src, bytes);
    };
    for (Stage &S : p.stages) {
        put(S.off_row_ptr, S.row_ptr.data(), S.row_ptr.size() * 4);
        put(S.off_row_len, S.row_len.data(), S.row_len.size() * 4);
        put(S.off_ent, S.ent.data(), S.ent.size() * 8);
        put(S.off_grp_rows, S.grp_rows.data(), S.grp_rows.size() * 4);
        put(S.off_batch_ptr, S.batch_ptr.data(), S.batch_ptr.size() * 4);
        put(S.off_batches, S.batches.data(), S.batches.size() * 4);
        put(S.off_instrs, S.instrs.data(), S.instrs.size() * 4);
        put(S.off_ldsb, S.ldsb.data(), S.ldsb.size() * 4);
        put(S.off_node_closes, S.node_closes.data(), S.node_closes.size() * 4);
        put(S.off_lin, S.lin.data(), S.lin.size() * 4);
        put(S.off_lin_smem, S.lin_smem.data(), S.lin_smem.size() * 4);
        put(S.off_nodes, S.nodes.data(), S.nodes.size() * 4);
        put(S.off_tiles, S.tiles.data(), S.tiles.size() * 4);
        put(S.off_row_lo, S.row_lo.data(), S.row_lo.size() * 4);
    }
    int64_t ws = 0;
    for (Stage &S : p.stages) {
        if (S.final_stage) continue;
        S.ws_off = ws;
        ws = round_up(ws + dtype_bytes(S.dst_dtype, S.rows * S.pitch), 256);
    }
    // a graded u8 leaf plane read by the packed final stage: one bound word per leaf workgroup
    // and the reduced one after them
    p.bound_off = -1;
    p.bound_n = 0;
    if (p.stages.size() == 2 && p.stages[0].kernel == kKernelAnchored && p.stages[0].dst_dtype == SND_DT_U8 &&
        p.desc.mode == SND_MODE_GRADED && p.stages[1].kernel == kKernelGroupLds && p.stages[1].group_pack &&
        p.stages[0].ntiles > 0) {
        p.bound_off = ws;
        p.bound_n = p.stages[0].ntiles;
        ws = round_up(ws + 4 * (p.bound_n + 1), 256);
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
            in_bytes = dtype_bytes(S.src_dtype, (int64_t)nc * p.nsamp);
        } else {
            const Level &SL = p.lev[S.src_level];
            in_bytes = 0;
            for (int64_t r = 0; r < SL.rows; ++r) in_bytes += (p.n_out + SL.hi[r] - SL.lo[r]);
            in_bytes = dtype_bytes(S.src_dtype, in_bytes);
        }
        int64_t out_bytes = 0;
        for (int64_t r = 0; r < S.rows; ++r) out_bytes += S.row_len[r];
        out_bytes = dtype_bytes(S.dst_dtype, out_bytes);
        S.alg_bytes = in_bytes + out_bytes;
        alg += S.alg_bytes;
        I.stage_alg_bytes[si] = S.alg_bytes;
        I.stage_rows[si] = S.rows;
        I.stage_entries[si] = (int64_t)S.ent.size();
        I.stage_kernel[si] = S.kernel == kKernelGroupLds && S.group_pack                   ? 7
                             : S.kernel == kKernelGroupLds && S.group_lin                  ? 6
                             : S.kernel == kKernelAnchored && S.src_dtype == SND_DT_BITS ? 5
                             : S.kernel == kKernelGroupLds && S.src_dtype == SND_DT_BITS ? 4
                             : (S.kernel == kKernelGroupLds && S.group_f1 > 0) ? 3
                                                                                : S.kernel;
        if (S.kernel == kKernelGroupLds) {
            int64_t staged = 0;
            for (size_t i = 0; i < S.slots.size(); i += 4) staged += S.slots[i + 2] + S.group_tile;
            I.stage_staged[si] = staged;
            I.stage_batches[si] = (int64_t)(S.batches.size() / 4);
            I.stage_windows[si] = (int64_t)(S.slots.size() / 4);
        }
    }
    I.alg_bytes = alg;
    I.build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    return SND_OK;
}

}  // namespace snd
