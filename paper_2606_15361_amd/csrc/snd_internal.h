// Internal declarations shared by the plan builder, the C ABI and the HIP kernels.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "snd.h"

namespace snd {

// Dispersion constant in MHz^2 ms per (pc cm^-3) (Methods, "Incoherent dedispersion").
constexpr double kDM = 4.148808e6;
// Deepest sub-tree one kernel stage evaluates in registers.
constexpr int kMaxDepth = 16;
// Source rows addressable by a table entry (low 24 bits of Entry::rowc).
constexpr uint32_t kRowMask = 0x00FFFFFFu;

// One input of a stage output row: source row (low 24 bits), the number of sub-tree levels
// that complete after this input (high 8 bits), and the time offset into the source row.
struct Entry {
    uint32_t rowc;
    int32_t off;
};

// Kernel stage: every output row is the value of one tree node's neuron (or, in the final
// stage, of the root for one DM), computed from rows of a lower materialised level (or the
// input channels) by evaluating the sub-tree between them in registers.
struct Stage {
    int src_level = -1;      // -1 = input channels
    int dst_level = 0;       // tree level computed by this stage
    int depth = 1;           // dst_level - src_level
    bool final_stage = false;
    int64_t rows = 0;
    int64_t max_len = 0;     // longest output row (samples)
    int64_t pitch = 0;       // output pitch in elements (non-final stages)
    int src_dtype = 0, dst_dtype = 0;
    int64_t src_rows = 0;
    std::vector<uint32_t> row_ptr;  // rows + 1
    std::vector<int32_t> row_len;   // samples computed per output row
    std::vector<Entry> ent;
    int64_t off_row_ptr = 0, off_row_len = 0, off_ent = 0;  // byte offsets in the table image
    int64_t ws_off = 0;            // byte offset of the output plane in the workspace
    int64_t alg_bytes = 0;

    // Kernel chosen for the stage.
    int kernel = 0;  // kKernelGeneric, kKernelGroupLds or kKernelAnchored

    // kKernelGroupLds: rows in groups of kGroupRows sharing LDS-staged source windows.
    int64_t ngroups = 0;
    int32_t n_entries = 0;          // entries per row (identical for every row)
    int32_t lds_bytes = 0;          // dynamic LDS per workgroup
    int32_t lds_buf_elems = 0;      // elements per LDS buffer (group kernel)
    int32_t group_f1 = 0;           // inputs per level-1 node when regular (specialised kernel), else 0
    int32_t group_tile = 0;         // time samples per workgroup
    int32_t xcd_chunk = 1;          // DM groups of one time tile dealt to each XCD in turn
    int32_t group_rpw = 1;          // rows per wave (kFastRows for the specialised kernel)
    std::vector<int32_t> grp_rows;  // [ngroups * kGroupRows * rows per wave], -1 = padding
    std::vector<int32_t> batch_ptr; // [ngroups + 1] into batches
    std::vector<int32_t> batches;   // 4 ints per batch: entry begin, entry end, window begin, window end
    std::vector<int32_t> slots;     // 4 ints per staged window: source row, start offset, span, LDS element
                                    // offset (host only: plan statistics)
    std::vector<int32_t> instrs;    // 4 ints per staged window, as copied: source row, element offset of
                                    // its 16-byte aligned footprint, LDS byte offset of the footprint,
                                    // head + span (elements from the footprint start, tile excluded)
    std::vector<uint32_t> ldsb;     // [ngroups][kGroupRows][n_entries][rows per wave]: LDS element offset |
                                    // closes << 24 (general kernel) or LDS byte offset (specialised kernel)
    std::vector<int32_t> node_closes;  // specialised kernel: levels completed by each level-1 node
    // Linear kernel (float mode: the final stage is one sum over its inputs, no activation).  Per
    // (global batch index, wave): kLinWords offset words, copied to LDS with the batch: words
    // q * n .. q * n + n - 1 are the LDS byte offsets of the first samples of the n inputs of the
    // wave's row q (16-bit rows: those that start a dword first, each part in plan order); and
    // kLinSmemWords words read as scalars: the number of copy chunks of the wave, then for its
    // chunks (global -> LDS copies of up to 64 16-byte units) the source unit index from the
    // plane start, the LDS byte offset and the unit count, then (16-bit rows) the count of each
    // row's inputs that start a dword (4 bits per row), and last n.  The packed kernel keeps its
    // tables (kPackWords and kPackSmemWords per batch and wave) in the same two vectors.
    bool group_lin = false;
    bool group_pack = false;
    std::vector<uint32_t> lin;
    std::vector<uint32_t> lin_smem;
    int64_t off_grp_rows = 0, off_batch_ptr = 0, off_batches = 0, off_instrs = 0, off_ldsb = 0;
    int64_t off_node_closes = 0, off_lin = 0, off_lin_smem = 0;

    // kKernelAnchored: one workgroup per (node, window of anchor_tile reference samples).
    std::vector<int32_t> nodes;     // 6 ints per node: row begin, row end, channel begin, channel end, rho max,
                                    // reach of its rows past n_out
    std::vector<int32_t> tiles;     // 2 ints per workgroup: node index, window start
    std::vector<int32_t> row_lo;    // [rows]
    int32_t anchor_tile = 0;        // reference samples per workgroup window
    int64_t off_nodes = 0, off_tiles = 0, off_row_lo = 0;
    int64_t ntiles = 0;
};

constexpr int kKernelGeneric = 0;
constexpr int kKernelGroupLds = 1;
constexpr int kKernelAnchored = 2;
constexpr int kGroupRows = 16;       // rows (waves) per LDS-group workgroup
constexpr int kGroupTile = 256;      // time samples per LDS-group workgroup
constexpr int kGroupLdsBytes = 20480;  // per LDS buffer
constexpr int kGroupBuffers = 3;       // batches b, b+1, b+2 in LDS at once
// Specialised group kernel: regular level-1 nodes of f1 inputs, compile-time depth; each wave
// computes kFastRows DM rows of 64 * kFastV samples, so a workgroup covers kGroupRows *
// kFastRows rows (more rows share each staged window) and a tile of kGroupTileFast samples.
constexpr int kFastRows = 2;
constexpr int kFastV = 8;
constexpr int kGroupTileFast = 64 * kFastV;
constexpr int kFastBuffers = 2;           // batch b + 1 lands while b is read
constexpr int kGroupFastLdsBytes = 81920; // per buffer (two fill the 160 KB of LDS)
constexpr int kGroupTileBits = 2048;  // bit rows: 32 samples (one word) per lane
// Linear kernel shape per row storage.  f32 rows: eight DM rows per wave (128 DM-adjacent rows
// per workgroup share the staged windows) over tiles of 512 samples, lane i owning samples
// i + 64 v (v = 0 .. 7).  16-bit rows: four rows per wave (64-row groups) over tiles of 1024
// samples, lane i owning the sample pairs 2 i + 128 v (v = 0 .. 7); an input that starts in the
// upper half of a dword reads one dword past the tile, so those windows stage one 16-byte unit
// more.  (The 16-bit sums are bound by instruction issue, which the longer tile eases; f32 rows
// are bound by LDS reads, and the larger groups stage fewer bytes per output.)
constexpr int lin_rows(int src_dtype) { return src_dtype == SND_DT_F32 ? 8 : 4; }
constexpr int lin_tile(int src_dtype) { return src_dtype == SND_DT_F32 ? 512 : 1024; }
inline int lin_cover(int src_dtype) { return src_dtype == SND_DT_F32 ? lin_tile(src_dtype) : lin_tile(src_dtype) + 8; }
// inputs per row and batch: the wave's offset words fit 64 lanes, and the 16-bit kernels pack
// each row's count of inputs of one dword phase in 4 bits
constexpr int lin_max_batch_entries(int src_dtype) { return 64 / lin_rows(src_dtype) < 15 ? 64 / lin_rows(src_dtype) : 15; }
constexpr int kLinWords = 64;                  // offset words per (batch, wave)
constexpr int kLinMaxChunks = 7;               // copy chunks per (batch, wave)
constexpr int kLinSmemWords = 24;              // chunk count, 7 units, 7 LDS offsets, 7 lengths, counts, n
constexpr int kLinBuffers = 2;                 // batch b + 1 lands while b is read
constexpr int kLinWordBytes = kGroupRows * kLinWords * 4;  // each buffer's copy of its batch's offset words
constexpr int kLinLdsBytes = (163840 / kLinBuffers - kLinWordBytes) / 16 * 16;  // window bytes per buffer
// Packed kernel (graded mode on u8 rows, regular level-1 nodes of 4 or 8 inputs): the staging
// and copy tables of the linear kernel; each wave computes pack_rows DM rows over tiles of
// pack_tile samples: two rows over 1024 samples where the open level sums of the shape fit the
// registers (four inputs per level-1 node, depth <= 4: 32-row groups), four rows over 512
// samples otherwise (64-row groups).  Lane i owns samples 4 i + 256 v as two pairs of 16-bit
// counts, and reads each input as two aligned dwords (its first four samples may start in
// either), so windows stage one 16-byte unit beyond the tile.  Offset words: lane i, component
// q of a 16-byte word holds input i of row q.  Scalar words: those of the linear kernel, then
// the levels each level-1 node of the batch completes (4 bits per node, two words), then n.
constexpr int pack_rows(int f1, int depth) { return f1 == 4 && depth <= 4 ? 2 : 4; }
constexpr int pack_tile(int f1, int depth) { return pack_rows(f1, depth) == 2 ? 1024 : 512; }
constexpr int kPackRowsMax = 4;
constexpr int kPackMaxBatchEntries = 64;
constexpr int kPackWords = 256;                // offset words per (batch, wave)
constexpr int kPackSmemWords = 25;
constexpr int kPackWordBytes = kGroupRows * kPackWords * 4;
constexpr int kPackLdsBytes = (163840 / 2 - kPackWordBytes) / 16 * 16;
inline bool group_fast_types(int mode, int src_dt, int dst_dt)
{
    if (mode == SND_MODE_BINARY) return (src_dt == SND_DT_U8 || src_dt == SND_DT_BITS) && dst_dt == SND_DT_U8;
    if (mode == SND_MODE_GRADED) return src_dt == dst_dt && (src_dt == SND_DT_U8 || src_dt == SND_DT_U16);
    return dst_dt == SND_DT_F32;
}
inline bool group_fast_supported(int f1, int depth)
{
    return (f1 == 2 && depth >= 1 && depth <= 8) || (f1 == 4 && depth >= 1 && depth <= 5) ||
           (f1 == 8 && depth >= 1 && depth <= 4);
}
constexpr int kGroupMaxSpan = 256;   // offset spread of one staged window (window <= span + tile)
constexpr int kGroupSlotsPerWave = 8;  // staged windows per wave per batch
constexpr int kAnchorTile = 512;     // reference samples per anchored sub-tile (8 per lane)
constexpr int kAnchorMaxTile = 2048;  // largest anchored window per workgroup
constexpr int kAnchorWaves = 16;     // waves per anchored workgroup
constexpr int kAnchorLdsBytes = 65536;
constexpr int kAnchorLdsTarget = 40960;  // larger windows only while four workgroups fit a CU
constexpr int kAnchorBitsW = 4;                         // bit input: words per lane
constexpr int kAnchorTileBits = 64 * 32 * kAnchorBitsW;  // bit input: samples per workgroup
// words of one staged channel window on bit input: the tile, the largest offset, one more word
// for the funnel shift
inline int64_t anchor_bits_words(int32_t rho_max) { return 64 * kAnchorBitsW + (rho_max >> 5) + 1; }

struct Level {
    int nnodes = 0;
    std::vector<int32_t> chlo, chhi, kidlo, kidhi, ref;
    std::vector<int32_t> nid;       // [nnodes][ndm]: neuron (within the node) serving each DM
    std::vector<int32_t> nneu;      // [nnodes]
    std::vector<int64_t> row_base;  // [nnodes]: first row of the node within the level
    std::vector<int32_t> rep;       // [rows]: one DM served by the row's neuron
    std::vector<int32_t> lo, hi;    // [rows]: range of the node reference delay over its DMs
    std::vector<int32_t> node_of;   // [rows]
    int64_t rows = 0;
    int64_t synapses = 0;
};

struct PlanImpl {
    snd_plan_desc desc{};
    std::vector<double> freq, dm;
    int nchan = 0, ndm = 0;
    int64_t nsamp = 0, n_out = 0, max_delay = 0;
    double fref = 0.0;
    std::vector<int32_t> delay;  // [ndm][nchan]
    std::vector<Level> lev;
    std::vector<Stage> stages;
    std::vector<uint8_t> table;  // host image of the device tables
    int64_t workspace_bytes = 0;
    // graded plans of an input-anchored leaf stage and a packed final stage: workspace offset of
    // the leaf stage's per-workgroup bound words and their count (bound word after them); -1: none
    int64_t bound_off = -1;
    int64_t bound_n = 0;
    int out_dtype = SND_DT_F32;
    void *d_table = nullptr;
    snd_plan_info info{};
};

int dtype_size(int dt);
int64_t dtype_bytes(int dt, int64_t elems);  // storage bytes of elems elements (bit rows: rounded up)

// One execution of a plan: n_run <= n_out output samples from a source window of src_len
// samples per channel; the input rows are rings of ring_len samples whose window starts at
// column ring_start when ring_len > 0 (streaming), plain rows otherwise.
struct Run {
    int64_t n_run;
    int64_t src_len;
    int64_t ring_len;
    int64_t ring_start;
};
inline Run full_run(const PlanImpl &p) { return Run{p.n_out, p.nsamp, 0, 0}; }
// Enqueue stage si of one run (defined with the C ABI).
snd_status run_stage(PlanImpl &P, size_t si, const Run &run, const void *d_in, int64_t in_pitch, void *d_out,
                     int64_t out_pitch, void *d_workspace, void *stream);
// Depth classes of the kernels whose open-level stack is sized at compile time.
inline int depth_bucket(int d) { return d <= 1 ? 1 : d <= 2 ? 2 : d <= 4 ? 4 : d <= 8 ? 8 : 16; }
void set_error(const std::string &msg);
// Builds the whole plan; returns SND_OK or an error with a message in `err`.
snd_status build_plan(const snd_plan_desc &d, PlanImpl &p, std::string &err);

// ---- device launchers (kernels.hip) ----

// Several stage launches of one kernel class in a single grid: record r (an argument struct of
// the kernel in device memory) owns the workgroups [prefix[r], prefix[r + 1]).  n == 0 means a
// plain launch whose arguments are passed by value.
struct Multi {
    const void *recs;
    const int32_t *prefix;
    int32_t n;
};
struct StageArgs {
    const void *src;
    int64_t src_pitch;
    void *dst;
    int64_t dst_pitch;
    const uint32_t *row_ptr;
    const int32_t *row_len;
    const Entry *ent;
    int32_t rows;
    int32_t n_ttiles;
    int32_t n_rgroups;
    int32_t depth;
    int32_t src_is_input;
    int32_t k_leaf, k_int, cap;
    float scale;
    int32_t len_cut;  // samples dropped from the end of every row (runs with fewer outputs than n_out)
};

// Workgroups of one generic stage launch; fills a.n_ttiles and a.n_rgroups.
int64_t stage_blocks(StageArgs &a, int64_t max_len);
// Enqueue one stage; returns 0 or a HIP error code.  With m.n > 0 the arguments come from the
// records of m and the grid has `nblocks` workgroups (a is only used to choose the instance).
int launch_stage(int mode, int src_dtype, int dst_dtype, const StageArgs &a, int64_t max_len, void *stream,
                 const Multi &m = Multi{nullptr, nullptr, 0}, int64_t nblocks = 0);

struct GroupArgs {
    const void *src;
    int64_t src_pitch;
    void *dst;
    int64_t dst_pitch;
    const int32_t *grp_rows;
    const int32_t *batch_ptr;
    const int32_t *batches;  // 4 ints per batch
    const int32_t *instrs;   // 4 ints per staged window (copy descriptor)
    const uint32_t *ldsb;
    const int32_t *node_closes;  // specialised kernel only
    const uint32_t *lin_smem;    // linear kernel only
    const uint32_t *lin;
    int32_t lin_kernel;          // 1: linear kernel, 2: packed kernel
    int32_t xcd_chunk;           // DM groups of one time tile dealt to each XCD in turn
    int32_t ngroups;
    int32_t n_entries;
    int32_t buf_elems;
    int32_t f1;  // > 0: specialised kernel with level-1 nodes of f1 inputs
    int32_t n_out;
    int32_t depth;
    int32_t src_is_input;
    int32_t k_leaf, k_int, cap;
    float scale;
    // packed graded kernel: the largest value of its input plane, written by the stage that
    // produced it (k_bound_reduce); nullptr: no bound known, the kernel takes its general path
    const uint32_t *bound;
};
int launch_group(int mode, int src_dtype, int dst_dtype, const GroupArgs &a, int64_t n_out, int lds_bytes, void *stream,
                 const Multi &m = Multi{nullptr, nullptr, 0}, int64_t nblocks = 0);

struct AnchorArgs {
    const void *src;
    int64_t src_pitch;
    int64_t src_len;     // valid samples per source row, counted from the window start
    int64_t ring_len;    // > 0: source rows are rings of this many samples
    int64_t ring_start;  // ring column of the window start (0 when not a ring)
    void *dst;
    int64_t dst_pitch;
    const uint32_t *row_ptr;
    const int32_t *row_len;
    const Entry *ent;
    const int32_t *nodes;
    const int32_t *tiles;    // 2 ints per workgroup
    const int32_t *row_lo;
    int32_t depth;
    int32_t k_leaf, k_int, cap;
    float scale;
    int32_t n_run;    // output samples of this run (<= n_out)
    int32_t len_cut;  // n_out - n_run: samples dropped from the end of every row
    int32_t tile;     // reference samples per workgroup window (a multiple of kAnchorTile)
    // graded u8 output: one word per workgroup receives the largest value it computed, and
    // the word after the last the largest of them all (k_bound_reduce); nullptr: not tracked
    uint32_t *bound_slots;
};
int launch_anchored(int mode, int src_dtype, int dst_dtype, const AnchorArgs &a, int64_t ntiles, int lds_bytes,
                    void *stream, const Multi &m = Multi{nullptr, nullptr, 0});
// max of the n per-workgroup words at slots into slots[n] (one workgroup)
int launch_bound_reduce(uint32_t *slots, int64_t n, void *stream);
// the same for every record of a batched leaf grid that tracks its words (one workgroup each)
int launch_bound_reduce_records(const Multi &m, void *stream);
int launch_encode(const float *z, int64_t z_pitch, int time_major, int nchan, int64_t nsamp, const float *thr,
                  int nthr, uint8_t *out, int64_t out_pitch, void *stream);
int launch_encode_bits(const float *z, int64_t z_pitch, int time_major, int nchan, int64_t nsamp, float thr,
                       uint32_t *out, int64_t out_words, void *stream);
int launch_chanstats(const float *p, int64_t p_pitch, int nchan, int64_t n, double clip, double *stats, void *stream);
int launch_zero_dm(float *z, int64_t zp, int nchan, int64_t n, double gamma, int32_t *count, void *stream);
int launch_flag_channels(float *z, int64_t zp, int nchan, int64_t n, int64_t w, double k, double *sigma,
                         uint8_t *flags, int64_t fp, void *stream);
int launch_normalize(const float *p, int64_t p_pitch, int nchan, int64_t n, const double *stats, float *z,
                     int64_t z_pitch, void *stream);
int launch_cast(const float *src, int64_t src_pitch, int64_t rows, int64_t cols, void *dst, int64_t dst_pitch,
                int dst_dtype, void *stream);
// Bit rows: copy L bits of each of nchan chunk rows (from bit 0) into a ring of R bits per row
// (R a multiple of 32) at ring bit position pos, wrapping at R; the ring's other bits keep.
int launch_ring_put_bits(const uint32_t *chunk, int64_t chunk_words, uint32_t *ring, int64_t ring_words, int64_t R,
                         int64_t pos, int64_t L, int nchan, void *stream);

// Compile-time shape of the kernel instance that runs stage S: the depth class, or, for the
// specialised row-group kernel, 1000 * (inputs per level-1 node) + depth; -1 for the linear
// kernel; minus the specialised shape for the packed kernel.
inline int stage_shape(const Stage &S)
{
    if (S.kernel == kKernelGroupLds && S.group_lin) return -1;
    if (S.kernel == kKernelGroupLds && S.group_pack) return -(1000 * S.group_f1 + S.depth);
    if (S.kernel == kKernelGroupLds && S.group_f1 > 0) return 1000 * S.group_f1 + S.depth;
    return depth_bucket(S.depth);
}

// One stage launch with its arguments filled in, ready to run alone or as one record of a
// batched launch.  Launches may share a grid when kind, mode, dtypes and shape agree.
struct Prepared {
    int kind, mode, src_dt, dst_dt;
    int shape;   // compile-time shape of the instance: depth class, or 1000 * f1 + depth
    int lds;     // dynamic LDS bytes
    int64_t nblocks;
    int64_t n_run;    // LDS row groups: output samples of the run
    int64_t max_len;  // generic: longest row of the run
    bool bad_pitch;   // LDS row groups: source pitch the kernel cannot address
    StageArgs st;
    GroupArgs gr;
    AnchorArgs an;
};
// bound: track the leaf plane's largest value for the packed graded final stage (a batched leaf
// grid is followed by launch_bound_reduce_records, a single leaf launch by launch_bound_reduce)
Prepared prepare_stage(const PlanImpl &P, size_t si, const Run &run, const void *d_in, int64_t in_pitch, void *d_out,
                       int64_t out_pitch, void *d_workspace, bool bound = false);
snd_status launch_prepared(const Prepared &pr, void *stream, const Multi &m, int64_t nblocks);

// One beam of a batched execution: its plan, run and buffers.
struct Job {
    const PlanImpl *P;
    Run run;
    const void *in;
    int64_t in_pitch;
    void *out;
    int64_t out_pitch;
    void *ws;
};
// Device record bytes a batch of these plans needs, and the number of grids it launches.
int64_t batch_record_bytes(const std::vector<const PlanImpl *> &plans, int *n_launches);
// Every stage of every job, one grid per (stage wave, kernel class); records in d_records.
snd_status run_batch(const std::vector<Job> &jobs, void *d_records, int64_t records_bytes, void *stream,
                     int *n_launches);

}  // namespace snd

struct snd_plan_s {
    snd::PlanImpl impl;
};
