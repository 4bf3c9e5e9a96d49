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
};

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
    int out_dtype = SND_DT_F32;
    void *d_table = nullptr;
    snd_plan_info info{};
};

int dtype_size(int dt);
// Builds the whole plan; returns SND_OK or an error with a message in `err`.
snd_status build_plan(const snd_plan_desc &d, PlanImpl &p, std::string &err);

// ---- device launchers (kernels.hip) ----
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
};

// Enqueue one stage; returns 0 or a HIP error code.
int launch_stage(int mode, int src_dtype, int dst_dtype, const StageArgs &a, int64_t max_len, void *stream);
int launch_encode(const float *z, int64_t z_pitch, int time_major, int nchan, int64_t nsamp, const float *thr,
                  int nthr, uint8_t *out, int64_t out_pitch, void *stream);
int launch_cast(const float *src, int64_t src_pitch, int64_t rows, int64_t cols, void *dst, int64_t dst_pitch,
                int dst_dtype, void *stream);

}  // namespace snd

struct snd_plan_s {
    snd::PlanImpl impl;
};
