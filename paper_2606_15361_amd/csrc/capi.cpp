// C ABI entry points (include/snd.h).  Argument checking, error reporting and the stage
// schedule of one execute; all device arithmetic is in the HIP kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "snd_internal.h"

namespace {

thread_local std::string g_err;

snd_status fail(snd_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

snd_status hip_fail(int code, const char *what)
{
    g_err = std::string(what) + ": " + hipGetErrorString((hipError_t)code);
    return SND_ERR_HIP;
}

bool aligned256(const void *p) { return ((uintptr_t)p & 255u) == 0; }

}  // namespace

namespace snd {
void set_error(const std::string &msg) { g_err = msg; }
}  // namespace snd

extern "C" {

const char *snd_last_error(void) { return g_err.c_str(); }

const char *snd_version(void) { return "snd-mi355x 0.1 (gfx950)"; }

snd_status snd_plan_create(const snd_plan_desc *desc, snd_plan *out)
{
    if (!desc || !out) return fail(SND_ERR_INVALID, "null descriptor or output handle");
    *out = nullptr;
    snd_plan p = new (std::nothrow) snd_plan_s;
    if (!p) return fail(SND_ERR_NOMEM, "host allocation failed");
    std::string err;
    snd_status s;
    try {
        s = snd::build_plan(*desc, p->impl, err);
    } catch (const std::bad_alloc &) {
        s = SND_ERR_NOMEM;
        err = "host allocation failed while building the plan";
    }
    if (s != SND_OK) {
        delete p;
        return fail(s, err);
    }
    *out = p;
    return SND_OK;
}

snd_status snd_plan_query(snd_plan plan, snd_plan_info *out)
{
    if (!plan || !out) return fail(SND_ERR_INVALID, "null plan or output");
    *out = plan->impl.info;
    return SND_OK;
}

snd_status snd_plan_delays(snd_plan plan, int32_t *h_delays, int64_t count)
{
    if (!plan || !h_delays) return fail(SND_ERR_INVALID, "null plan or buffer");
    const auto &d = plan->impl.delay;
    if (count < (int64_t)d.size()) return fail(SND_ERR_NOMEM, "delay buffer smaller than ndm * nchan");
    std::memcpy(h_delays, d.data(), d.size() * sizeof(int32_t));
    return SND_OK;
}

snd_status snd_plan_upload(snd_plan plan, void *d_tables, int64_t bytes, void *stream)
{
    if (!plan || !d_tables) return fail(SND_ERR_INVALID, "null plan or table buffer");
    auto &P = plan->impl;
    if (bytes < (int64_t)P.table.size()) return fail(SND_ERR_NOMEM, "table buffer smaller than table_bytes");
    if (!aligned256(d_tables)) return fail(SND_ERR_INVALID, "table buffer must be 256-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(d_tables, P.table.data(), P.table.size(), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(tables)");
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize(tables)");
    P.d_table = d_tables;
    return SND_OK;
}

snd_status snd_plan_destroy(snd_plan plan)
{
    delete plan;
    return SND_OK;
}

}  // extern "C"

namespace {

snd_status check_exec(snd_plan plan, const void *d_in, int64_t in_pitch, void *d_out, int64_t out_pitch,
                      void *d_workspace, int64_t workspace_bytes)
{
    if (!plan || !d_in || !d_out) return fail(SND_ERR_INVALID, "null plan, input or output");
    auto &P = plan->impl;
    if (!P.d_table) return fail(SND_ERR_STATE, "plan tables not uploaded");
    if (in_pitch < P.nsamp) return fail(SND_ERR_INVALID, "input pitch smaller than nsamp");
    if (P.desc.in_dtype == SND_DT_BITS && in_pitch % 32 != 0)
        return fail(SND_ERR_INVALID, "bit input pitch must be a multiple of 32 bits");
    if (out_pitch < P.n_out) return fail(SND_ERR_INVALID, "output pitch smaller than n_out");
    if (P.workspace_bytes > 0 && (!d_workspace || workspace_bytes < P.workspace_bytes))
        return fail(SND_ERR_NOMEM, "workspace smaller than workspace_bytes");
    if (P.workspace_bytes > 0 && !aligned256(d_workspace)) return fail(SND_ERR_INVALID, "workspace must be 256-byte aligned");
    return SND_OK;
}

}  // namespace

namespace snd {

Prepared prepare_stage(const PlanImpl &P, size_t si, const Run &run, const void *d_in, int64_t in_pitch, void *d_out,
                       int64_t out_pitch, void *d_workspace, bool bound)
{
    const int32_t len_cut = (int32_t)(P.n_out - run.n_run);
    const uint8_t *tb = static_cast<const uint8_t *>(P.d_table);
    uint8_t *ws = static_cast<uint8_t *>(d_workspace);
    const Stage &S = P.stages[si];
    Prepared pr{};
    pr.kind = S.kernel;
    pr.mode = P.desc.mode;
    pr.src_dt = S.src_dtype;
    pr.dst_dt = S.dst_dtype;
    pr.lds = S.lds_bytes;
    StageArgs &a = pr.st;
    if (si == 0) {
        a.src = d_in;
        a.src_pitch = in_pitch;
    } else {
        const Stage &Q = P.stages[si - 1];
        a.src = ws + Q.ws_off;
        a.src_pitch = Q.pitch;
    }
    if (S.final_stage) {
        a.dst = d_out;
        a.dst_pitch = out_pitch;
    } else {
        a.dst = ws + S.ws_off;
        a.dst_pitch = S.pitch;
    }
    a.row_ptr = reinterpret_cast<const uint32_t *>(tb + S.off_row_ptr);
    a.row_len = reinterpret_cast<const int32_t *>(tb + S.off_row_len);
    a.ent = reinterpret_cast<const Entry *>(tb + S.off_ent);
    const float scale = (S.final_stage && P.desc.mode == SND_MODE_FLOAT && P.desc.root_norm)
                            ? (float)(1.0 / std::sqrt((double)P.nchan))
                            : 1.0f;
    if (S.kernel == kKernelGroupLds) {
        GroupArgs &g = pr.gr;
        pr.bad_pitch = a.src_pitch < 0 || a.src_pitch * dtype_size(S.src_dtype) >= (int64_t(1) << 32);
        g.src = a.src;
        g.src_pitch = a.src_pitch;
        g.dst = a.dst;
        g.dst_pitch = a.dst_pitch;
        g.grp_rows = reinterpret_cast<const int32_t *>(tb + S.off_grp_rows);
        g.batch_ptr = reinterpret_cast<const int32_t *>(tb + S.off_batch_ptr);
        g.batches = reinterpret_cast<const int32_t *>(tb + S.off_batches);
        g.instrs = reinterpret_cast<const int32_t *>(tb + S.off_instrs);
        g.ldsb = reinterpret_cast<const uint32_t *>(tb + S.off_ldsb);
        g.node_closes = reinterpret_cast<const int32_t *>(tb + S.off_node_closes);
        g.lin_smem = reinterpret_cast<const uint32_t *>(tb + S.off_lin_smem);
        g.lin = reinterpret_cast<const uint32_t *>(tb + S.off_lin);
        g.lin_kernel = S.group_lin ? 1 : S.group_pack ? 2 : 0;
        g.xcd_chunk = S.xcd_chunk;
        g.ngroups = (int32_t)S.ngroups;
        g.n_entries = S.n_entries;
        g.buf_elems = S.lds_buf_elems;
        g.f1 = S.group_f1;
        g.n_out = (int32_t)run.n_run;
        g.depth = S.depth;
        g.src_is_input = S.src_level < 0;
        g.k_leaf = P.desc.k_leaf;
        g.k_int = P.desc.k_int;
        g.cap = P.desc.cap;
        g.scale = scale;
        if (bound && S.group_pack && si == 1 && P.bound_off >= 0)
            g.bound = reinterpret_cast<const uint32_t *>(ws + P.bound_off) + P.bound_n;
        pr.n_run = run.n_run;
        pr.shape = stage_shape(S);
        const int64_t tile = S.group_tile;
        pr.nblocks = S.ngroups * ((run.n_run + tile - 1) / tile);
        return pr;
    }
    if (S.kernel == kKernelAnchored) {
        AnchorArgs &g = pr.an;
        g.src = a.src;
        g.src_pitch = a.src_pitch;
        g.src_len = run.src_len;
        g.ring_len = run.ring_len;
        g.ring_start = run.ring_start;
        g.dst = a.dst;
        g.dst_pitch = a.dst_pitch;
        g.row_ptr = a.row_ptr;
        g.row_len = a.row_len;
        g.ent = a.ent;
        g.nodes = reinterpret_cast<const int32_t *>(tb + S.off_nodes);
        g.tiles = reinterpret_cast<const int32_t *>(tb + S.off_tiles);
        g.row_lo = reinterpret_cast<const int32_t *>(tb + S.off_row_lo);
        g.depth = S.depth;
        g.k_leaf = P.desc.k_leaf;
        g.k_int = P.desc.k_int;
        g.cap = P.desc.cap;
        g.scale = scale;
        g.n_run = (int32_t)run.n_run;
        g.len_cut = len_cut;
        g.tile = S.anchor_tile;
        if (bound && si == 0 && P.bound_off >= 0) g.bound_slots = reinterpret_cast<uint32_t *>(ws + P.bound_off);
        pr.shape = stage_shape(S);
        pr.nblocks = S.ntiles;
        return pr;
    }
    a.rows = (int32_t)S.rows;
    a.depth = S.depth;
    a.src_is_input = S.src_level < 0;
    a.k_leaf = P.desc.k_leaf;
    a.k_int = P.desc.k_int;
    a.cap = P.desc.cap;
    a.scale = scale;
    a.len_cut = len_cut;
    pr.max_len = S.max_len - len_cut;
    pr.shape = stage_shape(S);
    pr.nblocks = stage_blocks(a, pr.max_len);
    return pr;
}

snd_status launch_prepared(const Prepared &pr, void *stream, const Multi &m, int64_t nblocks)
{
    int e = 0;
    const char *what = "stage launch";
    if (pr.kind == kKernelGroupLds) {
        if (pr.bad_pitch) {
            set_error("source row pitch of 4 GiB or more is not supported by the LDS row-group kernels");
            return SND_ERR_UNSUPPORTED;
        }
        e = launch_group(pr.mode, pr.src_dt, pr.dst_dt, pr.gr, pr.n_run, pr.lds, stream, m, nblocks);
        what = "stage launch (LDS groups)";
    } else if (pr.kind == kKernelAnchored) {
        e = launch_anchored(pr.mode, pr.src_dt, pr.dst_dt, pr.an, m.n > 0 ? nblocks : pr.nblocks, pr.lds, stream, m);
        what = "stage launch (input-anchored)";
        if (!e && pr.an.bound_slots && m.n == 0) {
            e = launch_bound_reduce(pr.an.bound_slots, pr.nblocks, stream);
            what = "leaf bound reduction";
        }
    } else {
        e = launch_stage(pr.mode, pr.src_dt, pr.dst_dt, pr.st, pr.max_len, stream, m, nblocks);
    }
    if (e) return hip_fail(e, what);
    return SND_OK;
}

snd_status run_stage(PlanImpl &P, size_t si, const Run &run, const void *d_in, int64_t in_pitch, void *d_out,
                     int64_t out_pitch, void *d_workspace, void *stream)
{
    // a marker range per stage on the host timeline (rocprofv3 --marker-trace); no cost otherwise
    static const char *kStageNames[] = {"snd stage 0", "snd stage 1", "snd stage 2", "snd stage 3",
                                        "snd stage 4", "snd stage 5", "snd stage 6", "snd stage 7"};
    roctxRangePushA(si < 8 ? kStageNames[si] : "snd stage");
    const Prepared pr = prepare_stage(P, si, run, d_in, in_pitch, d_out, out_pitch, d_workspace, true);
    const snd_status s = launch_prepared(pr, stream, Multi{nullptr, nullptr, 0}, 0);
    roctxRangePop();
    return s;
}

}  // namespace snd

extern "C" {

snd_status snd_execute(snd_plan plan, const void *d_in, int64_t in_pitch, void *d_out, int64_t out_pitch,
                       void *d_workspace, int64_t workspace_bytes, void *stream)
{
    snd_status s = check_exec(plan, d_in, in_pitch, d_out, out_pitch, d_workspace, workspace_bytes);
    if (s != SND_OK) return s;
    for (size_t si = 0; si < plan->impl.stages.size(); ++si) {
        s = snd::run_stage(plan->impl, si, snd::full_run(plan->impl), d_in, in_pitch, d_out, out_pitch, d_workspace,
                           stream);
        if (s != SND_OK) return s;
    }
    return SND_OK;
}

snd_status snd_execute_stage(snd_plan plan, int32_t stage, const void *d_in, int64_t in_pitch, void *d_out,
                             int64_t out_pitch, void *d_workspace, int64_t workspace_bytes, void *stream)
{
    snd_status s = check_exec(plan, d_in, in_pitch, d_out, out_pitch, d_workspace, workspace_bytes);
    if (s != SND_OK) return s;
    if (stage < 0 || stage >= (int32_t)plan->impl.stages.size()) return fail(SND_ERR_INVALID, "stage index out of range");
    return snd::run_stage(plan->impl, (size_t)stage, snd::full_run(plan->impl), d_in, in_pitch, d_out, out_pitch,
                          d_workspace, stream);
}

snd_status snd_encode(const float *d_z, int64_t z_pitch, int32_t time_major, int32_t nchan, int64_t nsamp,
                      const float *h_thresholds, int32_t nthr, uint8_t *d_out, int64_t out_pitch, void *stream)
{
    if (!d_z || !d_out || !h_thresholds) return fail(SND_ERR_INVALID, "null pointer");
    if (nchan < 1 || nsamp < 1 || nthr < 1 || nthr > 8) return fail(SND_ERR_INVALID, "bad nchan, nsamp or nthr (1..8)");
    if (z_pitch < (time_major ? nchan : nsamp) || out_pitch < nsamp) return fail(SND_ERR_INVALID, "pitch too small");
    if (!time_major && nchan > 65535) return fail(SND_ERR_INVALID, "too many channels");
    int e = snd::launch_encode(d_z, z_pitch, time_major, nchan, nsamp, h_thresholds, nthr, d_out, out_pitch, stream);
    if (e) return hip_fail(e, "encode launch");
    return SND_OK;
}

snd_status snd_encode_bits(const float *d_z, int64_t z_pitch, int32_t time_major, int32_t nchan, int64_t nsamp,
                           float threshold, uint32_t *d_out, int64_t out_pitch, void *stream)
{
    if (!d_z || !d_out) return fail(SND_ERR_INVALID, "null pointer");
    if (nchan < 1 || nsamp < 1) return fail(SND_ERR_INVALID, "bad nchan or nsamp");
    if (z_pitch < (time_major ? nchan : nsamp) || out_pitch < nsamp || out_pitch % 32 != 0)
        return fail(SND_ERR_INVALID, "pitch too small, or output pitch not a multiple of 32 bits");
    if (nchan > 65535 * (time_major ? 64 : 1) || nsamp > (int64_t)0x7fffffff * 64)
        return fail(SND_ERR_INVALID, "too many channels or samples");
    int e = snd::launch_encode_bits(d_z, z_pitch, time_major, nchan, nsamp, threshold, d_out, out_pitch / 32, stream);
    if (e) return hip_fail(e, "encode launch");
    return SND_OK;
}

snd_status snd_channel_stats(const float *d_p, int64_t p_pitch, int32_t nchan, int64_t nsamp, double clip,
                             double *d_stats, void *stream)
{
    if (!d_p || !d_stats) return fail(SND_ERR_INVALID, "null pointer");
    if (nchan < 1 || nsamp < 1 || p_pitch < nsamp || !(clip > 0.0) || !std::isfinite(clip))
        return fail(SND_ERR_INVALID, "bad nchan, nsamp, pitch or clip");
    int e = snd::launch_chanstats(d_p, p_pitch, nchan, nsamp, clip, d_stats, stream);
    if (e) return hip_fail(e, "channel statistics launch");
    return SND_OK;
}

snd_status snd_normalize(const float *d_p, int64_t p_pitch, int32_t nchan, int64_t nsamp, const double *d_stats,
                         float *d_z, int64_t z_pitch, void *stream)
{
    if (!d_p || !d_stats || !d_z) return fail(SND_ERR_INVALID, "null pointer");
    if (nchan < 1 || nchan > 65535 || nsamp < 1 || p_pitch < nsamp || z_pitch < nsamp)
        return fail(SND_ERR_INVALID, "bad nchan, nsamp or pitch");
    int e = snd::launch_normalize(d_p, p_pitch, nchan, nsamp, d_stats, d_z, z_pitch, stream);
    if (e) return hip_fail(e, "normalize launch");
    return SND_OK;
}

snd_status snd_zero_dm(float *d_z, int64_t z_pitch, int32_t nchan, int64_t nsamp, double gamma, int32_t *d_count,
                       void *stream)
{
    if (!d_z) return fail(SND_ERR_INVALID, "null pointer");
    if (nchan < 1 || nsamp < 1 || z_pitch < nsamp || nsamp > (int64_t)0xffffffff * 256 || !(gamma >= 0.0) ||
        !std::isfinite(gamma))
        return fail(SND_ERR_INVALID, "bad nchan, nsamp, pitch or gamma");
    int e = snd::launch_zero_dm(d_z, z_pitch, nchan, nsamp, gamma, d_count, stream);
    if (e) return hip_fail(e, "zero-DM launch");
    return SND_OK;
}

snd_status snd_flag_channels(float *d_z, int64_t z_pitch, int32_t nchan, int64_t nsamp, int64_t window, double k,
                             double *d_sigma, uint8_t *d_flags, int64_t flags_pitch, void *stream)
{
    if (!d_z || !d_sigma) return fail(SND_ERR_INVALID, "null pointer");
    if (nchan < 1 || nchan > 8192 || nsamp < 1 || z_pitch < nsamp || window < 1 || !(k >= 0.0) || !std::isfinite(k))
        return fail(SND_ERR_INVALID, "1 <= nchan <= 8192, nsamp >= 1, pitch >= nsamp, window >= 1, finite k >= 0 needed");
    const int64_t nwin = (nsamp + window - 1) / window;
    if (nwin > 0x7fffffff) return fail(SND_ERR_INVALID, "too many windows");
    if (d_flags && flags_pitch < nchan) return fail(SND_ERR_INVALID, "flags_pitch < nchan");
    if (nwin > 65535) return fail(SND_ERR_INVALID, "at most 65535 windows");
    int e = snd::launch_flag_channels(d_z, z_pitch, nchan, nsamp, window, k, d_sigma, d_flags, flags_pitch, stream);
    if (e) return hip_fail(e, "channel flagging launch");
    return SND_OK;
}

snd_status snd_cast(const float *d_src, int64_t src_pitch, int64_t rows, int64_t cols, void *d_dst, int64_t dst_pitch,
                    int32_t dst_dtype, void *stream)
{
    if (!d_src || !d_dst) return fail(SND_ERR_INVALID, "null pointer");
    if (rows < 1 || cols < 1 || rows > 65535 || src_pitch < cols || dst_pitch < cols)
        return fail(SND_ERR_INVALID, "bad shape or pitch");
    if (dst_dtype != SND_DT_BF16 && dst_dtype != SND_DT_F16) return fail(SND_ERR_UNSUPPORTED, "cast target must be BF16 or F16");
    int e = snd::launch_cast(d_src, src_pitch, rows, cols, d_dst, dst_pitch, dst_dtype, stream);
    if (e) return hip_fail(e, "cast launch");
    return SND_OK;
}

}  // extern "C"
