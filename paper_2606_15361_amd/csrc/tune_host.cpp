// Schedule autotuner: builds the plan of each candidate (stage schedule, time chunk), uploads
// it, and times executes over the caller's buffers with HIP events.  The fastest candidate whose
// tables and workspace fit the buffers wins.  Results of every candidate are identical; only
// their speed and memory differ.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "snd_internal.h"

namespace {

snd_status tfail(snd_status s, const std::string &msg)
{
    snd::set_error(msg);
    return s;
}

// One pass of plan P over the block: a single run, or runs of P.n_out output samples at
// increasing time offsets until n_total outputs are written.
snd_status pass(snd::PlanImpl &P, int64_t n_total, const uint8_t *in, int64_t in_pitch, int64_t in_es, uint8_t *out,
                int64_t out_pitch, int64_t out_es, void *ws, hipStream_t st)
{
    for (int64_t t = 0; t < n_total; t += P.n_out) {
        const int64_t n = std::min<int64_t>(P.n_out, n_total - t);
        const snd::Run run{n, P.max_delay + n, 0, 0};
        for (size_t si = 0; si < P.stages.size(); ++si) {
            snd_status s = snd::run_stage(P, si, run, in + t * in_es, in_pitch, out + t * out_es, out_pitch, ws, st);
            if (s != SND_OK) return s;
        }
    }
    return SND_OK;
}

}  // namespace

extern "C" {

snd_status snd_autotune(const snd_plan_desc *desc, snd_tune_candidate *cands, int32_t ncand, const void *d_in,
                        int64_t in_pitch, void *d_out, int64_t out_pitch, void *d_workspace, int64_t workspace_bytes,
                        void *d_tables, int64_t table_bytes, int32_t reps, int32_t *h_best, void *stream)
{
    if (!desc || !cands || ncand < 1 || !d_in || !d_out || !d_tables || !h_best || reps < 1)
        return tfail(SND_ERR_INVALID, "null argument, no candidates or reps < 1");
    if (desc->chunk > 0) return tfail(SND_ERR_INVALID, "the descriptor to tune must describe a whole block (chunk 0)");
    if (((uintptr_t)d_tables & 255u) || (d_workspace && ((uintptr_t)d_workspace & 255u)))
        return tfail(SND_ERR_INVALID, "table and workspace buffers must be 256-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return tfail(SND_ERR_HIP, "hipEventCreate");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return tfail(SND_ERR_HIP, "hipEventCreate");
    }
    snd_status ret = SND_OK;
    int best = -1;
    int64_t n_total = -1;
    for (int32_t i = 0; i < ncand && ret == SND_OK; ++i) {
        snd_tune_candidate &c = cands[i];
        c.ms = -1.0;
        c.workspace_bytes = c.table_bytes = 0;
        snd_plan_desc d = *desc;
        d.stage_levels = c.stage_levels;
        d.chunk = c.chunk > 0 ? c.chunk : 0;
        d.tune = c.tune;
        snd::PlanImpl P;
        std::string err;
        snd_status s = snd::build_plan(d, P, err);
        if (s == SND_ERR_UNSUPPORTED) continue;  // e.g. a leaf window the LDS cannot hold: skipped
        if (s != SND_OK) {
            ret = tfail(s, "candidate " + std::to_string(i) + ": " + err);
            break;
        }
        if (n_total < 0) {  // output samples of the whole block
            n_total = desc->nsamp - P.max_delay;
            if (n_total < 1 || in_pitch < desc->nsamp || out_pitch < n_total) {
                ret = tfail(SND_ERR_INVALID, "block too short or pitches too small");
                break;
            }
        }
        c.workspace_bytes = P.workspace_bytes;
        c.table_bytes = (int64_t)P.table.size();
        if (c.table_bytes > table_bytes || P.workspace_bytes > workspace_bytes ||
            (P.workspace_bytes > 0 && !d_workspace))
            continue;  // does not fit the buffers: skipped
        if (hipMemcpyAsync(d_tables, P.table.data(), P.table.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            ret = tfail(SND_ERR_HIP, "table upload");
            break;
        }
        P.d_table = d_tables;
        const int64_t in_es = snd::dtype_size(d.in_dtype), out_es = snd::dtype_size(P.out_dtype);
        const uint8_t *in = static_cast<const uint8_t *>(d_in);
        uint8_t *out = static_cast<uint8_t *>(d_out);
        s = pass(P, n_total, in, in_pitch, in_es, out, out_pitch, out_es, d_workspace, st);  // warm-up
        if (s == SND_OK && hipEventRecord(e0, st) != hipSuccess) s = tfail(SND_ERR_HIP, "hipEventRecord");
        for (int32_t r = 0; r < reps && s == SND_OK; ++r)
            s = pass(P, n_total, in, in_pitch, in_es, out, out_pitch, out_es, d_workspace, st);
        if (s == SND_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
            s = tfail(SND_ERR_HIP, "timing events");
        if (s != SND_OK) {
            ret = s;
            break;
        }
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            ret = tfail(SND_ERR_HIP, "hipEventElapsedTime");
            break;
        }
        c.ms = ms / reps;
        if (best < 0 || c.ms < cands[best].ms) best = i;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (ret != SND_OK) return ret;
    if (best < 0) return tfail(SND_ERR_NOMEM, "no candidate fits the table and workspace buffers");
    *h_best = best;
    return SND_OK;
}

}  // extern "C"
