// Batched execution: the stage launches of many beams, each with its own plan, grouped so that
// every (stage wave, kernel class) is one grid.  A kernel class is a kernel kind, mode, storage
// pair and compile-time shape; beams whose DM grids, lengths or tables differ still share a
// class.  Each grid reads its per-beam argument records and a workgroup prefix table from a
// caller-owned device buffer, written by one host-to-device copy per grid.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "snd_internal.h"

namespace snd {

namespace {

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

using ClassKey = std::tuple<int, int, int, int, int>;  // kind, mode, src dtype, dst dtype, shape

ClassKey class_key(const PlanImpl &P, size_t si)
{
    const Stage &S = P.stages[si];
    return ClassKey{S.kernel, P.desc.mode, S.src_dtype, S.dst_dtype, stage_shape(S)};
}

size_t args_size(int kind)
{
    if (kind == kKernelGroupLds) return sizeof(GroupArgs);
    if (kind == kKernelAnchored) return sizeof(AnchorArgs);
    return sizeof(StageArgs);
}

// Device bytes of one grid's records: n argument structs, then n + 1 prefix entries.
int64_t class_bytes(int kind, int64_t n)
{
    return round_up(round_up((int64_t)args_size(kind) * n, 16) + 4 * (n + 1), 256);
}

}  // namespace

int64_t batch_record_bytes(const std::vector<const PlanImpl *> &plans, int *n_launches)
{
    size_t waves = 0;
    for (const PlanImpl *P : plans) waves = std::max(waves, P->stages.size());
    int64_t bytes = 0;
    int nl = 0;
    for (size_t w = 0; w < waves; ++w) {
        std::map<ClassKey, int64_t> cls;
        for (const PlanImpl *P : plans)
            if (w < P->stages.size()) cls[class_key(*P, w)] += 1;
        for (const auto &kv : cls) {
            bytes += class_bytes(std::get<0>(kv.first), kv.second);
            ++nl;
        }
    }
    if (n_launches) *n_launches = nl;
    return bytes;
}

snd_status run_batch(const std::vector<Job> &jobs, void *d_records, int64_t records_bytes, void *stream,
                     int *n_launches)
{
    std::vector<const PlanImpl *> plans;
    for (const Job &j : jobs) plans.push_back(j.P);
    if (batch_record_bytes(plans, nullptr) > records_bytes) {
        set_error("record buffer smaller than the batch needs");
        return SND_ERR_NOMEM;
    }
    size_t waves = 0;
    for (const Job &j : jobs) waves = std::max(waves, j.P->stages.size());
    uint8_t *rec = static_cast<uint8_t *>(d_records);
    std::vector<uint8_t> host;
    int nl = 0;
    for (size_t w = 0; w < waves; ++w) {
        std::map<ClassKey, std::vector<Prepared>> cls;
        for (const Job &j : jobs) {
            if (w >= j.P->stages.size()) continue;
            if (j.run.n_run <= 0) continue;
            cls[class_key(*j.P, w)].push_back(
                prepare_stage(*j.P, w, j.run, j.in, j.in_pitch, j.out, j.out_pitch, j.ws, true));
        }
        for (auto &kv : cls) {
            std::vector<Prepared> &v = kv.second;
            const int kind = std::get<0>(kv.first);
            const int64_t n = (int64_t)v.size();
            const size_t asz = args_size(kind);
            const int64_t bytes = class_bytes(kind, n);
            const int64_t pre_off = round_up((int64_t)asz * n, 16);
            host.assign((size_t)bytes, 0);
            std::vector<int32_t> prefix((size_t)n + 1, 0);
            Prepared merged = v[0];
            for (int64_t r = 0; r < n; ++r) {
                const Prepared &p = v[(size_t)r];
                const void *src = kind == kKernelGroupLds ? (const void *)&p.gr
                                  : kind == kKernelAnchored ? (const void *)&p.an
                                                            : (const void *)&p.st;
                std::memcpy(host.data() + (size_t)r * asz, src, asz);
                if (p.nblocks > 0x7fffffffLL - prefix[(size_t)r]) {
                    set_error("batched grid exceeds 2^31 workgroups");
                    return SND_ERR_UNSUPPORTED;
                }
                prefix[(size_t)r + 1] = prefix[(size_t)r] + (int32_t)p.nblocks;
                merged.lds = std::max(merged.lds, p.lds);
                merged.max_len = std::max(merged.max_len, p.max_len);
                merged.n_run = std::max(merged.n_run, p.n_run);
                merged.bad_pitch = merged.bad_pitch || p.bad_pitch;
            }
            std::memcpy(host.data() + pre_off, prefix.data(), prefix.size() * sizeof(int32_t));
            // pageable source: the copy has consumed it when the call returns
            hipError_t e = hipMemcpyAsync(rec, host.data(), (size_t)bytes, hipMemcpyHostToDevice, (hipStream_t)stream);
            if (e != hipSuccess) {
                set_error(std::string("hipMemcpyAsync(batch records): ") + hipGetErrorString(e));
                return SND_ERR_HIP;
            }
            const Multi m{rec, reinterpret_cast<const int32_t *>(rec + pre_off), (int32_t)n};
            const int64_t total = prefix[(size_t)n];
            if (total > 0) {
                snd_status s = launch_prepared(merged, stream, m, total);
                if (s != SND_OK) return s;
                ++nl;
                // leaf grids of graded beams: each record's largest leaf value for its final stage
                bool bound = false;
                for (const Prepared &p : v) bound = bound || (kind == kKernelAnchored && p.an.bound_slots);
                if (bound) {
                    const int e = launch_bound_reduce_records(m, stream);
                    if (e) {
                        set_error(std::string("leaf bound reduction: ") + hipGetErrorString((hipError_t)e));
                        return SND_ERR_HIP;
                    }
                }
            }
            rec += bytes;
        }
    }
    if (n_launches) *n_launches = nl;
    return SND_OK;
}

}  // namespace snd

extern "C" {

snd_status snd_batch_records_bytes(int32_t nbeams, const snd_plan *plans, int64_t *bytes, int32_t *n_launches)
{
    if (nbeams < 1 || !plans || !bytes) {
        snd::set_error("nbeams must be >= 1 with non-null plans and output");
        return SND_ERR_INVALID;
    }
    std::vector<const snd::PlanImpl *> v;
    for (int32_t i = 0; i < nbeams; ++i) {
        if (!plans[i]) {
            snd::set_error("null plan");
            return SND_ERR_INVALID;
        }
        v.push_back(&plans[i]->impl);
    }
    int nl = 0;
    *bytes = snd::batch_record_bytes(v, &nl);
    if (n_launches) *n_launches = nl;
    return SND_OK;
}

snd_status snd_batch_execute(int32_t nbeams, const snd_plan *plans, const void *const *d_in, const int64_t *in_pitch,
                             void *const *d_out, const int64_t *out_pitch, void *const *d_workspace,
                             const int64_t *workspace_bytes, const int64_t *n_run, void *d_records,
                             int64_t records_bytes, void *stream, int32_t *h_launches)
{
    if (nbeams < 1 || !plans || !d_in || !in_pitch || !d_out || !out_pitch || !d_workspace || !workspace_bytes ||
        !d_records) {
        snd::set_error("null argument array or nbeams < 1");
        return SND_ERR_INVALID;
    }
    if (((uintptr_t)d_records & 255u) != 0) {
        snd::set_error("record buffer must be 256-byte aligned");
        return SND_ERR_INVALID;
    }
    std::vector<snd::Job> jobs;
    for (int32_t i = 0; i < nbeams; ++i) {
        const std::string who = "beam " + std::to_string(i) + ": ";
        if (!plans[i] || !d_in[i] || !d_out[i]) {
            snd::set_error(who + "null plan, input or output");
            return SND_ERR_INVALID;
        }
        const snd::PlanImpl &P = plans[i]->impl;
        if (!P.d_table) {
            snd::set_error(who + "plan tables not uploaded");
            return SND_ERR_STATE;
        }
        const int64_t nr = n_run ? n_run[i] : P.n_out;
        if (nr < 0 || nr > P.n_out) {
            snd::set_error(who + "n_run must be in 0..n_out");
            return SND_ERR_INVALID;
        }
        if (P.desc.in_dtype == SND_DT_BITS && in_pitch[i] % 32 != 0) {
            snd::set_error(who + "bit input pitch must be a multiple of 32 bits");
            return SND_ERR_INVALID;
        }
        if (in_pitch[i] < P.max_delay + nr || out_pitch[i] < nr) {
            snd::set_error(who + "input pitch below max_delay + n_run or output pitch below n_run");
            return SND_ERR_INVALID;
        }
        if (P.workspace_bytes > 0 &&
            (!d_workspace[i] || workspace_bytes[i] < P.workspace_bytes || ((uintptr_t)d_workspace[i] & 255u))) {
            snd::set_error(who + "workspace smaller than workspace_bytes or not 256-byte aligned");
            return SND_ERR_NOMEM;
        }
        for (int32_t j = 0; j < i; ++j)
            if (P.workspace_bytes > 0 && d_workspace[j] == d_workspace[i]) {
                snd::set_error(who + "beams of one batch need separate workspaces");
                return SND_ERR_INVALID;
            }
        snd::Job jb;
        jb.P = &P;
        jb.run = snd::Run{nr, P.max_delay + nr, 0, 0};
        jb.in = d_in[i];
        jb.in_pitch = in_pitch[i];
        jb.out = d_out[i];
        jb.out_pitch = out_pitch[i];
        jb.ws = d_workspace[i];
        jobs.push_back(jb);
    }
    int nl = 0;
    snd_status s = snd::run_batch(jobs, d_records, records_bytes, stream, &nl);
    if (h_launches) *h_launches = nl;
    return s;
}

}  // extern "C"
