// Streaming form of the SND path (include/snd.h, "Streaming"): per-beam input rings in
// caller-owned device memory, admission against a byte budget, chunk pushes that compute the
// output samples whose dispersive sweep has fully arrived.
//
// A beam of plan P keeps the last R = max_delay + n_out input samples of every channel in a
// ring (row pitch padded to 256 bytes).  With S samples received and E = max(0, S - max_delay)
// outputs emitted, a chunk of L samples is copied to ring columns [S, S + L) mod R and the
// plan runs once over the window [E, S + L) of the ring: its n_run = max(0, S + L - max_delay)
// - E new outputs are bit-identical to those of a plain execute over the concatenated input,
// because the same kernels evaluate the same sums for every output time.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "snd_internal.h"

namespace {

constexpr uint64_t kMagic = 0x31564548444e53ULL;  // checkpoint tag
constexpr int64_t kHeaderBytes = 64;

snd_status fail(snd_status s, const std::string &msg)
{
    snd::set_error(msg);
    return s;
}

snd_status hip_fail(hipError_t e, const char *what)
{
    snd::set_error(std::string(what) + ": " + hipGetErrorString(e));
    return SND_ERR_HIP;
}

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

struct RingShape {
    int64_t ring_len;  // R
    int64_t pitch;     // elements per ring row
    int64_t es;        // bytes per element; 0 for bit input (one bit per sample)
    int64_t bytes;
};

// Bit input keeps one bit per sample: R is a whole number of 32-bit words, so that ring
// positions wrap at a word boundary, and rows are padded to 256 bytes.
RingShape ring_shape(const snd::PlanImpl &P)
{
    RingShape r{};
    if (P.desc.in_dtype == SND_DT_BITS) {
        r.es = 0;
        r.ring_len = round_up(P.max_delay + P.n_out, 32);
        r.pitch = round_up(r.ring_len, 2048);
        r.bytes = (int64_t)P.nchan * r.pitch / 8;
        return r;
    }
    r.es = snd::dtype_size(P.desc.in_dtype);
    r.ring_len = P.max_delay + P.n_out;
    r.pitch = round_up(r.ring_len * r.es, 256) / r.es;
    r.bytes = (int64_t)P.nchan * r.pitch * r.es;
    return r;
}

struct Beam {
    snd_plan plan = nullptr;
    uint8_t *ring = nullptr;
    RingShape shape{};
    int64_t received = 0;    // S
    int64_t emitted = 0;     // E
    int64_t next_chunk = -1; // -1: any index starts the history
    int64_t charge = 0;      // bytes charged against the budget (admission_charge)
};

// The state a beam can be in: nothing received (any chunk index starts it), or S >= 1 samples
// received with E = max(0, S - max_delay) outputs emitted and the next chunk index >= 1.
bool valid_state(int64_t received, int64_t emitted, int64_t next_chunk, int64_t max_delay)
{
    if (received == 0) return emitted == 0 && next_chunk == -1;
    return received > 0 && emitted == std::max<int64_t>(0, received - max_delay) && next_chunk >= 1;
}

struct Header {
    uint64_t magic;
    int64_t received, emitted, next_chunk, ring_len, pitch, es, nchan;
};
static_assert(sizeof(Header) == kHeaderBytes, "checkpoint header is 64 bytes");

// Bytes of one beam's share of a batched push workspace.
int64_t ws_share(const snd::PlanImpl &P) { return round_up(P.workspace_bytes, 256); }

// Device bytes a beam is charged at admission: its input ring plus its share of the workspace
// of a batched push, so that a budget that admits a set of beams also holds a batched push of
// all of them.
int64_t admission_charge(const snd::PlanImpl &P) { return ring_shape(P).bytes + ws_share(P); }

}  // namespace

struct snd_stream_s {
    int64_t budget = 0;
    int64_t used = 0;
    std::map<int32_t, Beam> beams;
};

extern "C" {

snd_status snd_stream_history_bytes(snd_plan plan, int64_t *bytes)
{
    if (!plan || !bytes) return fail(SND_ERR_INVALID, "null plan or output");
    *bytes = ring_shape(plan->impl).bytes;
    return SND_OK;
}

snd_status snd_stream_admission_bytes(snd_plan plan, int64_t *bytes)
{
    if (!plan || !bytes) return fail(SND_ERR_INVALID, "null plan or output");
    *bytes = admission_charge(plan->impl);
    return SND_OK;
}

snd_status snd_stream_create(int64_t hbm_budget_bytes, snd_stream *out)
{
    if (!out) return fail(SND_ERR_INVALID, "null output handle");
    *out = nullptr;
    if (hbm_budget_bytes <= 0) return fail(SND_ERR_INVALID, "budget must be > 0");
    snd_stream s = new (std::nothrow) snd_stream_s;
    if (!s) return fail(SND_ERR_NOMEM, "host allocation failed");
    s->budget = hbm_budget_bytes;
    *out = s;
    return SND_OK;
}

snd_status snd_stream_destroy(snd_stream s)
{
    delete s;
    return SND_OK;
}

snd_status snd_stream_admit(snd_stream s, int32_t beam_id, snd_plan plan, void *d_history, int64_t bytes)
{
    if (!s || !plan || !d_history) return fail(SND_ERR_INVALID, "null stream, plan or history buffer");
    if (beam_id < 0) return fail(SND_ERR_INVALID, "beam id must be >= 0");
    if (s->beams.count(beam_id)) return fail(SND_ERR_INVALID, "beam already admitted");
    const snd::PlanImpl &P = plan->impl;
    if (P.stages.empty() || P.stages[0].kernel != snd::kKernelAnchored || P.stages[0].final_stage)
        return fail(SND_ERR_UNSUPPORTED,
                    "streaming needs a plan whose first stage is the input-anchored kernel (default schedule)");
    if (((uintptr_t)d_history & 255u) != 0) return fail(SND_ERR_INVALID, "history buffer must be 256-byte aligned");
    const RingShape r = ring_shape(P);
    if (bytes < r.bytes) return fail(SND_ERR_NOMEM, "history buffer smaller than snd_stream_history_bytes");
    const int64_t charge = admission_charge(P);
    if (s->used + charge > s->budget)
        return fail(SND_ERR_CAPACITY, "admission would exceed the stream's device-memory budget (" +
                                          std::to_string(s->used) + " + " + std::to_string(charge) +
                                          " bytes of history ring and batched-push workspace > " +
                                          std::to_string(s->budget) + " bytes)");
    Beam b;
    b.plan = plan;
    b.ring = static_cast<uint8_t *>(d_history);
    b.shape = r;
    b.charge = charge;
    s->beams[beam_id] = b;
    s->used += charge;
    return SND_OK;
}

snd_status snd_stream_evict(snd_stream s, int32_t beam_id)
{
    if (!s) return fail(SND_ERR_INVALID, "null stream");
    auto it = s->beams.find(beam_id);
    if (it == s->beams.end()) return fail(SND_ERR_STATE, "beam not admitted");
    s->used -= it->second.charge;
    s->beams.erase(it);
    return SND_OK;
}

}  // extern "C"

namespace {

snd_status push_impl(snd_stream s, int32_t n, snd_stream_item *items, void *d_workspace, int64_t workspace_bytes,
                     void *d_records, int64_t records_bytes, bool batched, void *stream)
{
    if (!s || (n > 0 && !items)) return fail(SND_ERR_INVALID, "null stream or items");
    if (n < 0) return fail(SND_ERR_INVALID, "negative item count");
    // validate everything before any work
    std::vector<Beam *> bp((size_t)n);
    int64_t ws_total = 0;
    std::vector<const snd::PlanImpl *> plans;
    for (int32_t i = 0; i < n; ++i) {
        snd_stream_item &it = items[i];
        auto f = s->beams.find(it.beam_id);
        if (f == s->beams.end()) return fail(SND_ERR_STATE, "item " + std::to_string(i) + ": beam not admitted");
        for (int32_t j = 0; j < i; ++j)
            if (items[j].beam_id == it.beam_id) return fail(SND_ERR_INVALID, "a beam appears twice in one push");
        Beam &b = f->second;
        const snd::PlanImpl &P = b.plan->impl;
        if (!it.d_chunk || !it.d_out) return fail(SND_ERR_INVALID, "item " + std::to_string(i) + ": null chunk or output");
        if (it.chunk_len < 1 || it.chunk_len > P.n_out)
            return fail(SND_ERR_INVALID, "item " + std::to_string(i) + ": chunk_len must be in 1..n_out of the plan");
        if (it.chunk_pitch < it.chunk_len) return fail(SND_ERR_INVALID, "item " + std::to_string(i) + ": chunk pitch");
        if (P.desc.in_dtype == SND_DT_BITS && (it.chunk_pitch % 32 || ((uintptr_t)it.d_chunk & 3u)))
            return fail(SND_ERR_INVALID, "item " + std::to_string(i) + ": bit chunks need whole 32-bit words per row");
        if (it.out_pitch < P.n_out) return fail(SND_ERR_INVALID, "item " + std::to_string(i) + ": output pitch < n_out");
        if (it.chunk_idx < 0) return fail(SND_ERR_INVALID, "item " + std::to_string(i) + ": negative chunk index");
        if (!P.d_table) return fail(SND_ERR_STATE, "item " + std::to_string(i) + ": plan tables not uploaded");
        {
            // the outputs this chunk completes must fit the plan's output and workspace rows
            const bool gap = b.next_chunk >= 0 && it.chunk_idx != b.next_chunk;
            const int64_t S0 = gap ? 0 : b.received, E0 = gap ? 0 : b.emitted;
            const int64_t n_run = std::max<int64_t>(0, S0 + it.chunk_len - P.max_delay) - E0;
            if (n_run < 0 || n_run > P.n_out)
                return fail(SND_ERR_STATE, "item " + std::to_string(i) + ": beam state inconsistent with its plan");
        }
        ws_total += batched ? ws_share(P) : 0;
        if (!batched && P.workspace_bytes > 0 &&
            (!d_workspace || workspace_bytes < P.workspace_bytes || ((uintptr_t)d_workspace & 255u)))
            return fail(SND_ERR_NOMEM, "workspace smaller than the plan's workspace_bytes or not 256-byte aligned");
        plans.push_back(&P);
        bp[(size_t)i] = &b;
    }
    if (batched) {
        if (ws_total > 0 && (!d_workspace || workspace_bytes < ws_total || ((uintptr_t)d_workspace & 255u)))
            return fail(SND_ERR_NOMEM, "workspace smaller than the batch needs (snd_stream_batch_bytes) or not "
                                       "256-byte aligned");
        if (n > 0 && (!d_records || ((uintptr_t)d_records & 255u) ||
                      records_bytes < snd::batch_record_bytes(plans, nullptr)))
            return fail(SND_ERR_NOMEM, "record buffer smaller than the batch needs or not 256-byte aligned");
    }
    hipStream_t st = (hipStream_t)stream;
    snd_status ret = SND_OK;
    std::string gap_msg;
    std::vector<snd::Job> jobs;
    uint8_t *wsp = static_cast<uint8_t *>(d_workspace);
    for (int32_t i = 0; i < n; ++i) {
        snd_stream_item &it = items[i];
        Beam &b = *bp[(size_t)i];
        snd::PlanImpl &P = b.plan->impl;
        it.status = SND_OK;
        if (b.next_chunk >= 0 && it.chunk_idx != b.next_chunk) {  // lost or repeated chunk: start over
            it.status = SND_ERR_GAP;
            ret = SND_ERR_GAP;
            gap_msg += "beam " + std::to_string(it.beam_id) + " expected chunk " + std::to_string(b.next_chunk) +
                       ", got " + std::to_string(it.chunk_idx) + "; ";
            b.received = 0;
            b.emitted = 0;
        }
        const RingShape &r = b.shape;
        const int64_t L = it.chunk_len;
        // append the chunk at ring columns [S, S + L) mod R (two pieces when it wraps)
        const int64_t c0 = b.received % r.ring_len;
        const int64_t n1 = std::min(L, r.ring_len - c0);
        const uint8_t *src = static_cast<const uint8_t *>(it.d_chunk);
        hipError_t e = hipSuccess;
        if (r.es == 0) {  // bit rows: a kernel merges the chunk's bits into the ring's words
            const int rc = snd::launch_ring_put_bits(static_cast<const uint32_t *>(it.d_chunk), it.chunk_pitch / 32,
                                                     reinterpret_cast<uint32_t *>(b.ring), r.pitch / 32, r.ring_len,
                                                     c0, L, P.nchan, st);
            e = (hipError_t)rc;
        } else {
            e = hipMemcpy2DAsync(b.ring + c0 * r.es, (size_t)(r.pitch * r.es), src, (size_t)(it.chunk_pitch * r.es),
                                 (size_t)(n1 * r.es), (size_t)P.nchan, hipMemcpyDeviceToDevice, st);
            if (e == hipSuccess && n1 < L)
                e = hipMemcpy2DAsync(b.ring, (size_t)(r.pitch * r.es), src + n1 * r.es,
                                     (size_t)(it.chunk_pitch * r.es), (size_t)((L - n1) * r.es), (size_t)P.nchan,
                                     hipMemcpyDeviceToDevice, st);
        }
        if (e != hipSuccess) return hip_fail(e, "chunk into history");
        const int64_t S1 = b.received + L;
        const int64_t E1 = std::max<int64_t>(0, S1 - P.max_delay);
        const int64_t n_run = E1 - b.emitted;
        it.out_t0 = b.emitted;
        it.out_n = n_run;
        if (n_run > 0) {
            const snd::Run run{n_run, P.max_delay + n_run, r.ring_len, b.emitted % r.ring_len};
            if (batched) {
                jobs.push_back(snd::Job{&P, run, b.ring, r.pitch, it.d_out, it.out_pitch, wsp});
                wsp += ws_share(P);
            } else {
                for (size_t si = 0; si < P.stages.size(); ++si) {
                    snd_status rs =
                        snd::run_stage(P, si, run, b.ring, r.pitch, it.d_out, it.out_pitch, d_workspace, st);
                    if (rs != SND_OK) return rs;
                }
            }
        }
        b.received = S1;
        b.emitted = E1;
        b.next_chunk = it.chunk_idx + 1;
    }
    if (!jobs.empty()) {
        snd_status rs = snd::run_batch(jobs, d_records, records_bytes, st, nullptr);
        if (rs != SND_OK) return rs;
    }
    if (ret != SND_OK) snd::set_error("history reset after a chunk gap: " + gap_msg);
    return ret;
}

}  // namespace

extern "C" {

snd_status snd_stream_push(snd_stream s, int32_t n, snd_stream_item *items, void *d_workspace,
                           int64_t workspace_bytes, void *stream)
{
    return push_impl(s, n, items, d_workspace, workspace_bytes, nullptr, 0, false, stream);
}

snd_status snd_stream_push_batched(snd_stream s, int32_t n, snd_stream_item *items, void *d_workspace,
                                   int64_t workspace_bytes, void *d_records, int64_t records_bytes, void *stream)
{
    return push_impl(s, n, items, d_workspace, workspace_bytes, d_records, records_bytes, true, stream);
}

snd_status snd_stream_batch_bytes(snd_stream s, int32_t n, const int32_t *beam_ids, int64_t *workspace_bytes,
                                  int64_t *records_bytes)
{
    if (!s || n < 0 || (n > 0 && !beam_ids) || !workspace_bytes || !records_bytes)
        return fail(SND_ERR_INVALID, "null argument or negative count");
    std::vector<const snd::PlanImpl *> plans;
    int64_t ws = 0;
    for (int32_t i = 0; i < n; ++i) {
        auto f = s->beams.find(beam_ids[i]);
        if (f == s->beams.end()) return fail(SND_ERR_STATE, "beam not admitted");
        plans.push_back(&f->second.plan->impl);
        ws += ws_share(f->second.plan->impl);
    }
    *workspace_bytes = ws;
    *records_bytes = n > 0 ? snd::batch_record_bytes(plans, nullptr) : 0;
    return SND_OK;
}

snd_status snd_stream_beam_state(snd_stream s, int32_t beam_id, int64_t *received, int64_t *next_chunk,
                                 int64_t *emitted)
{
    if (!s) return fail(SND_ERR_INVALID, "null stream");
    auto it = s->beams.find(beam_id);
    if (it == s->beams.end()) return fail(SND_ERR_STATE, "beam not admitted");
    if (received) *received = it->second.received;
    if (next_chunk) *next_chunk = it->second.next_chunk;
    if (emitted) *emitted = it->second.emitted;
    return SND_OK;
}

snd_status snd_stream_usage(snd_stream s, int64_t *budget, int64_t *used, int32_t *n_beams)
{
    if (!s) return fail(SND_ERR_INVALID, "null stream");
    if (budget) *budget = s->budget;
    if (used) *used = s->used;
    if (n_beams) *n_beams = (int32_t)s->beams.size();
    return SND_OK;
}

snd_status snd_stream_export_bytes(snd_stream s, int32_t beam_id, int64_t *bytes)
{
    if (!s || !bytes) return fail(SND_ERR_INVALID, "null stream or output");
    auto it = s->beams.find(beam_id);
    if (it == s->beams.end()) return fail(SND_ERR_STATE, "beam not admitted");
    *bytes = kHeaderBytes + it->second.shape.bytes;
    return SND_OK;
}

snd_status snd_stream_export(snd_stream s, int32_t beam_id, void *h_buf, int64_t bytes, void *stream)
{
    if (!s || !h_buf) return fail(SND_ERR_INVALID, "null stream or buffer");
    auto it = s->beams.find(beam_id);
    if (it == s->beams.end()) return fail(SND_ERR_STATE, "beam not admitted");
    const Beam &b = it->second;
    if (bytes < kHeaderBytes + b.shape.bytes) return fail(SND_ERR_NOMEM, "buffer smaller than snd_stream_export_bytes");
    Header h{kMagic, b.received, b.emitted, b.next_chunk, b.shape.ring_len, b.shape.pitch, b.shape.es,
             (int64_t)b.plan->impl.nchan};
    std::memcpy(h_buf, &h, sizeof h);
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(static_cast<uint8_t *>(h_buf) + kHeaderBytes, b.ring, (size_t)b.shape.bytes,
                                  hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "export copy");
    return SND_OK;
}

snd_status snd_stream_import(snd_stream s, int32_t beam_id, const void *h_buf, int64_t bytes, void *stream)
{
    if (!s || !h_buf) return fail(SND_ERR_INVALID, "null stream or buffer");
    auto it = s->beams.find(beam_id);
    if (it == s->beams.end()) return fail(SND_ERR_STATE, "beam not admitted");
    Beam &b = it->second;
    if (bytes < kHeaderBytes) return fail(SND_ERR_INVALID, "buffer too small for a checkpoint");
    Header h;
    std::memcpy(&h, h_buf, sizeof h);
    if (h.magic != kMagic) return fail(SND_ERR_INVALID, "not a stream checkpoint");
    if (h.ring_len != b.shape.ring_len || h.pitch != b.shape.pitch || h.es != b.shape.es ||
        h.nchan != b.plan->impl.nchan)
        return fail(SND_ERR_INVALID, "checkpoint ring shape differs from the beam's plan");
    if (bytes < kHeaderBytes + b.shape.bytes) return fail(SND_ERR_INVALID, "checkpoint truncated");
    if (!valid_state(h.received, h.emitted, h.next_chunk, b.plan->impl.max_delay))
        return fail(SND_ERR_INVALID, "corrupt checkpoint state (received, emitted and next chunk index do not "
                                     "fit the beam's plan)");
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(b.ring, static_cast<const uint8_t *>(h_buf) + kHeaderBytes, (size_t)b.shape.bytes,
                                  hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "import copy");
    b.received = h.received;
    b.emitted = h.emitted;
    b.next_chunk = h.next_chunk;
    return SND_OK;
}

}  // extern "C"
