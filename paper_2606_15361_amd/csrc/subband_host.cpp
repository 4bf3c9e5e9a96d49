// Approximate sub-band dedispersion, second step (snd_subband_combine): argument checks, the
// tables into the caller's workspace, one launch.
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>
#include <vector>

#include "snd_internal.h"

namespace snd {
int launch_subband_combine(const float *const *planes, const int64_t *pitches, const int32_t *coarse,
                           const int32_t *offs, int nsub, int ndm, float *out, int64_t op, int64_t n, void *stream);
}

namespace {

int64_t up256(int64_t x) { return (x + 255) / 256 * 256; }

struct Layout {
    int64_t planes = 0, pitches = 0, coarse = 0, offs = 0, end = 0;
};

Layout layout(int64_t ndm, int64_t nsub)
{
    Layout L;
    L.planes = 0;
    L.pitches = up256(L.planes + nsub * 8);
    L.coarse = up256(L.pitches + nsub * 8);
    L.offs = up256(L.coarse + ndm * 4);
    L.end = up256(L.offs + ndm * nsub * 4);
    return L;
}

snd_status fail(snd_status s, const std::string &m)
{
    snd::set_error(m);
    return s;
}

}  // namespace

extern "C" {

snd_status snd_subband_workspace_bytes(int32_t ndm, int32_t nsub, int64_t *bytes)
{
    if (ndm < 1 || nsub < 1 || !bytes) return fail(SND_ERR_INVALID, "ndm and nsub must be >= 1");
    *bytes = layout(ndm, nsub).end;
    return SND_OK;
}

snd_status snd_subband_combine(int32_t ndm, int32_t nsub, const float *const *d_planes, const int64_t *pitches,
                               const int64_t *n_valid, int32_t ncoarse, const int32_t *coarse_row,
                               const int32_t *offsets, float *d_out, int64_t out_pitch, int64_t n_out,
                               void *d_workspace, int64_t workspace_bytes, void *stream)
{
    if (ndm < 1 || nsub < 1 || ncoarse < 1 || !d_planes || !pitches || !n_valid || !coarse_row || !offsets ||
        !d_out || !d_workspace || n_out < 1 || out_pitch < n_out)
        return fail(SND_ERR_INVALID, "null argument, empty shape or output pitch below n_out");
    const Layout L = layout(ndm, nsub);
    if (workspace_bytes < L.end || ((uintptr_t)d_workspace & 255u))
        return fail(SND_ERR_NOMEM, "sub-band workspace too small or not 256-byte aligned");
    for (int32_t s = 0; s < nsub; ++s)
        if (!d_planes[s] || pitches[s] < n_valid[s]) return fail(SND_ERR_INVALID, "null plane or pitch below its samples");
    for (int32_t k = 0; k < ndm; ++k) {
        if (coarse_row[k] < 0 || coarse_row[k] >= ncoarse) return fail(SND_ERR_INVALID, "coarse row out of range");
        for (int32_t s = 0; s < nsub; ++s) {
            const int64_t o = offsets[(int64_t)k * nsub + s];
            if (o < 0 || o + n_out > n_valid[s]) return fail(SND_ERR_INVALID, "a read would pass a plane's valid samples");
        }
    }
    uint8_t *ws = static_cast<uint8_t *>(d_workspace);
    hipStream_t st = (hipStream_t)stream;
    // pageable sources: consumed when each copy call returns
    hipError_t e = hipMemcpyAsync(ws + L.planes, d_planes, (size_t)nsub * 8, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(ws + L.pitches, pitches, (size_t)nsub * 8, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(ws + L.coarse, coarse_row, (size_t)ndm * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ws + L.offs, offsets, (size_t)ndm * nsub * 4, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return fail(SND_ERR_HIP, std::string("sub-band tables: ") + hipGetErrorString(e));
    const int r = snd::launch_subband_combine(reinterpret_cast<const float *const *>(ws + L.planes),
                                              reinterpret_cast<const int64_t *>(ws + L.pitches),
                                              reinterpret_cast<const int32_t *>(ws + L.coarse),
                                              reinterpret_cast<const int32_t *>(ws + L.offs), nsub, ndm, d_out,
                                              out_pitch, n_out, stream);
    if (r) return fail(SND_ERR_HIP, std::string("sub-band combine: ") + hipGetErrorString((hipError_t)r));
    return SND_OK;
}

}  // extern "C"
