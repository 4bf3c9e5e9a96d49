// snd_detect_launch_noalloc: the asynchronous detection launch with its device workspace in a
// fixed, file-scope device array instead of a caller-allocated buffer, for callers that cannot
// allocate device memory (code under graph capture, tight serving loops).
//
// The array lives once per GPU, at its own address on each.  Its name in host code is only a
// host-side stand-in, so its device address is taken with hipGetSymbolAddress, once per device
// with that device current, and only that address is ever handed to the kernels.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "snd.h"
#include "snd_internal.h"

namespace {

constexpr int64_t kScratchBytes = SND_DETECT_NOALLOC_MAX_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

snd_status fail(snd_status s, const std::string &msg)
{
    snd::set_error(msg);
    return s;
}

// Device address of this device's copy of the array, looked up on first use with the device
// current (and the caller's current device restored afterwards).
snd_status scratch_for(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(SND_ERR_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
        void *p = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur >= 0 && cur != dev) {
            const hipError_t r = hipSetDevice(cur);
            if (e == hipSuccess) e = r;
        }
        if (e != hipSuccess || !p)
            return fail(SND_ERR_HIP, std::string("hipGetSymbolAddress(detect scratch): ") + hipGetErrorString(e));
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return SND_OK;
}

}  // namespace

extern "C" snd_status snd_detect_launch_noalloc(snd_plan plan, const void *d_plane, int64_t plane_pitch,
                                                const snd_detect_desc *desc, void *h_stage, int64_t stage_bytes,
                                                void *stream)
{
    int64_t need = 0;
    snd_status s = snd_detect_workspace(plan, desc, &need);
    if (s != SND_OK) return s;
    if (need > kScratchBytes)
        return fail(SND_ERR_NOMEM, "detection needs a " + std::to_string(need) +
                                       "-byte workspace; the static scratch holds " + std::to_string(kScratchBytes) +
                                       " bytes (use snd_detect_launch with a caller workspace)");
    int dev = -1;
    hipError_t e = stream ? hipStreamGetDevice((hipStream_t)stream, &dev) : hipGetDevice(&dev);
    if (e != hipSuccess) return fail(SND_ERR_HIP, std::string("device of the stream: ") + hipGetErrorString(e));
    void *ws = nullptr;
    s = scratch_for(dev, &ws);
    if (s != SND_OK) return s;
    // the same launch as snd_detect_launch; its kernels clear the cell counter themselves
    return snd_detect_launch(plan, d_plane, plane_pitch, desc, ws, kScratchBytes, h_stage, stage_bytes, stream);
}
