// Device pieces shared by the LDS row-group kernels: asynchronous global-to-LDS copy of a
// batch's windows, and a wait on a run-time count of outstanding vector-memory operations.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "snd_internal.h"
#include "stage_common.h"

namespace snd {

// Wait until at most n vector-memory operations of this wave are outstanding (n < 64).  Loads
// complete in issue order, so this waits for everything but the n most recent.  The count is
// known only at run time, so branch to the matching immediate.
__device__ inline void wait_vmcnt(int n)
{
#define SND_VM(N) __builtin_amdgcn_s_waitcnt(((N) & 15) | (((N) >> 4) << 14) | (7 << 4) | (15 << 8))
    switch (n) {
#define SND_VM4(B) case B: SND_VM(B); break; case B + 1: SND_VM(B + 1); break; \
                   case B + 2: SND_VM(B + 2); break; case B + 3: SND_VM(B + 3); break;
    SND_VM4(0) SND_VM4(4) SND_VM4(8) SND_VM4(12) SND_VM4(16) SND_VM4(20) SND_VM4(24) SND_VM4(28)
    SND_VM4(32) SND_VM4(36) SND_VM4(40) SND_VM4(44) SND_VM4(48) SND_VM4(52) SND_VM4(56) SND_VM4(60)
    default: SND_VM(0); break;
#undef SND_VM4
    }
#undef SND_VM
}

// Copy this wave's windows of batch b (windows wave, wave + kGroupRows, ...) into LDS buffer
// `dst` in 16-byte units straight from global memory to LDS (1 KB per instruction).  A window
// is (source row, start offset, span, LDS element offset); it covers span + vt samples from
// sample t0 + start, and its LDS footprint starts `start mod (elements per 16 bytes)` elements
// before its offset so that 16-byte copies from the 16-byte aligned source row land every
// element in place.  Returns the number of copy instructions issued.
template <typename TI>
__device__ inline int issue_windows(const_ptr<int32_t> batches, const_ptr<int32_t> slots, int b, int wave, int lane,
                                    const unsigned char *srcb, int64_t src_pitch, int t0, int vt, TI *dst)
{
    constexpr int ES = (int)sizeof(TI);
    constexpr int EPU = 16 / ES;  // elements per 16-byte unit
    const int bz = batches[4 * b + 2], bw = batches[4 * b + 3];
    int n_ins = 0;
#pragma unroll
    for (int k = 0; k < kGroupSlotsPerWave; ++k) {
        const int si = bz + wave + kGroupRows * k;
        if (si < bw) {
            const int srow = slots[4 * si], start = slots[4 * si + 1], span = slots[4 * si + 2];
            const int lofs = slots[4 * si + 3];
            const int head = start % EPU;
            const uint4 *gp =
                reinterpret_cast<const uint4 *>(srcb + ((int64_t)srow * src_pitch + t0 + start - head) * ES);
            uint4 *lp = reinterpret_cast<uint4 *>(dst + lofs - head);
            const int nu = ((head + span + vt) * ES + 15) / 16;  // 16-byte units
            int u0 = 0;
            for (; u0 + 64 <= nu; u0 += 64) {  // whole instructions, no mask
                __builtin_amdgcn_global_load_lds(gp + u0 + lane, (__attribute__((address_space(3))) void *)(lp + u0), 16,
                                                 0, 0);
                ++n_ins;
            }
            if (u0 < nu) {
                if (u0 + lane < nu)
                    __builtin_amdgcn_global_load_lds(gp + u0 + lane, (__attribute__((address_space(3))) void *)(lp + u0),
                                                     16, 0, 0);
                ++n_ins;
            }
        }
    }
    return n_ins;
}

int launch_group_fast_binary(int src_dt, int dst_dt, const GroupArgs &a, int64_t n_out, int lds, void *stream,
                             const Multi &m, int64_t nblocks);
int launch_group_fast_graded(int src_dt, int dst_dt, const GroupArgs &a, int64_t n_out, int lds, void *stream,
                             const Multi &m, int64_t nblocks);
int launch_group_fast_float(int src_dt, int dst_dt, const GroupArgs &a, int64_t n_out, int lds, void *stream,
                            const Multi &m, int64_t nblocks);

}  // namespace snd
