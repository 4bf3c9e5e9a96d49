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

// Asynchronous copy of this wave's windows of batch b (windows wave, wave + kGroupRows, ...)
// into the LDS buffer `dst`, straight from global memory to LDS in 16-byte units, 64 units (one
// per lane, 1 KB) per instruction.  A window's descriptor is (source row, element offset of its
// 16-byte aligned footprint, LDS byte offset of the footprint, head + span); for a tile of vt
// samples it covers head + span + vt elements.  Returns the number of copy instructions issued.
template <typename TI>
__device__ inline int issue_batch(const_ptr<int32_t> batches, const_ptr<int32_t> instrs, int b, int wave, int lane,
                                  const unsigned char *srcb, int64_t pitch_bytes, int t0, int vt, TI *dst)
{
    constexpr int ES = (int)sizeof(TI);
    const int bz = batches[4 * b + 2], bw = batches[4 * b + 3];
    unsigned char *ldsb = reinterpret_cast<unsigned char *>(dst);
    int n_ins = 0;
    for (int si = bz + wave; si < bw; si += kGroupRows) {
        {
            const int srow = instrs[4 * si], eoff = instrs[4 * si + 1], lbyte = instrs[4 * si + 2];
            const int hs = instrs[4 * si + 3];
            // row and offsets are non-negative and a row pitch is below 4 GiB (checked on the host)
            const uint4 *gp = reinterpret_cast<const uint4 *>(srcb + (uint64_t)(uint32_t)srow * (uint32_t)pitch_bytes +
                                                              (uint64_t)(uint32_t)(eoff + t0) * ES) + lane;
            unsigned char *lp = ldsb + lbyte;
            const int nu = ((hs + vt) * ES + 15) >> 4;  // 16-byte units of the window for this tile
            int u0 = 0;
            for (; u0 + 64 <= nu; u0 += 64) {  // whole instructions, no mask
                __builtin_amdgcn_global_load_lds(gp + u0, (__attribute__((address_space(3))) void *)(lp + 16 * u0), 16,
                                                 0, 0);
                ++n_ins;
            }
            if (u0 < nu) {
                if (u0 + lane < nu)
                    __builtin_amdgcn_global_load_lds(gp + u0, (__attribute__((address_space(3))) void *)(lp + 16 * u0),
                                                     16, 0, 0);
                ++n_ins;
            }
        }
    }
    return n_ins;
}

// Copy one window (descriptor as in issue_batch) of the tile into LDS; returns the number of
// copy instructions issued.
template <typename TI>
__device__ inline int issue_window(int srow, int eoff, int lbyte, int hs, int lane, const unsigned char *srcb,
                                   int64_t pitch_bytes, int t0, int vt, unsigned char *ldsb)
{
    constexpr int ES = (int)sizeof(TI);
    // row and offsets are non-negative and a row pitch is below 4 GiB (checked on the host)
    const uint4 *gp = reinterpret_cast<const uint4 *>(srcb + (uint64_t)(uint32_t)srow * (uint32_t)pitch_bytes +
                                                      (uint64_t)(uint32_t)(eoff + t0) * ES) + lane;
    unsigned char *lp = ldsb + lbyte;
    const int nu = ((hs + vt) * ES + 15) >> 4;  // 16-byte units of the window for this tile
    int u0 = 0;
    for (; u0 + 64 <= nu; u0 += 64)  // whole instructions, no mask
        __builtin_amdgcn_global_load_lds(gp + u0, (__attribute__((address_space(3))) void *)(lp + 16 * u0), 16, 0, 0);
    if (u0 < nu && u0 + lane < nu)
        __builtin_amdgcn_global_load_lds(gp + u0, (__attribute__((address_space(3))) void *)(lp + 16 * u0), 16, 0, 0);
    return (nu + 63) >> 6;
}

// A batch's table words for one wave: its entry range and window range, and the descriptors
// of the wave's first two windows.  Loaded a batch ahead of use, so that no wave waits for
// scalar loads between a barrier and its copies or its first LDS reads.
struct BatchWords {
    int ex, ey, bz, bw;
    int d[2][4];
};

__device__ inline void load_batch_words(const_ptr<int32_t> batches, const_ptr<int32_t> instrs, int b, int wave,
                                        BatchWords &w)
{
    w.ex = batches[4 * b];
    w.ey = batches[4 * b + 1];
    w.bz = batches[4 * b + 2];
    w.bw = batches[4 * b + 3];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int si = w.bz + wave + j * kGroupRows;
        if (si < w.bw) {  // uniform; windows past the batch are not read
#pragma unroll
            for (int i = 0; i < 4; ++i) w.d[j][i] = instrs[4 * si + i];
        }
    }
}

// issue_batch from preloaded words: the first two windows from w, any further ones loaded here.
// Returns the number of copy instructions issued.
template <typename TI>
__device__ inline int issue_batch_words(const BatchWords &w, const_ptr<int32_t> instrs, int wave, int lane,
                                        const unsigned char *srcb, int64_t pitch_bytes, int t0, int vt, TI *dst)
{
    unsigned char *ldsb = reinterpret_cast<unsigned char *>(dst);
    int si = w.bz + wave, n = 0;
#pragma unroll
    for (int j = 0; j < 2; ++j, si += kGroupRows)
        if (si < w.bw)
            n += issue_window<TI>(w.d[j][0], w.d[j][1], w.d[j][2], w.d[j][3], lane, srcb, pitch_bytes, t0, vt, ldsb);
    for (; si < w.bw; si += kGroupRows)
        n += issue_window<TI>(instrs[4 * si], instrs[4 * si + 1], instrs[4 * si + 2], instrs[4 * si + 3], lane, srcb,
                              pitch_bytes, t0, vt, ldsb);
    return n;
}

// Workgroup barrier for the staged kernels.  Every wave has already waited for its own copies
// into the buffer about to be read (wait_vmcnt), and every LDS read of the buffer about to be
// refilled has returned (its values were summed), so only the execution barrier is needed:
// unlike __syncthreads() this does not wait for the copies of the batches still in flight.  The
// empty asm statements keep the compiler from moving memory accesses across it.
__device__ inline void stage_barrier()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

int launch_group_bits(const GroupArgs &a, int64_t n_out, int lds, void *stream, const Multi &m, int64_t nblocks);
int launch_group_lin(int src_dt, const GroupArgs &a, int64_t n_out, int lds, void *stream, const Multi &m,
                     int64_t nblocks);
int launch_group_pack(const GroupArgs &a, int64_t n_out, int lds, void *stream, const Multi &m, int64_t nblocks);
int launch_anchored_bits(const AnchorArgs &a, int64_t ntiles, int lds, void *stream, const Multi &m);
int launch_group_fast_binary(int src_dt, int dst_dt, const GroupArgs &a, int64_t n_out, int lds, void *stream,
                             const Multi &m, int64_t nblocks);
int launch_group_fast_graded(int src_dt, int dst_dt, const GroupArgs &a, int64_t n_out, int lds, void *stream,
                             const Multi &m, int64_t nblocks);
int launch_group_fast_float(int src_dt, int dst_dt, const GroupArgs &a, int64_t n_out, int lds, void *stream,
                            const Multi &m, int64_t nblocks);

}  // namespace snd
