// Staging pipeline of the table-driven row-group kernels (the one-sum float kernel and the
// packed graded kernel): 16 waves of 1024 threads, each wave computing Sum::kRows DM rows of
// one DM group over a time tile of Sum::kStep samples.  The leaf windows of a batch of inputs
// are copied global -> LDS into one of two buffers while the other batch is summed: in full
// tiles by the 64-unit chunks the plan lists per (batch, wave), in the last tile window by
// window.  Each buffer also receives the wave's offset words of its batch (Sum::kWords per
// wave, Sum::kWords / 64 per lane); the scalar words of batch b + 1 (chunks, counts) are
// loaded while the wave waits for the barrier of batch b.
//
// A Sum policy provides the element types, the sizes above, the per-batch scalars it needs
// (Carry, taken from the scalar words before they are overwritten), the per-batch arithmetic
// and the store of one row; the sums live in a plain array of this function (`st`).
#pragma once

#include "group_common.h"

namespace snd {

// The pipeline for workgroup bid of nblk over the arguments s (its record, already selected).
template <class Sum>
__device__ __forceinline__ void group_tab_run(const GroupArgs &s, uint32_t bid, uint32_t nblk)
{
    using TI = typename Sum::TI;
    using A = typename Sum::A;
    constexpr int ES = (int)sizeof(TI);
    constexpr int R = Sum::kRows, T = Sum::kStep, NW = Sum::kWords, NSM = Sum::kSmemWords;
    constexpr int WPL = NW / 64;  // offset words per lane
    static_assert(WPL == 1 || WPL == 4, "one global_load_lds of 4 or 16 bytes per lane");
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    // logical tile = time tile * ngroups + DM group, dealt so that the XCDs share time tiles
    const uint32_t L = xcd_remap_chunked(bid, nblk, (uint32_t)s.xcd_chunk);
    const int g = (int)(L % (uint32_t)s.ngroups);
    const int t0 = (int)(L / (uint32_t)s.ngroups) * T;
    const int vt = s.n_out - t0 < T ? s.n_out - t0 : T;
    int row[R];
#pragma unroll
    for (int q = 0; q < R; ++q)
        row[q] = __builtin_amdgcn_readfirstlane(as_const(s.grp_rows)[(g * kGroupRows + wave) * R + q]);
    const unsigned char *srcb = static_cast<const unsigned char *>(s.src);
    const_ptr<int32_t> batches = as_const(s.batches);
    const_ptr<int32_t> instrs = as_const(s.instrs);
    const int64_t pitch_bytes = s.src_pitch * (int64_t)ES;
    const int buf_bytes = s.buf_elems * ES;
    const int stride = buf_bytes + kGroupRows * NW * 4;  // bytes of one buffer: windows, then offset words
    const bool full = vt == T;  // full tiles copy from the chunk table; the last tile by window

    A st[Sum::kState];
#pragma unroll
    for (int i = 0; i < Sum::kState; ++i) st[i] = 0;

    const_ptr<uint32_t> smem_tab = as_const(s.lin_smem);
    // this lane's 16-byte unit of the tile's first sample (t0 is a multiple of the unit's
    // samples); chunk sources add their unit index
    const uint4 *tile_src = reinterpret_cast<const uint4 *>(srcb) + (uint32_t)(t0 * ES) / 16u + lane;
    // Copies of batch bb into buffer j: this wave's chunks of its windows (scalar words blk), or
    // its windows one by one in the last tile, and the wave's offset words.
    auto issue = [&](int bb, const uint32_t (&blk)[NSM], int j) {
        unsigned char *buf_base = smem + j * stride;
        if (full) {
            const int nch = (int)blk[0];
#pragma unroll
            for (int c = 0; c < kLinMaxChunks; ++c) {
                if (c >= nch) break;
                const uint4 *gp = tile_src + blk[1 + c];
                auto lp = (__attribute__((address_space(3))) void *)(buf_base + blk[1 + kLinMaxChunks + c]);
                if (lane < (int)blk[1 + 2 * kLinMaxChunks + c]) __builtin_amdgcn_global_load_lds(gp, lp, 16, 0, 0);
            }
        } else {
            issue_batch<TI>(batches, instrs, bb, wave, lane, srcb, pitch_bytes, t0, vt,
                            reinterpret_cast<TI *>(buf_base));
        }
        const uint32_t *wp = s.lin + ((int64_t)bb * kGroupRows + wave) * NW + WPL * lane;
        __builtin_amdgcn_global_load_lds(wp, (__attribute__((address_space(3))) void *)(buf_base + buf_bytes + 4 * NW * wave),
                                         Sum::kWords / 16, 0, 0);
    };
    auto load_blk = [&](int bb, uint32_t (&blk)[NSM]) {
        const_ptr<uint32_t> p = smem_tab + ((int64_t)bb * kGroupRows + wave) * NSM;
#pragma unroll
        for (int i = 0; i < NSM; ++i) blk[i] = p[i];
    };

    const int b0 = as_const(s.batch_ptr)[g], b1 = as_const(s.batch_ptr)[g + 1];
    uint32_t blk[NSM];
    typename Sum::Carry cur{};
    if (b0 < b1) {
        load_blk(b0, blk);
        issue(b0, blk, 0);
        cur = Sum::carry(blk);
    }
    int slot = 0;
    for (int b = b0; b < b1; ++b) {
        // the scalar words of batch b + 1 load while this wave waits for its copies and the barrier
        if (b + 1 < b1) load_blk(b + 1, blk);
        __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0): this wave's copies of batch b have landed
        stage_barrier();  // everyone's have; everyone is done reading batch b - 1
        typename Sum::Carry nxt{};
        if (b + 1 < b1) {  // into the buffer of batch b - 1
            issue(b + 1, blk, slot ^ 1);
            nxt = Sum::carry(blk);
        }
        const unsigned char *buf_base = smem + slot * stride;
        Sum::add_batch(st, buf_base, buf_base + buf_bytes + 4 * NW * wave + 4 * WPL * lane, lane, cur, s);
        cur = nxt;
        slot ^= 1;
    }

#pragma unroll
    for (int q = 0; q < R; ++q) {
        if (row[q] < 0) continue;
        Sum::store(st, q, static_cast<typename Sum::TO *>(s.dst) + (int64_t)row[q] * s.dst_pitch + t0, lane, vt, s);
    }
}

template <class Sum>
__device__ __forceinline__ void group_tab_body(const GroupArgs &s0, const Multi &m)
{
    GroupArgs s;
    uint32_t bid, nblk;
    select_record(s0, m, s, bid, nblk);
    group_tab_run<Sum>(s, bid, nblk);
}

}  // namespace snd
