// Final stage of a float-mode plan as one sum per DM row (Methods, "Tree activation modes":
// float mode applies no activation, so the root of DM d is the plain sum of its leaf neurons,
// each read at its own delay; Eq. for y_d in "Incoherent dedispersion").
//
// Staging is that of the other row-group kernels: 16 waves of 1024 threads, leaf windows copied
// global -> LDS in double-buffered batches, full tiles by 64-unit chunks listed in the plan.  Each
// wave sums eight DM rows, so 128 DM-adjacent rows share the staged windows.  Lane i owns tile
// samples i + 64 v (v = 0 .. 7): an input starting at LDS byte offset o is read as eight dwords
// at o + 4 i + 256 v, which pair into stride-64 reads of two dwords; that read needs 4-byte
// alignment only, so every input takes the same path whatever its offset.
//
// Each row is summed in FP32 in the order the plan lists its inputs: an association of the exact
// sum that differs from the tree's, within the float tolerance of the FP64 definition.
#include <hip/hip_runtime.h>

#include "group_common.h"

namespace snd {

__global__ __launch_bounds__(1024) void k_group_lin(GroupArgs s0, Multi m)
{
    GroupArgs s;
    uint32_t bid, nblk;
    select_record(s0, m, s, bid, nblk);
    constexpr int T = kLinTile, R = kLinRows, V = kLinTile / 64;
    static_assert(R % 2 == 0, "rows are read two at a time");
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    // logical tile = time tile * ngroups + DM group, dealt so that the XCDs share time tiles
    const uint32_t L = xcd_remap_chunked(bid, nblk, (uint32_t)(s.ngroups >= 8 ? s.ngroups / 8 : 1));
    const int g = (int)(L % (uint32_t)s.ngroups);
    const int t0 = (int)(L / (uint32_t)s.ngroups) * T;
    const int vt = s.n_out - t0 < T ? s.n_out - t0 : T;
    const unsigned char *srcb = static_cast<const unsigned char *>(s.src);
    const_ptr<int32_t> batches = as_const(s.batches);
    const_ptr<int32_t> instrs = as_const(s.instrs);
    const int64_t pitch_bytes = s.src_pitch * (int64_t)sizeof(float);
    const int buf_bytes = s.buf_elems * (int)sizeof(float);
    static_assert(kLinBuffers == 2, "the table words below are loaded one batch ahead of a double buffer");
    const int stride = buf_bytes + kLinWordBytes;  // bytes of one buffer: windows, then offset words
    const bool full = vt == T;  // full tiles copy from the chunk table; the last tile by window

    float acc[R][V];
#pragma unroll
    for (int q = 0; q < R; ++q)
#pragma unroll
        for (int v = 0; v < V; ++v) acc[q][v] = 0.0f;

    const_ptr<uint32_t> smem_tab = as_const(s.lin_smem);
    // this lane's 16-byte unit of the tile's first sample; chunk sources add their unit index
    const uint4 *tile_src = reinterpret_cast<const uint4 *>(srcb) + (t0 >> 2) + lane;
    // Copies of batch bb into buffer j: this wave's chunks of its windows (scalar words blk), or
    // its windows one by one in the last tile, and the wave's offset words.
    auto issue = [&](int bb, const uint32_t (&blk)[kLinSmemWords], int j) {
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
            issue_batch<float>(batches, instrs, bb, wave, lane, srcb, pitch_bytes, t0, vt,
                               reinterpret_cast<float *>(buf_base));
        }
        const uint32_t *wp = s.lin + ((int64_t)bb * kGroupRows + wave) * kLinWords + lane;
        __builtin_amdgcn_global_load_lds(wp, (__attribute__((address_space(3))) void *)(buf_base + buf_bytes + 256 * wave),
                                         4, 0, 0);
    };
    auto load_blk = [&](int bb, uint32_t (&blk)[kLinSmemWords]) {
        const_ptr<uint32_t> p = smem_tab + ((int64_t)bb * kGroupRows + wave) * kLinSmemWords;
#pragma unroll
        for (int i = 0; i < kLinSmemWords; ++i) blk[i] = p[i];
    };

    const int b0 = as_const(s.batch_ptr)[g], b1 = as_const(s.batch_ptr)[g + 1];
    uint32_t blk[kLinSmemWords];
    int n_cur = 0;
    if (b0 < b1) {
        load_blk(b0, blk);
        issue(b0, blk, 0);
        n_cur = (int)blk[kLinSmemWords - 1];
    }
    int slot = 0;
    for (int b = b0; b < b1; ++b) {
        // the scalar words of batch b + 1 load while this wave waits for its copies and the barrier
        if (b + 1 < b1) load_blk(b + 1, blk);
        __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0): this wave's copies of batch b have landed
        stage_barrier();  // everyone's have; everyone is done reading batch b - 1
        int n_nxt = 0;
        if (b + 1 < b1) {  // into the buffer of batch b - 1
            issue(b + 1, blk, slot ^ 1);
            n_nxt = (int)blk[kLinSmemWords - 1];
        }
        const unsigned char *buf_base = smem + slot * stride;
        const uint32_t vw = *reinterpret_cast<const uint32_t *>(buf_base + buf_bytes + 256 * wave + 4 * lane);
        const unsigned char *lane_base = buf_base + 4 * lane;
        const int n = n_cur;
        for (int i = 0; i < n; ++i) {
#pragma unroll
            for (int q0 = 0; q0 < R; q0 += 2) {
                float x[2][V];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const uint32_t o = (uint32_t)__builtin_amdgcn_readlane((int)vw, (q0 + u) * n + i);
                    const float *p = reinterpret_cast<const float *>(lane_base + o);
#pragma unroll
                    for (int v = 0; v < V; ++v) x[u][v] = p[64 * v];
                }
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int v = 0; v < V; ++v) acc[q0 + u][v] += x[u][v];
            }
        }
        n_cur = n_nxt;
        slot ^= 1;
    }

#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = __builtin_amdgcn_readfirstlane(as_const(s.grp_rows)[(g * kGroupRows + wave) * R + q]);
        if (r < 0) continue;
        auto drow = as_global(static_cast<float *>(s.dst) + (int64_t)r * s.dst_pitch + t0);
#pragma unroll
        for (int v = 0; v < V; ++v)
            if (lane + 64 * v < vt) drow[lane + 64 * v] = acc[q][v] * s.scale;
    }
}

int launch_group_lin(const GroupArgs &a, int64_t n_out, int lds, void *stream, const Multi &m, int64_t nb_multi)
{
    const int64_t ntt = (n_out + kLinTile - 1) / kLinTile;
    const int64_t nb = m.n > 0 ? nb_multi : (int64_t)a.ngroups * ntt;
    if (nb <= 0) return 0;
    if (nb > 0x7fffffffLL) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(k_group_lin, dim3((uint32_t)nb), dim3(1024), lds, (hipStream_t)stream, a, m);
    return (int)hipGetLastError();
}

}  // namespace snd
