// Specialised LDS row-group kernel for final stages whose level-1 nodes all have F1 inputs
// (regular trees) and whose depth D is known at compile time.  Same staging pipeline as the
// general row-group kernel; the sums differ only in how the work is scheduled: the F1 inputs
// of a level-1 node are summed directly (the first one assigned, no zeroing), the node is
// activated, and levels 2..D are closed with compile-time control.  The node arithmetic, its
// order and its association are the tree's, so results equal every other schedule.
#pragma once

#include "group_common.h"

namespace snd {

// Levels J..D of the open sub-tree after an input that completes c levels: when c >= J the
// level-J node is complete, its activated sum goes to level J + 1 (or is the root's value)
// and its accumulator restarts at zero; only then can level J + 1 be complete as well.
template <int MODE, typename A, int J, int D, int NS, int R, int V>
__device__ inline void close_levels_from(int c, A (&stk)[NS][R][V], A (&out)[R][V], int src_is_input, int k_leaf,
                                         int k_int, int cap)
{
    if constexpr (J <= D) {
        if (c >= J) {
#pragma unroll
            for (int q = 0; q < R; ++q)
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const A y = activate<MODE>(stk[J - 2][q][v], J, src_is_input, k_leaf, k_int, cap);
                    stk[J - 2][q][v] = 0;
                    if constexpr (J == D) out[q][v] = y;
                    else stk[J - 1][q][v] += y;
                }
            close_levels_from<MODE, A, J + 1, D, NS, R, V>(c, stk, out, src_is_input, k_leaf, k_int, cap);
        }
    }
}

template <int MODE, typename TI, typename TO, int F1, int D>
__global__ __launch_bounds__(1024) void k_group_fast(GroupArgs s0, Multi m)
{
    using A = typename Acc<MODE>::type;
    GroupArgs s;
    uint32_t bid, nblk;
    select_record(s0, m, s, bid, nblk);
    constexpr int T = kGroupTileFast;
    constexpr int V = kFastV;            // samples per lane
    constexpr int R = kFastRows;         // DM rows per wave
    // inputs whose reads are issued together (fewer when the row registers are many)
    constexpr int SC = V * R > 8 ? (F1 < 2 ? F1 : 2) : (F1 < 4 ? F1 : 4);
    constexpr int NS = D > 1 ? D - 1 : 1;
    extern __shared__ __align__(16) unsigned char smem[];
    TI *lds = reinterpret_cast<TI *>(smem);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    // logical tile L = time tile * ngroups + DM group: each XCD takes an eighth of the DM groups
    // of a time tile, and the XCDs work on the same time tiles, whose leaf windows the DM
    // groups share
    const uint32_t L = xcd_remap_chunked(bid, nblk, (uint32_t)s.xcd_chunk);
    const int g = (int)(L % (uint32_t)s.ngroups);
    const int t0 = (int)(L / (uint32_t)s.ngroups) * T;
    const int vt = s.n_out - t0 < T ? s.n_out - t0 : T;
    int row[R];
#pragma unroll
    for (int q = 0; q < R; ++q)
        row[q] = __builtin_amdgcn_readfirstlane(as_const(s.grp_rows)[(g * kGroupRows + wave) * R + q]);
    // LDS byte offset of entry e of row q of this wave: lb[e * R + q]
    const_ptr<uint32_t> lb = as_const(s.ldsb) + (int64_t)(g * kGroupRows + wave) * s.n_entries * R;
    const_ptr<int32_t> closes = as_const(s.node_closes);
    const unsigned char *srcb = static_cast<const unsigned char *>(s.src);
    const_ptr<int32_t> batches = as_const(s.batches);
    const_ptr<int32_t> instrs = as_const(s.instrs);
    const int64_t pitch_bytes = s.src_pitch * (int64_t)sizeof(TI);

    A stk[NS][R][V];  // stk[j - 2]: partial sums of the open level-j node, j = 2 .. D
    A out[R][V];
#pragma unroll
    for (int j = 0; j < NS; ++j)
#pragma unroll
        for (int q = 0; q < R; ++q)
#pragma unroll
            for (int v = 0; v < V; ++v) stk[j][q][v] = 0;
#pragma unroll
    for (int q = 0; q < R; ++q)
#pragma unroll
        for (int v = 0; v < V; ++v) out[q][v] = 0;

    const int b0 = as_const(s.batch_ptr)[g], b1 = as_const(s.batch_ptr)[g + 1];
    static_assert(kFastBuffers == 2, "the pipeline below double-buffers");
    // table words of batches b (cur) and b + 1 (nxt); those of b + 2 are loaded during batch b
    BatchWords cur{}, nxt{};
    if (b0 < b1) {
        load_batch_words(batches, instrs, b0, wave, cur);
        issue_batch_words<TI>(cur, instrs, wave, lane, srcb, pitch_bytes, t0, vt, lds);
    }
    if (b0 + 1 < b1) load_batch_words(batches, instrs, b0 + 1, wave, nxt);
    int buf = 0;
    for (int b = b0; b < b1; ++b) {
        __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0): this wave's copies of batch b have landed
        stage_barrier();  // everyone's have; everyone is done reading batch b - 1
        if (b + 1 < b1)   // into the buffer of batch b - 1
            issue_batch_words<TI>(nxt, instrs, wave, lane, srcb, pitch_bytes, t0, vt, lds + (buf ^ 1) * s.buf_elems);
        const int ex = cur.ex, ey = cur.ey;
        cur = nxt;
        if (b + 2 < b1) load_batch_words(batches, instrs, b + 2, wave, nxt);
        if (row[0] >= 0) {
            const unsigned char *base = reinterpret_cast<const unsigned char *>(lds + buf * s.buf_elems + lane);
            for (int c0 = ex; c0 < ey; c0 += F1) {  // one level-1 node per step
                const int c = closes[(uint32_t)c0 / F1];  // levels completed by this node's last input
                uint32_t x[F1][R];
#pragma unroll
                for (int u = 0; u < F1; ++u)
#pragma unroll
                    for (int q = 0; q < R; ++q) x[u][q] = lb[(c0 + u) * R + q];
                A a1[R][V];
#pragma unroll
                for (int u0 = 0; u0 < F1; u0 += SC) {
                    A val[SC][R][V];
#pragma unroll
                    for (int u = 0; u < SC; ++u)
#pragma unroll
                        for (int q = 0; q < R; ++q) {
                            const TI *p = reinterpret_cast<const TI *>(base + x[u0 + u][q]);
#pragma unroll
                            for (int v = 0; v < V; ++v) {
                                A y = (A)Load<TI>::get(p + 64 * v);
                                if constexpr (MODE == SND_MODE_BINARY) y = y != 0;
                                val[u][q][v] = y;
                            }
                        }
#pragma unroll
                    for (int u = 0; u < SC; ++u)
#pragma unroll
                        for (int q = 0; q < R; ++q)
#pragma unroll
                            for (int v = 0; v < V; ++v) {
                                if (u0 + u == 0) a1[q][v] = val[u][q][v];
                                else a1[q][v] += val[u][q][v];
                            }
                }
#pragma unroll
                for (int q = 0; q < R; ++q)
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        const A y = activate<MODE>(a1[q][v], 1, s.src_is_input, s.k_leaf, s.k_int, s.cap);
                        if constexpr (D == 1) out[q][v] = y;
                        else stk[0][q][v] += y;
                    }
                // closing level j implies closing every level below it: nested tests
                close_levels_from<MODE, A, 2, D, NS, R, V>(c, stk, out, s.src_is_input, s.k_leaf, s.k_int, s.cap);
            }
        }
        buf ^= 1;
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
        if (row[q] < 0) continue;
        const auto dst = as_global(static_cast<TO *>(s.dst)) + (int64_t)row[q] * s.dst_pitch + t0 + lane;
#pragma unroll
        for (int v = 0; v < V; ++v)
            if (lane + 64 * v < vt) {
                if constexpr (MODE == SND_MODE_FLOAT) Store<TO>::put(dst + 64 * v, out[q][v] * s.scale);
                else Store<TO>::put(dst + 64 * v, out[q][v]);
            }
    }
}

template <int MODE, typename TI, typename TO, int F1, int D>
int launch_fast_shape(const GroupArgs &a, int64_t n_out, int lds, hipStream_t st, const Multi &m, int64_t nb_multi)
{
    const int64_t ntt = (n_out + kGroupTileFast - 1) / kGroupTileFast;
    const int64_t nb = m.n > 0 ? nb_multi : (int64_t)a.ngroups * ntt;
    if (nb <= 0) return 0;
    if (nb > 0x7fffffffLL) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL((k_group_fast<MODE, TI, TO, F1, D>), dim3((uint32_t)nb), dim3(1024), lds, st, a, m);
    return (int)hipGetLastError();
}

// Every (F1, depth) pair listed by group_fast_supported().
template <int MODE, typename TI, typename TO>
int launch_fast_typed(const GroupArgs &a, int64_t n_out, int lds, hipStream_t st, const Multi &m, int64_t nb)
{
#define SND_FAST(F, DD) \
    if (a.f1 == F && a.depth == DD) return launch_fast_shape<MODE, TI, TO, F, DD>(a, n_out, lds, st, m, nb);
    SND_FAST(2, 1) SND_FAST(2, 2) SND_FAST(2, 3) SND_FAST(2, 4) SND_FAST(2, 5) SND_FAST(2, 6) SND_FAST(2, 7) SND_FAST(2, 8)
    SND_FAST(4, 1) SND_FAST(4, 2) SND_FAST(4, 3) SND_FAST(4, 4) SND_FAST(4, 5)
    SND_FAST(8, 1) SND_FAST(8, 2) SND_FAST(8, 3) SND_FAST(8, 4)
#undef SND_FAST
    return (int)hipErrorInvalidValue;
}

}  // namespace snd
