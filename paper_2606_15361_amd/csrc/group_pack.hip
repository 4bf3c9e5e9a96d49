// Final stage of a graded-mode plan on u8 rows with regular level-1 nodes (Methods, "Tree
// activation modes": every node's output is the sum of its inputs clipped at the cap, at every
// level up to the root).
//
// Staging is the table pipeline of the one-sum float kernel (group_tab.h).  Each wave computes
// two DM rows over a tile of 1024 samples (32 DM-adjacent rows per workgroup) where the open
// level sums of the shape allow (four inputs per level-1 node, depth <= 4), else four rows over
// 512 samples; lane i owns samples 4 i + 256 v.  An input at LDS byte offset o is read as the two aligned
// dwords that hold its four samples for the lane (one ds_read2_b32), and one byte permute per
// pair picks them out as two 16-bit counts: (samples 0, 2) and (samples 1, 3), whichever byte of
// the dword the input starts at.  Level sums are then formed two samples per instruction with
// 32-bit adds (fan-in x cap < 2^16, so the halves never carry into each other) and clipped with
// a packed 16-bit minimum; levels 2 .. D close with compile-time control as the plan's closing
// counts say.  Integer arithmetic in the tree's own order: the result is the tree's, bit for bit.
//
// When the stage that wrote the input plane reports its largest value m and F1 m < 256, a
// level-1 node's sums fit a byte per sample: each input's four samples are aligned into one
// dword (v_alignbyte_b32, whatever its byte phase), the F1 dwords are added as four bytes at
// once, and only the node's sum is split into 16-bit counts for the clip.  A sample position
// that holds no valid output (past the last tile's valid length) may carry out of its byte, but
// only into higher positions, which hold none either.
#include <hip/hip_runtime.h>

#include "group_tab.h"

namespace snd {

namespace {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ inline uint32_t pk_min_u16(uint32_t a, uint32_t b)
{
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_min(__builtin_bit_cast(u16x2, a),
                                                                   __builtin_bit_cast(u16x2, b)));
}

// st[(j * R + q) * K + k]: j = 0 .. D - 2 the open partial sums of levels 2 .. D, j = D - 1 the
// root; k = 2 v + h holds samples (h, h + 2) of the lane's four in block v.  BYTES: level-1 sums
// as four bytes per dword (the input plane's bound allows it).
template <int F1, int D, bool BYTES>
struct PackGraded {
    using TI = uint8_t;
    using TO = uint8_t;
    using A = uint32_t;
    static constexpr int kRows = pack_rows(F1, D), kStep = pack_tile(F1, D), kWords = kPackWords,
                         kSmemWords = kPackSmemWords;
    static constexpr int R = kRows, V = kStep / 256, K = 2 * V;
    static constexpr int OUT = D - 1;  // slot of the root
    static constexpr int kState = D * R * K;
    static_assert(F1 >= 3, "three-input adds");
    struct Carry {
        uint32_t close0, close1;  // levels completed by each level-1 node, 4 bits per node
        int n;
    };
    static __device__ __forceinline__ Carry carry(const uint32_t (&blk)[kPackSmemWords])
    {
        return Carry{blk[22], blk[23], (int)blk[kPackSmemWords - 1]};
    }
    static __device__ __forceinline__ A &at(A (&st)[kState], int j, int q, int k) { return st[(j * R + q) * K + k]; }

    // close levels J .. D after a node that completes c levels (closing level j implies every
    // level below it)
    template <int J>
    static __device__ __forceinline__ void close_from(A (&st)[kState], int c, uint32_t cap2)
    {
        if constexpr (J <= D) {
            if (c >= J) {
#pragma unroll
                for (int q = 0; q < R; ++q)
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        const uint32_t y = pk_min_u16(at(st, J - 2, q, k), cap2);
                        at(st, J - 2, q, k) = 0;
                        if constexpr (J == D) at(st, OUT, q, k) = y;
                        else at(st, J - 1, q, k) += y;
                    }
                close_from<J + 1>(st, c, cap2);
            }
        }
    }

    // the dword pairs holding the lane's samples of the F1 inputs of level-1 node j of one row
    // (offset words w), and per input the byte selector of its samples (0, 2); +0x00010001
    // gives samples (1, 3), and 0x0c fills a zero byte
    static __device__ __forceinline__ void load_row(uint32_t (&d)[F1][V][2], uint32_t (&sel)[F1], uint32_t w,
                                                    const unsigned char *lane_base, int j)
    {
#pragma unroll
        for (int u = 0; u < F1; ++u) {
            const uint32_t o = (uint32_t)__builtin_amdgcn_readlane((int)w, j * F1 + u);
            sel[u] = 0x0c020c00u + (o & 3u) * 0x00010001u;
            const uint32_t *p = reinterpret_cast<const uint32_t *>(lane_base + (o & ~3u));
#pragma unroll
            for (int v = 0; v < V; ++v) {
                d[u][v][0] = p[64 * v];
                d[u][v][1] = p[64 * v + 1];
            }
        }
    }

    // the same dword pairs, and per input its byte phase
    static __device__ __forceinline__ void load_row_bytes(uint32_t (&d)[F1][V][2], uint32_t (&ph)[F1], uint32_t w,
                                                          const unsigned char *lane_base, int j)
    {
#pragma unroll
        for (int u = 0; u < F1; ++u) {
            const uint32_t o = (uint32_t)__builtin_amdgcn_readlane((int)w, j * F1 + u);
            ph[u] = o & 3u;
            const uint32_t *p = reinterpret_cast<const uint32_t *>(lane_base + (o & ~3u));
#pragma unroll
            for (int v = 0; v < V; ++v) {
                d[u][v][0] = p[64 * v];
                d[u][v][1] = p[64 * v + 1];
            }
        }
    }

    // the level-1 nodes of one batch: for each, its F1 inputs per row, then the closes
    static __device__ __forceinline__ void add_batch(A (&st)[kState], const unsigned char *buf, const unsigned char *w,
                                                     int lane, const Carry &cr, const GroupArgs &s)
    {
        const uint4 w4 = *reinterpret_cast<const uint4 *>(w);  // component q: row q's input `lane`
        const uint32_t wq[4] = {w4.x, w4.y, w4.z, w4.w};
        const uint32_t cap2 = (uint32_t)s.cap * 0x00010001u;
        const unsigned char *lane_base = buf + 4 * lane;
        const int nn = cr.n / F1;
        if constexpr (BYTES) {
            for (int j = 0; j < nn; ++j) {
                const int c = (int)(((j < 8 ? cr.close0 : cr.close1) >> (4 * (j & 7))) & 15u);
#pragma unroll
                for (int q = 0; q < R; ++q) {
                    uint32_t d[F1][V][2], ph[F1];
                    load_row_bytes(d, ph, wq[q], lane_base, j);
                    uint32_t a[K];
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        uint32_t x[F1];
#pragma unroll
                        for (int u = 0; u < F1; ++u) x[u] = __builtin_amdgcn_alignbyte(d[u][v][1], d[u][v][0], ph[u]);
                        // four byte sums below 256 each: no carries between valid samples
                        uint32_t acc = x[0] + x[1] + x[2];
#pragma unroll
                        for (int u = 3; u < F1; u += 2) acc = u + 1 < F1 ? acc + x[u] + x[u + 1] : acc + x[u];
                        a[2 * v] = __builtin_amdgcn_perm(0u, acc, 0x0c020c00u);      // samples (0, 2)
                        a[2 * v + 1] = __builtin_amdgcn_perm(0u, acc, 0x0c030c01u);  // samples (1, 3)
                    }
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        const uint32_t y = pk_min_u16(a[k], cap2);
                        if constexpr (D == 1) at(st, OUT, q, k) = y;
                        else at(st, 0, q, k) += y;
                    }
                }
                close_from<2>(st, c, cap2);
            }
            return;
        }
        for (int j = 0; j < nn; ++j) {
            const int c = (int)(((j < 8 ? cr.close0 : cr.close1) >> (4 * (j & 7))) & 15u);
#pragma unroll
            for (int q = 0; q < R; ++q) {
                uint32_t d[F1][V][2], sel[F1];
                load_row(d, sel, wq[q], lane_base, j);
                // the node's sum of F1 permuted inputs, three at a time (v_add3_u32)
                uint32_t a[K];
#pragma unroll
                for (int v = 0; v < V; ++v)
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        uint32_t x[F1];
#pragma unroll
                        for (int u = 0; u < F1; ++u)
                            x[u] = __builtin_amdgcn_perm(d[u][v][1], d[u][v][0], sel[u] + (h ? 0x00010001u : 0u));
                        uint32_t acc = x[0] + x[1] + x[2];
#pragma unroll
                        for (int u = 3; u < F1; u += 2) acc = u + 1 < F1 ? acc + x[u] + x[u + 1] : acc + x[u];
                        a[2 * v + h] = acc;
                    }
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const uint32_t y = pk_min_u16(a[k], cap2);
                    if constexpr (D == 1) at(st, OUT, q, k) = y;
                    else at(st, 0, q, k) += y;
                }
            }
            close_from<2>(st, c, cap2);
        }
    }

    // root counts (<= cap <= 255) back to bytes: (s0, s2) | (s1, s3) << 8
    static __device__ __forceinline__ void store(const A (&st)[kState], int q, uint8_t *drow, int lane, int vt,
                                                 const GroupArgs &)
    {
        auto d = as_global(drow);
        const bool vec = (reinterpret_cast<uintptr_t>(drow) & 3u) == 0;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const uint32_t x = st[(OUT * R + q) * K + 2 * v] | (st[(OUT * R + q) * K + 2 * v + 1] << 8);
            const int t = 4 * lane + 256 * v;
            if (vec && t + 4 <= vt) {
                *reinterpret_cast<__attribute__((address_space(1))) uint32_t *>(d + t) = x;
            } else {
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    if (t + b < vt) d[t + b] = (uint8_t)(x >> (8 * b));
            }
        }
    }
};

}  // namespace

template <int F1, int D>
__global__ __launch_bounds__(1024) void k_group_pack(GroupArgs s0, Multi m)
{
    GroupArgs s;
    uint32_t bid, nblk;
    select_record(s0, m, s, bid, nblk);
    // per record (uniform per workgroup); the two bodies are separate so that neither holds the
    // other's registers
    if (s.bound && (uint32_t)F1 * as_const(s.bound)[0] <= 255u)
        group_tab_run<PackGraded<F1, D, true>>(s, bid, nblk);
    else
        group_tab_run<PackGraded<F1, D, false>>(s, bid, nblk);
}

namespace {

template <int F1, int D>
int launch_pack(const GroupArgs &a, int64_t n_out, int lds, void *stream, const Multi &m, int64_t nb_multi)
{
    const int64_t ntt = (n_out + pack_tile(F1, D) - 1) / pack_tile(F1, D);
    const int64_t nb = m.n > 0 ? nb_multi : (int64_t)a.ngroups * ntt;
    if (nb <= 0) return 0;
    if (nb > 0x7fffffffLL) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL((k_group_pack<F1, D>), dim3((uint32_t)nb), dim3(1024), lds, (hipStream_t)stream, a, m);
    return (int)hipGetLastError();
}

}  // namespace

// Every (inputs per level-1 node, depth) pair the plan builder admits for this kernel.
int launch_group_pack(const GroupArgs &a, int64_t n_out, int lds, void *stream, const Multi &m, int64_t nblocks)
{
#define SND_PACK(F, DD) \
    if (a.f1 == F && a.depth == DD) return launch_pack<F, DD>(a, n_out, lds, stream, m, nblocks);
    SND_PACK(4, 1) SND_PACK(4, 2) SND_PACK(4, 3) SND_PACK(4, 4) SND_PACK(4, 5)
    SND_PACK(8, 1) SND_PACK(8, 2) SND_PACK(8, 3) SND_PACK(8, 4)
#undef SND_PACK
    return (int)hipErrorInvalidValue;
}

}  // namespace snd
