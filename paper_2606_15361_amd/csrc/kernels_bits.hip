// Binary tree kernels on bit rows (Methods, "Tree activation modes", Mode A): the final stage
// and, for bit input, the leaf stage.
//
// The leaf stage stores every leaf neuron's output as one bit per sample.  Here a lane holds 32
// consecutive samples of a DM row in one 32-bit word, so every tree operation works on 32
// samples at once with bitwise logic:
//   - an input is the 32 bits of a staged leaf window at the row's offset, read as two aligned
//     words from LDS and funnel-shifted;
//   - a node's input count is kept bit-sliced (plane i holds bit i of every sample's count) and
//     incremented with a ripple of AND / XOR;
//   - the quorum count >= K is a bit-sliced comparison with the constant K;
//   - the root's bits are expanded to the 0/1 bytes of the output plane.
// Staging, batches, row groups and the closing pattern are those of the specialised row-group
// kernel (two DM rows per wave), with tiles of 2048 samples.  The counts and quorums are exact
// integers, so the output equals the byte-row kernels and the oracle bit for bit.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "group_common.h"

namespace snd {
namespace {

constexpr int kPlanes = 4;  // counts up to 15: leaf clusters of at most 15 channels
// bit planes for counts up to n
constexpr int planes_for(int n) { return n < 2 ? 1 : n < 4 ? 2 : n < 8 ? 3 : 4; }

// count += x (bit-sliced, one increment per set bit of x)
template <int NP>
__device__ inline void bs_add(uint32_t (&c)[NP], uint32_t x)
{
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        const uint32_t t = c[i] & x;
        c[i] ^= x;
        x = t;
    }
}

// bits where count >= k (k uniform, >= 1)
template <int NP>
__device__ inline uint32_t bs_ge(const uint32_t (&c)[NP], int k)
{
    if (k >= (1 << NP)) return 0u;
    uint32_t gt = 0u, eq = ~0u;
#pragma unroll
    for (int i = NP - 1; i >= 0; --i) {
        if ((k >> i) & 1) {
            eq &= c[i];
        } else {
            gt |= eq & c[i];
            eq &= ~c[i];
        }
    }
    return gt | eq;
}

// Copy this wave's windows of batch b into LDS: as issue_batch, with elements of one bit (the
// element offset and the window length are in bits, the copy units are 128 bits).
__device__ inline void issue_bits(const_ptr<int32_t> batches, const_ptr<int32_t> instrs, int b, int wave, int lane,
                                  const unsigned char *srcb, int64_t pitch_bytes, int t0, int vt, unsigned char *dst)
{
    const int bz = batches[4 * b + 2], bw = batches[4 * b + 3];
    for (int si = bz + wave; si < bw; si += kGroupRows) {
        const int srow = instrs[4 * si], eoff = instrs[4 * si + 1], lbyte = instrs[4 * si + 2];
        const int hs = instrs[4 * si + 3];
        // eoff and t0 are multiples of 128 bits: the footprint starts on a 16-byte boundary
        const uint4 *gp = reinterpret_cast<const uint4 *>(srcb + (uint64_t)(uint32_t)srow * (uint32_t)pitch_bytes +
                                                          ((uint64_t)(uint32_t)(eoff + t0) >> 3)) + lane;
        unsigned char *lp = dst + lbyte;
        const int nu = (hs + vt + 127) >> 7;  // 128-bit units of the window for this tile
        int u0 = 0;
        for (; u0 + 64 <= nu; u0 += 64)
            __builtin_amdgcn_global_load_lds(gp + u0, (__attribute__((address_space(3))) void *)(lp + 16 * u0), 16, 0, 0);
        if (u0 < nu && u0 + lane < nu)
            __builtin_amdgcn_global_load_lds(gp + u0, (__attribute__((address_space(3))) void *)(lp + 16 * u0), 16, 0, 0);
    }
}

// Levels J..D after an input that completes c levels (see the byte-row kernel): the level-J
// count's quorum goes to level J + 1 (or is the root) and the count restarts at zero.
template <int J, int D, int NS, int R, int NP>
__device__ inline void close_bits_from(int c, uint32_t (&cnt)[NS][R][NP], uint32_t (&out)[R], int k)
{
    if constexpr (J <= D) {
        if (c >= J) {
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const uint32_t y = bs_ge(cnt[J - 2][q], k);
#pragma unroll
                for (int i = 0; i < NP; ++i) cnt[J - 2][q][i] = 0u;
                if constexpr (J == D) out[q] = y;
                else bs_add(cnt[J - 1][q], y);
            }
            close_bits_from<J + 1, D, NS, R, NP>(c, cnt, out, k);
        }
    }
}

template <int F1, int D>
__global__ __launch_bounds__(1024) void k_group_bits(GroupArgs s0, Multi m)
{
    GroupArgs s;
    uint32_t bid, nblk;
    select_record(s0, m, s, bid, nblk);
    constexpr int T = kGroupTileBits;  // 32 samples per lane
    constexpr int R = kFastRows;       // DM rows per wave
    constexpr int NS = D > 1 ? D - 1 : 1;
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    // time tile * ngroups + DM group, dealt so that the XCDs share time tiles (as k_group_fast)
    const uint32_t L = xcd_remap_chunked(bid, nblk, (uint32_t)s.xcd_chunk);
    const int g = (int)(L % (uint32_t)s.ngroups);
    const int t0 = (int)(L / (uint32_t)s.ngroups) * T;
    const int vt = s.n_out - t0 < T ? s.n_out - t0 : T;
    int row[R];
#pragma unroll
    for (int q = 0; q < R; ++q)
        row[q] = __builtin_amdgcn_readfirstlane(as_const(s.grp_rows)[(g * kGroupRows + wave) * R + q]);
    // entry e of row q: byte offset of the word holding its first sample | bit offset << 27
    const_ptr<uint32_t> lb = as_const(s.ldsb) + (int64_t)(g * kGroupRows + wave) * s.n_entries * R;
    const_ptr<int32_t> closes = as_const(s.node_closes);
    const unsigned char *srcb = static_cast<const unsigned char *>(s.src);
    const_ptr<int32_t> batches = as_const(s.batches);
    const_ptr<int32_t> instrs = as_const(s.instrs);
    const int64_t pitch_bytes = s.src_pitch / 8;  // row pitch in bits (a multiple of 128)
    const int buf_bytes = s.buf_elems / 8;
    const int k1 = s.src_is_input ? s.k_leaf : s.k_int;  // quorum of the level-1 nodes

    // every node of the tree has at most F1 inputs (level-1 nodes exactly F1, the branching
    // factor; higher levels at most that), so counts fit NP bit planes
    constexpr int NP = planes_for(F1);
    uint32_t cnt[NS][R][NP];  // cnt[j - 2]: input count of the open level-j node, j = 2 .. D
    uint32_t out[R];
#pragma unroll
    for (int j = 0; j < NS; ++j)
#pragma unroll
        for (int q = 0; q < R; ++q)
#pragma unroll
            for (int i = 0; i < NP; ++i) cnt[j][q][i] = 0u;
#pragma unroll
    for (int q = 0; q < R; ++q) out[q] = 0u;

    const int b0 = as_const(s.batch_ptr)[g], b1 = as_const(s.batch_ptr)[g + 1];
    if (b0 < b1) issue_bits(batches, instrs, b0, wave, lane, srcb, pitch_bytes, t0, vt, smem);
    int buf = 0;
    for (int b = b0; b < b1; ++b) {
        __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0): this wave's copies of batch b have landed
        stage_barrier();                     // everyone's have; everyone is done reading batch b - 1
        if (b + 1 < b1) issue_bits(batches, instrs, b + 1, wave, lane, srcb, pitch_bytes, t0, vt, smem + (buf ^ 1) * buf_bytes);
        if (row[0] >= 0) {
            const int ex = batches[4 * b], ey = batches[4 * b + 1];
            const unsigned char *base = smem + buf * buf_bytes + 4 * lane;
            for (int c0 = ex; c0 < ey; c0 += F1) {  // one level-1 node per step
                const int c = closes[(uint32_t)c0 / F1];
                uint32_t x[F1][R];
#pragma unroll
                for (int u = 0; u < F1; ++u)
#pragma unroll
                    for (int q = 0; q < R; ++q) x[u][q] = lb[(c0 + u) * R + q];
                uint32_t a[R][NP];
#pragma unroll
                for (int q = 0; q < R; ++q)
#pragma unroll
                    for (int i = 0; i < NP; ++i) a[q][i] = 0u;
#pragma unroll
                for (int u = 0; u < F1; ++u)
#pragma unroll
                    for (int q = 0; q < R; ++q) {
                        const uint32_t w = x[u][q];
                        const uint32_t *p = reinterpret_cast<const uint32_t *>(base + (w & 0x07ffffffu));
                        const uint32_t lo = p[0], hi = p[1];
                        bs_add(a[q], __builtin_amdgcn_alignbit(hi, lo, w >> 27));
                    }
#pragma unroll
                for (int q = 0; q < R; ++q) {
                    const uint32_t y = bs_ge(a[q], k1);
                    if constexpr (D == 1) out[q] = y;
                    else bs_add(cnt[0][q], y);
                }
                close_bits_from<2, D, NS, R, NP>(c, cnt, out, s.k_int);
            }
        }
        buf ^= 1;
    }
    // root bits -> 0/1 bytes: lane holds samples t0 + 32 lane .. + 31
#pragma unroll
    for (int q = 0; q < R; ++q) {
        if (row[q] < 0) continue;
        const auto dst = as_global(static_cast<uint8_t *>(s.dst)) + (int64_t)row[q] * s.dst_pitch + t0 + 32 * lane;
        const int nv = vt - 32 * lane;  // valid samples of this lane
        if (nv >= 32 && ((uintptr_t)dst & 3u) == 0) {
            uint32_t wds[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const uint32_t nib = (out[q] >> (4 * k)) & 0xfu;
                wds[k] = (nib & 1u) | ((nib & 2u) << 7) | ((nib & 4u) << 14) | ((nib & 8u) << 21);
            }
            const auto d32 = reinterpret_cast<global_ptr<uint32_t>>(dst);
#pragma unroll
            for (int k = 0; k < 8; ++k) d32[k] = wds[k];
        } else {
            for (int i = 0; i < 32 && i < nv; ++i) dst[i] = (uint8_t)((out[q] >> i) & 1u);
        }
    }
}

// Leaf stage on bit input: one 256-thread workgroup per (leaf node, window of kAnchorTileBits
// reference samples), as the byte-input anchored kernel.  The node's channel windows are staged
// in LDS as words (bits past the valid input are cleared); a wave evaluates one leaf neuron row
// at a time, a lane holding the 32-sample words lane + 64 u of the tile: each input is a funnel
// shift of two staged words, the count is bit-sliced and the quorum count >= K_L is one
// bit-sliced comparison.  Row anchors and tiles are 64-aligned, so every output word is whole.
template <int W>
__global__ __launch_bounds__(256) void k_anchored_bits(AnchorArgs s0, Multi m)
{
    AnchorArgs s;
    uint32_t bid, nblk;
    select_record(s0, m, s, bid, nblk);
    constexpr int T = 64 * 32 * W;
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t *lds = reinterpret_cast<uint32_t *>(smem);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    // every table value below is uniform: scalar loads through the constant address space
    const int node = __builtin_amdgcn_readfirstlane(as_const(s.tiles)[2 * bid]);
    const int tau0 = __builtin_amdgcn_readfirstlane(as_const(s.tiles)[2 * bid + 1]);
    const_ptr<int32_t> nd = as_const(s.nodes) + 6 * node;
    const int r0 = __builtin_amdgcn_readfirstlane(nd[0]), r1 = __builtin_amdgcn_readfirstlane(nd[1]);
    const int c0 = __builtin_amdgcn_readfirstlane(nd[2]), c1 = __builtin_amdgcn_readfirstlane(nd[3]);
    const int rho_max = __builtin_amdgcn_readfirstlane(nd[4]);
    if (tau0 >= nd[5] + s.n_run) return;  // past every row of the node in this run (uniform per block)
    const_ptr<int32_t> row_lo = as_const(s.row_lo), row_len = as_const(s.row_len);
    const_ptr<uint32_t> row_ptr = as_const(s.row_ptr);
    const_ptr<uint32_t> ent = as_const(reinterpret_cast<const uint32_t *>(s.ent));  // (rowc, off) word pairs
    const int nw = 64 * W + (rho_max >> 5) + 1;  // staged words per channel
    const auto src = as_global(static_cast<const uint32_t *>(s.src));
    const int64_t wp = s.src_pitch >> 5;  // words per input row
    const int64_t w0 = tau0 >> 5;         // first staged word
    const int ntot = (c1 - c0) * nw;
    // a ring (streaming): sample i of the run sits at ring bit (ring_start + i) mod ring_len,
    // ring_len a whole number of words, so the run's word k is a funnel shift of ring words
    // q, q + 1 (mod the ring) with q = ring_start / 32 + k
    const int64_t rw = s.ring_len >> 5, q0 = s.ring_start >> 5;
    const uint32_t rb = (uint32_t)(s.ring_start & 31);
    for (int j = tid; j < ntot; j += 256) {
        const int c = j / nw, k = j - c * nw;
        const int64_t sb = 32 * (w0 + k);  // first sample of the word
        uint32_t v = 0u;
        if (sb < s.src_len) {
            const auto row = src + (int64_t)(c0 + c) * wp;
            if (rw > 0) {
                int64_t q = q0 + w0 + k;
                q = q >= rw ? q % rw : q;
                const int64_t q1 = q + 1 == rw ? 0 : q + 1;
                v = rb ? __builtin_amdgcn_alignbit(row[q1], row[q], rb) : row[q];
            } else {
                v = row[w0 + k];
            }
            const int64_t left = s.src_len - sb;
            if (left < 32) v &= (1u << left) - 1u;
        }
        lds[j] = v;
    }
    __syncthreads();
    for (int r = r0 + wave; r < r1; r += 4) {
        const int lo = row_lo[r], len = row_len[r] - s.len_cut;
        const int i0 = tau0 - lo;  // output index at the window start (a multiple of 64)
        if (i0 >= len || i0 + T <= 0) continue;
        uint32_t cnt[W][kPlanes];
#pragma unroll
        for (int u = 0; u < W; ++u)
#pragma unroll
            for (int i = 0; i < kPlanes; ++i) cnt[u][i] = 0u;
        const uint32_t eb = row_ptr[r], ee = row_ptr[r + 1];
        for (uint32_t e = eb; e < ee; ++e) {
            const int rho = (int32_t)ent[2 * e + 1] - lo;
            const uint32_t *p = lds + ((int)(ent[2 * e] & kRowMask) - c0) * nw + (rho >> 5) + lane;
            const uint32_t sh = (uint32_t)rho & 31u;
#pragma unroll
            for (int u = 0; u < W; ++u) bs_add(cnt[u], __builtin_amdgcn_alignbit(p[64 * u + 1], p[64 * u], sh));
        }
        const auto rowp = as_global(static_cast<uint32_t *>(s.dst)) + (int64_t)r * (s.dst_pitch >> 5);
#pragma unroll
        for (int u = 0; u < W; ++u) {
            const int wi = (i0 >> 5) + lane + 64 * u;  // output word of the row
            if (wi < 0 || 32 * wi >= len) continue;
            uint32_t y = bs_ge(cnt[u], s.k_leaf);
            const int left = len - 32 * wi;
            if (left < 32) y &= (1u << left) - 1u;
            rowp[wi] = y;
        }
    }
}

template <int F1, int D>
int launch_bits_shape(const GroupArgs &a, int64_t n_out, int lds, hipStream_t st, const Multi &m, int64_t nb_multi)
{
    const int64_t ntt = (n_out + kGroupTileBits - 1) / kGroupTileBits;
    const int64_t nb = m.n > 0 ? nb_multi : (int64_t)a.ngroups * ntt;
    if (nb <= 0) return 0;
    if (nb > 0x7fffffffLL) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL((k_group_bits<F1, D>), dim3((uint32_t)nb), dim3(1024), lds, st, a, m);
    return (int)hipGetLastError();
}

// A streamed bit chunk into its beam's ring: L bits of chunk row c (from bit 0) go to ring bit
// positions pos, pos + 1, ... of row c, wrapping at R (a whole number of words).  One thread per
// ring word touched (the positions [pos, min(pos + L, R)) and then [0, pos + L - R)); each word
// keeps its bits outside that range.  Bit by bit: a chunk is a few thousand bits per row.
__global__ __launch_bounds__(256) void k_ring_put_bits(const uint32_t *chunk, int64_t cw, uint32_t *ring, int64_t rwp,
                                                       int64_t R, int64_t pos, int64_t L)
{
    const int c = blockIdx.y;
    const int64_t e0 = pos + L < R ? pos + L : R;  // first segment [pos, e0), source bits from 0
    const int64_t e1 = pos + L - R;                // second segment [0, e1) when > 0, from R - pos
    const int64_t n0 = (e0 - 1) / 32 - pos / 32 + 1, n1 = e1 > 0 ? (e1 - 1) / 32 + 1 : 0;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n0 + n1) return;
    const int64_t a = i < n0 ? pos : 0, b = i < n0 ? e0 : e1, so = i < n0 ? 0 : R - pos;
    const int64_t w = i < n0 ? pos / 32 + i : i - n0;
    const uint32_t *src = chunk + (int64_t)c * cw;
    uint32_t v = ring[(int64_t)c * rwp + w];
    for (int k = 0; k < 32; ++k) {
        const int64_t p = 32 * w + k;
        if (p < a || p >= b) continue;
        const int64_t sbit = so + (p - a);
        const uint32_t bit = (src[sbit >> 5] >> (sbit & 31)) & 1u;
        v = (v & ~(1u << k)) | (bit << k);
    }
    ring[(int64_t)c * rwp + w] = v;
}

}  // namespace

int launch_ring_put_bits(const uint32_t *chunk, int64_t chunk_words, uint32_t *ring, int64_t ring_words, int64_t R,
                         int64_t pos, int64_t L, int nchan, void *stream)
{
    if (L < 1 || nchan < 1) return 0;
    if ((R & 31) != 0 || pos < 0 || pos >= R || L > R || 32 * chunk_words < L || 32 * ring_words < R)
        return (int)hipErrorInvalidValue;
    const int64_t words = L / 32 + 2;  // ring words one chunk can touch, at most
    hipLaunchKernelGGL(k_ring_put_bits, dim3((uint32_t)((words + 255) / 256), (uint32_t)nchan), dim3(256), 0,
                       (hipStream_t)stream, chunk, chunk_words, ring, ring_words, R, pos, L);
    return (int)hipGetLastError();
}

int launch_anchored_bits(const AnchorArgs &a, int64_t ntiles, int lds, void *stream, const Multi &m)
{
    if (ntiles <= 0) return 0;
    if (ntiles > 0x7fffffffLL || a.depth != 1 || (a.ring_len & 31) != 0) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL((k_anchored_bits<kAnchorBitsW>), dim3((uint32_t)ntiles), dim3(256), lds, (hipStream_t)stream, a,
                       m);
    return (int)hipGetLastError();
}

int launch_group_bits(const GroupArgs &a, int64_t n_out, int lds, void *stream, const Multi &m, int64_t nb)
{
    hipStream_t st = (hipStream_t)stream;
#define SND_BITS(F, DD) \
    if (a.f1 == F && a.depth == DD) return launch_bits_shape<F, DD>(a, n_out, lds, st, m, nb);
    SND_BITS(2, 1) SND_BITS(2, 2) SND_BITS(2, 3) SND_BITS(2, 4) SND_BITS(2, 5) SND_BITS(2, 6) SND_BITS(2, 7) SND_BITS(2, 8)
    SND_BITS(4, 1) SND_BITS(4, 2) SND_BITS(4, 3) SND_BITS(4, 4) SND_BITS(4, 5)
    SND_BITS(8, 1) SND_BITS(8, 2) SND_BITS(8, 3) SND_BITS(8, 4)
#undef SND_BITS
    return (int)hipErrorInvalidValue;
}

}  // namespace snd
