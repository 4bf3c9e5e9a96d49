// LDS-staged SND stage kernels for gfx950.
//
// k_group (final stage): a 1024-thread workgroup evaluates kGroupRows DMs adjacent in value
// over kGroupTile samples.  Adjacent DMs use the same lower-level neuron rows at nearly the
// same shifts, so for each batch of entries the workgroup stages one window per distinct
// (source row, offset cluster) in LDS, then every wave walks its DM's entries reading the
// shifted samples from LDS and evaluates the sub-tree in registers exactly as the generic
// stage kernel does (same node arithmetic, order and association).  Windows are copied from
// global memory straight into LDS (global_load_lds) two batches ahead into a ring of three
// buffers, so every copy has two batches of sums to land and one barrier per batch suffices.
//
// k_anchored (first stage from the input): one workgroup of kAnchorWaves waves per (tree node,
// window of the stage's anchor tile of reference samples, in sub-tiles of kAnchorTile).  Every neuron row of a node is anchored at its own smallest
// reference delay, so the neurons of one node read the node's channels at widely different
// offsets; staging the node's channels over the absolute window once and producing the
// overlapping segment of every neuron row reads each input sample once instead of once per
// neuron.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "group_common.h"

namespace snd {
namespace {

template <int MODE, typename TI, typename TO, int MAXD>
__global__ __launch_bounds__(1024) void k_group(GroupArgs s0, Multi m)
{
    using A = typename Acc<MODE>::type;
    GroupArgs s;
    uint32_t bid, nblk;
    select_record(s0, m, s, bid, nblk);
    constexpr int V = kGroupTile / 64;  // samples per lane
    constexpr int EU = MAXD <= 8 ? 8 : 4;  // entries per step
    extern __shared__ __align__(16) unsigned char smem[];
    TI *lds = reinterpret_cast<TI *>(smem);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    // time tile * ngroups + DM group, dealt so that the XCDs share time tiles (as k_group_fast)
    const uint32_t L = xcd_remap_chunked(bid, nblk, (uint32_t)s.xcd_chunk);
    const int g = (int)(L % (uint32_t)s.ngroups);
    const int t0 = (int)(L / (uint32_t)s.ngroups) * kGroupTile;
    const int vt = s.n_out - t0 < kGroupTile ? s.n_out - t0 : kGroupTile;
    const int row = __builtin_amdgcn_readfirstlane(as_const(s.grp_rows)[g * kGroupRows + wave]);
    const_ptr<uint32_t> lb = as_const(s.ldsb) + (int64_t)(g * kGroupRows + wave) * s.n_entries;
    const unsigned char *srcb = static_cast<const unsigned char *>(s.src);
    const_ptr<int32_t> batches = as_const(s.batches);  // 4 ints per batch
    const_ptr<int32_t> instrs = as_const(s.instrs);    // 4 ints per copy instruction
    const int64_t pitch_bytes = s.src_pitch * (int64_t)sizeof(TI);

    A acc[MAXD][V];
    A out[V];
#pragma unroll
    for (int j = 0; j < MAXD; ++j)
#pragma unroll
        for (int v = 0; v < V; ++v) acc[j][v] = 0;
#pragma unroll
    for (int v = 0; v < V; ++v) out[v] = 0;

    // asynchronous copy of this wave's windows of batch b into LDS buffer buf
    auto issue = [&](int b, int buf) {
        return issue_batch<TI>(batches, instrs, b, wave, lane, srcb, pitch_bytes, t0, vt, lds + buf * s.buf_elems);
    };

    const int b0 = as_const(s.batch_ptr)[g], b1 = as_const(s.batch_ptr)[g + 1];
    int n1 = 0, n2 = 0;  // copies outstanding for batches b+1 and b+2
    if (b0 < b1) issue(b0, 0);
    if (b0 + 1 < b1) n1 = issue(b0 + 1, 1);
    int buf = 0;
    for (int b = b0; b < b1; ++b) {
        wait_vmcnt(n1);   // this wave's copies of batch b have landed
        stage_barrier();  // everyone's have; everyone is done reading batch b - 1
        n2 = 0;
        if (b + 2 < b1) n2 = issue(b + 2, buf == 0 ? 2 : buf - 1);  // the buffer of batch b - 1
        if (row >= 0) {
            const int ex = batches[4 * b], ey = batches[4 * b + 1];
            const TI *base = lds + buf * s.buf_elems + lane;
            int e0 = ex;
            // full chunks: all table words, then all LDS reads, then the sums
            for (; e0 + EU <= ey; e0 += EU) {
                uint32_t x[EU];
#pragma unroll
                for (int u = 0; u < EU; ++u) x[u] = lb[e0 + u];
                A val[EU][V];
#pragma unroll
                for (int u = 0; u < EU; ++u) {
                    const TI *p = base + (x[u] & kRowMask);
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        A y = (A)Load<TI>::get(p + 64 * v);
                        if constexpr (MODE == SND_MODE_BINARY) y = y != 0;
                        val[u][v] = y;
                    }
                }
#pragma unroll
                for (int u = 0; u < EU; ++u) {
#pragma unroll
                    for (int v = 0; v < V; ++v) acc[0][v] += val[u][v];
                    close_levels<MODE, A, MAXD, V>(acc, out, (int)(x[u] >> 24), s.depth, s.src_is_input, s.k_leaf,
                                                   s.k_int, s.cap);
                }
            }
            for (; e0 < ey; ++e0) {
                const uint32_t x = lb[e0];
                const TI *p = base + (x & kRowMask);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    A y = (A)Load<TI>::get(p + 64 * v);
                    if constexpr (MODE == SND_MODE_BINARY) y = y != 0;
                    acc[0][v] += y;
                }
                close_levels<MODE, A, MAXD, V>(acc, out, (int)(x >> 24), s.depth, s.src_is_input, s.k_leaf, s.k_int,
                                               s.cap);
            }
        }
        n1 = n2;
        buf = buf == 2 ? 0 : buf + 1;
    }
    if (row >= 0) {
        const auto dst = as_global(static_cast<TO *>(s.dst)) + (int64_t)row * s.dst_pitch + t0 + lane;
#pragma unroll
        for (int v = 0; v < V; ++v)
            if (lane + 64 * v < vt) {
                if constexpr (MODE == SND_MODE_FLOAT) Store<TO>::put(dst + 64 * v, out[v] * s.scale);
                else Store<TO>::put(dst + 64 * v, out[v]);
            }
    }
}

template <int MODE, typename TI, typename TO, int MAXD>
__global__ __launch_bounds__(64 * kAnchorWaves) void k_anchored(AnchorArgs s0, Multi m)
{
    using A = typename Acc<MODE>::type;
    AnchorArgs s;
    uint32_t bid, nblk;
    select_record(s0, m, s, bid, nblk);
    constexpr int ST = kAnchorTile;  // samples per sub-tile: V per lane
    constexpr int V = ST / 64;
    constexpr int EU = 4;
    constexpr int NT = 64 * kAnchorWaves;
    extern __shared__ __align__(16) unsigned char smem[];
    TI *lds = reinterpret_cast<TI *>(smem);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    // every table value below is uniform: scalar loads through the constant address space
    const int node = __builtin_amdgcn_readfirstlane(as_const(s.tiles)[2 * bid]);
    const int tau0 = __builtin_amdgcn_readfirstlane(as_const(s.tiles)[2 * bid + 1]);
    const_ptr<int32_t> nd = as_const(s.nodes) + 6 * node;
    const int r0 = __builtin_amdgcn_readfirstlane(nd[0]), r1 = __builtin_amdgcn_readfirstlane(nd[1]);
    const int c0 = __builtin_amdgcn_readfirstlane(nd[2]), c1 = __builtin_amdgcn_readfirstlane(nd[3]);
    const int rho_max = __builtin_amdgcn_readfirstlane(nd[4]);
    // graded u8 rows: the largest value this workgroup computes, for the packed final stage
    constexpr bool kBound = MODE == SND_MODE_GRADED && std::is_same<TO, uint8_t>::value;
    uint32_t vmax = 0;
    if (tau0 >= nd[5] + s.n_run) {  // past every row of the node in this run (uniform per block)
        if (kBound && s.bound_slots && tid == 0) s.bound_slots[bid] = 0;
        return;
    }
    const_ptr<int32_t> row_lo = as_const(s.row_lo), row_len = as_const(s.row_len);
    const_ptr<uint32_t> row_ptr = as_const(s.row_ptr);
    const_ptr<uint32_t> ent = as_const(reinterpret_cast<const uint32_t *>(s.ent));  // (rowc, off) word pairs
    const int T = s.tile;  // a multiple of ST
    const int wst = T + rho_max;
    // staged as raw storage words of the element type
    using RT = typename std::conditional<sizeof(TI) == 1, uint8_t,
                                         typename std::conditional<sizeof(TI) == 2, uint16_t, uint32_t>::type>::type;
    static_assert(sizeof(RT) == sizeof(TI), "element storage");
    const auto src = as_global(static_cast<const RT *>(s.src));
    for (int c = c0; c < c1; ++c) {  // stage the node's channels over [tau0, tau0 + wst)
        const auto p = src + (int64_t)c * s.src_pitch;
        RT *l = reinterpret_cast<RT *>(lds) + (c - c0) * wst;
        for (int j0 = 0; j0 < wst; j0 += 4 * NT) {
            RT tmp[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int j = j0 + tid + NT * u;
                const int64_t idx = (int64_t)tau0 + j;
                int64_t col = idx + s.ring_start;  // ring column of window sample idx
                if (s.ring_len > 0 && col >= s.ring_len) col -= s.ring_len;
                tmp[u] = (j < wst && idx < s.src_len) ? p[col] : (RT)0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int j = j0 + tid + NT * u;
                if (j < wst) l[j] = tmp[u];
            }
        }
    }
    __syncthreads();
    for (int r = r0 + wave; r < r1; r += kAnchorWaves) {
        const int lo = row_lo[r], len = row_len[r] - s.len_cut;
        const uint32_t eb = row_ptr[r], ee = row_ptr[r + 1];
        if constexpr (MAXD == 1 && !std::is_same<TO, bits_t>::value) if (ee - eb == (uint32_t)EU) {
            // one-level rows of EU inputs (the leaf level of clusters of four channels): table
            // words once per row, stores without per-sample tests inside the row
            // rows of 1- or 2-byte elements: lane i owns the PK consecutive samples PK i + j
            // + 64 PK w (j < PK) of a sub-tile, so that each store writes a whole dword
            constexpr int PK = sizeof(TO) < 4 ? 4 / (int)sizeof(TO) : 1;
            static_assert(V % PK == 0, "whole dwords per lane");
            const TI *p[EU];
#pragma unroll
            for (int u = 0; u < EU; ++u)
                p[u] = lds - lo + PK * lane + ((int)(ent[2 * (eb + u)] & kRowMask) - c0) * wst +
                       (int32_t)ent[2 * (eb + u) + 1];
            // sample slot v of the lane: offset PK lane + off(v) in the sub-tile
            auto off = [](int v) { return (v % PK) + 64 * PK * (v / PK); };
            for (int sub = 0; sub < T; sub += ST) {
                const int i0 = tau0 + sub - lo;  // output index at the sub-tile start
                if (i0 >= len || i0 + ST <= 0) continue;
                A val[EU][V];
#pragma unroll
                for (int u = 0; u < EU; ++u)
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        A y = (A)Load<TI>::get(p[u] + sub + off(v));
                        if constexpr (MODE == SND_MODE_BINARY) y = y != 0;
                        val[u][v] = y;
                    }
                A out[V];
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    A a = val[0][v];
#pragma unroll
                    for (int u = 1; u < EU; ++u) a += val[u][v];
                    out[v] = activate<MODE>(a, 1, 1, s.k_leaf, s.k_int, s.cap);
                    if constexpr (kBound) vmax = max(vmax, (uint32_t)out[v]);
                }
                const auto dst = as_global(static_cast<TO *>(s.dst)) + (int64_t)r * s.dst_pitch + i0 + PK * lane;
                if constexpr (MODE == SND_MODE_FLOAT) {
#pragma unroll
                    for (int v = 0; v < V; ++v) out[v] *= s.scale;
                }
                // uniform: the whole sub-tile is inside the row (and, for packed stores, starts
                // on a dword)
                if (i0 >= 0 && i0 + ST <= len && (PK == 1 || ((uintptr_t)(dst - PK * lane) & 3u) == 0)) {
                    if constexpr (PK == 1) {
#pragma unroll
                        for (int v = 0; v < V; ++v) Store<TO>::put(dst + 64 * v, out[v]);
                    } else {
                        auto d32 = reinterpret_cast<global_ptr<uint32_t>>(dst);
#pragma unroll
                        for (int w = 0; w < V / PK; ++w) {
                            uint32_t word = 0;
#pragma unroll
                            for (int j = 0; j < PK; ++j)
                                word |= store_bits<TO>(out[PK * w + j]) << (8 * (int)sizeof(TO) * j);
                            d32[64 * w] = word;  // samples 64 PK w + PK lane .. + PK - 1
                        }
                    }
                } else {
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        const int i = i0 + PK * lane + off(v);
                        if (i >= 0 && i < len) Store<TO>::put(dst + off(v), out[v]);
                    }
                }
            }
            continue;
        }
        for (int sub = 0; sub < T; sub += ST) {  // sub-tiles of the window: the row's table words stay cached
            const int i0 = tau0 + sub - lo;  // output index at the sub-tile start
            if (i0 >= len || i0 + ST <= 0) continue;
            const TI *lsub = lds + sub - lo + lane;
            A acc[MAXD][V];
            A out[V];
#pragma unroll
            for (int j = 0; j < MAXD; ++j)
#pragma unroll
                for (int v = 0; v < V; ++v) acc[j][v] = 0;
#pragma unroll
            for (int v = 0; v < V; ++v) out[v] = 0;
            uint32_t e0 = eb;
            for (; e0 + EU <= ee; e0 += EU) {  // full chunks: table words, then LDS reads, then sums
                Entry en[EU];
#pragma unroll
                for (int u = 0; u < EU; ++u) en[u] = Entry{ent[2 * (e0 + u)], (int32_t)ent[2 * (e0 + u) + 1]};
                A val[EU][V];
#pragma unroll
                for (int u = 0; u < EU; ++u) {
                    const TI *p = lsub + ((int)(en[u].rowc & kRowMask) - c0) * wst + en[u].off;
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        A y = (A)Load<TI>::get(p + 64 * v);
                        if constexpr (MODE == SND_MODE_BINARY) y = y != 0;
                        val[u][v] = y;
                    }
                }
#pragma unroll
                for (int u = 0; u < EU; ++u) {
#pragma unroll
                    for (int v = 0; v < V; ++v) acc[0][v] += val[u][v];
                    close_levels<MODE, A, MAXD, V>(acc, out, (int)(en[u].rowc >> 24), s.depth, 1, s.k_leaf, s.k_int,
                                                   s.cap);
                }
            }
            for (; e0 < ee; ++e0) {
                const Entry en{ent[2 * e0], (int32_t)ent[2 * e0 + 1]};
                const TI *p = lsub + ((int)(en.rowc & kRowMask) - c0) * wst + en.off;
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    A y = (A)Load<TI>::get(p + 64 * v);
                    if constexpr (MODE == SND_MODE_BINARY) y = y != 0;
                    acc[0][v] += y;
                }
                close_levels<MODE, A, MAXD, V>(acc, out, (int)(en.rowc >> 24), s.depth, 1, s.k_leaf, s.k_int, s.cap);
            }
            if constexpr (std::is_same<TO, bits_t>::value) {
                // bit rows: i0 is a multiple of 64 (row anchors, tiles and sub-tiles are), so the
                // 64 samples lane + 64 v of a wave are the two words (i0 + 64 v) / 32 and the next;
                // samples outside the row are zero and words outside it are not written
                const auto rowp = as_global(reinterpret_cast<uint32_t *>(s.dst)) + (int64_t)r * (s.dst_pitch / 32);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const int i = i0 + lane + 64 * v;
                    const uint64_t mask = __ballot(i >= 0 && i < len && out[v] != 0);
                    const int w = ((i0 + 64 * v) >> 5) + (lane & 1);
                    if (lane < 2 && w >= 0 && 32 * w < len) rowp[w] = lane ? (uint32_t)(mask >> 32) : (uint32_t)mask;
                }
            } else {
                const auto dst = as_global(static_cast<TO *>(s.dst)) + (int64_t)r * s.dst_pitch + i0 + lane;
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const int i = i0 + lane + 64 * v;
                    if constexpr (kBound) vmax = max(vmax, (uint32_t)out[v]);
                    if (i >= 0 && i < len) {
                        if constexpr (MODE == SND_MODE_FLOAT) Store<TO>::put(dst + 64 * v, out[v] * s.scale);
                        else Store<TO>::put(dst + 64 * v, out[v]);
                    }
                }
            }
        }
    }
    if constexpr (kBound) {
        if (s.bound_slots) {  // uniform: every thread of the block gets here
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) vmax = max(vmax, (uint32_t)__shfl_xor((int)vmax, o, 64));
            // the staged window's first words, once every wave is done reading it (no static LDS,
            // which would cost the stage a resident workgroup per CU at its LDS target)
            uint32_t *wave_max = reinterpret_cast<uint32_t *>(smem);
            __syncthreads();
            if (lane == 0) wave_max[wave] = vmax;
            __syncthreads();
            if (tid == 0) {
                uint32_t m = 0;
                for (int w = 0; w < kAnchorWaves; ++w) m = max(m, wave_max[w]);
                s.bound_slots[bid] = m;
            }
        }
    }
}

// The largest of n per-workgroup words into slots[n]: one workgroup of 1024 threads, four
// independent loads in flight per thread.
__device__ __forceinline__ void bound_reduce(uint32_t *slots, int64_t n)
{
    __shared__ uint32_t wave_max[16];
    const auto src = as_global(static_cast<const uint32_t *>(slots));
    uint32_t m[4] = {0, 0, 0, 0};
    int64_t i = threadIdx.x;
    for (; i + 3 * 1024 < n; i += 4 * 1024) {
#pragma unroll
        for (int u = 0; u < 4; ++u) m[u] = max(m[u], src[i + 1024 * u]);
    }
    for (; i < n; i += 1024) m[0] = max(m[0], src[i]);
    uint32_t r = max(max(m[0], m[1]), max(m[2], m[3]));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) r = max(r, (uint32_t)__shfl_xor((int)r, o, 64));
    if ((threadIdx.x & 63) == 0) wave_max[threadIdx.x >> 6] = r;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < 16; ++w) t = max(t, wave_max[w]);
        slots[n] = t;
    }
}

__global__ __launch_bounds__(1024) void k_bound_reduce(uint32_t *slots, int64_t n) { bound_reduce(slots, n); }

// Batched leaf grids: workgroup r reduces the words of record r (its workgroup count from the
// prefix table), when the record tracks them.
__global__ __launch_bounds__(1024) void k_bound_reduce_records(Multi m)
{
    const int r = (int)blockIdx.x;
    const_ptr<int32_t> pre = as_const(m.prefix);
    const int64_t n = pre[r + 1] - pre[r];
    const auto *rec = static_cast<const AnchorArgs *>(m.recs) + r;
    uint32_t *slots = rec->bound_slots;
    if (!slots || n <= 0) return;
    bound_reduce(slots, n);
}

template <int MODE, typename TI, typename TO>
int launch_group_typed(const GroupArgs &a, int64_t n_out, int lds, hipStream_t st, const Multi &m, int64_t nb_multi)
{
    const int64_t ntt = (n_out + kGroupTile - 1) / kGroupTile;
    const int64_t nb = m.n > 0 ? nb_multi : (int64_t)a.ngroups * ntt;
    if (nb <= 0) return 0;
    if (nb > 0x7fffffffLL) return (int)hipErrorInvalidValue;
    dim3 grid((uint32_t)nb), block(1024);
    if (a.depth <= 1) hipLaunchKernelGGL((k_group<MODE, TI, TO, 1>), grid, block, lds, st, a, m);
    else if (a.depth <= 2) hipLaunchKernelGGL((k_group<MODE, TI, TO, 2>), grid, block, lds, st, a, m);
    else if (a.depth <= 4) hipLaunchKernelGGL((k_group<MODE, TI, TO, 4>), grid, block, lds, st, a, m);
    else if (a.depth <= 8) hipLaunchKernelGGL((k_group<MODE, TI, TO, 8>), grid, block, lds, st, a, m);
    else hipLaunchKernelGGL((k_group<MODE, TI, TO, 16>), grid, block, lds, st, a, m);
    return (int)hipGetLastError();
}

template <int MODE, typename TI, typename TO>
int launch_anchored_typed(const AnchorArgs &a, int64_t ntiles, int lds, hipStream_t st, const Multi &m)
{
    if (ntiles <= 0) return 0;
    if (ntiles > 0x7fffffffLL || a.depth > 8) return (int)hipErrorInvalidValue;
    if (a.tile < kAnchorTile || a.tile % kAnchorTile) return (int)hipErrorInvalidValue;
    dim3 grid((uint32_t)ntiles), block(64 * kAnchorWaves);
    if (a.depth <= 1) hipLaunchKernelGGL((k_anchored<MODE, TI, TO, 1>), grid, block, lds, st, a, m);
    else if (a.depth <= 2) hipLaunchKernelGGL((k_anchored<MODE, TI, TO, 2>), grid, block, lds, st, a, m);
    else if (a.depth <= 4) hipLaunchKernelGGL((k_anchored<MODE, TI, TO, 4>), grid, block, lds, st, a, m);
    else hipLaunchKernelGGL((k_anchored<MODE, TI, TO, 8>), grid, block, lds, st, a, m);
    return (int)hipGetLastError();
}

struct GroupLauncher {
    const GroupArgs &a;
    int64_t n_out;
    int lds;
    const Multi &m;
    int64_t nblocks;
    template <int MODE, typename TI, typename TO> int run(hipStream_t st) const
    {
        return launch_group_typed<MODE, TI, TO>(a, n_out, lds, st, m, nblocks);
    }
};

struct AnchorLauncher {
    const AnchorArgs &a;
    int64_t ntiles;
    int lds;
    const Multi &m;
    template <int MODE, typename TI, typename TO> int run(hipStream_t st) const
    {
        return launch_anchored_typed<MODE, TI, TO>(a, ntiles, lds, st, m);
    }
};

}  // namespace

int launch_group(int mode, int src_dt, int dst_dt, const GroupArgs &a, int64_t n_out, int lds_bytes, void *stream,
                 const Multi &m, int64_t nblocks)
{
    if (src_dt == SND_DT_BITS) {
        if (mode != SND_MODE_BINARY || dst_dt != SND_DT_U8 || a.f1 <= 0) return (int)hipErrorInvalidValue;
        return launch_group_bits(a, n_out, lds_bytes, stream, m, nblocks);
    }
    if (a.lin_kernel == 2) {
        if (mode != SND_MODE_GRADED || src_dt != SND_DT_U8 || dst_dt != SND_DT_U8) return (int)hipErrorInvalidValue;
        return launch_group_pack(a, n_out, lds_bytes, stream, m, nblocks);
    }
    if (a.lin_kernel) {
        if (mode != SND_MODE_FLOAT || dst_dt != SND_DT_F32) return (int)hipErrorInvalidValue;
        return launch_group_lin(src_dt, a, n_out, lds_bytes, stream, m, nblocks);
    }
    if (a.f1 > 0) {
        if (mode == SND_MODE_BINARY)
            return launch_group_fast_binary(src_dt, dst_dt, a, n_out, lds_bytes, stream, m, nblocks);
        if (mode == SND_MODE_GRADED)
            return launch_group_fast_graded(src_dt, dst_dt, a, n_out, lds_bytes, stream, m, nblocks);
        if (mode == SND_MODE_FLOAT)
            return launch_group_fast_float(src_dt, dst_dt, a, n_out, lds_bytes, stream, m, nblocks);
        return (int)hipErrorInvalidValue;
    }
    return dispatch_types(mode, src_dt, dst_dt, GroupLauncher{a, n_out, lds_bytes, m, nblocks}, (hipStream_t)stream);
}

int launch_anchored(int mode, int src_dt, int dst_dt, const AnchorArgs &a, int64_t ntiles, int lds_bytes, void *stream,
                    const Multi &m)
{
    if (src_dt == SND_DT_BITS) {
        if (mode != SND_MODE_BINARY || dst_dt != SND_DT_BITS) return (int)hipErrorInvalidValue;
        return launch_anchored_bits(a, ntiles, lds_bytes, stream, m);
    }
    if (dst_dt == SND_DT_BITS) {
        if (mode != SND_MODE_BINARY || src_dt != SND_DT_U8) return (int)hipErrorInvalidValue;
        return launch_anchored_typed<SND_MODE_BINARY, uint8_t, bits_t>(a, ntiles, lds_bytes, (hipStream_t)stream, m);
    }
    return dispatch_types(mode, src_dt, dst_dt, AnchorLauncher{a, ntiles, lds_bytes, m}, (hipStream_t)stream);
}

int launch_bound_reduce(uint32_t *slots, int64_t n, void *stream)
{
    if (!slots || n <= 0) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(k_bound_reduce, dim3(1), dim3(1024), 0, (hipStream_t)stream, slots, n);
    return (int)hipGetLastError();
}

int launch_bound_reduce_records(const Multi &m, void *stream)
{
    if (m.n <= 0) return 0;
    hipLaunchKernelGGL(k_bound_reduce_records, dim3((uint32_t)m.n), dim3(1024), 0, (hipStream_t)stream, m);
    return (int)hipGetLastError();
}

}  // namespace snd
