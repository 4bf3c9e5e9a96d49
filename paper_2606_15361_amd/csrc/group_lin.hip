// Final stage of a float-mode plan as one sum per DM row (Methods, "Tree activation modes":
// float mode applies no activation, so the root of DM d is the plain sum of its leaf neurons,
// each read at its own delay; Eq. for y_d in "Incoherent dedispersion").
//
// Staging is that of the other row-group kernels: 16 waves of 1024 threads, leaf windows copied
// global -> LDS in double-buffered batches, full tiles by 64-unit chunks listed in the plan.  Each
// wave sums eight DM rows, so 128 DM-adjacent rows share the staged windows.  Every read is a
// dword at o + 4 i + 256 v for an input at LDS byte offset o (lane i, v = 0 .. 3 or 7), which
// pairs into stride-64 reads of two dwords and needs 4-byte alignment only:
//  * f32 rows: lane i owns samples i + 64 v, one per dword, and every input takes one path.
//  * bf16 / f16 rows: lane i owns the sample pairs (2 i + 128 v, 2 i + 1 + 128 v), one dword.
//    An input whose first sample sits in the upper half of a dword takes the upper half of that
//    dword and the lower half of the next one (a second read); the branch on that is uniform.
//    Samples are widened to FP32 exactly before they are added.
//
// Each row is summed in FP32 in the order the plan lists its inputs: an association of the
// exact sum that differs from the tree's, within the float tolerance of the FP64 definition.
#include <hip/hip_runtime.h>

#include "group_common.h"

namespace snd {

namespace {

constexpr int R = kLinRows;

// The sums of a wave live in a plain array of the kernel, `st`, which the policies below index
// (a struct holding them ended up in scratch memory).
//
// f32 rows: st[q * V + v] is sample lane + 64 v of row q.
struct LinF32 {
    using TI = float;
    static constexpr int kStep = kLinTile;
    static constexpr int V = kLinTile / 64;
    static constexpr int kState = R * V;

    // the n inputs of every row of the wave from the batch at buf; vw: the wave's offset words
    static __device__ __forceinline__ void add_batch(float (&st)[kState], const unsigned char *buf, int lane,
                                                     uint32_t vw, int n, uint32_t)
    {
        const unsigned char *lane_base = buf + 4 * lane;
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
                    for (int v = 0; v < V; ++v) st[(q0 + u) * V + v] += x[u][v];
            }
        }
    }
    static __device__ __forceinline__ void store(const float (&st)[kState], int q, float *drow, int lane, int vt,
                                                 float scale)
    {
        auto d = as_global(drow);
#pragma unroll
        for (int v = 0; v < V; ++v)
            if (lane + 64 * v < vt) d[lane + 64 * v] = st[q * V + v] * scale;
    }
};

// bf16 / f16 rows: st[LO + q * V + v] and st[HI + q * V + v] are samples 2 lane + 128 v and
// 2 lane + 1 + 128 v of row q.  An input whose first sample starts a dword is read as one
// dword per pair; one whose first sample sits in the upper half of a dword as the upper half of
// that dword and the lower half of the next (two reads per pair).  The plan lists each row's
// inputs of the first kind first.
template <bool F16>
struct Lin16 {
    using TI = uint16_t;
    static constexpr int kStep = kLinTile;
    static constexpr int V = kLinTile / 128;
    static constexpr int LO = 0, HI = R * V, kState = 2 * R * V;

    static __device__ inline float lower(uint32_t d)
    {
        if constexpr (F16) return (float)__builtin_bit_cast(_Float16, (uint16_t)(d & 0xffffu));
        else return __uint_as_float(d << 16);
    }
    static __device__ inline float upper(uint32_t d)
    {
        if constexpr (F16) return (float)__builtin_bit_cast(_Float16, (uint16_t)(d >> 16));
        else return __uint_as_float(d & 0xffff0000u);
    }
    // Row q's inputs that start a dword (the first even_q of its n words), then the others: two
    // loops per row without a branch per input, two inputs in flight.
    static __device__ __forceinline__ void add_batch(float (&st)[kState], const unsigned char *buf, int lane,
                                                     uint32_t vw, int n, uint32_t even)
    {
        const unsigned char *lane_base = buf + 4 * lane;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int k0 = q * n, ke = k0 + (int)((even >> (4 * q)) & 15u), k1 = k0 + n;
            int k = k0;
            for (; k + 2 <= ke; k += 2) {
                uint32_t x[2][V];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const uint32_t o = (uint32_t)__builtin_amdgcn_readlane((int)vw, k + u);
                    const uint32_t *p = reinterpret_cast<const uint32_t *>(lane_base + o);
#pragma unroll
                    for (int v = 0; v < V; ++v) x[u][v] = p[64 * v];
                }
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        st[LO + q * V + v] += lower(x[u][v]);
                        st[HI + q * V + v] += upper(x[u][v]);
                    }
            }
            if (k < ke) {
                const uint32_t o = (uint32_t)__builtin_amdgcn_readlane((int)vw, k);
                const uint32_t *p = reinterpret_cast<const uint32_t *>(lane_base + o);
                uint32_t x[V];
#pragma unroll
                for (int v = 0; v < V; ++v) x[v] = p[64 * v];
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    st[LO + q * V + v] += lower(x[v]);
                    st[HI + q * V + v] += upper(x[v]);
                }
                ++k;
            }
            // first sample in the upper half: that half of the dword, then the lower half of the next
            for (; k < k1; ++k) {
                const uint32_t o = (uint32_t)__builtin_amdgcn_readlane((int)vw, k);
                const uint32_t *p = reinterpret_cast<const uint32_t *>(lane_base + (o & ~3u));
                uint32_t x[V], y[V];
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    x[v] = p[64 * v];
                    y[v] = p[64 * v + 1];
                }
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    st[LO + q * V + v] += upper(x[v]);
                    st[HI + q * V + v] += lower(y[v]);
                }
            }
        }
    }
    static __device__ __forceinline__ void store(const float (&st)[kState], int q, float *drow, int lane, int vt,
                                                 float scale)
    {
        auto d = as_global(drow);
        const bool vec = (reinterpret_cast<uintptr_t>(drow) & 7u) == 0;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const float y0 = st[LO + q * V + v] * scale, y1 = st[HI + q * V + v] * scale;
            const int t = 2 * lane + 128 * v;
            if (vec && t + 1 < vt) {
                typedef float f32x2 __attribute__((ext_vector_type(2)));
                *reinterpret_cast<__attribute__((address_space(1))) f32x2 *>(d + t) = f32x2{y0, y1};
            } else {
                if (t < vt) d[t] = y0;
                if (t + 1 < vt) d[t + 1] = y1;
            }
        }
    }
};

}  // namespace

template <class Sum>
__global__ __launch_bounds__(1024) void k_group_lin(GroupArgs s0, Multi m)
{
    using TI = typename Sum::TI;
    constexpr int ES = (int)sizeof(TI);
    GroupArgs s;
    uint32_t bid, nblk;
    select_record(s0, m, s, bid, nblk);
    constexpr int T = Sum::kStep;
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    // logical tile = time tile * ngroups + DM group, dealt so that the XCDs share time tiles
    const uint32_t L = xcd_remap_chunked(bid, nblk, (uint32_t)(s.ngroups >= 8 ? s.ngroups / 8 : 1));
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
    static_assert(kLinBuffers == 2, "the table words below are loaded one batch ahead of a double buffer");
    const int stride = buf_bytes + kLinWordBytes;  // bytes of one buffer: windows, then offset words
    const bool full = vt == T;  // full tiles copy from the chunk table; the last tile by window

    float st[Sum::kState];
#pragma unroll
    for (int i = 0; i < Sum::kState; ++i) st[i] = 0.0f;

    const_ptr<uint32_t> smem_tab = as_const(s.lin_smem);
    // this lane's 16-byte unit of the tile's first sample (t0 is a multiple of the unit's
    // samples); chunk sources add their unit index
    const uint4 *tile_src = reinterpret_cast<const uint4 *>(srcb) + (uint32_t)(t0 * ES) / 16u + lane;
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
            issue_batch<TI>(batches, instrs, bb, wave, lane, srcb, pitch_bytes, t0, vt,
                            reinterpret_cast<TI *>(buf_base));
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
    uint32_t e_cur = 0;
    if (b0 < b1) {
        load_blk(b0, blk);
        issue(b0, blk, 0);
        n_cur = (int)blk[kLinSmemWords - 1];
        e_cur = blk[kLinSmemWords - 2];
    }
    int slot = 0;
    for (int b = b0; b < b1; ++b) {
        // the scalar words of batch b + 1 load while this wave waits for its copies and the barrier
        if (b + 1 < b1) load_blk(b + 1, blk);
        __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0): this wave's copies of batch b have landed
        stage_barrier();  // everyone's have; everyone is done reading batch b - 1
        int n_nxt = 0;
        uint32_t e_nxt = 0;
        if (b + 1 < b1) {  // into the buffer of batch b - 1
            issue(b + 1, blk, slot ^ 1);
            n_nxt = (int)blk[kLinSmemWords - 1];
            e_nxt = blk[kLinSmemWords - 2];
        }
        const unsigned char *buf_base = smem + slot * stride;
        const uint32_t vw = *reinterpret_cast<const uint32_t *>(buf_base + buf_bytes + 256 * wave + 4 * lane);
        Sum::add_batch(st, buf_base, lane, vw, n_cur, e_cur);
        n_cur = n_nxt;
        e_cur = e_nxt;
        slot ^= 1;
    }

#pragma unroll
    for (int q = 0; q < R; ++q) {
        if (row[q] < 0) continue;
        Sum::store(st, q, static_cast<float *>(s.dst) + (int64_t)row[q] * s.dst_pitch + t0, lane, vt, s.scale);
    }
}

namespace {

template <class Sum>
int launch_lin(const GroupArgs &a, int64_t n_out, int lds, void *stream, const Multi &m, int64_t nb_multi)
{
    const int64_t ntt = (n_out + Sum::kStep - 1) / Sum::kStep;
    const int64_t nb = m.n > 0 ? nb_multi : (int64_t)a.ngroups * ntt;
    if (nb <= 0) return 0;
    if (nb > 0x7fffffffLL) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(k_group_lin<Sum>, dim3((uint32_t)nb), dim3(1024), lds, (hipStream_t)stream, a, m);
    return (int)hipGetLastError();
}

}  // namespace

int launch_group_lin(int src_dt, const GroupArgs &a, int64_t n_out, int lds, void *stream, const Multi &m,
                     int64_t nblocks)
{
    switch (src_dt) {
    case SND_DT_F32: return launch_lin<LinF32>(a, n_out, lds, stream, m, nblocks);
    case SND_DT_BF16: return launch_lin<Lin16<false>>(a, n_out, lds, stream, m, nblocks);
    case SND_DT_F16: return launch_lin<Lin16<true>>(a, n_out, lds, stream, m, nblocks);
    default: return (int)hipErrorInvalidValue;
    }
}

}  // namespace snd
