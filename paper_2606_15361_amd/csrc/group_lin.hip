// Final stage of a float-mode plan as one sum per DM row (Methods, "Tree activation modes":
// float mode applies no activation, so the root of DM d is the plain sum of its leaf neurons,
// each read at its own delay; Eq. for y_d in "Incoherent dedispersion").
//
// Staging is that of the other row-group kernels: 16 waves, two DM rows each (32 DM-adjacent
// rows per workgroup), leaf windows copied global -> LDS in double-buffered batches.  The sums
// differ: a lane owns the 4-sample units at tile samples 4i and 252 + 4i and reads each input
// as two aligned 16-byte units (ds_read_b128) starting at the unit that holds the input's first
// sample.  An input whose offset is p (mod 4) therefore lands p samples early; it is added to the
// accumulator of phase p, and each of the four accumulators is shifted back by its phase once
// per tile (the last p values of a unit come from the next lane's unit, via a lane shuffle).
// Lane 63 only supplies those values to lane 62, so a tile holds 504 output samples.
//
// Inputs are summed per phase in the order the plan lists them, and the four phase sums are
// added at the end: an FP32 association of the exact sum that differs from the tree's, within
// the float tolerance of the FP64 definition.
#include <hip/hip_runtime.h>

#include "group_common.h"

namespace snd {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline f32x4 lds_unit(const unsigned char *p) { return *reinterpret_cast<const f32x4 *>(p); }

__device__ inline void add4(float (&a)[8], int h, const f32x4 &v)
{
    a[4 * h + 0] += v.x;
    a[4 * h + 1] += v.y;
    a[4 * h + 2] += v.z;
    a[4 * h + 3] += v.w;
}

// One input of one row: the two 16-byte units at byte offset o of this lane's window position.
__device__ inline void add_input(float (&a)[8], const unsigned char *lane_base, uint32_t o)
{
    const unsigned char *p = lane_base + o;
    const f32x4 u0 = lds_unit(p), u1 = lds_unit(p + 4 * kLinHalf);
    add4(a, 0, u0);
    add4(a, 1, u1);
}

// The n (<= 8) inputs of one (row, phase) segment: their offsets sit in lanes L .. L + n - 1 of
// the wave's offset word v (static lane indices: no scalar work per input but the count test).
// The inputs of one phase of one row: n offsets from lane k of the wave's offset word v, two at a
// time so that four 16-byte reads are in flight.
__device__ inline void add_phase(float (&a)[8], const unsigned char *lane_base, uint32_t v, int k, int n)
{
    int i = 0;
    for (; i + 2 <= n; i += 2) {
        const uint32_t o0 = (uint32_t)__builtin_amdgcn_readlane((int)v, k + i);
        const uint32_t o1 = (uint32_t)__builtin_amdgcn_readlane((int)v, k + i + 1);
        const unsigned char *p0 = lane_base + o0, *p1 = lane_base + o1;
        const f32x4 x0 = lds_unit(p0), y0 = lds_unit(p0 + 4 * kLinHalf);
        const f32x4 x1 = lds_unit(p1), y1 = lds_unit(p1 + 4 * kLinHalf);
        add4(a, 0, x0);
        add4(a, 1, y0);
        add4(a, 0, x1);
        add4(a, 1, y1);
    }
    if (i < n) add_input(a, lane_base, (uint32_t)__builtin_amdgcn_readlane((int)v, k + i));
}

}  // namespace

__global__ __launch_bounds__(1024) void k_group_lin(GroupArgs s0, Multi m)
{
    GroupArgs s;
    uint32_t bid, nblk;
    select_record(s0, m, s, bid, nblk);
    constexpr int T = kLinTile, H = kLinHalf, R = kLinRows;
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
    const int64_t pitch_bytes = s.src_pitch * (int64_t)sizeof(float);
    const int buf_bytes = s.buf_elems * (int)sizeof(float);
    static_assert(kLinBuffers == 2, "the table words below are loaded one batch ahead of a double buffer");
    const int stride = buf_bytes + kLinWordBytes;  // bytes of one buffer: windows, then offset words
    const bool full = vt == T;  // full tiles copy from the chunk table; the last tile by window

    float acc[R][4][8];
#pragma unroll
    for (int q = 0; q < R; ++q)
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int j = 0; j < 8; ++j) acc[q][p][j] = 0.0f;

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
        const unsigned char *lane_base = buf_base + 16 * lane;
        const int n = n_cur;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const uint32_t cw = (uint32_t)__builtin_amdgcn_readlane((int)vw, 2 * n + q);
            int k = q * n;
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const int np = (int)((cw >> (8 * p)) & 255u);
                add_phase(acc[q][p], lane_base, vw, k, np);
                k += np;
            }
        }
        n_cur = n_nxt;
        slot ^= 1;
    }

    // shift each phase sum back by its phase and add the four; lanes 0..62 store their units
#pragma unroll
    for (int q = 0; q < R; ++q) {
        float y[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) y[j] = acc[q][0][j];
#pragma unroll
        for (int p = 1; p < 4; ++p)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                float nb[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) nb[j] = j < p ? __shfl_down(acc[q][p][4 * h + j], 1) : 0.0f;
#pragma unroll
                for (int j = 0; j < 4; ++j) y[4 * h + j] += j + p < 4 ? acc[q][p][4 * h + j + p] : nb[j + p - 4];
            }
        if (row[q] < 0 || lane == 63) continue;
        float *const drow = static_cast<float *>(s.dst) + (int64_t)row[q] * s.dst_pitch + t0;
        const bool vec = ((reinterpret_cast<uintptr_t>(drow) & 15u) == 0);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int t = h * H + 4 * lane;
            auto d = as_global(drow + t);
            const float v0 = y[4 * h] * s.scale, v1 = y[4 * h + 1] * s.scale, v2 = y[4 * h + 2] * s.scale,
                        v3 = y[4 * h + 3] * s.scale;
            if (vec && t + 4 <= vt) {
                *reinterpret_cast<__attribute__((address_space(1))) f32x4 *>(d) = f32x4{v0, v1, v2, v3};
            } else {
                if (t < vt) d[0] = v0;
                if (t + 1 < vt) d[1] = v1;
                if (t + 2 < vt) d[2] = v2;
                if (t + 3 < vt) d[3] = v3;
            }
        }
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
