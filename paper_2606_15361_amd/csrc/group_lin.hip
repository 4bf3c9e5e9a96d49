// Final stage of a float-mode plan as one sum per DM row (Methods, "Tree activation modes":
// float mode applies no activation, so the root of DM d is the plain sum of its leaf neurons,
// each read at its own delay; Eq. for y_d in "Incoherent dedispersion").
//
// Staging is that of the other row-group kernels: 16 waves of 1024 threads, leaf windows copied
// global -> LDS in double-buffered batches, full tiles by 64-unit chunks listed in the plan.  Each
// wave sums eight DM rows over a tile of 512 samples (f32 rows: 128 DM-adjacent rows share the
// staged windows) or four rows over 1024 samples (16-bit rows: 64-row groups).  Every read is a
// dword at o + 4 i + 256 v for an input at LDS byte offset o (lane i, v = 0 .. 7), which pairs
// into stride-64 reads of two dwords and needs 4-byte alignment only:
//  * f32 rows: lane i owns samples i + 64 v, one per dword, and every input takes one path.
//  * bf16 / f16 rows: lane i owns the sample pairs (2 i + 128 v, 2 i + 1 + 128 v), one dword.
//    An input whose first sample sits in the upper half of a dword takes the upper half of that
//    dword and the lower half of the next one (a second read); the branch on that is uniform.
//    f16 samples are added by v_fma_mix_f32 with a multiplier of 1.0 (the f16 half widened
//    exactly, the product exact, one rounding: the FP32 add of the widened sample, in one
//    instruction).  bf16 inputs go in twos: one
//    byte permute puts the two inputs' samples of one output sample into one dword, and one
//    v_dot2_f32_bf16 with weights (1, 1) adds both to the FP32 sum (one instruction per sample
//    instead of a widening and an add).  Only samples of the output being formed enter a dot.
//
// Each row is summed in FP32 in the order the plan lists its inputs (16-bit rows: batch by batch,
// each batch's inputs that start a dword before the others): an association of the exact sum
// that differs from the tree's, within the float tolerance of the FP64 definition.  A bf16 dot
// does not round like FP32 adds: measured on gfx950, its error stays below 1.5 x 2^-23 times the
// sum of its three terms' magnitudes (against 2^-24 times the result for an add), with a slight
// bias toward -infinity.  A row of n inputs is therefore within n 2^-23 sum|x| of the exact sum,
// the bound the parity tests check element by element.
#include <hip/hip_runtime.h>

#include "group_tab.h"

namespace snd {

namespace {

// The policies below index the sums of a wave in a plain array of the pipeline (a struct
// holding them ended up in scratch memory).
//
// f32 rows: st[q * V + v] is sample lane + 64 v of row q.
// Interface shared with the linear 16-bit sums: output element types, words per (batch, wave),
// the batch's inputs n (and the 16-bit dword-phase counts) as per-batch scalars; each policy
// sets its rows per wave and tile.
struct LinBase {
    using A = float;
    using TO = float;
    static constexpr int kWords = kLinWords, kSmemWords = kLinSmemWords;
    struct Carry {
        int n;
        uint32_t even;
    };
    static __device__ __forceinline__ Carry carry(const uint32_t (&blk)[kLinSmemWords])
    {
        return Carry{(int)blk[kLinSmemWords - 1], blk[kLinSmemWords - 2]};
    }
};

struct LinF32 : LinBase {
    using TI = float;
    static constexpr int R = lin_rows(SND_DT_F32), kRows = R, kStep = lin_tile(SND_DT_F32);
    static constexpr int V = kStep / 64;
    static constexpr int kState = R * V;

    // the n inputs of every row of the wave from the batch at buf; the lane's offset word at w
    static __device__ __forceinline__ void add_batch(float (&st)[kState], const unsigned char *buf,
                                                     const unsigned char *w, int lane, const Carry &c,
                                                     const GroupArgs &)
    {
        const uint32_t vw = *reinterpret_cast<const uint32_t *>(w);
        const int n = c.n;
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
                                                 const GroupArgs &s)
    {
        auto d = as_global(drow);
#pragma unroll
        for (int v = 0; v < V; ++v)
            if (lane + 64 * v < vt) d[lane + 64 * v] = st[q * V + v] * s.scale;
    }
};

// bf16 / f16 rows: st[LO + q * V + v] and st[HI + q * V + v] are samples 2 lane + 128 v and
// 2 lane + 1 + 128 v of row q.  An input whose first sample starts a dword is read as one
// dword per pair; one whose first sample sits in the upper half of a dword as the upper half of
// that dword and the lower half of the next (two reads per pair).  The plan lists each row's
// inputs of the first kind first.
template <bool F16>
struct Lin16 : LinBase {
    using TI = uint16_t;
    static constexpr int R = lin_rows(SND_DT_BF16), kRows = R, kStep = lin_tile(SND_DT_BF16);
    static constexpr int V = kStep / 128;
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
    // f16: acc + the lower or upper half of d, widened, as one FP32 add (v_fma_mix_f32 with a
    // multiplier of 1.0 in a scalar register)
    static __device__ __forceinline__ float mix_lo(float acc, uint32_t d, uint32_t one)
    {
        float r;
        asm("v_fma_mix_f32 %0, %1, %2, %3 op_sel_hi:[1,0,0]" : "=v"(r) : "v"(d), "s"(one), "v"(acc));
        return r;
    }
    static __device__ __forceinline__ float mix_hi(float acc, uint32_t d, uint32_t one)
    {
        float r;
        asm("v_fma_mix_f32 %0, %1, %2, %3 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(r) : "v"(d), "s"(one), "v"(acc));
        return r;
    }
    // acc + lower(d) / upper(d): one instruction for f16, widening and add for bf16
    static __device__ __forceinline__ float add_lo(float acc, uint32_t d, uint32_t one)
    {
        if constexpr (F16) return mix_lo(acc, d, one);
        else return acc + lower(d);
    }
    static __device__ __forceinline__ float add_hi(float acc, uint32_t d, uint32_t one)
    {
        if constexpr (F16) return mix_hi(acc, d, one);
        else return acc + upper(d);
    }
    // byte selectors of v_perm_b32 (a, b): the lower halves of b and a, or their upper halves
    static constexpr uint32_t kLoLo = 0x05040100u, kHiHi = 0x07060302u;
    // acc + the two bf16 samples that the selector picks from a and b (weights one2 = (1, 1))
    static __device__ __forceinline__ float add2(float acc, uint32_t a, uint32_t b, uint32_t sel, uint32_t one2)
    {
        typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
        const uint32_t pr = __builtin_amdgcn_perm(a, b, sel);
        return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, pr), __builtin_bit_cast(bf16x2, one2), acc,
                                               false);
    }
    // Row q's inputs that start a dword (the first even_q of its n words), then the others: two
    // loops per row without a branch per input, two inputs in flight.
    static __device__ __forceinline__ void add_batch(float (&st)[kState], const unsigned char *buf,
                                                     const unsigned char *w, int lane, const Carry &c,
                                                     const GroupArgs &)
    {
        const uint32_t vw = *reinterpret_cast<const uint32_t *>(w);
        const int n = c.n;
        const uint32_t even = c.even;
        // (1.0, 1.0) in bf16, materialised in a scalar register so that the compiler cannot encode
        // it as an inline constant (which the hardware would apply to one half only); 1.0f for f16
        uint32_t one2;
        if constexpr (F16) asm volatile("s_mov_b32 %0, 0x3f800000" : "=s"(one2));
        else asm volatile("s_mov_b32 %0, 0x3f803f80" : "=s"(one2));
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
                if constexpr (F16) {
#pragma unroll
                    for (int u = 0; u < 2; ++u)
#pragma unroll
                        for (int v = 0; v < V; ++v) {
                            st[LO + q * V + v] = add_lo(st[LO + q * V + v], x[u][v], one2);
                            st[HI + q * V + v] = add_hi(st[HI + q * V + v], x[u][v], one2);
                        }
                } else {
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        st[LO + q * V + v] = add2(st[LO + q * V + v], x[1][v], x[0][v], kLoLo, one2);
                        st[HI + q * V + v] = add2(st[HI + q * V + v], x[1][v], x[0][v], kHiHi, one2);
                    }
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
                    st[LO + q * V + v] = add_lo(st[LO + q * V + v], x[v], one2);
                    st[HI + q * V + v] = add_hi(st[HI + q * V + v], x[v], one2);
                }
                ++k;
            }
            // first sample in the upper half: that half of the dword, then the lower half of the next
            if constexpr (!F16) {
                for (; k + 2 <= k1; k += 2) {
                    uint32_t x[2][V], y[2][V];
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        const uint32_t o = (uint32_t)__builtin_amdgcn_readlane((int)vw, k + u);
                        const uint32_t *p = reinterpret_cast<const uint32_t *>(lane_base + (o & ~3u));
#pragma unroll
                        for (int v = 0; v < V; ++v) {
                            x[u][v] = p[64 * v];
                            y[u][v] = p[64 * v + 1];
                        }
                    }
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        st[LO + q * V + v] = add2(st[LO + q * V + v], x[1][v], x[0][v], kHiHi, one2);
                        st[HI + q * V + v] = add2(st[HI + q * V + v], y[1][v], y[0][v], kLoLo, one2);
                    }
                }
            }
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
                    st[LO + q * V + v] = add_hi(st[LO + q * V + v], x[v], one2);
                    st[HI + q * V + v] = add_lo(st[HI + q * V + v], y[v], one2);
                }
            }
        }
    }
    static __device__ __forceinline__ void store(const float (&st)[kState], int q, float *drow, int lane, int vt,
                                                 const GroupArgs &s)
    {
        const float scale = s.scale;
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
    group_tab_body<Sum>(s0, m);
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
