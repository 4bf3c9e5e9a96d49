// Device helpers shared by the SND stage kernels: storage types, node activation, the
// level-closing step of the in-register sub-tree evaluation, the XCD-aware block remap and
// the (mode, source type, destination type) dispatch.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "snd.h"
#include "snd_internal.h"

namespace snd {

// Plan tables are never written while a kernel runs: read them through the constant address
// space so that wave-uniform reads become scalar loads (counted apart from vector memory).
template <typename T> using const_ptr = const __attribute__((address_space(4))) T *;
template <typename T> __device__ inline const_ptr<T> as_const(const T *p) { return (const_ptr<T>)p; }
// Device-memory pointers as global-address-space pointers: loads and stores through them are
// global_* instructions, which count on the vector-memory counter only (flat ones also count on
// the LDS counter, so every LDS wait would wait for them too).
template <typename T> using global_ptr = __attribute__((address_space(1))) T *;
template <typename T> __device__ inline global_ptr<T> as_global(T *p) { return (global_ptr<T>)p; }
template <typename T> __device__ inline global_ptr<const T> as_global(const T *p) { return (global_ptr<const T>)p; }

struct bf16_t { uint16_t bits; };
struct f16_t { _Float16 v; };
// Bit rows (binary mode): one bit per sample in 32-bit words; rows are written word-wise by the
// leaf stage and read word-wise by the bit-row final stage, never through Load / Store.
struct bits_t { uint32_t w; };

// Element access through any pointer type (generic, global or LDS).
template <typename T> struct Load;
template <> struct Load<uint8_t> { template <typename P> __device__ static int get(P p) { return *p; } };
template <> struct Load<uint16_t> { template <typename P> __device__ static int get(P p) { return *p; } };
template <> struct Load<float> { template <typename P> __device__ static float get(P p) { return *p; } };
template <> struct Load<bf16_t> {
    template <typename P> __device__ static float get(P p) { return __uint_as_float((uint32_t)p->bits << 16); }
};
template <> struct Load<f16_t> { template <typename P> __device__ static float get(P p) { return (float)p->v; } };

template <typename T> struct Zero { __device__ static T get() { return T{}; } };

__device__ inline uint16_t f32_to_bf16_rne(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

template <typename T> struct Store;
template <> struct Store<uint8_t> {
    template <typename P, typename A> __device__ static void put(P p, A v) { *p = (uint8_t)v; }
};
template <> struct Store<uint16_t> {
    template <typename P, typename A> __device__ static void put(P p, A v) { *p = (uint16_t)v; }
};
template <> struct Store<float> {
    template <typename P, typename A> __device__ static void put(P p, A v) { *p = (float)v; }
};
template <> struct Store<bf16_t> {
    template <typename P, typename A> __device__ static void put(P p, A v) { p->bits = f32_to_bf16_rne((float)v); }
};
template <> struct Store<f16_t> {
    template <typename P, typename A> __device__ static void put(P p, A v) { p->v = (_Float16)(float)v; }
};

// The storage bits of one element as Store<T>::put writes them, for packed stores.
template <typename T, typename A> __device__ inline uint32_t store_bits(A v);
template <> __device__ inline uint32_t store_bits<uint8_t, int>(int v) { return (uint32_t)(uint8_t)v; }
template <> __device__ inline uint32_t store_bits<uint16_t, int>(int v) { return (uint32_t)(uint16_t)v; }
template <> __device__ inline uint32_t store_bits<bf16_t, float>(float v) { return f32_to_bf16_rne(v); }
template <> __device__ inline uint32_t store_bits<f16_t, float>(float v)
{
    return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)v);
}

template <int MODE> struct Acc { using type = int; };
template <> struct Acc<SND_MODE_FLOAT> { using type = float; };

// Node activation at relative level j of a stage (Methods, "Tree activation modes"): binary
// quorum (K_L for the leaf level, K_I above), graded clip, or identity.
template <int MODE, typename A>
__device__ inline A activate(A a, int j, int src_is_input, int k_leaf, int k_int, int cap)
{
    if constexpr (MODE == SND_MODE_BINARY) {
        const int k = (j == 1 && src_is_input) ? k_leaf : k_int;
        return a >= k ? 1 : 0;
    } else if constexpr (MODE == SND_MODE_GRADED) {
        return a < cap ? a : cap;
    } else {
        return a;
    }
}

// After an input that completes c sub-tree levels: activate each completed node in turn and
// add its output to the parent's partial sum; the stage's own level goes to `out`.
template <int MODE, typename A, int MAXD, int V>
__device__ inline void close_levels(A (&acc)[MAXD][V], A (&out)[V], int c, int depth, int src_is_input, int k_leaf,
                                    int k_int, int cap)
{
#pragma unroll
    for (int j = 1; j <= MAXD; ++j) {
        if (j <= c) {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const A y = activate<MODE>(acc[j - 1][v], j, src_is_input, k_leaf, k_int, cap);
                acc[j - 1][v] = 0;
                if (j == depth) out[v] = y;
                else if (j < MAXD) acc[j][v] += y;
            }
        }
    }
}

// Workgroups are dealt round-robin to the 8 XCDs; remap so that each XCD (own L2) works on a
// contiguous range of logical tiles, which share source rows.
__device__ inline uint32_t xcd_remap(uint32_t b, uint32_t nb)
{
    const uint32_t x = b & 7u, i = b >> 3, q = nb >> 3, r = nb & 7u;
    return x * q + (x < r ? x : r) + i;
}

// The same idea in chunks of 8 m workgroups: within each chunk XCD x takes the x-th run of m
// consecutive logical tiles, so that all XCDs advance through the logical range together (the
// data that the tiles of one chunk share stays in the Infinity Cache) while each XCD's tiles
// are neighbours (they share lines in its L2).  The tail that does not fill a chunk keeps the
// contiguous map above.  A bijection on [0, nb) for every m >= 1.
__device__ inline uint32_t xcd_remap_chunked(uint32_t b, uint32_t nb, uint32_t m)
{
    const uint32_t C = 8u * m, full = nb / C * C;
    if (b >= full) return full + xcd_remap(b - full, nb - full);
    const uint32_t base = b / C * C, r = b - base;
    return base + (r & 7u) * m + (r >> 3);
}

// The arguments and the workgroup index of this workgroup: those passed by value for a plain
// launch, else those of the record whose workgroup range holds blockIdx.x (binary search over
// the prefix table; every value is wave-uniform, so this is scalar work).
template <typename A>
__device__ inline void select_record(const A &a0, const Multi &m, A &a, uint32_t &bid, uint32_t &nblk)
{
    if (m.n == 0) {
        a = a0;
        bid = blockIdx.x;
        nblk = gridDim.x;
        return;
    }
    const_ptr<int32_t> pre = as_const(m.prefix);
    const int32_t b = (int32_t)blockIdx.x;
    int lo = 0, hi = m.n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pre[mid] <= b) lo = mid;
        else hi = mid;
    }
    static_assert(sizeof(A) % 4 == 0, "argument records are copied as dwords");
    const_ptr<uint32_t> src = as_const(reinterpret_cast<const uint32_t *>(static_cast<const A *>(m.recs) + lo));
    uint32_t w[sizeof(A) / 4];
#pragma unroll
    for (size_t i = 0; i < sizeof(A) / 4; ++i) w[i] = src[i];
    __builtin_memcpy(&a, w, sizeof(A));
    bid = (uint32_t)(b - pre[lo]);
    nblk = (uint32_t)(pre[lo + 1] - pre[lo]);
}

// Calls f.template run<MODE, TI, TO>(stream) for the supported storage combinations.
template <typename F>
int dispatch_types(int mode, int src_dt, int dst_dt, const F &f, hipStream_t st)
{
    if (mode == SND_MODE_BINARY) {
        if (src_dt == SND_DT_U8 && dst_dt == SND_DT_U8) return f.template run<SND_MODE_BINARY, uint8_t, uint8_t>(st);
    } else if (mode == SND_MODE_GRADED) {
        if (src_dt == SND_DT_U8 && dst_dt == SND_DT_U8) return f.template run<SND_MODE_GRADED, uint8_t, uint8_t>(st);
        if (src_dt == SND_DT_U8 && dst_dt == SND_DT_U16) return f.template run<SND_MODE_GRADED, uint8_t, uint16_t>(st);
        if (src_dt == SND_DT_U16 && dst_dt == SND_DT_U16) return f.template run<SND_MODE_GRADED, uint16_t, uint16_t>(st);
        if (src_dt == SND_DT_U16 && dst_dt == SND_DT_U8) return f.template run<SND_MODE_GRADED, uint16_t, uint8_t>(st);
    } else if (mode == SND_MODE_FLOAT) {
#define SND_FLOAT_DST(TI)                                                                             \
    switch (dst_dt) {                                                                                 \
    case SND_DT_F32: return f.template run<SND_MODE_FLOAT, TI, float>(st);                            \
    case SND_DT_BF16: return f.template run<SND_MODE_FLOAT, TI, bf16_t>(st);                          \
    case SND_DT_F16: return f.template run<SND_MODE_FLOAT, TI, f16_t>(st);                            \
    }                                                                                                 \
    break;
        switch (src_dt) {
        case SND_DT_F32: SND_FLOAT_DST(float)
        case SND_DT_BF16: SND_FLOAT_DST(bf16_t)
        case SND_DT_F16: SND_FLOAT_DST(f16_t)
        }
#undef SND_FLOAT_DST
    }
    return (int)hipErrorInvalidValue;
}

}  // namespace snd
