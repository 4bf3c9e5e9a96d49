// SND tree kernels for gfx950 (CDNA4).
//
// One generic stage kernel evaluates, for a block of output rows and a time tile, the SND
// sub-tree between two materialised levels (Methods, "The Spiking Neural Dedispersion
// algorithm": leaf clusters, B-ary levels, shared-pattern neurons; "Tree activation modes").
// Each output row owns a list of (source row, time offset, closing depth) entries in
// depth-first tree order.  A wave walks that list with scalar loads, reads the 64 x V
// shifted source samples of each entry with coalesced vector loads, and keeps one partial
// sum per open tree level in registers; when an entry closes k levels the node activation
// (quorum, clip or none) is applied level by level exactly as in the tree.  The node
// arithmetic, its order and its association are those of a level-by-level evaluation, so
// the result does not depend on which levels are materialised.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "snd_internal.h"

namespace snd {
namespace {

constexpr int kWaves = 4;      // output rows per workgroup (one per wave)
constexpr int kV = 4;          // time samples per lane (strided by 64)
constexpr int kTile = 64 * kV; // time samples per wave
constexpr int kUnroll = 8;     // entries whose loads are issued together

template <typename T> struct Load;
template <> struct Load<uint8_t> {
    using acc = int;
    __device__ static int get(const uint8_t *p) { return *p; }
};
template <> struct Load<uint16_t> {
    __device__ static int get(const uint16_t *p) { return *p; }
};
template <> struct Load<float> {
    __device__ static float get(const float *p) { return *p; }
};
struct bf16_t { uint16_t bits; };
struct f16_t { _Float16 v; };
template <> struct Load<bf16_t> {
    __device__ static float get(const bf16_t *p) { return __uint_as_float((uint32_t)p->bits << 16); }
};
template <> struct Load<f16_t> {
    __device__ static float get(const f16_t *p) { return (float)p->v; }
};

__device__ inline uint16_t f32_to_bf16_rne(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

template <typename T> struct Store;
template <> struct Store<uint8_t> {
    template <typename A> __device__ static void put(uint8_t *p, A v) { *p = (uint8_t)v; }
};
template <> struct Store<uint16_t> {
    template <typename A> __device__ static void put(uint16_t *p, A v) { *p = (uint16_t)v; }
};
template <> struct Store<float> {
    template <typename A> __device__ static void put(float *p, A v) { *p = (float)v; }
};
template <> struct Store<bf16_t> {
    template <typename A> __device__ static void put(bf16_t *p, A v) { p->bits = f32_to_bf16_rne((float)v); }
};
template <> struct Store<f16_t> {
    template <typename A> __device__ static void put(f16_t *p, A v) { p->v = (_Float16)(float)v; }
};

template <int MODE> struct Acc { using type = int; };
template <> struct Acc<SND_MODE_FLOAT> { using type = float; };

// Node activation at relative level j of the stage (Methods, "Tree activation modes").
template <int MODE, typename A>
__device__ inline A activate(A a, int j, const StageArgs &s)
{
    if constexpr (MODE == SND_MODE_BINARY) {
        int k = (j == 1 && s.src_is_input) ? s.k_leaf : s.k_int;
        return a >= k ? 1 : 0;
    } else if constexpr (MODE == SND_MODE_GRADED) {
        return a < s.cap ? a : s.cap;
    } else {
        return a;
    }
}

// Blocks are dealt round-robin to the 8 XCDs; remap so that each XCD (own L2) works on a
// contiguous range of logical tiles, which share source rows.
__device__ inline uint32_t xcd_remap(uint32_t b, uint32_t nb)
{
    uint32_t x = b & 7u, i = b >> 3, q = nb >> 3, r = nb & 7u;
    return x * q + (x < r ? x : r) + i;
}

template <int MODE, typename TI, typename TO, int MAXD>
__global__ __launch_bounds__(256) void k_stage(StageArgs s)
{
    using A = typename Acc<MODE>::type;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const uint32_t L = xcd_remap(blockIdx.x, gridDim.x);
    const int rg = (int)(L % (uint32_t)s.n_rgroups);
    const int tt = (int)(L / (uint32_t)s.n_rgroups);
    int row = rg * kWaves + wave;
    if (row >= s.rows) return;
    row = __builtin_amdgcn_readfirstlane(row);
    const int len = s.row_len[row];
    const int t0 = tt * kTile;
    if (t0 >= len) return;
    const uint32_t beg = s.row_ptr[row], end = s.row_ptr[row + 1];
    const int depth = s.depth;

    bool ok[kV];
#pragma unroll
    for (int v = 0; v < kV; ++v) ok[v] = t0 + lane + 64 * v < len;

    A acc[MAXD][kV];
    A out[kV];
#pragma unroll
    for (int j = 0; j < MAXD; ++j)
#pragma unroll
        for (int v = 0; v < kV; ++v) acc[j][v] = 0;
#pragma unroll
    for (int v = 0; v < kV; ++v) out[v] = 0;

    const TI *src = static_cast<const TI *>(s.src);
    for (uint32_t e0 = beg; e0 < end; e0 += kUnroll) {
        const int n = (int)(end - e0) < kUnroll ? (int)(end - e0) : kUnroll;
        A val[kUnroll][kV];
        int cl[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            cl[u] = 0;
#pragma unroll
            for (int v = 0; v < kV; ++v) val[u][v] = 0;
            if (u < n) {
                const Entry en = s.ent[e0 + u];
                cl[u] = (int)(en.rowc >> 24);
                const TI *p = src + (int64_t)(en.rowc & kRowMask) * s.src_pitch + en.off + t0 + lane;
#pragma unroll
                for (int v = 0; v < kV; ++v)
                    if (ok[v]) {
                        A x = (A)Load<TI>::get(p + 64 * v);
                        if constexpr (MODE == SND_MODE_BINARY) x = x != 0;
                        val[u][v] = x;
                    }
            }
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            if (u < n) {
#pragma unroll
                for (int v = 0; v < kV; ++v) acc[0][v] += val[u][v];
                const int c = cl[u];
#pragma unroll
                for (int j = 1; j <= MAXD; ++j) {
                    if (j <= c) {
#pragma unroll
                        for (int v = 0; v < kV; ++v) {
                            A y = activate<MODE>(acc[j - 1][v], j, s);
                            acc[j - 1][v] = 0;
                            if (j == depth) out[v] = y;
                            else if (j < MAXD) acc[j][v] += y;
                        }
                    }
                }
            }
        }
    }

    TO *dst = static_cast<TO *>(s.dst) + (int64_t)row * s.dst_pitch + t0 + lane;
#pragma unroll
    for (int v = 0; v < kV; ++v) {
        if (ok[v]) {
            if constexpr (MODE == SND_MODE_FLOAT) Store<TO>::put(dst + 64 * v, out[v] * s.scale);
            else Store<TO>::put(dst + 64 * v, out[v]);
        }
    }
}

template <int MODE, typename TI, typename TO>
int launch_typed(const StageArgs &a, int64_t max_len, hipStream_t st)
{
    const int64_t ntt = (max_len + kTile - 1) / kTile;
    StageArgs s = a;
    s.n_ttiles = (int32_t)ntt;
    s.n_rgroups = (a.rows + kWaves - 1) / kWaves;
    const int64_t nblocks = (int64_t)s.n_rgroups * ntt;
    if (nblocks <= 0) return 0;
    if (nblocks > 0x7fffffffLL || max_len > 0x7fffffffLL) return (int)hipErrorInvalidValue;
    dim3 grid((uint32_t)nblocks), block(256);
    if (a.depth <= 1) hipLaunchKernelGGL((k_stage<MODE, TI, TO, 1>), grid, block, 0, st, s);
    else if (a.depth <= 2) hipLaunchKernelGGL((k_stage<MODE, TI, TO, 2>), grid, block, 0, st, s);
    else if (a.depth <= 4) hipLaunchKernelGGL((k_stage<MODE, TI, TO, 4>), grid, block, 0, st, s);
    else if (a.depth <= 8) hipLaunchKernelGGL((k_stage<MODE, TI, TO, 8>), grid, block, 0, st, s);
    else hipLaunchKernelGGL((k_stage<MODE, TI, TO, 16>), grid, block, 0, st, s);
    return (int)hipGetLastError();
}

template <typename TI>
int launch_float_out(int dst_dt, const StageArgs &a, int64_t max_len, hipStream_t st)
{
    switch (dst_dt) {
    case SND_DT_F32: return launch_typed<SND_MODE_FLOAT, TI, float>(a, max_len, st);
    case SND_DT_BF16: return launch_typed<SND_MODE_FLOAT, TI, bf16_t>(a, max_len, st);
    case SND_DT_F16: return launch_typed<SND_MODE_FLOAT, TI, f16_t>(a, max_len, st);
    }
    return (int)hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------------------
// Delta encoder (Methods, "Input encoding"): level = number of thresholds z exceeds.
// Time-major input is transposed through LDS in 64 x 64 tiles so both the read (along
// channels) and the write (along time) are coalesced.
// ---------------------------------------------------------------------------------------
struct Thresholds { float v[8]; int n; };

__global__ __launch_bounds__(256) void k_encode_cm(const float *z, int64_t zp, int nchan, int64_t nsamp, Thresholds th,
                                                   uint8_t *out, int64_t op)
{
    const int c = blockIdx.y;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= nchan || t >= nsamp) return;
    const float x = z[(int64_t)c * zp + t];
    int l = 0;
    for (int j = 0; j < th.n; ++j) l += x > th.v[j];
    out[(int64_t)c * op + t] = (uint8_t)l;
}

__global__ __launch_bounds__(256) void k_encode_tm(const float *z, int64_t zp, int nchan, int64_t nsamp, Thresholds th,
                                                   uint8_t *out, int64_t op)
{
    __shared__ uint8_t tile[64][65];
    const int64_t tb = (int64_t)blockIdx.x * 64;
    const int cb = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int i = ty; i < 64; i += 4) {  // i: time within tile, tx: channel within tile
        const int64_t t = tb + i;
        const int c = cb + tx;
        uint8_t l = 0;
        if (t < nsamp && c < nchan) {
            const float x = z[t * zp + c];
            for (int j = 0; j < th.n; ++j) l += x > th.v[j];
        }
        tile[i][tx] = l;
    }
    __syncthreads();
    for (int i = ty; i < 64; i += 4) {  // i: channel within tile, tx: time within tile
        const int c = cb + i;
        const int64_t t = tb + tx;
        if (c < nchan && t < nsamp) out[(int64_t)c * op + t] = tile[tx][i];
    }
}

template <typename TO>
__global__ __launch_bounds__(256) void k_cast(const float *src, int64_t sp, int64_t cols, TO *dst, int64_t dp)
{
    const int64_t r = blockIdx.y;
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= cols) return;
    Store<TO>::put(dst + r * dp + c, src[r * sp + c]);
}

}  // namespace

int launch_stage(int mode, int src_dt, int dst_dt, const StageArgs &a, int64_t max_len, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    if (mode == SND_MODE_BINARY) {
        if (src_dt == SND_DT_U8 && dst_dt == SND_DT_U8) return launch_typed<SND_MODE_BINARY, uint8_t, uint8_t>(a, max_len, st);
    } else if (mode == SND_MODE_GRADED) {
        if (src_dt == SND_DT_U8 && dst_dt == SND_DT_U8) return launch_typed<SND_MODE_GRADED, uint8_t, uint8_t>(a, max_len, st);
        if (src_dt == SND_DT_U8 && dst_dt == SND_DT_U16) return launch_typed<SND_MODE_GRADED, uint8_t, uint16_t>(a, max_len, st);
        if (src_dt == SND_DT_U16 && dst_dt == SND_DT_U16) return launch_typed<SND_MODE_GRADED, uint16_t, uint16_t>(a, max_len, st);
        if (src_dt == SND_DT_U16 && dst_dt == SND_DT_U8) return launch_typed<SND_MODE_GRADED, uint16_t, uint8_t>(a, max_len, st);
    } else if (mode == SND_MODE_FLOAT) {
        switch (src_dt) {
        case SND_DT_F32: return launch_float_out<float>(dst_dt, a, max_len, st);
        case SND_DT_BF16: return launch_float_out<bf16_t>(dst_dt, a, max_len, st);
        case SND_DT_F16: return launch_float_out<f16_t>(dst_dt, a, max_len, st);
        }
    }
    return (int)hipErrorInvalidValue;
}

int launch_encode(const float *z, int64_t zp, int time_major, int nchan, int64_t nsamp, const float *thr, int nthr,
                  uint8_t *out, int64_t op, void *stream)
{
    Thresholds th{};
    th.n = nthr;
    for (int i = 0; i < nthr; ++i) th.v[i] = thr[i];
    hipStream_t st = (hipStream_t)stream;
    if (time_major) {
        dim3 grid((uint32_t)((nsamp + 63) / 64), (uint32_t)((nchan + 63) / 64));
        hipLaunchKernelGGL(k_encode_tm, grid, dim3(256), 0, st, z, zp, nchan, nsamp, th, out, op);
    } else {
        dim3 grid((uint32_t)((nsamp + 255) / 256), (uint32_t)nchan);
        hipLaunchKernelGGL(k_encode_cm, grid, dim3(256), 0, st, z, zp, nchan, nsamp, th, out, op);
    }
    return (int)hipGetLastError();
}

int launch_cast(const float *src, int64_t sp, int64_t rows, int64_t cols, void *dst, int64_t dp, int dst_dt, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    dim3 grid((uint32_t)((cols + 255) / 256), (uint32_t)rows);
    if (dst_dt == SND_DT_BF16) hipLaunchKernelGGL(k_cast<bf16_t>, grid, dim3(256), 0, st, src, sp, cols, (bf16_t *)dst, dp);
    else if (dst_dt == SND_DT_F16) hipLaunchKernelGGL(k_cast<f16_t>, grid, dim3(256), 0, st, src, sp, cols, (f16_t *)dst, dp);
    else return (int)hipErrorInvalidValue;
    return (int)hipGetLastError();
}

}  // namespace snd
