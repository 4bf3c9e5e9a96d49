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
#include "stage_common.h"

namespace snd {
namespace {

constexpr int kWaves = 4;      // output rows per workgroup (one per wave)
constexpr int kV = 4;          // time samples per lane (strided by 64)
constexpr int kTile = 64 * kV; // time samples per wave
constexpr int kUnroll = 8;     // entries whose loads are issued together

template <int MODE, typename TI, typename TO, int MAXD>
__global__ __launch_bounds__(256) void k_stage(StageArgs s0, Multi m)
{
    using A = typename Acc<MODE>::type;
    StageArgs s;
    uint32_t bid, nblk;
    select_record(s0, m, s, bid, nblk);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const uint32_t L = xcd_remap(bid, nblk);
    const int rg = (int)(L % (uint32_t)s.n_rgroups);
    const int tt = (int)(L / (uint32_t)s.n_rgroups);
    int row = rg * kWaves + wave;
    if (row >= s.rows) return;
    row = __builtin_amdgcn_readfirstlane(row);
    const int len = s.row_len[row] - s.len_cut;
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
    uint32_t e0 = beg;
    // full chunks: all table entries, then all loads, then the sums (no per-entry guards, so the
    // loads of a chunk are in flight together)
    for (; e0 + kUnroll <= end; e0 += kUnroll) {
        Entry en[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) en[u] = s.ent[e0 + u];
        A val[kUnroll][kV];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const TI *p = src + (int64_t)(en[u].rowc & kRowMask) * s.src_pitch + en[u].off + t0 + lane;
#pragma unroll
            for (int v = 0; v < kV; ++v) {
                A x = 0;
                if (ok[v]) x = (A)Load<TI>::get(p + 64 * v);
                if constexpr (MODE == SND_MODE_BINARY) x = x != 0;
                val[u][v] = x;
            }
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
#pragma unroll
            for (int v = 0; v < kV; ++v) acc[0][v] += val[u][v];
            close_levels<MODE, A, MAXD, kV>(acc, out, (int)(en[u].rowc >> 24), depth, s.src_is_input, s.k_leaf,
                                            s.k_int, s.cap);
        }
    }
    for (; e0 < end; ++e0) {
        const Entry en = s.ent[e0];
        const TI *p = src + (int64_t)(en.rowc & kRowMask) * s.src_pitch + en.off + t0 + lane;
#pragma unroll
        for (int v = 0; v < kV; ++v) {
            A x = 0;
            if (ok[v]) x = (A)Load<TI>::get(p + 64 * v);
            if constexpr (MODE == SND_MODE_BINARY) x = x != 0;
            acc[0][v] += x;
        }
        close_levels<MODE, A, MAXD, kV>(acc, out, (int)(en.rowc >> 24), depth, s.src_is_input, s.k_leaf, s.k_int,
                                        s.cap);
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
int launch_typed(const StageArgs &a, int64_t max_len, hipStream_t st, const Multi &m, int64_t nb_multi)
{
    StageArgs s = a;
    const int64_t nblocks = m.n > 0 ? nb_multi : stage_blocks(s, max_len);
    if (nblocks <= 0) return 0;
    if (nblocks > 0x7fffffffLL || max_len > 0x7fffffffLL) return (int)hipErrorInvalidValue;
    dim3 grid((uint32_t)nblocks), block(256);
    if (a.depth <= 1) hipLaunchKernelGGL((k_stage<MODE, TI, TO, 1>), grid, block, 0, st, s, m);
    else if (a.depth <= 2) hipLaunchKernelGGL((k_stage<MODE, TI, TO, 2>), grid, block, 0, st, s, m);
    else if (a.depth <= 4) hipLaunchKernelGGL((k_stage<MODE, TI, TO, 4>), grid, block, 0, st, s, m);
    else if (a.depth <= 8) hipLaunchKernelGGL((k_stage<MODE, TI, TO, 8>), grid, block, 0, st, s, m);
    else hipLaunchKernelGGL((k_stage<MODE, TI, TO, 16>), grid, block, 0, st, s, m);
    return (int)hipGetLastError();
}

struct StageLauncher {
    const StageArgs &a;
    int64_t max_len;
    const Multi &m;
    int64_t nblocks;
    template <int MODE, typename TI, typename TO> int run(hipStream_t st) const
    {
        return launch_typed<MODE, TI, TO>(a, max_len, st, m, nblocks);
    }
};

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

// Bits: one wave tests 64 consecutive samples of a channel; the ballot is two output words.
__global__ __launch_bounds__(256) void k_encode_bits_cm(const float *z, int64_t zp, int64_t nsamp, float th,
                                                        uint32_t *out, int64_t ow)
{
    const int c = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int64_t tb = (int64_t)blockIdx.x * 256 + (threadIdx.x >> 6) * 64;  // first sample of the wave
    const int64_t t = tb + lane;
    const uint64_t mask = __ballot(t < nsamp && z[(int64_t)c * zp + t] > th);
    const int64_t w = (tb >> 5) + lane;
    if (lane < 2 && 32 * w < nsamp) out[(int64_t)c * ow + w] = lane ? (uint32_t)(mask >> 32) : (uint32_t)mask;
}

// Bits from time-major input: a 64 x 64 (time, channel) tile through LDS, then one ballot per
// channel of the tile.
__global__ __launch_bounds__(256) void k_encode_bits_tm(const float *z, int64_t zp, int nchan, int64_t nsamp,
                                                        float th, uint32_t *out, int64_t ow)
{
    __shared__ uint8_t tile[64][65];
    const int64_t tb = (int64_t)blockIdx.x * 64;
    const int cb = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int i = ty; i < 64; i += 4) {  // i: time within tile, tx: channel within tile
        const int64_t t = tb + i;
        const int c = cb + tx;
        tile[i][tx] = (t < nsamp && c < nchan) ? (uint8_t)(z[t * zp + c] > th) : (uint8_t)0;
    }
    __syncthreads();
    for (int i = ty; i < 64; i += 4) {  // i: channel within tile, tx: time within tile
        const uint64_t mask = __ballot(tile[tx][i] != 0);
        const int c = cb + i;
        const int64_t w = (tb >> 5) + tx;
        if (tx < 2 && c < nchan && 32 * w < nsamp) out[(int64_t)c * ow + w] = tx ? (uint32_t)(mask >> 32) : (uint32_t)mask;
    }
}

// Time scrunch: each thread sums s consecutive samples of one channel in order (FP32, no
// contraction) and scales by r.
__global__ __launch_bounds__(256) void k_scrunch(const float *z, int64_t zp, int64_t nout, int s, float r, float *out,
                                                 int64_t op)
{
    const int c = blockIdx.y;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= nout) return;
    const float *p = z + (int64_t)c * zp + t * s;
    float acc = p[0];
    for (int j = 1; j < s; ++j) acc = acc + p[j];
    out[(int64_t)c * op + t] = acc * r;
}

// Sigma-clip statistics of one channel per workgroup: a first FP64 pass about the channel's
// first sample gives mu0 and sigma0, a second pass the same statistics of the clipped values
// (about the clip range's centre, mu0).  Loads are coalesced across the workgroup.
__device__ inline void block_sum2(double &a, double &b, double (*sh)[256], int tid)
{
    sh[0][tid] = a;
    sh[1][tid] = b;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) {
            sh[0][tid] += sh[0][tid + w];
            sh[1][tid] += sh[1][tid + w];
        }
        __syncthreads();
    }
    a = sh[0][0];
    b = sh[1][0];
    __syncthreads();
}

__global__ __launch_bounds__(256) void k_chanstats(const float *p, int64_t pp, int64_t n, double clip, double *stats)
{
    __shared__ double sh[2][256];
    const int c = blockIdx.x, tid = threadIdx.x;
    const float *row = p + (int64_t)c * pp;
    const double shift = (double)row[0];
    double a = 0.0, b = 0.0;
    for (int64_t t = tid; t < n; t += 256) {
        const double d = (double)row[t] - shift;
        a += d;
        b += d * d;
    }
    block_sum2(a, b, sh, tid);
    const double dn = (double)n;
    const double m1 = a / dn;
    const double mu0 = shift + m1;
    const double v0 = b / dn - m1 * m1;
    const double s0 = v0 > 0.0 ? sqrt(v0) : 0.0;
    const double lo = mu0 - clip * s0, hi = mu0 + clip * s0;
    a = 0.0;
    b = 0.0;
    for (int64_t t = tid; t < n; t += 256) {
        double v = (double)row[t];
        v = v < lo ? lo : (v > hi ? hi : v);
        const double d = v - mu0;
        a += d;
        b += d * d;
    }
    block_sum2(a, b, sh, tid);
    if (tid == 0) {
        const double m = a / dn;
        const double v = b / dn - m * m;
        stats[2 * c] = mu0 + m;
        stats[2 * c + 1] = v > 0.0 ? sqrt(v) : 0.0;
    }
}

__global__ __launch_bounds__(256) void k_normalize(const float *p, int64_t pp, int64_t n, const double *stats,
                                                   float *z, int64_t zp)
{
    const int c = blockIdx.y;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n) return;
    const double mu = stats[2 * c], sg = stats[2 * c + 1];
    z[(int64_t)c * zp + t] = (float)(((double)p[(int64_t)c * pp + t] - mu) / sg);
}

// Zero-DM subtraction: one thread per sample t sums the channels in order in FP64 (the
// threads of a wave read consecutive samples of a channel row); when the zero-DM S/N
// |sum| / sqrt(nchan) exceeds gamma, the channel mean sum / nchan is subtracted from every
// channel, each result rounded once to FP32.
__global__ __launch_bounds__(256) void k_zero_dm(float *z, int64_t zp, int nchan, int64_t n, double gamma,
                                                 int32_t *count)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n) return;
    double s = 0.0;
    for (int c = 0; c < nchan; ++c) s += (double)z[(int64_t)c * zp + t];
    if (__builtin_fabs(s) / __builtin_sqrt((double)nchan) > gamma) {
        const double mean = s / (double)nchan;
        for (int c = 0; c < nchan; ++c) z[(int64_t)c * zp + t] = (float)((double)z[(int64_t)c * zp + t] - mean);
        if (count) atomicAdd(count, 1);
    }
}

// Index of the element of rank r (0-based, increasing; equal values ordered by index) among
// v[0..n) in LDS: each thread ranks its elements against all others.
__device__ inline void lds_rank_select(const double *v, int n, int r, int *out)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double x = v[i];
        int below = 0;
        for (int j = 0; j < n; ++j) below += (v[j] < x) || (v[j] == x && j < i);
        if (below == r) *out = i;
    }
}

// Windowed channel flagging by median absolute deviation, in two kernels.
// k_chan_window_sigma: one wave per (channel, window of w samples): s = the population standard
//   deviation over the window, each of its two FP64 sums (samples, then squared deviations from
//   the mean) taken as 64 interleaved partial sums -- lane j sums samples j, j + 64, ... in
//   order -- added in lane order.  Writes sigma[window][channel].
// k_flag_window: one workgroup per window: m = the lower median of the window's s over the
//   channels, MAD = the lower median of |s_c - m|; channel c is flagged when |s_c - m| >
//   k * (kMad * MAD), kMad = 1 / Phi^-1(3/4), and its samples in the window are set to 0.
constexpr double kFlagMadScale = 1.4826022185056018;

__device__ inline double wave_sum_in_lane_order(double v, double *lds64)
{
    const int lane = threadIdx.x & 63;
    lds64[lane] = v;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double s = 0.0;
    for (int j = 0; j < 64; ++j) s += lds64[j];
    __builtin_amdgcn_wave_barrier();
    return s;
}

__global__ __launch_bounds__(256) void k_chan_window_sigma(const float *z, int64_t zp, int nchan, int64_t n,
                                                           int64_t w, double *sigma)
{
    __shared__ double part[4][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int c = blockIdx.x * 4 + wave;
    const int64_t b = blockIdx.y;
    if (c >= nchan) return;  // whole waves
    const int64_t t0 = b * w;
    const int64_t len = n - t0 < w ? n - t0 : w;
    const float *row = z + (int64_t)c * zp + t0;
    double a = 0.0;
    for (int64_t t = lane; t < len; t += 64) a += (double)row[t];
    const double mu = wave_sum_in_lane_order(a, part[wave]) / (double)len;
    double q = 0.0;
    for (int64_t t = lane; t < len; t += 64) q += ((double)row[t] - mu) * ((double)row[t] - mu);
    const double qs = wave_sum_in_lane_order(q, part[wave]);
    if (lane == 0) sigma[b * nchan + c] = __builtin_sqrt(qs / (double)len);
}


__global__ __launch_bounds__(1024) void k_flag_window(float *z, int64_t zp, int nchan, int64_t n, int64_t w,
                                                      double k, const double *sigma, uint8_t *flags, int64_t fp)
{
    extern __shared__ double sv[];  // [2 * nchan]: the window's sigmas, then their deviations
    __shared__ int s_idx;
    const int64_t b = blockIdx.x;
    const int64_t t0 = b * w;
    const int64_t len = n - t0 < w ? n - t0 : w;
    for (int c = threadIdx.x; c < nchan; c += blockDim.x) sv[c] = sigma[b * nchan + c];
    __syncthreads();
    const int r = (nchan - 1) / 2;
    lds_rank_select(sv, nchan, r, &s_idx);
    __syncthreads();
    const double m = sv[s_idx];
    for (int c = threadIdx.x; c < nchan; c += blockDim.x) sv[nchan + c] = __builtin_fabs(sv[c] - m);
    __syncthreads();
    lds_rank_select(sv + nchan, nchan, r, &s_idx);
    __syncthreads();
    const double thr = k * (kFlagMadScale * sv[nchan + s_idx]);
    for (int c = 0; c < nchan; ++c) {  // uniform: every thread sees the same flag
        const bool f = sv[nchan + c] > thr;
        if (threadIdx.x == 0 && flags) flags[b * fp + c] = f ? 1 : 0;
        if (f) {
            float *row = z + (int64_t)c * zp + t0;
            for (int64_t t = threadIdx.x; t < len; t += blockDim.x) row[t] = 0.0f;
        }
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

int64_t stage_blocks(StageArgs &a, int64_t max_len)
{
    const int64_t ntt = (max_len + kTile - 1) / kTile;
    a.n_ttiles = (int32_t)ntt;
    a.n_rgroups = (a.rows + kWaves - 1) / kWaves;
    return (int64_t)a.n_rgroups * ntt;
}

int launch_stage(int mode, int src_dt, int dst_dt, const StageArgs &a, int64_t max_len, void *stream, const Multi &m,
                 int64_t nblocks)
{
    return dispatch_types(mode, src_dt, dst_dt, StageLauncher{a, max_len, m, nblocks}, (hipStream_t)stream);
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

int launch_encode_bits(const float *z, int64_t zp, int time_major, int nchan, int64_t nsamp, float thr, uint32_t *out,
                       int64_t ow, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    if (time_major) {
        dim3 grid((uint32_t)((nsamp + 63) / 64), (uint32_t)((nchan + 63) / 64));
        hipLaunchKernelGGL(k_encode_bits_tm, grid, dim3(256), 0, st, z, zp, nchan, nsamp, thr, out, ow);
    } else {
        dim3 grid((uint32_t)((nsamp + 255) / 256), (uint32_t)nchan);
        hipLaunchKernelGGL(k_encode_bits_cm, grid, dim3(256), 0, st, z, zp, nsamp, thr, out, ow);
    }
    return (int)hipGetLastError();
}

int launch_scrunch(const float *z, int64_t zp, int nchan, int64_t nout, int s, float r, float *out, int64_t op,
                   void *stream)
{
    dim3 grid((uint32_t)((nout + 255) / 256), (uint32_t)nchan);
    hipLaunchKernelGGL(k_scrunch, grid, dim3(256), 0, (hipStream_t)stream, z, zp, nout, s, r, out, op);
    return (int)hipGetLastError();
}

int launch_chanstats(const float *p, int64_t pp, int nchan, int64_t n, double clip, double *stats, void *stream)
{
    hipLaunchKernelGGL(k_chanstats, dim3((uint32_t)nchan), dim3(256), 0, (hipStream_t)stream, p, pp, n, clip, stats);
    return (int)hipGetLastError();
}

// One FDMT merge: output row r = source row U (tab[4r]) plus source row L (tab[4r + 1]) read
// tab[4r + 2] samples later, zero past n.  A workgroup covers 2048 samples of a strided set of
// rows; the table words are uniform (scalar loads).
__global__ __launch_bounds__(256) void k_fdmt_merge(const float *src, int64_t sp, float *dst, int64_t dp,
                                                    const int32_t *tab, int64_t rows, int64_t n)
{
    const int64_t t0 = (int64_t)blockIdx.x * 2048 + threadIdx.x;
    for (int64_t r = blockIdx.y; r < rows; r += gridDim.y) {
        const int64_t ru = tab[4 * r], rl = tab[4 * r + 1], du = tab[4 * r + 2];
        const float *u = src + ru * sp;
        const float *l = src + rl * sp + du;
        float *o = dst + r * dp;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int64_t t = t0 + 256 * j;
            if (t < n) o[t] = u[t] + (t + du < n ? l[t] : 0.0f);
        }
    }
}

int launch_fdmt_merge(const float *src, int64_t sp, float *dst, int64_t dp, const int32_t *tab, int64_t rows, int64_t n,
                      void *stream)
{
    if (rows < 1) return 0;
    const int64_t nx = (n + 2047) / 2048;
    const int64_t ny = rows < 4096 ? rows : 4096;
    hipLaunchKernelGGL(k_fdmt_merge, dim3((uint32_t)nx, (uint32_t)ny), dim3(256), 0, (hipStream_t)stream, src, sp,
                       dst, dp, tab, rows, n);
    return (int)hipGetLastError();
}

// Approximate sub-band dedispersion, second step: out row k = sum over sub-bands s of row
// coarse[k] of sub-band plane s, read offs[k * nsub + s] samples later, in FP32 in sub-band
// order.  A workgroup covers 1024 samples of one row, 4 per lane (coalesced reads of each plane
// row); the table words are uniform (scalar loads).
__global__ __launch_bounds__(256) void k_subband_combine(const float *const *planes, const int64_t *pitches,
                                                         const int32_t *coarse, const int32_t *offs, int nsub,
                                                         float *out, int64_t op, int64_t n)
{
    const int k = blockIdx.y;
    const int64_t t0 = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    const int j = coarse[k];
    float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int s = 0; s < nsub; ++s) {
        const float *row = planes[s] + (int64_t)j * pitches[s] + offs[(int64_t)k * nsub + s];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t t = t0 + 256 * i;
            if (t < n) acc[i] += row[t];
        }
    }
    float *o = out + (int64_t)k * op;
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (t0 + 256 * i < n) o[t0 + 256 * i] = acc[i];
}

int launch_subband_combine(const float *const *planes, const int64_t *pitches, const int32_t *coarse,
                           const int32_t *offs, int nsub, int ndm, float *out, int64_t op, int64_t n, void *stream)
{
    if (ndm < 1 || n < 1) return 0;
    hipLaunchKernelGGL(k_subband_combine, dim3((uint32_t)((n + 1023) / 1024), (uint32_t)ndm), dim3(256), 0,
                       (hipStream_t)stream, planes, pitches, coarse, offs, nsub, out, op, n);
    return (int)hipGetLastError();
}

int launch_zero_dm(float *z, int64_t zp, int nchan, int64_t n, double gamma, int32_t *count, void *stream)
{
    const int64_t nb = (n + 255) / 256;
    hipLaunchKernelGGL(k_zero_dm, dim3((uint32_t)nb), dim3(256), 0, (hipStream_t)stream, z, zp, nchan, n, gamma, count);
    return (int)hipGetLastError();
}

int launch_flag_channels(float *z, int64_t zp, int nchan, int64_t n, int64_t w, double k, double *sigma,
                         uint8_t *flags, int64_t fp, void *stream)
{
    const int64_t nwin = (n + w - 1) / w;
    hipLaunchKernelGGL(k_chan_window_sigma, dim3((uint32_t)((nchan + 3) / 4), (uint32_t)nwin), dim3(256), 0,
                       (hipStream_t)stream, z, zp, nchan, n, w, sigma);
    hipLaunchKernelGGL(k_flag_window, dim3((uint32_t)nwin), dim3(1024), (size_t)(2 * nchan) * sizeof(double),
                       (hipStream_t)stream, z, zp, nchan, n, w, k, sigma, flags, fp);
    return (int)hipGetLastError();
}

int launch_normalize(const float *p, int64_t pp, int nchan, int64_t n, const double *stats, float *z, int64_t zp,
                     void *stream)
{
    dim3 grid((uint32_t)((n + 255) / 256), (uint32_t)nchan);
    hipLaunchKernelGGL(k_normalize, grid, dim3(256), 0, (hipStream_t)stream, p, pp, n, stats, z, zp);
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
