// Boxcar matched filter and candidate-pixel compaction for gfx950 (Methods, "Matched
// filtering" and "Candidate detection").
//
// k_rowstats: mean and population standard deviation of each DM row over its valid samples.
//   Integer planes use exact 64-bit sums S1, S2 and sigma = sqrt(n*S2 - S1*S1)/n in one fixed
//   FP64 expression; float planes use one FP64 pass about the row's first sample.  A floor
//   sigma_min applies.
// k_snr: one workgroup per (row, tile of 8192 samples for integer planes, 2048 for float).  The tile plus the widest boxcar is
//   staged in LDS as an inclusive prefix sum (int32 for integer planes: exact; FP64 for float
//   planes), every sample then evaluates all widths with two LDS reads each:
//   SNR(t, W) = (S_W(t) - mu W) / (sigma sqrt W), maximum over widths (first width on ties).
//   Either the full S/N plane and width index are written, or the cells whose S/N reaches the
//   threshold are appended to a global pixel list, each workgroup's cells as one segment in
//   increasing t.  For the list, a per-width bound on the boxcar sum (in the prefix type)
//   skips the cells that cannot reach the threshold; every cell that can takes the exact
//   quotient.  u8 planes whose widths are 1 and even widths up to 256 (every boxcar sum below
//   2^16) take the bound tests on two cells per 32-bit lane: the prefix is kept modulo 2^16 in
//   16-bit halves (differences stay exact), one dword read brings the prefix at t + W and
//   t + 1 + W, and packed 16-bit subtractions test both cells.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "snd_detect.h"

namespace snd {
namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
template <typename T> using global_ptr = __attribute__((address_space(1))) T *;
template <typename T> __device__ inline global_ptr<const T> as_global(const T *p) { return (global_ptr<const T>)p; }

constexpr int kThreads = 256;

template <typename T> struct IsInt { static constexpr bool value = true; };
template <typename P> struct BoundNever { __device__ static P value() { return (P)2147483647; } };
template <> struct BoundNever<double> { __device__ static double value() { return __builtin_inf(); } };
template <> struct IsInt<float> { static constexpr bool value = false; };
// Samples of one row per S/N workgroup: integer planes carry a 4-byte prefix per sample and
// little arithmetic per byte read, so their tiles are longer (fewer workgroups, a smaller share
// of re-read halo; 4096 keeps seven workgroups on a CU, 8192 and 2048 measured slower); float
// planes carry an 8-byte prefix.
template <typename T> constexpr int snr_tile() { return IsInt<T>::value ? 4096 : 2048; }

// Row sums with 16-byte loads: a scalar head up to the first 16-byte boundary of the row, then
// 16-byte vectors (four in flight per thread), then a scalar tail.  f(x, j) folds one sample;
// j is its place in a vector (0 for the scalar head and tail), for independent accumulators.
template <typename T, typename F>
__device__ inline void row_fold(const T *row, int64_t n, int tid, F &&f)
{
    constexpr int E = 16 / (int)sizeof(T);  // samples per vector
    int64_t head = (int64_t)(((16u - ((uint32_t)(uintptr_t)row & 15u)) & 15u) / sizeof(T));
    if (((uintptr_t)row % sizeof(T)) != 0 || head > n) head = n;  // misaligned element type: all scalar
    if (tid < head) f(row[tid], 0);
    const int64_t nv = (n - head) / E;
    const auto vec = as_global(reinterpret_cast<const u32x4 *>(row + head));
    int64_t i = tid;
    for (; i + 3 * kThreads < nv; i += 4 * kThreads) {
        u32x4 q[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) q[u] = vec[i + u * kThreads];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const T *e = reinterpret_cast<const T *>(&q[u]);
#pragma unroll
            for (int j = 0; j < E; ++j) f(e[j], j);
        }
    }
    for (; i < nv; i += kThreads) {
        const u32x4 q = vec[i];
        const T *e = reinterpret_cast<const T *>(&q);
#pragma unroll
        for (int j = 0; j < E; ++j) f(e[j], j);
    }
    for (int64_t t = head + nv * E + tid; t < n; t += kThreads) f(row[t], 0);
}

// Row k of a launch: a row of the single plane, or (BATCH) batch row row0 + k of the plane
// whose row range holds it (a scan of the table: every value is wave-uniform, so scalar work).
template <bool BATCH, typename T>
__device__ inline void locate_row(const T *plane, int64_t pitch, int64_t n, const int32_t *row_nw, const DetBeam *beams,
                                  int nbeams, int row0, int k_launch, const T *&row, int64_t &nr, const int32_t *&nw,
                                  int &k, int &kl)
{
    k = row0 + k_launch;
    if constexpr (!BATCH) {
        row = plane + (int64_t)k * pitch;
        nr = n;
        nw = row_nw;
        kl = k;
        return;
    }
    int i = 0;
    while (i + 1 < nbeams && k >= beams[i + 1].row_base) ++i;
    const DetBeam b = beams[i];
    kl = k - b.row_base;
    row = static_cast<const T *>(b.plane) + (int64_t)kl * b.pitch;
    nr = b.n;
    nw = b.row_nw;
}

template <typename T, bool BATCH>
__global__ __launch_bounds__(kThreads) void k_rowstats(const T *plane, int64_t pitch, int64_t n_, double sigma_min,
                                                       double *stats, const DetBeam *beams, int nbeams, int row0)
{
    const T *row;
    int64_t n;
    const int32_t *nw_unused;
    int k, kl;
    locate_row<BATCH>(plane, pitch, n_, nullptr, beams, nbeams, row0, (int)blockIdx.x, row, n, nw_unused, k, kl);
    const int tid = threadIdx.x;
    if constexpr (IsInt<T>::value) {
        __shared__ unsigned long long s1[kThreads], s2[kThreads];
        // per-thread sums stay exact in 64 bits (at most n / kThreads + 1 samples of < 2^16 each)
        unsigned long long a = 0, b = 0;
        row_fold(row, n, tid, [&](T x, int) {
            const unsigned long long v = (unsigned long long)x;
            a += v;
            b += v * v;
        });
        s1[tid] = a;
        s2[tid] = b;
        __syncthreads();
        for (int s = kThreads / 2; s > 0; s >>= 1) {
            if (tid < s) {
                s1[tid] += s1[tid + s];
                s2[tid] += s2[tid + s];
            }
            __syncthreads();
        }
        if (tid == 0) {
            const double dn = (double)n;
            const double mu = (double)s1[0] / dn;
            const double num = __dsub_rn(__dmul_rn(dn, (double)s2[0]), __dmul_rn((double)s1[0], (double)s1[0]));
            double sg = num > 0.0 ? sqrt(num) / dn : 0.0;
            if (sg < sigma_min) sg = sigma_min;
            stats[2 * k] = mu;
            stats[2 * k + 1] = sg;
        }
    } else {
        // one pass in FP64 about a shift c (the row's first sample), so that a large mean does
        // not cancel: mu = c + S1 / n, sigma^2 = S2 / n - (S1 / n)^2 with S1, S2 the sums of
        // (y - c) and (y - c)^2; two accumulator pairs keep the FP64 adds independent
        __shared__ double r1[kThreads], r2[kThreads];
        const double c = (double)row[0];
        double a0 = 0.0, b0 = 0.0, a1 = 0.0, b1 = 0.0;
        row_fold(row, n, tid, [&](T x, int j) {
            const double d = (double)x - c;
            if (j & 1) {
                a1 += d;
                b1 += d * d;
            } else {
                a0 += d;
                b0 += d * d;
            }
        });
        r1[tid] = a0 + a1;
        r2[tid] = b0 + b1;
        __syncthreads();
        for (int s = kThreads / 2; s > 0; s >>= 1) {
            if (tid < s) {
                r1[tid] += r1[tid + s];
                r2[tid] += r2[tid + s];
            }
            __syncthreads();
        }
        if (tid == 0) {
            const double m1 = r1[0] / (double)n;
            const double var = r2[0] / (double)n - m1 * m1;
            double sg = var > 0.0 ? sqrt(var) : 0.0;
            if (sg < sigma_min) sg = sigma_min;
            stats[2 * k] = c + m1;
            stats[2 * k + 1] = sg;
        }
    }
}

// Per-row constants of S/N(t, W) = (S_W(t) - mu W) / (sigma sqrt W), for threads tid < nw:
// mu W, sigma sqrt W and the bound on the boxcar sum below which a cell cannot reach the
// threshold at width W.
template <typename P>
__device__ inline void row_constants(int tid, const SnrArgs &a, double mu, double sg, double *muw, double *den,
                                     P *sthr, bool is_int)
{
    if (tid >= a.nw) return;
    muw[tid] = __dmul_rn(mu, (double)a.w[tid]);
    den[tid] = __dmul_rn(sg, a.sqrtw[tid]);
    // S/N >= Theta needs S >= mu W + Theta sigma sqrt W up to the rounding of the exact
    // quotient (relative 1e-16); the bound takes a relative margin of 1e-9 below that
    const double b = muw[tid] + a.threshold * den[tid];
    const double thr = b - 1e-9 * (fabs(muw[tid]) + a.threshold * den[tid]);
    if (is_int) {  // integer sums: the largest integer at or below the bound
        sthr[tid] = thr <= -2147483648.0 ? (P)(-2147483647 - 1) : thr >= 2147483647.0 ? (P)2147483647 : (P)floor(thr);
    } else {
        sthr[tid] = (P)thr;
    }
}

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
__device__ inline uint32_t pk_sub(uint32_t x, uint32_t y)  // two 16-bit differences modulo 2^16
{
    return __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, x) - __builtin_bit_cast(u16x2, y));
}
__device__ inline uint32_t pk_sub_sat(uint32_t x, uint32_t y)  // two max(x - y, 0)
{
    return __builtin_bit_cast(uint32_t,
                              __builtin_elementwise_sub_sat(__builtin_bit_cast(u16x2, x), __builtin_bit_cast(u16x2, y)));
}
// (p mod 2^16, (p + x) mod 2^16) from p and a word whose byte 2 holds x (other bytes zero)
__device__ inline uint32_t pair_word(uint32_t p, uint32_t x_hi)
{
    return __builtin_amdgcn_perm(p, p, 0x01000100u) + x_hi;
}

// Inclusive sum over the 64 lanes of a wave with DPP moves: within each row of 16 lanes by
// shifts of 1, 2, 4 and 8 (lanes shifted in from outside the row add zero), then lane 15's total
// into rows 1 and 3, then lane 31's into rows 2 and 3.
__device__ inline uint32_t wave_inclusive_sum(uint32_t x)
{
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);  // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);  // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);  // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);  // row_shr:8
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);  // row_bcast:15
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return x;
}

// The same scan for FP64 values (each DPP move carries the two halves of a value).
template <int CTRL, int ROW_MASK>
__device__ inline double dpp_f64(double x)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, ROW_MASK, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, ROW_MASK, 0xf, false);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ inline double wave_inclusive_sum(double x)
{
    x += dpp_f64<0x111, 0xf>(x);
    x += dpp_f64<0x112, 0xf>(x);
    x += dpp_f64<0x114, 0xf>(x);
    x += dpp_f64<0x118, 0xf>(x);
    x += dpp_f64<0x142, 0xa>(x);
    x += dpp_f64<0x143, 0xc>(x);
    return x;
}
__device__ inline int32_t wave_inclusive_sum(int32_t x) { return (int32_t)wave_inclusive_sum((uint32_t)x); }

// The paired path applies to a u8 list whose first width is 1 and whose other widths are even
// and at most 256 (every boxcar sum of u8 samples is then below 2^16).
template <int NW>
__device__ inline bool pairs_usable(const SnrArgs &a)
{
    if (a.w[0] != 1 || a.w[NW - 1] > 256) return false;
#pragma unroll
    for (int w = 1; w < NW; ++w)
        if (a.w[w] & 1) return false;
    return true;
}

// Compaction on the paired path for one interior tile of a u8 row (16-byte aligned): every
// width fits every cell of the tile.  The tile's bytes are loaded into registers before the
// row's statistics, so that the two loads overlap.  The cells whose bound test passes take the
// exact quotient, as on the general path; the output is the same list (none when sigma is 0).
template <int NW>
__device__ void snr_pairs(const uint8_t *row, int k, int64_t t0, int nwk, int wmax, const double *stats,
                          const SnrArgs &a, unsigned char *dyn, int32_t *wtot, int (*slab_off)[kThreads / 64],
                          unsigned int &base_s, double *muw, double *den, int32_t *sthr)
{
    __shared__ uint64_t smask[snr_tile<uint8_t>() / 2 / kThreads][kThreads / 64][2];
    constexpr int kTile = snr_tile<uint8_t>();
    constexpr int kPairs = kTile / 2 / kThreads;  // pairs of cells per thread
    static_assert(kTile == 16 * kThreads, "sixteen staged bytes per thread");
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    uint16_t *pre16 = reinterpret_cast<uint16_t *>(dyn);  // pre16[j] = P(j) mod 2^16
    // thread t: samples 16 t .. 16 t + 15 (one 16-byte load); wave 0 also the halo samples
    // 4096 + 4 lane .. + 3 that exist in the tile's window (L = 4096 + wmax - 1 samples; the
    // others read as zero and feed prefix entries no width of the row reads)
    const u32x4 q = as_global(reinterpret_cast<const u32x4 *>(row))[tid];
    uint32_t hq = 0u;
    if (wv == 0) {
        const auto grow = as_global(row + kTile);
#pragma unroll
        for (int b = 0; b < 4; ++b)
            if (4 * lane + b < wmax - 1) hq |= (uint32_t)grow[4 * lane + b] << (8 * b);
    }
    const double mu = stats[2 * k], sg = stats[2 * k + 1];
    if (!(sg > 0.0)) return;  // uniform: no cell of the row has a non-zero S/N
    row_constants(tid, a, mu, sg, muw, den, sthr, true);
    // per-width thresholds as two 16-bit copies of sthr - 1: a cell's sum S passes when
    // max(S - (sthr - 1), 0) > 0; widths past the row's set never pass; a bound at or below
    // zero passes every cell (flag word all ones)
    __shared__ uint2 thw[NW];
    if (tid < NW) {
        const int32_t sb = sthr[tid];
        uint32_t t = 0xFFFFu, all = 0u;
        if (tid < nwk) {
            if (sb <= 0) all = 0xFFFFFFFFu;
            else t = (uint32_t)min(sb - 1, 65535);
        }
        thw[tid] = uint2{t * 0x00010001u, all};
    }
    constexpr uint32_t kOnes = 0x01010101u;
    uint32_t tot = __builtin_amdgcn_udot4(q.x, kOnes, 0u, false);
    tot = __builtin_amdgcn_udot4(q.y, kOnes, tot, false);
    tot = __builtin_amdgcn_udot4(q.z, kOnes, tot, false);
    tot = __builtin_amdgcn_udot4(q.w, kOnes, tot, false);
    const uint32_t htot = __builtin_amdgcn_udot4(hq, kOnes, 0u, false);
    const uint32_t inc = wave_inclusive_sum(tot);
    if (lane == 63) wtot[wv] = (int32_t)inc;
    __syncthreads();
    uint32_t B = inc - tot;
    for (int w = 0; w < wv; ++w) B += (uint32_t)wtot[w];
    uint32_t words[8];
    const uint32_t qd[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const uint32_t d = qd[m];
        words[2 * m] = pair_word(B, __builtin_amdgcn_perm(0u, d, 0x0c000c0cu));      // P(4m), P(4m + 1)
        const uint32_t B2 = __builtin_amdgcn_udot4(d, 0x00000101u, B, false);
        words[2 * m + 1] = pair_word(B2, __builtin_amdgcn_perm(0u, d, 0x0c020c0cu));  // P(4m + 2), P(4m + 3)
        B = __builtin_amdgcn_udot4(d, kOnes, B, false);
    }
    u32x4 *p4 = reinterpret_cast<u32x4 *>(pre16 + 16 * tid);
    p4[0] = u32x4{words[0], words[1], words[2], words[3]};
    p4[1] = u32x4{words[4], words[5], words[6], words[7]};
    if (wv == 0) {  // P(4096 + 4 lane + i), i = 0..3
        const uint32_t hinc = wave_inclusive_sum(htot);
        const uint32_t Bh = (uint32_t)wtot[0] + (uint32_t)wtot[1] + (uint32_t)wtot[2] + (uint32_t)wtot[3] + hinc - htot;
        const uint32_t w0 = pair_word(Bh, __builtin_amdgcn_perm(0u, hq, 0x0c000c0cu));
        const uint32_t w1 = pair_word(__builtin_amdgcn_udot4(hq, 0x00000101u, Bh, false),
                                      __builtin_amdgcn_perm(0u, hq, 0x0c020c0cu));
        uint32_t *h2 = reinterpret_cast<uint32_t *>(pre16 + kTile + 4 * lane);
        h2[0] = w0;
        h2[1] = w1;
    }
    __syncthreads();
    uint32_t th[NW];
    int hw[NW];
    uint32_t m0 = 0u;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        hw[w] = w == 0 ? 1 : (a.w[w] >> 1);
        const uint2 t = thw[w];
        th[w] = t.x;
        m0 |= t.y;
    }
    const uint32_t *dw = reinterpret_cast<const uint32_t *>(pre16);
    auto exact16 = [&](int i, double &best, int &bi) {
        best = 0.0;
        bi = -1;
        for (int w = 0; w < nwk; ++w) {
            const int W = a.w[w];
            const double s = (double)(uint16_t)(pre16[i + W] - pre16[i]);
            const double val = __dsub_rn(s, muw[w]) / den[w];
            if (bi < 0 || val > best) {
                best = val;
                bi = w;
            }
        }
    };
    // straight-line bound tests; mk[j]: the wave's lanes whose pair j has a cell that passes
    uint64_t mk[kPairs];
    uint64_t any = 0;
#pragma unroll
    for (int j = 0; j < kPairs; ++j) {
        const int qp = tid + kThreads * j;
        const uint32_t d0 = dw[qp];
        uint32_t m = m0 | pk_sub_sat(pk_sub(__builtin_amdgcn_alignbit(dw[qp + 1], d0, 16), d0), th[0]);
#pragma unroll
        for (int w = 1; w < NW; ++w) m |= pk_sub_sat(pk_sub(dw[qp + hw[w]], d0), th[w]);
        mk[j] = __ballot(m != 0u);
        any |= mk[j];
    }
    // the marked pairs (few) take the exact quotient on both cells; bit 2 j + h of `flags`:
    // cell 2 (tid + 256 j) + h reaches the threshold
    uint32_t maybe = 0;
    if (any) {  // uniform over the wave
#pragma unroll
        for (int j = 0; j < kPairs; ++j) maybe |= (uint32_t)((mk[j] >> lane) & 1u) << j;
    }
    uint32_t flags = 0;
    while (maybe) {
        const int j = __builtin_ctz(maybe);
        maybe &= maybe - 1u;
#pragma unroll 1
        for (int h = 0; h < 2; ++h) {
            double best;
            int bi;
            exact16(2 * (tid + kThreads * j) + h, best, bi);
            if (bi >= 0 && best >= a.threshold) flags |= 1u << (2 * j + h);
        }
    }
    // ordered output: pairs in increasing t (slab j, then thread), the even cell first; each
    // wave's ballots of its even and odd cells per slab go through LDS for the output loop
#pragma unroll
    for (int j = 0; j < kPairs; ++j) {
        const uint64_t b0 = __ballot((flags >> (2 * j)) & 1u), b1 = __ballot((flags >> (2 * j + 1)) & 1u);
        if (lane == 0) {
            slab_off[j][wv] = __popcll(b0) + __popcll(b1);
            smask[j][wv][0] = b0;
            smask[j][wv][1] = b1;
        }
    }
    __syncthreads();
    if (tid == 0) {
        int tsum = 0;
        for (int j = 0; j < kPairs; ++j)
            for (int w = 0; w < kThreads / 64; ++w) {
                const int c = slab_off[j][w];
                slab_off[j][w] = tsum;
                tsum += c;
            }
        base_s = tsum ? atomicAdd(a.counter, (unsigned int)tsum) : 0u;
    }
    __syncthreads();
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    uint32_t f = flags;
    while (f) {
        const int b = __builtin_ctz(f);
        f &= f - 1u;
        const int j = b >> 1, h = b & 1;
        const int64_t pos = (int64_t)base_s + slab_off[j][wv] + __popcll(smask[j][wv][0] & below) +
                            __popcll(smask[j][wv][1] & below) + (h ? ((flags >> (2 * j)) & 1u) : 0u);
        if (pos < a.max_pixels) {
            // the flagged cells are few: their exact maximum is taken again rather than kept
            const int i = 2 * (tid + kThreads * j) + h;
            double best;
            int bi;
            exact16(i, best, bi);
            Pixel px;
            px.k = k;
            px.t = (int32_t)(t0 + i);
            px.snr = best;
            px.widx = bi;
            px.pad = 0;
            a.pixels[pos] = px;
        }
    }
}

// NW > 0: exactly NW widths, known at compile time (per-row constants stay in registers);
// NW == 0: any number of widths.  BATCH: rows of several planes (SnrArgs::beams).
template <typename T, int NW, bool BATCH>
__global__ __launch_bounds__(kThreads) void k_snr(const T *plane, int64_t pitch, int64_t n_, const double *stats,
                                                  SnrArgs a)
{
    using P = typename PrefixType<T>::type;
    constexpr int kSnrTile = snr_tile<T>();
    constexpr int kMaxPer = (kSnrTile + kMaxWidth + kThreads - 1) / kThreads;  // elements per thread
    constexpr int kSlabs = kSnrTile / kThreads;                                // samples per thread
    static_assert(kSlabs <= 32, "one flag bit per slab");
    extern __shared__ __align__(16) unsigned char snr_dyn[];  // prefix sums: tile + widest width + 1
    P *pre = reinterpret_cast<P *>(snr_dyn);
    __shared__ P wtot[kThreads / 64];
    __shared__ int slab_off[kSlabs][kThreads / 64];
    __shared__ unsigned int base_s;
    __shared__ double muw[kMaxWidths], den[kMaxWidths];  // per-row constants
    __shared__ P sthr[kMaxWidths];                       // per-row boxcar-sum bounds
    const T *rowk;
    int64_t n;
    const int32_t *row_nw;
    int k, kl;
    locate_row<BATCH>(plane, pitch, n_, a.row_nw, a.beams, a.nbeams, a.row0, (int)blockIdx.y, rowk, n, row_nw, k, kl);
    const int64_t t0 = (int64_t)blockIdx.x * kSnrTile;
    if constexpr (BATCH) {
        if (t0 >= n) return;  // a shorter plane of the batch (uniform: before any barrier)
    }
    const T *row = rowk + t0;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // widths of this row: the first nwk of the list (all of them unless a DM-scaled set)
    const int nwk = row_nw ? row_nw[kl] : a.nw;
    const int wmax = a.w[nwk - 1];
    // elements t0 .. t0 + L - 1 are needed (and exist): L = min(tile + wmax - 1, n - t0)
    int64_t L64 = (int64_t)kSnrTile + wmax - 1;
    if (L64 > n - t0) L64 = n - t0;
    const int L = (int)L64;
    if constexpr (std::is_same<T, uint8_t>::value && NW >= 2) {
        // uniform over the workgroup: the list, the tile's place in the row and its alignment
        if (!a.snr && t0 + kSnrTile + wmax - 1 <= n && ((uintptr_t)row & 15u) == 0 && pairs_usable<NW>(a)) {
            snr_pairs<NW>(row, k, t0, nwk, wmax, stats, a, snr_dyn, wtot, slab_off, base_s, muw, den, sthr);
            return;
        }
    }
    // float tiles on a 16-byte boundary are read as 16-byte vectors: chunks of a multiple of
    // four samples (at most kMaxPer, since kMaxPer is itself a multiple of four)
    static_assert(kMaxPer % 4 == 0, "vector chunks");
    const bool vec4 = !IsInt<T>::value && sizeof(T) == 4 && ((uintptr_t)row & 15u) == 0;
    // integer tiles: every thread takes kMaxPer elements, those past L read as zero (the staged
    // bytes fit the prefix array for any L), and only prefix entries up to L are written
    const int per = IsInt<T>::value ? kMaxPer
                    : vec4          ? (L + 4 * kThreads - 1) / (4 * kThreads) * 4
                                    : (L + kThreads - 1) / kThreads;
    const int beg = tid * per;
    // prefix sums: per-thread chunk totals, wave scan, wave totals through LDS.  Integer
    // tiles are first read with coalesced loads into LDS (in the prefix array's storage, which
    // is written only after the barrier below); float tiles are read in place (measured faster)
    P v[kMaxPer];
    P run = 0;
    if constexpr (IsInt<T>::value) {
        T *raw = reinterpret_cast<T *>(pre);
        static_assert(sizeof(T) <= sizeof(P), "the staged tile fits the prefix array");
        const auto grow = as_global(row);
        // 16-byte loads where the tile starts on a 16-byte boundary (rows of 64-sample pitch do)
        constexpr int E = 16 / (int)sizeof(T);
        int j0 = 0;
        if (((uintptr_t)row & 15u) == 0) {
            const auto g4 = as_global(reinterpret_cast<const u32x4 *>(row));
            u32x4 *r4 = reinterpret_cast<u32x4 *>(raw);
            for (int j = tid; j < L / E; j += kThreads) r4[j] = g4[j];
            j0 = L / E * E;
        }
        for (int j = j0 + tid; j < L; j += kThreads) raw[j] = grow[j];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kMaxPer; ++i) {
            const int j = beg + i;
            const P x = (P)raw[j];
            v[i] = j < L ? x : (P)0;
            run += v[i];
        }
    } else if (vec4) {
        typedef float f32x4 __attribute__((ext_vector_type(4)));
        const auto g4 = as_global(reinterpret_cast<const f32x4 *>(row));
        const auto grow = as_global(row);
#pragma unroll
        for (int i = 0; i < kMaxPer; i += 4) {
            const int j = beg + i;
            if (i < per && j + 3 < L) {
                const f32x4 q = g4[j >> 2];
                v[i] = (P)q.x;
                v[i + 1] = (P)q.y;
                v[i + 2] = (P)q.z;
                v[i + 3] = (P)q.w;
            } else {
#pragma unroll
                for (int u = 0; u < 4; ++u) v[i + u] = (i < per && j + u < L) ? (P)grow[j + u] : (P)0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) run += v[i + u];
        }
    } else {
        const auto grow = as_global(row);
#pragma unroll
        for (int i = 0; i < kMaxPer; ++i) {
            const int j = beg + i;
            v[i] = (i < per && j < L) ? (P)grow[j] : (P)0;
            run += v[i];
        }
    }
    const P inc = wave_inclusive_sum(run);
    if (lane == 63) wtot[wv] = inc;
    __syncthreads();
    P acc = inc - run;
    for (int w = 0; w < wv; ++w) acc += wtot[w];
    if (tid == 0) pre[0] = 0;
    if constexpr (IsInt<T>::value) {
#pragma unroll
        for (int i = 0; i < kMaxPer; ++i) {
            acc += v[i];
            if (beg + i < L) pre[beg + i + 1] = acc;  // entries 1 .. L (the array holds tile + wmax + 1)
        }
    } else {
#pragma unroll
        for (int i = 0; i < kMaxPer; ++i) {
            const int j = beg + i;
            if (i < per && j < L) {
                acc += v[i];
                pre[j + 1] = acc;
            }
        }
    }
    const double mu = stats[2 * k], sg = stats[2 * k + 1];
    // per-row constants of S/N(t, W) = (S_W(t) - mu W) / (sigma sqrt W)
    row_constants(tid, a, mu, sg, muw, den, sthr, IsInt<T>::value);
    __syncthreads();
    // the exact maximum over widths of sample i (first width on ties)
    auto exact = [&](int i, int64_t t, double &best, int &bi) {
        best = 0.0;
        bi = -1;
        for (int w = 0; w < nwk; ++w) {
            const int W = a.w[w];
            if (t + W > n) break;
            double val = 0.0;
            if (sg > 0.0) {
                const double s = (double)(pre[i + W] - pre[i]);
                val = __dsub_rn(s, muw[w]) / den[w];
            }
            if (bi < 0 || val > best) {
                best = val;
                bi = w;
            }
        }
    };
    if (a.snr) {  // the whole S/N plane
        for (int i = tid; i < kSnrTile; i += kThreads) {
            const int64_t t = t0 + i;
            if (t >= n) break;
            double best;
            int bi;
            exact(i, t, best, bi);
            a.snr[(int64_t)k * a.snr_pitch + t] = (float)best;
            a.widx[(int64_t)k * a.widx_pitch + t] = (int8_t)bi;
        }
        return;
    }
    // compaction: a cell can reach the threshold at width W only if its boxcar sum reaches
    // the row's bound for W (one subtraction and one compare per width, in the prefix type);
    // the cells that do take the exact quotient
    constexpr int RW = NW > 0 ? NW : 1;
    P rthr[RW];
    int rw[RW];
    if constexpr (NW > 0) {
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            // widths beyond the row's set get a bound no sum reaches (their prefix reads stay
            // inside the prefix array; the values there are not this row's and are never used)
            rthr[w] = w < nwk ? sthr[w] : BoundNever<P>::value();
            rw[w] = a.w[w];
        }
    }
    // every width fits every sample of the tile: no end-of-row tests
    const bool interior = t0 + kSnrTile + wmax - 1 <= n;
    uint32_t flags = 0;
    if (NW > 0 && interior && sg > 0.0) {  // straight-line bound tests; the exact quotient is rare
#pragma unroll
        for (int j = 0; j < kSlabs; ++j) {
            const int i = tid + kThreads * j;
            const P p0 = pre[i];
            bool maybe = false;
#pragma unroll
            for (int w = 0; w < RW; ++w) maybe |= (P)(pre[i + rw[w]] - p0) >= rthr[w];
            if (maybe) {
                double best;
                int bi;
                exact(i, t0 + i, best, bi);
                if (bi >= 0 && best >= a.threshold) flags |= 1u << j;
            }
        }
    } else {
#pragma unroll
    for (int j = 0; j < kSlabs; ++j) {
        const int i = tid + kThreads * j;
        const int64_t t = t0 + i;
        if (t >= n || !(sg > 0.0)) continue;
        const P p0 = pre[i];
        bool maybe = false;
        if (NW > 0 && interior) {
#pragma unroll
            for (int w = 0; w < RW; ++w) maybe |= (P)(pre[i + rw[w]] - p0) >= rthr[w];
        } else {
            for (int w = 0; w < nwk; ++w) {
                if (t + a.w[w] > n) break;
                maybe |= (P)(pre[i + a.w[w]] - p0) >= sthr[w];
            }
        }
        if (!maybe) continue;
        double best;
        int bi;
        exact(i, t, best, bi);
        if (bi >= 0 && best >= a.threshold) flags |= 1u << j;
    }
    }
    // ordered output: the block's cells in increasing t (slab by slab, thread by thread)
    uint64_t masks[kSlabs];
#pragma unroll
    for (int j = 0; j < kSlabs; ++j) {
        masks[j] = __ballot((flags >> j) & 1u);
        if (lane == 0) slab_off[j][wv] = __popcll(masks[j]);
    }
    __syncthreads();
    if (tid == 0) {
        int tot = 0;
        for (int j = 0; j < kSlabs; ++j)
            for (int w = 0; w < kThreads / 64; ++w) {
                const int c = slab_off[j][w];
                slab_off[j][w] = tot;
                tot += c;
            }
        base_s = tot ? atomicAdd(a.counter, (unsigned int)tot) : 0u;
    }
    __syncthreads();
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
#pragma unroll
    for (int j = 0; j < kSlabs; ++j) {
        if (!((flags >> j) & 1u)) continue;
        const int64_t pos = (int64_t)base_s + slab_off[j][wv] + __popcll(masks[j] & below);
        if (pos < a.max_pixels) {
            // the flagged cells are few: their exact maximum is taken again rather than kept
            const int i = tid + kThreads * j;
            double best;
            int bi;
            exact(i, t0 + i, best, bi);
            Pixel px;
            px.k = k;
            px.t = (int32_t)(t0 + i);
            px.snr = best;
            px.widx = bi;
            px.pad = 0;
            a.pixels[pos] = px;
        }
    }
}

// Robust row sigma, the MAD option of the matched filter: sigma = kMadScale * MAD, MAD the lower
// median of |y - m| over the row's valid samples and m the row's lower median (rank
// floor((n - 1) / 2) of the sorted values; kMadScale = 1 / Phi^-1(3/4) makes it the standard
// deviation of Gaussian noise).  Both medians are exact: a radix select over an order-preserving
// integer key of the values, 8 bits per pass over the row, with one histogram per wave in LDS.
// The deviation is taken in the plane's own arithmetic: exact for integer planes, one FP32
// subtraction for float planes.  The floor sigma_min applies as for the standard deviation.
constexpr double kMadScale = 1.4826022185056018;

template <typename T> struct MadKeys;
template <> struct MadKeys<uint8_t> {
    static constexpr int kBits = 8;
    __device__ static uint32_t key(uint8_t v) { return v; }
    __device__ static uint8_t value(uint32_t k) { return (uint8_t)k; }
    __device__ static uint32_t dev_key(uint8_t v, uint8_t m) { return v > m ? (uint32_t)(v - m) : (uint32_t)(m - v); }
    __device__ static double dev_value(uint32_t k) { return (double)k; }
};
template <> struct MadKeys<uint16_t> {
    static constexpr int kBits = 16;
    __device__ static uint32_t key(uint16_t v) { return v; }
    __device__ static uint16_t value(uint32_t k) { return (uint16_t)k; }
    __device__ static uint32_t dev_key(uint16_t v, uint16_t m) { return v > m ? (uint32_t)(v - m) : (uint32_t)(m - v); }
    __device__ static double dev_value(uint32_t k) { return (double)k; }
};
template <> struct MadKeys<float> {
    static constexpr int kBits = 32;
    // IEEE order as unsigned order: negative values reversed below the positive ones
    __device__ static uint32_t key(float v)
    {
        const uint32_t u = __float_as_uint(v);
        return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    }
    __device__ static float value(uint32_t k) { return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k); }
    __device__ static uint32_t dev_key(float v, float m) { return key(__builtin_fabsf(v - m)); }
    __device__ static double dev_value(uint32_t k) { return (double)value(k); }
};

// Key of rank `rank` (0-based, in increasing order) among key(y) over the row.
template <typename T, int BITS, typename K>
__device__ uint32_t radix_select(const T *row, int64_t n, int64_t rank, K key, uint32_t (*hist)[256],
                                 uint32_t *s_digit, long long *s_rank)
{
    const int tid = threadIdx.x, wave = tid >> 6;
    uint32_t prefix = 0;
    for (int shift = BITS - 8; shift >= 0; shift -= 8) {
        for (int i = tid; i < (kThreads / 64) * 256; i += kThreads) (&hist[0][0])[i] = 0u;
        __syncthreads();
        const int hs = shift + 8;  // keys that agree with the prefix above this digit take part
        row_fold(row, n, tid, [&](T v, int) {
            const uint32_t k = key(v);
            if ((uint32_t)((uint64_t)(k ^ prefix) >> hs) == 0u) atomicAdd(&hist[wave][(k >> shift) & 255u], 1u);
        });
        __syncthreads();
        if (tid < 256) {
            uint32_t c = 0;
#pragma unroll
            for (int w = 0; w < kThreads / 64; ++w) c += hist[w][tid];
            hist[0][tid] = c;
        }
        __syncthreads();
        if (tid == 0) {  // the digit whose bin holds the rank; the taking part outnumber it
            long long r = rank;
            uint32_t b = 0;
            for (; b < 255u && r >= (long long)hist[0][b]; ++b) r -= hist[0][b];
            *s_digit = b;
            *s_rank = r;
        }
        __syncthreads();
        prefix |= *s_digit << shift;
        rank = *s_rank;
        __syncthreads();  // everyone has read the digit before the histogram is cleared
    }
    return prefix;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_rowmad(const T *plane, int64_t pitch, int64_t n, double sigma_min,
                                                       double *stats)
{
    __shared__ uint32_t hist[kThreads / 64][256];
    __shared__ uint32_t s_digit;
    __shared__ long long s_rank;
    const int64_t k = blockIdx.x;
    const T *row = plane + k * pitch;
    const int64_t r = (n - 1) / 2;
    using MK = MadKeys<T>;
    const T m = MK::value(radix_select<T, MK::kBits>(row, n, r, [](T v) { return MK::key(v); }, hist, &s_digit, &s_rank));
    const uint32_t d = radix_select<T, MK::kBits>(row, n, r, [m](T v) { return MK::dev_key(v, m); }, hist, &s_digit,
                                                  &s_rank);
    if (threadIdx.x == 0) {
        double sg = kMadScale * MK::dev_value(d);
        if (sg < sigma_min) sg = sigma_min;
        stats[2 * k + 1] = sg;
    }
}

__global__ void k_zero_counter(unsigned int *c) { *c = 0u; }

template <typename T, bool BATCH>
int launch_snr_grid(dim3 grid, const T *p, int64_t pitch, int64_t n, double *stats, const SnrArgs &a, hipStream_t st);

template <typename T>
int launch_typed(const void *plane, int64_t pitch, int ndm, int64_t n, double sigma_min, int sigma_mad,
                 double *stats, const SnrArgs &a, hipStream_t st)
{
    const T *p = static_cast<const T *>(plane);
    if (!a.snr) hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(1), 0, st, a.counter);
    hipLaunchKernelGGL((k_rowstats<T, false>), dim3((uint32_t)ndm), dim3(kThreads), 0, st, p, pitch, n, sigma_min,
                       stats, (const DetBeam *)nullptr, 0, 0);
    if (sigma_mad)  // sigma from the median absolute deviation instead (the mean stays)
        hipLaunchKernelGGL((k_rowmad<T>), dim3((uint32_t)ndm), dim3(kThreads), 0, st, p, pitch, n, sigma_min, stats);
    constexpr int kSnrTile = snr_tile<T>();
    dim3 grid((uint32_t)((n + kSnrTile - 1) / kSnrTile), (uint32_t)ndm);
    return launch_snr_grid<T, false>(grid, p, pitch, n, stats, a, st);
}

// Batched: statistics and S/N of batch rows a.row0 .. a.row0 + nrows - 1; the grid spans the
// longest plane, the tiles past a shorter plane's end return at once.
template <typename T>
int launch_typed_batch(int nrows, int64_t n_max, double sigma_min, double *stats, const SnrArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL((k_rowstats<T, true>), dim3((uint32_t)nrows), dim3(kThreads), 0, st, (const T *)nullptr,
                       (int64_t)0, (int64_t)0, sigma_min, stats, a.beams, a.nbeams, a.row0);
    constexpr int kSnrTile = snr_tile<T>();
    dim3 grid((uint32_t)((n_max + kSnrTile - 1) / kSnrTile), (uint32_t)nrows);
    return launch_snr_grid<T, true>(grid, (const T *)nullptr, 0, 0, stats, a, st);
}

template <typename T, bool BATCH>
int launch_snr_grid(dim3 grid, const T *p, int64_t pitch, int64_t n, double *stats, const SnrArgs &a, hipStream_t st)
{
    constexpr int kSnrTile = snr_tile<T>();
    // the prefix array holds the tile plus the widest boxcar of the list (every row's set is a
    // leading part of the list); integer tiles are first staged in its storage, at most
    // kThreads * kMaxPer samples of sizeof(T) <= 2 bytes each
    constexpr int64_t kStageBytes = IsInt<T>::value ? (int64_t)kThreads * ((kSnrTile + kMaxWidth + kThreads - 1) / kThreads) * 2 : 0;
    const int64_t entries = std::max<int64_t>(kSnrTile + a.w[a.nw - 1] + 1,
                                              (kStageBytes + (int64_t)sizeof(typename PrefixType<T>::type) - 1) /
                                                  (int64_t)sizeof(typename PrefixType<T>::type));
    const size_t lds = (size_t)entries * sizeof(typename PrefixType<T>::type);
    switch (a.nw) {
#define SND_NW(N) case N: hipLaunchKernelGGL((k_snr<T, N, BATCH>), grid, dim3(kThreads), lds, st, p, pitch, n, stats, a); break;
    SND_NW(1) SND_NW(2) SND_NW(3) SND_NW(4) SND_NW(5) SND_NW(6) SND_NW(7) SND_NW(8)
#undef SND_NW
    default: hipLaunchKernelGGL((k_snr<T, 0, BATCH>), grid, dim3(kThreads), lds, st, p, pitch, n, stats, a); break;
    }
    return (int)hipGetLastError();
}

}  // namespace

int launch_detect(int plane_dtype, const void *plane, int64_t pitch, int ndm, int64_t n, double sigma_min,
                  int sigma_mad, double *stats, const SnrArgs &a, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    switch (plane_dtype) {
    case SND_DT_U8: return launch_typed<uint8_t>(plane, pitch, ndm, n, sigma_min, sigma_mad, stats, a, st);
    case SND_DT_U16: return launch_typed<uint16_t>(plane, pitch, ndm, n, sigma_min, sigma_mad, stats, a, st);
    case SND_DT_F32: return launch_typed<float>(plane, pitch, ndm, n, sigma_min, sigma_mad, stats, a, st);
    }
    return (int)hipErrorInvalidValue;
}

int launch_zero_counter(unsigned int *counter, void *stream)
{
    hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(1), 0, (hipStream_t)stream, counter);
    return (int)hipGetLastError();
}

int launch_detect_batch(int plane_dtype, int nrows, int64_t n_max, double sigma_min, double *stats, const SnrArgs &a,
                        void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    switch (plane_dtype) {
    case SND_DT_U8: return launch_typed_batch<uint8_t>(nrows, n_max, sigma_min, stats, a, st);
    case SND_DT_U16: return launch_typed_batch<uint16_t>(nrows, n_max, sigma_min, stats, a, st);
    case SND_DT_F32: return launch_typed_batch<float>(nrows, n_max, sigma_min, stats, a, st);
    }
    return (int)hipErrorInvalidValue;
}

}  // namespace snd
