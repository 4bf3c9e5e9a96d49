// Boxcar matched filter and candidate-pixel compaction for gfx950 (Methods, "Matched
// filtering" and "Candidate detection").
//
// k_rowstats: mean and population standard deviation of each DM row over its valid samples.
//   Integer planes use exact 64-bit sums S1, S2 and sigma = sqrt(n*S2 - S1*S1)/n in one fixed
//   FP64 expression; float planes use a two-pass FP64 reduction.  A floor sigma_min applies.
// k_snr: one workgroup per (row, 1024-sample tile).  The tile plus the widest boxcar is
//   staged in LDS as an inclusive prefix sum (int32 for integer planes: exact; FP64 for float
//   planes), every sample then evaluates all widths with two LDS reads each:
//   SNR(t, W) = (S_W(t) - mu W) / (sigma sqrt W), maximum over widths (first width on ties).
//   Cells whose S/N reaches the threshold are appended to a global pixel list, or the full
//   S/N plane and width index are written.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "snd_detect.h"

namespace snd {
namespace {

constexpr int kSnrTile = 1024;
constexpr int kThreads = 256;

template <typename T> struct IsInt { static constexpr bool value = true; };
template <> struct IsInt<float> { static constexpr bool value = false; };

template <typename T>
__global__ __launch_bounds__(kThreads) void k_rowstats(const T *plane, int64_t pitch, int64_t n, double sigma_min,
                                                       double *stats)
{
    const int k = blockIdx.x;
    const T *row = plane + (int64_t)k * pitch;
    const int tid = threadIdx.x;
    if constexpr (IsInt<T>::value) {
        __shared__ unsigned long long s1[kThreads], s2[kThreads];
        unsigned long long a = 0, b = 0;
        for (int64_t t = tid; t < n; t += kThreads) {
            unsigned long long v = (unsigned long long)row[t];
            a += v;
            b += v * v;
        }
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
        __shared__ double red[kThreads];
        double a = 0.0;
        for (int64_t t = tid; t < n; t += kThreads) a += (double)row[t];
        red[tid] = a;
        __syncthreads();
        for (int s = kThreads / 2; s > 0; s >>= 1) {
            if (tid < s) red[tid] += red[tid + s];
            __syncthreads();
        }
        const double mu = red[0] / (double)n;
        __syncthreads();
        double q = 0.0;
        for (int64_t t = tid; t < n; t += kThreads) {
            double d = (double)row[t] - mu;
            q += d * d;
        }
        red[tid] = q;
        __syncthreads();
        for (int s = kThreads / 2; s > 0; s >>= 1) {
            if (tid < s) red[tid] += red[tid + s];
            __syncthreads();
        }
        if (tid == 0) {
            double sg = sqrt(red[0] / (double)n);
            if (sg < sigma_min) sg = sigma_min;
            stats[2 * k] = mu;
            stats[2 * k + 1] = sg;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_snr(const T *plane, int64_t pitch, int64_t n, const double *stats,
                                                  SnrArgs a)
{
    using P = typename PrefixType<T>::type;
    __shared__ P pre[kSnrTile + kMaxWidth + 1];
    __shared__ P part[kThreads];
    const int k = blockIdx.y;
    const int64_t t0 = (int64_t)blockIdx.x * kSnrTile;
    const T *row = plane + (int64_t)k * pitch;
    const int tid = threadIdx.x;
    const int wmax = a.w[a.nw - 1];
    // elements t0 .. t0 + L - 1 are needed (and exist): L = min(tile + wmax - 1, n - t0)
    int64_t L64 = (int64_t)kSnrTile + wmax - 1;
    if (L64 > n - t0) L64 = n - t0;
    const int L = (int)L64;
    const int per = (L + kThreads - 1) / kThreads;
    const int beg = tid * per;
    P run = 0;
    for (int i = 0; i < per; ++i) {
        const int j = beg + i;
        if (j < L) run += (P)row[t0 + j];
    }
    part[tid] = run;
    __syncthreads();
    for (int s = 1; s < kThreads; s <<= 1) {  // inclusive scan of the per-thread totals
        P v = tid >= s ? part[tid - s] : (P)0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    P acc = tid > 0 ? part[tid - 1] : (P)0;
    if (tid == 0) pre[0] = 0;
    for (int i = 0; i < per; ++i) {
        const int j = beg + i;
        if (j < L) {
            acc += (P)row[t0 + j];
            pre[j + 1] = acc;
        }
    }
    __syncthreads();
    const double mu = stats[2 * k], sg = stats[2 * k + 1];
    for (int i = tid; i < kSnrTile; i += kThreads) {
        const int64_t t = t0 + i;
        if (t >= n) break;
        double best = 0.0;
        int bi = -1;
        for (int w = 0; w < a.nw; ++w) {
            const int W = a.w[w];
            if (t + W > n) break;
            double val = 0.0;
            if (sg > 0.0) {
                const double s = (double)(pre[i + W] - pre[i]);
                const double num = __dsub_rn(s, __dmul_rn(mu, (double)W));
                const double den = __dmul_rn(sg, a.sqrtw[w]);
                val = num / den;
            }
            if (bi < 0 || val > best) {
                best = val;
                bi = w;
            }
        }
        if (a.snr) {
            a.snr[(int64_t)k * a.snr_pitch + t] = (float)best;
            a.widx[(int64_t)k * a.widx_pitch + t] = (int8_t)bi;
        } else if (bi >= 0 && best >= a.threshold) {
            const unsigned int slot = atomicAdd(a.counter, 1u);
            if ((int64_t)slot < a.max_pixels) {
                Pixel px;
                px.k = k;
                px.t = (int32_t)t;
                px.snr = best;
                px.widx = bi;
                px.pad = 0;
                a.pixels[slot] = px;
            }
        }
    }
}

__global__ void k_zero_counter(unsigned int *c) { *c = 0u; }

template <typename T>
int launch_typed(const void *plane, int64_t pitch, int ndm, int64_t n, double sigma_min, double *stats,
                 const SnrArgs &a, hipStream_t st)
{
    const T *p = static_cast<const T *>(plane);
    if (!a.snr) hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(1), 0, st, a.counter);
    hipLaunchKernelGGL((k_rowstats<T>), dim3((uint32_t)ndm), dim3(kThreads), 0, st, p, pitch, n, sigma_min, stats);
    dim3 grid((uint32_t)((n + kSnrTile - 1) / kSnrTile), (uint32_t)ndm);
    hipLaunchKernelGGL((k_snr<T>), grid, dim3(kThreads), 0, st, p, pitch, n, stats, a);
    return (int)hipGetLastError();
}

}  // namespace

int launch_detect(int plane_dtype, const void *plane, int64_t pitch, int ndm, int64_t n, double sigma_min,
                  double *stats, const SnrArgs &a, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    switch (plane_dtype) {
    case SND_DT_U8: return launch_typed<uint8_t>(plane, pitch, ndm, n, sigma_min, stats, a, st);
    case SND_DT_U16: return launch_typed<uint16_t>(plane, pitch, ndm, n, sigma_min, stats, a, st);
    case SND_DT_F32: return launch_typed<float>(plane, pitch, ndm, n, sigma_min, stats, a, st);
    }
    return (int)hipErrorInvalidValue;
}

}  // namespace snd
