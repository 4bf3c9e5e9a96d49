// Candidate detection on the device (Methods, "Candidate detection"): binary closing of the
// thresholded cells with a (2r+1)^2 square on the zero-extended plane, 8-connected labelling of
// the closed mask cropped to the plane, island sizes and peaks.  Same results as the host path.
//
// The mask is a bit array of the plane padded by 2r on every side (bit j of word w of a row is
// column 64 w + j); closing is four separable passes (dilation along time and along DM, then
// erosion along time and along DM, outside the array counting as zero: the padding keeps every
// dilated bit at least r from its border).  Labelling works on runs, the maximal sequences of
// closed cells within a plane row: runs of adjacent rows that touch (8-connectivity: column
// ranges within one of each other) are joined by a lock-free union-find that always links the
// larger root under the smaller, so every chain of parents decreases and every find ends.  Each
// island's size is the sum of its runs' lengths; its peak is the thresholded cell of highest S/N,
// then lowest DM row, then earliest time (S/N >= threshold > 0, so the FP64 bit patterns order
// as unsigned integers).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "snd_detect.h"

namespace snd {
namespace {

constexpr int kT = 256;

__global__ void k_fill64(uint64_t *p, int64_t n, uint64_t v)
{
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_iota32(int32_t *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i < n) p[i] = (int32_t)i;
}

__global__ void k_mark(const Pixel *px, const unsigned int *count, int64_t max_pixels, uint64_t *mask, int64_t wd,
                       int pad)
{
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    const int64_t n = (int64_t)*count < max_pixels ? (int64_t)*count : max_pixels;
    if (i >= n) return;
    const int64_t col = (int64_t)px[i].t + pad;
    atomicOr(reinterpret_cast<unsigned long long *>(&mask[((int64_t)px[i].k + pad) * wd + (col >> 6)]),
             1ull << (col & 63));
}

// 64 bits of a row starting d columns after word w's first column (|d| <= 64), zero outside.
__device__ inline uint64_t window(const uint64_t *row, int64_t wd, int64_t w, int d)
{
    const uint64_t cur = row[w];
    const uint64_t prev = w > 0 ? row[w - 1] : 0ull, next = w + 1 < wd ? row[w + 1] : 0ull;
    if (d == 0) return cur;
    if (d == 64) return next;
    if (d == -64) return prev;
    if (d > 0) return (cur >> d) | (next << (64 - d));
    return (cur << -d) | (prev >> (64 + d));
}

// along time: out = OR (dilate) or AND (erode) of the row shifted by -r .. r
template <bool DILATE>
__global__ void k_close_t(const uint64_t *in, uint64_t *out, int64_t rows, int64_t wd, int r)
{
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= rows * wd) return;
    const int64_t row = i / wd, w = i % wd;
    const uint64_t *src = in + row * wd;
    uint64_t v = DILATE ? 0ull : ~0ull;
    for (int d = -r; d <= r; ++d) {
        const uint64_t x = window(src, wd, w, d);
        v = DILATE ? (v | x) : (v & x);
    }
    out[i] = v;
}

// along DM: out = OR (dilate) or AND (erode) of rows row - r .. row + r (outside: zero)
template <bool DILATE>
__global__ void k_close_k(const uint64_t *in, uint64_t *out, int64_t rows, int64_t wd, int r)
{
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= rows * wd) return;
    const int64_t row = i / wd, w = i % wd;
    uint64_t v = DILATE ? 0ull : ~0ull;
    for (int d = -r; d <= r; ++d) {
        const int64_t rr = row + d;
        const uint64_t x = (rr >= 0 && rr < rows) ? in[rr * wd + w] : 0ull;
        v = DILATE ? (v | x) : (v & x);
    }
    out[i] = v;
}

// word w of plane row k, cropped to the plane's columns [pad, pad + n)
__device__ inline uint64_t crop_word(const uint64_t *row, int64_t w, int pad, int64_t n)
{
    const int64_t c0 = 64 * w, lo = pad, hi = pad + n;
    uint64_t v = row[w];
    if (c0 < lo) v &= lo - c0 >= 64 ? 0ull : (~0ull << (lo - c0));
    if (c0 + 64 > hi) v &= hi <= c0 ? 0ull : (~0ull >> (c0 + 64 - hi));
    return v;
}

// runs of plane row k, one wave per row, 64 consecutive words per step (one per lane): count
// them (EMIT = false) or write them from run_ptr[k] on.  A run's start is a set bit whose left
// neighbour is clear, its end a set bit whose right neighbour is clear; the i-th start and the
// i-th end of a row belong to its i-th run, so starts and ends are placed by their own ranks.
template <bool EMIT>
__global__ void k_runs(const uint64_t *mask, int64_t wd, int ndm, int64_t n, int pad, int32_t *nruns,
                       const int32_t *run_ptr, int32_t *rs, int32_t *re, int32_t *rk, int64_t max_runs)
{
    const int lane = threadIdx.x & 63;
    const int k = blockIdx.x * (kT / 64) + (threadIdx.x >> 6);
    if (k >= ndm) return;  // whole waves
    const uint64_t *row = mask + ((int64_t)k + pad) * wd;
    const int64_t w0 = pad / 64, w1 = (pad + n + 63) / 64;
    const int64_t base = EMIT ? run_ptr[k] : 0;
    int64_t ns = 0, ne = 0;       // starts and ends of the row before this step
    uint64_t prev_last = 0;       // last word of the previous step (lane 63's)
    for (int64_t wb = w0; wb < w1; wb += 64) {
        const int64_t w = wb + lane;
        const uint64_t v = w < w1 ? crop_word(row, w, pad, n) : 0ull;
        // neighbouring words: lane - 1 (or the previous step's last) and lane + 1 (or the next
        // step's first, read directly)
        uint64_t left = __shfl_up(v, 1, 64);
        if (lane == 0) left = prev_last;
        uint64_t right = __shfl_down(v, 1, 64);
        if (lane == 63) right = w + 1 < w1 ? crop_word(row, w + 1, pad, n) : 0ull;
        const uint64_t s = v & ~((v << 1) | (left >> 63));
        const uint64_t e = v & ~((v >> 1) | (right << 63));
        const int cs = __popcll(s), ce = __popcll(e);
        // inclusive scans of the per-lane counts
        int is = cs, ie = ce;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int us = __shfl_up(is, d, 64), ue = __shfl_up(ie, d, 64);
            if (lane >= d) {
                is += us;
                ie += ue;
            }
        }
        if (EMIT) {
            int64_t r = base + ns + (is - cs);
            for (uint64_t x = s; x; x &= x - 1, ++r)
                if (r < max_runs) {
                    rs[r] = (int32_t)(64 * w + __builtin_ctzll(x) - pad);
                    rk[r] = k;
                }
            r = base + ne + (ie - ce);
            for (uint64_t x = e; x; x &= x - 1, ++r)
                if (r < max_runs) re[r] = (int32_t)(64 * w + __builtin_ctzll(x) - pad);
        }
        ns += __shfl(is, 63, 64);
        ne += __shfl(ie, 63, 64);
        prev_last = __shfl(v, 63, 64);
    }
    if (!EMIT && lane == 0) nruns[k] = (int32_t)ns;
}

// exclusive prefix sum of nruns[0..ndm) into run_ptr[0..ndm], one workgroup
__global__ void k_scan_runs(const int32_t *nruns, int ndm, int32_t *run_ptr)
{
    __shared__ int64_t part[kT];
    const int tid = threadIdx.x;
    const int per = (ndm + kT - 1) / kT, b = tid * per;
    int64_t s = 0;
    for (int i = 0; i < per && b + i < ndm; ++i) s += nruns[b + i];
    part[tid] = s;
    __syncthreads();
    if (tid == 0) {
        int64_t a = 0;
        for (int i = 0; i < kT; ++i) {
            const int64_t x = part[i];
            part[i] = a;
            a += x;
        }
        run_ptr[ndm] = a > 0x7fffffffLL ? 0x7fffffff : (int32_t)a;
    }
    __syncthreads();
    int64_t a = part[tid];
    for (int i = 0; i < per && b + i < ndm; ++i) {
        run_ptr[b + i] = a > 0x7fffffffLL ? 0x7fffffff : (int32_t)a;
        a += nruns[b + i];
    }
}

__device__ inline int32_t find_root(int32_t *parent, int32_t x)
{
    int32_t p = __atomic_load_n(&parent[x], __ATOMIC_RELAXED);
    while (p != x) {
        x = p;
        p = __atomic_load_n(&parent[x], __ATOMIC_RELAXED);
    }
    return x;
}

__device__ inline void unite(int32_t *parent, int32_t a, int32_t b)
{
    while (true) {
        a = find_root(parent, a);
        b = find_root(parent, b);
        if (a == b) return;
        if (a < b) {  // link the larger root under the smaller
            const int32_t t = a;
            a = b;
            b = t;
        }
        if (atomicCAS(&parent[a], a, b) == a) return;
    }
}

// join each run with the touching runs of the next row (column ranges within one of each other)
__global__ void k_union(const int32_t *run_ptr, int ndm, const int32_t *rs, const int32_t *re, const int32_t *rk,
                        int32_t *parent)
{
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    const int64_t nr = run_ptr[ndm];
    if (i >= nr) return;
    const int k = rk[i];
    if (k + 1 >= ndm) return;
    int64_t lo = run_ptr[k + 1], hi = run_ptr[k + 2];
    const int32_t s = rs[i], e = re[i];
    // first run of the next row ending at or after s - 1
    while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if (re[mid] < s - 1) lo = mid + 1;
        else hi = mid;
    }
    const int64_t end = run_ptr[k + 2];
    for (int64_t j = lo; j < end && rs[j] <= e + 1; ++j) unite(parent, (int32_t)i, (int32_t)j);
}

__global__ void k_flatten(const int32_t *run_ptr, int ndm, int32_t *parent)
{
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= run_ptr[ndm]) return;
    parent[i] = find_root(parent, (int32_t)i);
}

__global__ void k_island_size(const int32_t *run_ptr, int ndm, const int32_t *rs, const int32_t *re,
                              const int32_t *parent, unsigned long long *npix)
{
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= run_ptr[ndm]) return;
    atomicAdd(&npix[parent[i]], (unsigned long long)(re[i] - rs[i] + 1));
}

// the run of row k holding column t (every thresholded cell lies in a closed run)
__device__ inline int64_t run_of(const int32_t *run_ptr, const int32_t *rs, int k, int32_t t)
{
    int64_t lo = run_ptr[k], hi = run_ptr[k + 1];
    while (hi - lo > 1) {  // last run starting at or before t
        const int64_t mid = (lo + hi) / 2;
        if (rs[mid] <= t) lo = mid;
        else hi = mid;
    }
    return lo;
}

// PASS 0: the highest S/N of each island; 1: its lowest (row, time) at that S/N; 2: its width
template <int PASS>
__global__ void k_peak(const Pixel *px, const unsigned int *count, int64_t max_pixels, const int32_t *run_ptr,
                       const int32_t *rs, const int32_t *parent, unsigned long long *smax, unsigned long long *pkey,
                       int32_t *pwidx)
{
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    const int64_t n = (int64_t)*count < max_pixels ? (int64_t)*count : max_pixels;
    if (i >= n) return;
    const Pixel p = px[i];
    const int64_t ri = run_of(run_ptr, rs, p.k, p.t);
    if (ri >= run_ptr[p.k + 1]) return;  // a row without runs (the closing keeps every cell, so never)
    const int32_t root = parent[ri];
    const unsigned long long bits = (unsigned long long)__double_as_longlong(p.snr);
    const unsigned long long key = ((unsigned long long)(uint32_t)p.k << 32) | (uint32_t)p.t;
    if (PASS == 0) atomicMax(&smax[root], bits);
    else if (PASS == 1) {
        if (bits == smax[root]) atomicMin(&pkey[root], key);
    } else if (bits == smax[root] && key == pkey[root]) {
        pwidx[root] = p.widx;
    }
}

__global__ void k_emit(const int32_t *run_ptr, int ndm, const int32_t *parent, const unsigned long long *npix,
                       const unsigned long long *smax, const unsigned long long *pkey, const int32_t *pwidx,
                       int64_t n_min, unsigned int *ncand, Pixel *cand, int64_t *cand_npix)
{
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= run_ptr[ndm] || parent[i] != (int32_t)i || (int64_t)npix[i] < n_min || smax[i] == 0ull) return;
    const unsigned int j = atomicAdd(ncand, 1u);
    Pixel c;
    c.k = (int32_t)(pkey[i] >> 32);
    c.t = (int32_t)(pkey[i] & 0xffffffffull);
    c.snr = __longlong_as_double((long long)smax[i]);
    c.widx = pwidx[i];
    c.pad = 0;
    cand[j] = c;
    cand_npix[j] = (int64_t)npix[i];
}

inline unsigned int nblocks(int64_t n) { return (unsigned int)((n + kT - 1) / kT); }

}  // namespace

int launch_label(const LabelArgs &a, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    const int64_t words = a.rows * a.wd;
    const int pad = 2 * a.r;
    hipLaunchKernelGGL(k_fill64, dim3(nblocks(words)), dim3(kT), 0, st, a.mask_a, words, 0ull);
    hipLaunchKernelGGL(k_mark, dim3(nblocks(a.max_pixels)), dim3(kT), 0, st, a.pixels, a.count, a.max_pixels, a.mask_a,
                       a.wd, pad);
    hipLaunchKernelGGL((k_close_t<true>), dim3(nblocks(words)), dim3(kT), 0, st, a.mask_a, a.mask_b, a.rows, a.wd, a.r);
    hipLaunchKernelGGL((k_close_k<true>), dim3(nblocks(words)), dim3(kT), 0, st, a.mask_b, a.mask_a, a.rows, a.wd, a.r);
    hipLaunchKernelGGL((k_close_t<false>), dim3(nblocks(words)), dim3(kT), 0, st, a.mask_a, a.mask_b, a.rows, a.wd, a.r);
    hipLaunchKernelGGL((k_close_k<false>), dim3(nblocks(words)), dim3(kT), 0, st, a.mask_b, a.mask_a, a.rows, a.wd, a.r);
    const unsigned int nbr = (unsigned int)((a.ndm + kT / 64 - 1) / (kT / 64));  // one wave per row
    hipLaunchKernelGGL((k_runs<false>), dim3(nbr), dim3(kT), 0, st, a.mask_a, a.wd, a.ndm, a.n, pad, a.nruns,
                       a.run_ptr, a.rs, a.re, a.rk, a.max_runs);
    hipLaunchKernelGGL(k_scan_runs, dim3(1), dim3(kT), 0, st, a.nruns, a.ndm, a.run_ptr);
    return (int)hipGetLastError();
}

int launch_label_finish(const LabelArgs &a, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    const int pad = 2 * a.r;
    const unsigned int nb = nblocks(a.max_runs);
    const unsigned int nbr = (unsigned int)((a.ndm + kT / 64 - 1) / (kT / 64));  // one wave per row
    hipLaunchKernelGGL((k_runs<true>), dim3(nbr), dim3(kT), 0, st, a.mask_a, a.wd, a.ndm, a.n, pad, a.nruns,
                       a.run_ptr, a.rs, a.re, a.rk, a.max_runs);
    hipLaunchKernelGGL(k_iota32, dim3(nb), dim3(kT), 0, st, a.parent, a.max_runs);
    hipLaunchKernelGGL(k_fill64, dim3(nb), dim3(kT), 0, st, reinterpret_cast<uint64_t *>(a.npix), a.max_runs, 0ull);
    hipLaunchKernelGGL(k_fill64, dim3(nb), dim3(kT), 0, st, reinterpret_cast<uint64_t *>(a.smax), a.max_runs, 0ull);
    hipLaunchKernelGGL(k_fill64, dim3(nb), dim3(kT), 0, st, reinterpret_cast<uint64_t *>(a.pkey), a.max_runs, ~0ull);
    hipLaunchKernelGGL(k_union, dim3(nb), dim3(kT), 0, st, a.run_ptr, a.ndm, a.rs, a.re, a.rk, a.parent);
    hipLaunchKernelGGL(k_flatten, dim3(nb), dim3(kT), 0, st, a.run_ptr, a.ndm, a.parent);
    hipLaunchKernelGGL(k_island_size, dim3(nb), dim3(kT), 0, st, a.run_ptr, a.ndm, a.rs, a.re, a.parent, a.npix);
    const unsigned int np = nblocks(a.max_pixels);
    hipLaunchKernelGGL((k_peak<0>), dim3(np), dim3(kT), 0, st, a.pixels, a.count, a.max_pixels, a.run_ptr, a.rs, a.parent,
                       a.smax, a.pkey, a.pwidx);
    hipLaunchKernelGGL((k_peak<1>), dim3(np), dim3(kT), 0, st, a.pixels, a.count, a.max_pixels, a.run_ptr, a.rs, a.parent,
                       a.smax, a.pkey, a.pwidx);
    hipLaunchKernelGGL((k_peak<2>), dim3(np), dim3(kT), 0, st, a.pixels, a.count, a.max_pixels, a.run_ptr, a.rs, a.parent,
                       a.smax, a.pkey, a.pwidx);
    hipLaunchKernelGGL(k_fill64, dim3(1), dim3(kT), 0, st, reinterpret_cast<uint64_t *>(a.ncand), 1, 0ull);
    hipLaunchKernelGGL(k_emit, dim3(nb), dim3(kT), 0, st, a.run_ptr, a.ndm, a.parent, a.npix, a.smax, a.pkey, a.pwidx,
                       a.n_min, a.ncand, a.cand, a.cand_npix);
    return (int)hipGetLastError();
}

}  // namespace snd
