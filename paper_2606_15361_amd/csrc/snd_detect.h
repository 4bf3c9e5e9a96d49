// Internal declarations of the matched-filter / candidate stage.
#pragma once

#include <cstdint>

#include "snd.h"

namespace snd {

constexpr int kMaxWidths = 32;
constexpr int kMaxWidth = 1024;

// One thresholded S/N cell.
struct Pixel {
    int32_t k;
    int32_t t;
    double snr;
    int32_t widx;
    int32_t pad;
};

template <typename T> struct PrefixType { using type = int32_t; };
template <> struct PrefixType<float> { using type = double; };

// One plane of a batched detection: its rows are rows row_base .. row_base + ndm - 1 of the
// batch (statistics, cells and width counts are indexed by batch row).
struct DetBeam {
    const void *plane;
    int64_t pitch;
    int64_t n;              // valid samples per row
    const int32_t *row_nw;  // per-row width counts of this plane (null: every width)
    int32_t row_base;
    int32_t ndm;
};

struct SnrArgs {
    int32_t w[kMaxWidths];
    double sqrtw[kMaxWidths];
    int32_t nw;
    const int32_t *row_nw;  // per-row number of leading widths used (null: nw for every row)
    double threshold;
    // plane output (when snr != nullptr)
    float *snr;
    int64_t snr_pitch;
    int8_t *widx;
    int64_t widx_pitch;
    // compaction output (when snr == nullptr)
    unsigned int *counter;
    Pixel *pixels;
    int64_t max_pixels;
    // batched detection (beams != null): the launch covers batch rows row0 .. row0 + gridDim.y - 1
    // of the nbeams planes in `beams` (device table); plane, pitch and n of the launch are unused
    const DetBeam *beams;
    int32_t nbeams;
    int32_t row0;
};

int launch_detect(int plane_dtype, const void *plane, int64_t pitch, int ndm, int64_t n, double sigma_min,
                  int sigma_mad, double *stats, const SnrArgs &a, void *stream);
// Batched: rows a.row0 .. a.row0 + nrows - 1 of the planes in a.beams (all of plane_dtype), whose
// longest row has n_max samples.  The standard-deviation sigma only.
int launch_detect_batch(int plane_dtype, int nrows, int64_t n_max, double sigma_min, double *stats, const SnrArgs &a,
                        void *stream);
int launch_zero_counter(unsigned int *counter, void *stream);

// Closing and labelling on the device (label.hip).  launch_label builds the closed mask and
// counts its runs (run_ptr[ndm] = total); the caller checks the total against max_runs before
// launch_label_finish emits one candidate per island of at least n_min cells.
struct LabelArgs {
    const Pixel *pixels;          // thresholded cells and their count (from the S/N kernel)
    const unsigned int *count;
    int64_t max_pixels;
    int ndm;
    int64_t n;                    // valid samples per row
    int r;                        // closing radius
    int64_t rows, wd;             // mask: ndm + 4r rows of wd 64-bit words (n + 4r columns)
    uint64_t *mask_a, *mask_b;
    int32_t *nruns, *run_ptr;     // [ndm], [ndm + 1]
    int32_t *rs, *re, *rk, *parent;            // per run: first and last column, row, union-find
    unsigned long long *npix, *smax, *pkey;    // per run (roots): size, peak S/N bits, peak (row, t)
    int32_t *pwidx;
    int64_t max_runs, n_min;
    unsigned int *ncand;          // 8 bytes
    Pixel *cand;                  // [max_runs]
    int64_t *cand_npix;           // [max_runs]
};
int launch_label(const LabelArgs &a, void *stream);
int launch_label_finish(const LabelArgs &a, void *stream);

}  // namespace snd
