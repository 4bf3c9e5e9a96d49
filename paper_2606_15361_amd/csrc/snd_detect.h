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
};

int launch_detect(int plane_dtype, const void *plane, int64_t pitch, int ndm, int64_t n, double sigma_min,
                  int sigma_mad, double *stats, const SnrArgs &a, void *stream);

}  // namespace snd
