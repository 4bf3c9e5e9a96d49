/*
 * snd.h -- C ABI of the MI355X Spiking Neural Dedispersion (SND) library.
 *
 * SND (arXiv 2606.15361, Methods "The Spiking Neural Dedispersion algorithm") dedisperses
 * a spike-encoded filterbank over an arbitrary trial-DM grid with a hierarchical
 * delay-and-add tree: contiguous clusters of C channels form the leaves, B-ary levels
 * combine adjacent sub-bands, and at every node the DMs that share an integer delay
 * pattern share one "neuron" (one row of partial sums).
 *
 * Conventions for every entry point:
 *   - Return value: SND_OK (0) or a negative snd_status.  Nothing throws across the ABI.
 *     snd_last_error() returns a thread-local message for the last failure.
 *   - "d_" pointers are device (HIP) memory owned by the caller; "h_" pointers are host
 *     memory owned by the caller.  The library never allocates device memory.
 *   - "stream" is a hipStream_t passed as void* (NULL = the null stream).  Device work is
 *     enqueued asynchronously on it unless a function says it synchronises.
 *   - Pitches are in elements of the array's own type.  Row-major [rows][pitch].
 *   - A plan is immutable after snd_plan_create; one plan may be executed concurrently on
 *     several streams provided each call has its own workspace.
 */
#ifndef SND_H
#define SND_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SND_MAX_LEVELS 32
#define SND_STAGE_NONE 0x80000000u

typedef enum {
    SND_OK = 0,
    SND_ERR_INVALID = -1,     /* malformed argument or descriptor */
    SND_ERR_UNSUPPORTED = -2, /* valid but not implemented combination (e.g. dtype/mode) */
    SND_ERR_NOMEM = -3,       /* host allocation failed or a caller buffer is too small */
    SND_ERR_HIP = -4,         /* a HIP runtime call failed */
    SND_ERR_CAPACITY = -5,    /* admission beyond the configured device-memory budget */
    SND_ERR_STATE = -6,       /* call out of order (e.g. execute before upload) */
    SND_ERR_GAP = -7          /* streaming: a chunk index was skipped or repeated */
} snd_status;

/* Tree activation modes (Methods, "Tree activation modes"). */
typedef enum {
    SND_MODE_BINARY = 0, /* Mode A: node emits 1 when its active-input count >= K (K_L leaf, K_I above) */
    SND_MODE_GRADED = 1, /* Mode B: node emits its integer sum clipped to [0, cap] */
    SND_MODE_FLOAT = 2   /* Mode C: FP32 accumulation at every node */
} snd_mode;

typedef enum {
    SND_DT_U8 = 1,
    SND_DT_U16 = 2,
    SND_DT_F32 = 3,
    SND_DT_BF16 = 4,
    SND_DT_F16 = 5,
    SND_DT_BITS = 6   /* binary spikes, one bit per sample: bit i of 32-bit word w holds
                         sample 32 w + i of the row; pitches of such rows are counted in bits
                         (binary mode only: input and node storage) */
} snd_dtype;

/*
 * Plan descriptor (Methods, SND: "accepts an arbitrary trial-DM grid as input and
 * constructs a dedispersion plan").
 *
 * Delays: delta_c(d) = round_half_even(K_DM * d * (f_c^-2 - f_ref^-2) / tsamp_ms) with
 * K_DM = 4.148808e6 MHz^2 ms, evaluated in FP64 as ((K_DM * d) * (1/(f_c f_c) -
 * 1/(f_ref f_ref))) / tsamp_ms (Methods, "Incoherent dedispersion").
 * Output: y_k(t) = tree value of DM k at reference time t, for t in [0, n_out) with
 * n_out = nsamp - max_{k,c} delta_c(d_k); in the linear modes y_k(t) = sum_c x_c(t + delta_c(d_k)).
 * Tree: leaves are consecutive groups of `cluster` channels, each higher level groups
 * `branching` consecutive nodes; the last group of a level may be smaller.  A node's
 * reference channel is its highest-frequency channel; node shifts are differences of
 * the global channel delays.
 */
typedef struct {
    int32_t nchan;           /* N_f >= 1 */
    const double *freq_mhz;  /* [nchan] channel centre frequencies, > 0, any order (host) */
    double tsamp_s;          /* sampling interval, > 0 */
    double fref_mhz;         /* reference frequency; <= 0 selects max(freq); must be >= max(freq) */
    int32_t ndm;             /* N_DM >= 1 */
    const double *dm;        /* [ndm] trial DMs >= 0, any order, duplicates allowed (host) */
    int32_t branching;       /* B >= 2 */
    int32_t cluster;         /* C >= 1 */
    int32_t mode;            /* snd_mode */
    int32_t k_leaf;          /* binary quorum at leaves, >= 1 (ignored otherwise) */
    int32_t k_int;           /* binary quorum at every higher node incl. the root, >= 1 */
    int32_t cap;             /* graded clip N, 1..65535 (ignored otherwise) */
    int32_t in_dtype;        /* input samples: U8 for binary/graded (binary: non-zero = spike);
                                F32, BF16 or F16 for float.  Binary also takes BITS input (rows of
                                bits, in_pitch in bits and a multiple of 32), which needs
                                node_dtype BITS and cluster <= 15; UNSUPPORTED otherwise */
    int32_t node_dtype;      /* storage of materialised tree rows: BITS or U8 for binary; U8
                                (cap <= 255) or U16 for graded; F32, BF16 or F16 for float (FP32
                                accumulate).  BITS needs the default schedule (leaf level
                                materialised, no generic kernels) and a tree whose level-1 nodes
                                all have the same fan-in of 2, 4 or 8; UNSUPPORTED otherwise */
    int32_t root_norm;       /* float: divide the output by sqrt(nchan) (Methods, Mode C) */
    int64_t nsamp;           /* input samples per channel per execute (ignored when chunk > 0) */
    uint32_t stage_levels;   /* bit l (l below the root level) set: tree level l is written to
                                device memory and read by the next stage.  0 = library default
                                (leaves only); SND_STAGE_NONE = no level written (the whole tree is
                                evaluated from the input in one stage).  The output is identical
                                for every choice. */
    int32_t generic_kernels; /* 1: run every stage on the generic stage kernel instead of the
                                LDS-staged kernels (same results; for cross-checks) */
    int32_t chunk;           /* > 0: streaming plan for chunks of up to `chunk` samples; nsamp is
                                then max_delay + chunk, so that n_out = chunk */
    uint32_t tune;           /* launch-shape choices (0 = the library's defaults; the output is
                                identical for every value, only speed and memory differ):
                                bits 0-3  leaf-stage window of reference samples per workgroup:
                                          0 auto (the largest of 2048, 1024, 512 whose staging
                                          keeps four workgroups on a CU), 1..4 = 512, 1024, 2048,
                                          4096 (UNSUPPORTED when it exceeds the LDS);
                                bits 4-7  final-stage workgroups dealt per XCD and time tile:
                                          0 auto (an eighth of the DM groups), k = 1..7: 2^(k-1);
                                bits 8-11 final-stage LDS batch budget: 0 the whole buffer,
                                          1 three quarters, 2 half, 3 a quarter.
                                Other bits must be zero. */
    int32_t reserved[5];     /* must be zero */
} snd_plan_desc;

typedef struct snd_plan_s *snd_plan;

typedef struct {
    int64_t n_out;                          /* valid output samples per DM row */
    int64_t max_delay;                      /* max_{k,c} delta_c(d_k) */
    int32_t n_levels;                       /* tree levels, leaf .. root */
    int32_t n_stages;                       /* kernel stages per execute */
    int32_t out_dtype;                      /* U8 (binary, graded cap <= 255), U16, or F32 */
    int32_t pad0;
    int64_t n_neurons;                      /* shared-pattern neurons over all levels */
    int64_t n_synapses;                     /* inputs of those neurons */
    int64_t neurons_per_level[SND_MAX_LEVELS];
    int64_t synapses_per_level[SND_MAX_LEVELS];
    int64_t nodes_per_level[SND_MAX_LEVELS];
    int64_t table_bytes;                    /* device bytes needed by snd_plan_upload */
    int64_t workspace_bytes;                /* device bytes needed by snd_execute */
    int64_t alg_bytes;                      /* algorithmic device-memory bytes of one execute:
                                               every stage reads its source rows once and writes
                                               its output rows once */
    int64_t stage_alg_bytes[SND_MAX_LEVELS];/* the same per stage (last = final stage) */
    int64_t stage_rows[SND_MAX_LEVELS];     /* output rows per stage */
    int64_t stage_entries[SND_MAX_LEVELS];  /* (row, shift) inputs summed per stage per time sample */
    double build_seconds;                   /* host time of snd_plan_create */
    int32_t stage_kernel[SND_MAX_LEVELS];   /* kernel per stage: 0 generic, 1 LDS row groups,
                                               2 input-anchored, 3 LDS row groups specialised for
                                               regular level-1 nodes, 4 the same on bit rows,
                                               5 input-anchored on bit input, 6 LDS row groups
                                               summing float-mode rows as one sum each, 7 LDS
                                               row groups forming graded levels on packed
                                               16-bit counts */
    int64_t stage_staged[SND_MAX_LEVELS];   /* LDS row groups: source elements staged per time
                                               tile summed over groups (0 otherwise) */
    int64_t stage_batches[SND_MAX_LEVELS];  /* LDS row groups: batches summed over groups */
    int64_t stage_windows[SND_MAX_LEVELS];  /* LDS row groups: staged windows summed over groups */
} snd_plan_info;

/* Build a plan on the host (no device work).  INVALID on a malformed descriptor (n_out <= 0,
 * negative DM, f_ref < max frequency, B < 2, C < 1, bad quorum or cap), UNSUPPORTED for a
 * dtype/mode pair that is not provided.  On success *out owns host tables until destroy. */
snd_status snd_plan_create(const snd_plan_desc *desc, snd_plan *out);

snd_status snd_plan_query(snd_plan plan, snd_plan_info *out);

/* Copy the integer delay table int32 [ndm][nchan] into h_delays (host). */
snd_status snd_plan_delays(snd_plan plan, int32_t *h_delays, int64_t count);

/* Copy the plan's device tables into caller memory d_tables of at least table_bytes bytes
 * (256-byte aligned) and remember that address for later executes.  Synchronises the
 * stream.  Re-uploading moves the plan to the new address. */
snd_status snd_plan_upload(snd_plan plan, void *d_tables, int64_t bytes, void *stream);

snd_status snd_plan_destroy(snd_plan plan);

/*
 * One plain-form pass (Methods, SND; pipeline stage 2): dedisperse nsamp input samples
 * d_in [nchan][in_pitch] (in_dtype) into d_out [ndm][out_pitch] (out_dtype), rows in the
 * order of desc->dm, n_out valid samples per row.  d_workspace: workspace_bytes device
 * bytes, 256-byte aligned, contents irrelevant on entry.  Asynchronous on stream.
 * STATE before snd_plan_upload; INVALID for pitches smaller than nsamp / n_out, or a BITS
 * in_pitch that is not a multiple of 32.
 */
snd_status snd_execute(snd_plan plan, const void *d_in, int64_t in_pitch, void *d_out, int64_t out_pitch,
                       void *d_workspace, int64_t workspace_bytes, void *stream);

/*
 * One stage of snd_execute (0 <= stage < n_stages), for callers that time or interleave the
 * stages: stage 0 reads d_in, every later stage reads the workspace written by the stage
 * before it, the last stage writes d_out.  Running stages 0 .. n_stages-1 in order on one
 * stream is exactly snd_execute.  Same arguments and errors as snd_execute.  Besides the node
 * rows, the workspace carries what a stage records for the next: for graded plans whose final
 * stage is the packed kernel (stage_kernel 7), stage 0 writes the largest leaf value there, and
 * the final stage picks its level-1 arithmetic from it, so a final stage must follow the
 * stage 0 that wrote its workspace (as in snd_execute).
 */
snd_status snd_execute_stage(snd_plan plan, int32_t stage, const void *d_in, int64_t in_pitch, void *d_out,
                             int64_t out_pitch, void *d_workspace, int64_t workspace_bytes, void *stream);

/*
 * Delta encoder (Methods, "Input encoding": x = 1[z > theta]).  With several thresholds the
 * output level is the number of thresholds exceeded (thresholds compared in FP32).
 * d_z: float32, channel-major [nchan][z_pitch] or, with time_major = 1, [nsamp][z_pitch]
 * (one row per sample); d_out: uint8 [nchan][out_pitch] channel-major in both cases.
 * h_thresholds: host float[nthr], 1 <= nthr <= 8.  Asynchronous on stream.
 */
snd_status snd_encode(const float *d_z, int64_t z_pitch, int32_t time_major, int32_t nchan, int64_t nsamp,
                      const float *h_thresholds, int32_t nthr, uint8_t *d_out, int64_t out_pitch, void *stream);

/*
 * Delta encoder to bits (Methods, "Input encoding": x = 1[z > theta], one threshold, compared
 * in FP32): bit i of word w of channel c is 1[z_c(32 w + i) > theta].  d_z as for snd_encode;
 * d_out: uint32 [nchan][out_pitch / 32] channel-major, out_pitch in bits, a multiple of 32 and
 * >= nsamp.  Words past the last one holding a sample are not written; bits past nsamp in that
 * word are zero.  Asynchronous on stream.  The rows are BITS input for a binary plan.
 */
snd_status snd_encode_bits(const float *d_z, int64_t z_pitch, int32_t time_major, int32_t nchan, int64_t nsamp,
                           float threshold, uint32_t *d_out, int64_t out_pitch, void *stream);

/*
 * Front end (Methods, "Input encoding"): two-pass sigma-clip normalisation of raw power.
 * snd_channel_stats writes d_stats[2c] = mu_c and d_stats[2c+1] = sigma_c (device float64
 * [nchan][2]): the mean and population standard deviation of channel c's nsamp raw samples,
 * then of the same samples clipped to [mu0 - clip*sigma0, mu0 + clip*sigma0] (values outside
 * moved to the nearer bound), all in FP64.  snd_normalize writes d_z[c][t] = (P - mu_c) /
 * sigma_c, the quotient in FP64 rounded once to float32 (the encoders then threshold z in FP32).
 * d_p [nchan][p_pitch] and d_z [nchan][z_pitch] float32, channel-major; clip > 0.
 * Asynchronous on stream.
 */
snd_status snd_channel_stats(const float *d_p, int64_t p_pitch, int32_t nchan, int64_t nsamp, double clip,
                             double *d_stats, void *stream);
snd_status snd_normalize(const float *d_p, int64_t p_pitch, int32_t nchan, int64_t nsamp, const double *d_stats,
                         float *d_z, int64_t z_pitch, void *stream);

/*
 * Zero-DM subtraction (Results, "False-positive rate": optional zero-DM subtraction; Table S1:
 * gamma_zdm = 5).  On a z-scored filterbank d_z [nchan][z_pitch] (float32, channel-major, in
 * place): for every sample t, S(t) = sum_c z_c(t) in FP64 over the channels in order; where the
 * zero-DM S/N |S(t)| / sqrt(nchan) exceeds gamma, every channel gets z_c(t) <- z_c(t) - S(t) /
 * nchan, computed in FP64 and rounded once to float32.  The paper gives the threshold only; this
 * conditional form is the reading used here.  d_count (optional device int32, added to, not
 * cleared) counts the samples changed.  gamma >= 0.  Asynchronous on stream.
 */
snd_status snd_zero_dm(float *d_z, int64_t z_pitch, int32_t nchan, int64_t nsamp, double gamma, int32_t *d_count,
                       void *stream);

/*
 * Windowed channel flagging by median absolute deviation (Results, "False-positive rate").  On
 * a z-scored filterbank d_z [nchan][z_pitch] (float32, channel-major, in place), in windows of
 * `window` samples (the last one may be shorter): s_c = the population standard deviation of
 * channel c over the window, m = the lower median of the s_c over the channels (rank
 * floor((nchan - 1) / 2)), MAD = the lower median of |s_c - m|; channel c is flagged in the
 * window when |s_c - m| > k * (MAD / Phi^-1(3/4)), and its samples there are set to 0 (the
 * normalised mean: no spikes, no float contribution).  Each of the two FP64 sums behind s_c
 * (the samples, then the squared deviations from their mean) is taken as 64 interleaved
 * partial sums, partial j adding samples j, j + 64, ... of the window in order, and the
 * partials are added in order of j.  The paper names the method without parameters; window
 * and k are the caller's.  d_sigma (device float64 [nwin][nchan], nwin = ceil(nsamp / window),
 * caller-owned) receives the s_c; d_flags (optional device uint8 [nwin][flags_pitch]) 1 for
 * flagged (window, channel) pairs, 0 otherwise.  1 <= nchan <= 8192; window >= 1; nwin <=
 * 65535; k >= 0.  Asynchronous on stream.
 */
snd_status snd_flag_channels(float *d_z, int64_t z_pitch, int32_t nchan, int64_t nsamp, int64_t window, double k,
                             double *d_sigma, uint8_t *d_flags, int64_t flags_pitch, void *stream);

/* Float32 -> BF16 or F16 cast with round-to-nearest-even (input staging for the reduced-
 * precision float mode).  d_src [rows][src_pitch] float32, d_dst [rows][dst_pitch] of
 * dst_dtype.  Asynchronous on stream. */
snd_status snd_cast(const float *d_src, int64_t src_pitch, int64_t rows, int64_t cols, void *d_dst,
                    int64_t dst_pitch, int32_t dst_dtype, void *stream);

/* ------------------------------------------------------------------------------------
 * Matched filter and candidates (Methods, "Matched filtering" and "Candidate detection").
 * Per DM row k of a plane produced by snd_execute: mu_k and sigma_k are the mean and the
 * population standard deviation of the n_out valid samples (integer planes: from the exact
 * sums S1, S2 as mu = S1/n, sigma = sqrt(n*S2 - S1*S1)/n in FP64; float planes: two-pass FP64),
 * sigma_k is raised to sigma_min when smaller; for every width W that fits,
 *     SNR(k, t, W) = (sum_{t'=t}^{t+W-1} y_k(t') - mu_k W) / (sigma_k sqrt W),
 * the S/N plane is the maximum over widths (first width on ties; 0 and width index -1 where
 * no width fits; 0 on rows with sigma = 0).  Candidates: cells with S/N >= threshold, binary
 * closing with a (2r+1)^2 square on the zero-extended plane, 8-connected islands, islands
 * with fewer than n_min closed pixels dropped, one candidate per island at its peak cell
 * (highest S/N, then lowest DM index, then earliest sample), ordered by (dm_index, t).
 * ---------------------------------------------------------------------------------- */
#define SND_MAX_WIDTHS 32
#define SND_MAX_WIDTH 1024

typedef struct {
    const int32_t *widths;  /* host [nwidths], strictly increasing, 1..SND_MAX_WIDTH */
    int32_t nwidths;        /* 1..SND_MAX_WIDTHS */
    int32_t closing_radius; /* r >= 0; 4 gives the paper's 9 x 9 closing */
    double threshold;       /* > 0, compared with the FP64 S/N */
    double sigma_min;       /* >= 0; the paper floors sigma of binary planes (0.15-0.20) */
    int32_t n_min;          /* >= 1; the paper uses 10 */
    int32_t n_base_widths;  /* 0 (or nwidths): every row uses every width.  Else a DM-scaled set
                               (Methods, "Matched filtering", W(d_k)): row k uses the first
                               n_base_widths widths and every further width w <= width_alpha *
                               tau_sweep(d_k) / tsamp, tau_sweep being the unrounded delay of
                               the lowest channel frequency at d_k (evaluated as the channel
                               delays are); the paper uses {1,2,4,8} + {16..1024}, alpha 0.1 */
    int64_t max_pixels;     /* capacity of the device list of thresholded cells, >= 1 */
    double width_alpha;     /* >= 0, used when n_base_widths > 0 */
    int32_t sigma_estimator; /* 0: sigma_k is the row's standard deviation (Methods, "Matched
                                filtering").  1: sigma_k = MAD_k / Phi^-1(3/4), MAD_k the lower
                                median of |y_k(t) - m_k| and m_k the row's lower median (rank
                                floor((n_out - 1) / 2)), the deviation taken in the plane's own
                                arithmetic (FP32 for float planes); the robust per-row MAD the
                                paper mentions for bounded (graded) planes.  mu_k stays the mean
                                and sigma_min still floors sigma_k. */
    int32_t label_on_device; /* 0: closing and labelling on the host (from the thresholded cells
                                read back).  1: on the device as well, so that snd_detect reads
                                back only the candidates; the workspace then grows by two
                                bitmasks of the padded plane and per-run tables for max_pixels
                                runs (SND_ERR_CAPACITY beyond that).  Same candidates either way.
                                snd_detect_launch / snd_detect_collect label on the host. */
} snd_detect_desc;

typedef struct {
    int32_t dm_index; /* row of the peak cell (index into the plan's DM list) */
    int32_t width;    /* boxcar width of the peak, samples */
    int64_t t;        /* first sample of the peak boxcar */
    double snr;       /* S/N of the peak cell */
    double dm;        /* trial DM of the peak row */
    int64_t npix;     /* pixels of the closed island */
} snd_candidate;

/* Device workspace bytes needed by snd_detect / snd_snr_plane for this plan and descriptor. */
snd_status snd_detect_workspace(snd_plan plan, const snd_detect_desc *desc, int64_t *bytes);

/* Full S/N plane: d_snr float [ndm][snr_pitch] and d_widx int8 [ndm][widx_pitch] (width index,
 * -1 where none fits) for the plane d_plane [ndm][plane_pitch] of the plan's output dtype.
 * d_workspace: snd_detect_workspace bytes, 256-byte aligned; its first 2*ndm doubles (after a
 * 256-byte header) hold (mu_k, sigma_k) afterwards.  Asynchronous on stream. */
snd_status snd_snr_plane(snd_plan plan, const void *d_plane, int64_t plane_pitch, const snd_detect_desc *desc,
                         float *d_snr, int64_t snr_pitch, int8_t *d_widx, int64_t widx_pitch, void *d_workspace,
                         int64_t workspace_bytes, void *stream);

/* Candidates of the plane d_plane.  Synchronises the stream.  Writes up to cap candidates to
 * h_out, the number of candidates to *h_count and the number of thresholded cells to
 * *h_npixels.  CAPACITY (and no candidates) when the thresholded cells exceed max_pixels. */
snd_status snd_detect(snd_plan plan, const void *d_plane, int64_t plane_pitch, const snd_detect_desc *desc,
                      void *d_workspace, int64_t workspace_bytes, snd_candidate *h_out, int64_t cap,
                      int64_t *h_count, int64_t *h_npixels, void *stream);

/*
 * Asynchronous form of snd_detect, for pipelines that overlap the host's candidate extraction
 * with later device work (for example the next block's tree).
 *
 * snd_detect_launch enqueues on stream the kernels of snd_detect and the read-back of the
 * thresholded-cell count and of up to SND_DETECT_STAGE_CELLS(stage_bytes) cells into h_stage,
 * a caller-owned host buffer of stage_bytes (page-locked for the copy to be asynchronous;
 * >= SND_DETECT_STAGE_HEADER bytes; its first 4 bytes receive the count), and returns.  The
 * copy size is fixed by stage_bytes and max_pixels, not by the count.
 *
 * snd_detect_collect, called once that stream work has completed (e.g. after synchronising an
 * event recorded after snd_detect_launch), turns the staged cells into candidates on the host
 * without touching the device: same outputs as snd_detect.  CAPACITY (with *h_npixels set and
 * no candidates) when the count exceeds max_pixels or the cells h_stage holds; the caller can
 * then run snd_detect on the same plane.  The device workspace may be reused as soon as the
 * launch's stream work has completed; h_stage must stay untouched until collect returns.
 */
#define SND_DETECT_STAGE_HEADER 256
#define SND_DETECT_STAGE_CELLS(stage_bytes) (((stage_bytes) - SND_DETECT_STAGE_HEADER) / 24)
snd_status snd_detect_launch(snd_plan plan, const void *d_plane, int64_t plane_pitch, const snd_detect_desc *desc,
                             void *d_workspace, int64_t workspace_bytes, void *h_stage, int64_t stage_bytes,
                             void *stream);
snd_status snd_detect_collect(snd_plan plan, const snd_detect_desc *desc, const void *h_stage, int64_t stage_bytes,
                              snd_candidate *h_out, int64_t cap, int64_t *h_count, int64_t *h_npixels);

/*
 * Batched detection: the planes of n beams (each with its own plan: DM list, n_out, DM-scaled
 * width counts, output dtype) in shared grids -- one row-statistics and one S/N launch per plane
 * dtype for all beams, one cell counter and list, one read-back -- instead of one detection
 * per beam.  Same candidates as snd_detect per beam.  The descriptor is shared; the standard-
 * deviation sigma and host labelling only (sigma_estimator 1 or label_on_device 1:
 * UNSUPPORTED).  max_pixels bounds the cells of all beams together.
 *
 * snd_detect_batch_workspace: device bytes for these plans (256-byte aligned buffer).
 * snd_detect_batch_launch: enqueue on stream the detection of d_planes[i] [ndm_i][pitches[i]]
 * (plan i's output dtype) and the read-back of the cell count and of up to
 * SND_DETECT_STAGE_CELLS(stage_bytes) cells into h_stage (page-locked for an asynchronous copy;
 * first 4 bytes: the count), then return.
 * snd_detect_batch_collect: once that work has completed, the candidates of each beam from the
 * staged cells, on the host: beam i's at h_out + i * cap_per_beam (up to cap_per_beam), their
 * number in h_counts[i] and its thresholded cells in h_npixels[i] (host arrays of n).  CAPACITY
 * (no candidates) when the cells exceed max_pixels or the staged cells: run snd_detect per beam.
 * The plans, descriptor and n must be those of the launch.
 */
snd_status snd_detect_batch_workspace(int32_t n, const snd_plan *plans, const snd_detect_desc *desc, int64_t *bytes);
snd_status snd_detect_batch_launch(int32_t n, const snd_plan *plans, const void *const *d_planes, const int64_t *pitches,
                                   const snd_detect_desc *desc, void *d_workspace, int64_t workspace_bytes,
                                   void *h_stage, int64_t stage_bytes, void *stream);
snd_status snd_detect_batch_collect(int32_t n, const snd_plan *plans, const snd_detect_desc *desc, const void *h_stage,
                                    int64_t stage_bytes, snd_candidate *h_out, int64_t cap_per_beam, int64_t *h_counts,
                                    int64_t *h_npixels);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): snd_detect_launch with no workspace argument.  Its
 * kernels use a fixed device array of SND_DETECT_NOALLOC_MAX_BYTES held by the library on each
 * GPU it runs on until the process ends (looked up once per device on the first call there,
 * on the stream's device, or the current device for the null stream).  The call itself
 * allocates nothing.  Same arguments, outputs and errors as snd_detect_launch, collected with
 * snd_detect_collect; NOMEM (nothing launched) when snd_detect_workspace exceeds the maximum,
 * which holds e.g. 4096 DM rows with max_pixels up to 1.38 million.  Every call on one GPU
 * shares that GPU's array: the cell counter is cleared by the launch itself, and calls that
 * overlap on one GPU (other streams, other threads) race; order them, e.g. on one stream, and
 * collect a launch before the next one's stream work runs. */
#define SND_DETECT_NOALLOC_MAX_BYTES ((int64_t)32 << 20)
snd_status snd_detect_launch_noalloc(snd_plan plan, const void *d_plane, int64_t plane_pitch,
                                     const snd_detect_desc *desc, void *h_stage, int64_t stage_bytes, void *stream);

/* ---------------------------------------------------------------------------------------
 * Multi-rate extension (Methods, "Multi-rate extension").  The DM range is split into bands
 * by scrunch factor; each band runs its own plan (tsamp * S, nsamp / S samples, its DMs) on a
 * time-scrunched copy of the filterbank, re-encoded for binary and graded modes, and the
 * bands' candidates are merged in (DM, time).
 * --------------------------------------------------------------------------------------- */

/* Scrunch factor of each trial DM (Eq. scrunch): the largest power of two S <= s_max with
 * S * tsamp <= tau_smear(d) = K_DM * d * df / fc^3, 1 when S = 2 already fails; fc = mean of the
 * highest and lowest channel frequencies, df = channel spacing (highest - lowest) / (nchan - 1)
 * (0 for one channel), all in FP64.  h_factor: host int32[ndm].  s_max: 1..1024. */
snd_status snd_scrunch_factors(int32_t nchan, const double *freq_mhz, double tsamp_s, int32_t ndm, const double *dm,
                               int32_t s_max, int32_t *h_factor);

/* Time scrunch of a z-scored filterbank: d_out[c][t] = (sum_{j<s} d_z[c][s t + j]) * r for
 * t < nsamp / s, the sum taken in order in FP32 and r the FP32 value of 1 / sqrt(s) (unit
 * variance is kept, so encoder thresholds keep their meaning).  d_z [nchan][z_pitch] and d_out
 * [nchan][out_pitch] float32 device arrays; 1 <= s <= 1024; nothing is done (OK) when
 * nsamp < s.  Asynchronous on stream. */
snd_status snd_scrunch(const float *d_z, int64_t z_pitch, int32_t nchan, int64_t nsamp, int32_t s, float *d_out,
                       int64_t out_pitch, void *stream);

/* One candidate of one band, for the cross-band merge. */
typedef struct {
    double dm;        /* trial DM */
    double t_ms;      /* arrival time at the top of the band, ms from the block start */
    double snr;       /* S/N of the peak cell */
    int32_t band;     /* band index (caller's) */
    int32_t dm_index; /* row in the caller's full DM list */
    int32_t width;    /* boxcar width, band samples */
    int32_t reserved; /* ignored */
    int64_t t;        /* first sample of the peak boxcar, band samples */
    int64_t npix;     /* pixels of the band island */
} snd_band_candidate;

/* Cross-band merge (host): in decreasing S/N (ties: lower DM, then earlier time) a candidate
 * within |dDM| <= dm_tol and |dt| <= t_tol_ms of an already kept candidate is absorbed,
 * otherwise kept (the paper: 20 pc cm^-3, 200 ms; full ties keep input order).  Writes the kept
 * ones, ordered by (t_ms, dm), to h_out (room for n) and their number to *h_count. */
snd_status snd_merge_candidates(int64_t n, const snd_band_candidate *h_in, double dm_tol, double t_tol_ms,
                                snd_band_candidate *h_out, int64_t *h_count);

/* ---------------------------------------------------------------------------------------
 * FDMT baseline (Methods, "Classical dedispersion algorithms"), with the paper's no-smear
 * initialisation: a comparison point for the SND tree on the same GPU.  FDMT merges adjacent
 * sub-bands log2(nchan) times and outputs one row per integer band sweep delta = 0 .. D, D the
 * sweep at dm_max rounded up; row delta stands for DM = delta * dm_per_delay.
 *
 * Channels are intervals of width chan_bw_mhz around freq_mhz[c] (host, strictly descending,
 * lower edges > 0); nchan a power of two.  At each merge of a sub-band S into its upper half U
 * and lower half L, S's delay delta splits as delta_U = round_half_even(delta * (f_mid^-2 -
 * f_hi^-2) / (f_lo^-2 - f_hi^-2)) and delta_L = delta - delta_U (each clamped to the delays its
 * half holds: ceil(D r / r_band) + 1 for a sweep span r = f_lo^-2 - f_hi^-2), and P_S[delta](t)
 * = P_U[delta_U](t) + P_L[delta_L](t + delta_U), zero past nsamp; the time reference is each
 * sub-band's upper edge.  No-smear initialisation: every initial delay row of a channel is the
 * channel itself.  Sums in FP32.  Output row delta is valid for t < nsamp - D.
 * --------------------------------------------------------------------------------------- */
typedef struct snd_fdmt_s *snd_fdmt;

/* Host tables for one shape.  SND_ERR_INVALID on bad arguments, or when the sweep at dm_max
 * does not fit nsamp. */
snd_status snd_fdmt_create(int32_t nchan, const double *freq_mhz, double chan_bw_mhz, double tsamp_s, double dm_max,
                           int64_t nsamp, snd_fdmt *out);
/* Output rows (D + 1), valid samples per row, device bytes of the tables and of the workspace
 * (two buffers of the largest intermediate level), and the DM step per delay row.  Any output
 * pointer may be NULL. */
snd_status snd_fdmt_query(snd_fdmt p, int64_t *n_delays, int64_t *n_out, int64_t *table_bytes,
                          int64_t *workspace_bytes, double *dm_per_delay);
/* Copy the tables to caller-owned device memory (synchronises the stream); it must stay valid
 * while the handle executes. */
snd_status snd_fdmt_upload(snd_fdmt p, void *d_tables, int64_t bytes, void *stream);
/* d_in float32 [nchan][in_pitch], d_out float32 [n_delays][out_pitch], pitches >= nsamp,
 * d_ws >= workspace_bytes.  Asynchronous on stream; SND_ERR_STATE before upload. */
snd_status snd_fdmt_execute(snd_fdmt p, const float *d_in, int64_t in_pitch, float *d_out, int64_t out_pitch,
                            void *d_ws, int64_t ws_bytes, void *stream);
snd_status snd_fdmt_destroy(snd_fdmt p);

/* ---------------------------------------------------------------------------------------
 * Approximate (coarse-DM) sub-band dedispersion, a comparison baseline on the same GPU
 * (Methods, "Classical dedispersion algorithms": the hierarchical methods SND is set against).
 * The band is cut into sub-bands of adjacent channels.  Step one is an SND plan per sub-band
 * over a coarse DM grid (every channel at its delay relative to the band's top frequency):
 *     R_s[j](t) = sum_{c in s} x_c(t + delta_c(D_j)).
 * Step two, this call: every fine DM d_k takes the coarse row j = coarse_row[k] of each sub-band
 * and shifts it by the extra sweep of the sub-band's top channel c_s between D_j and d_k:
 *     y_k(t) = sum_s R_s[j](t + offsets[k][s]),   offsets[k][s] = delta_{c_s}(d_k) - delta_{c_s}(D_j),
 * exact when D_j = d_k, otherwise with each sub-band's internal sweep taken at D_j.
 * d_planes: host array of nsub device pointers, plane s float32 [ncoarse][pitches[s]] with
 * n_valid[s] valid samples per row; coarse_row [ndm] (0..ncoarse-1) and offsets [ndm][nsub]
 * (>= 0) host arrays, uploaded by the call into d_workspace (>= snd_subband_workspace_bytes,
 * 256-byte aligned); d_out float32 [ndm][out_pitch], n_out samples per row, each summed in FP32
 * in sub-band order.  INVALID when a read would pass a plane's valid samples.  Asynchronous on
 * stream.
 * --------------------------------------------------------------------------------------- */
snd_status snd_subband_workspace_bytes(int32_t ndm, int32_t nsub, int64_t *bytes);
snd_status snd_subband_combine(int32_t ndm, int32_t nsub, const float *const *d_planes, const int64_t *pitches,
                               const int64_t *n_valid, int32_t ncoarse, const int32_t *coarse_row,
                               const int32_t *offsets, float *d_out, int64_t out_pitch, int64_t n_out,
                               void *d_workspace, int64_t workspace_bytes, void *stream);

/* ---------------------------------------------------------------------------------------
 * Validation against injected pulses (Methods, "Validation methodology").  Host only.
 * --------------------------------------------------------------------------------------- */

/* Effective width of injected pulses at their DMs, in ms: the intrinsic width, the
 * dispersive smearing inside one channel and the sampling time added in quadrature,
 * sqrt(w^2 + tau^2 + dt^2), with tau = K_DM d df / fc^3 as in Eq. scrunch (fc the band
 * centre, the mean of the highest and lowest channel frequency; df the channel spacing).
 * The paper names this width without a formula; this is the reading used here.
 * freq_mhz [nchan] host, > 0; dm [n] >= 0 and w_int_ms [n] >= 0 host; h_weff_ms [n] host
 * output.  SND_ERR_INVALID on bad arguments (nothing written). */
snd_status snd_effective_width(int32_t nchan, const double *freq_mhz, double tsamp_s, int64_t n, const double *dm,
                               const double *w_int_ms, double *h_weff_ms);

/* Greedy one-to-one matching of candidates to injections.  Candidates are taken in
 * decreasing S/N (equal S/N: input order).  Each takes the unmatched injection j with
 * |dm - inj_dm[j]| <= dm_tol and |t_ms - inj_t_ms[j]| <= t_frac * inj_weff_ms[j] that is
 * nearest in time (ties: nearer in DM, then the lower index), or none.  The paper uses
 * dm_tol = 10 pc cm^-3 and t_frac = 0.5.  Candidate arrays [n_cand] and injection arrays
 * [n_inj] are host, finite; a candidate's time is the one the caller compares with the
 * injection's (e.g. the centre of its peak boxcar at the top of the band).  Writes h_match
 * [n_inj] (host): the matched candidate's index, or -1; and *h_nmatched, the number of
 * matched injections (completeness = *h_nmatched / n_inj).  SND_ERR_INVALID on bad
 * arguments, with h_match unspecified. */
snd_status snd_match_injections(int64_t n_cand, const double *cand_dm, const double *cand_t_ms, const double *cand_snr,
                                int64_t n_inj, const double *inj_dm, const double *inj_t_ms, const double *inj_weff_ms,
                                double dm_tol, double t_frac, int32_t *h_match, int64_t *h_nmatched);

/* ---------------------------------------------------------------------------------------
 * Batched execution.
 *
 * Several beams, each with its own uploaded plan (DM grids, lengths, modes and storage types
 * may all differ), run with one grid per (stage, kernel class) instead of one launch per beam
 * and stage.  A kernel class is a kernel kind, mode, storage pair and compile-time tree shape.
 * Each grid reads per-beam argument records and a workgroup prefix table from d_records
 * (caller-owned device memory, 256-byte aligned, snd_batch_records_bytes bytes, written by
 * one host-to-device copy per grid on `stream`).  Results equal one snd_execute per beam.
 * --------------------------------------------------------------------------------------- */

/* Record bytes for a batch of these plans, and the number of grids it launches. */
snd_status snd_batch_records_bytes(int32_t nbeams, const snd_plan *plans, int64_t *bytes, int32_t *n_launches);

/* Execute beam i of the batch on d_in[i] [nchan][in_pitch[i]] into d_out[i] [ndm][out_pitch[i]]
 * with its own workspace d_workspace[i] (workspace_bytes[i] >= the plan's, 256-byte aligned,
 * distinct per beam).  n_run: NULL for every plan's full n_out, else per beam 0..n_out output
 * samples (a shorter run reads max_delay + n_run[i] input samples), which lets a caller cut a
 * long beam into time chunks.  Asynchronous on stream; *h_launches (nullable) receives the
 * number of grids launched.  INVALID / STATE / NOMEM as for snd_execute, per beam. */
snd_status snd_batch_execute(int32_t nbeams, const snd_plan *plans, const void *const *d_in, const int64_t *in_pitch,
                             void *const *d_out, const int64_t *out_pitch, void *const *d_workspace,
                             const int64_t *workspace_bytes, const int64_t *n_run, void *d_records,
                             int64_t records_bytes, void *stream, int32_t *h_launches);

/* ---------------------------------------------------------------------------------------
 * Schedule autotuner.
 *
 * A candidate is a stage schedule (which tree levels are written to device memory, see
 * snd_plan_desc.stage_levels), a time chunk (0 = the whole block in one run, else runs of
 * `chunk` output samples, which bounds the workspace) and launch shapes (snd_plan_desc.tune).  Every candidate computes the same
 * output; they differ in speed and memory.  For each candidate the library builds its plan,
 * uploads the tables to d_tables and times `reps` passes over the block d_in -> d_out with HIP
 * events on `stream` (after one untimed pass).  A candidate whose tables or workspace exceed
 * table_bytes / workspace_bytes, or whose launch shapes the plan cannot take (UNSUPPORTED), is
 * skipped (ms = -1).  *h_best receives the index of the
 * fastest.  Synchronises the stream.  NOMEM when no candidate fits.
 * --------------------------------------------------------------------------------------- */
typedef struct {
    uint32_t stage_levels;     /* in: schedule (as in snd_plan_desc) */
    int32_t chunk;             /* in: output samples per run, 0 = whole block */
    uint32_t tune;             /* in: launch shapes (as snd_plan_desc.tune) */
    int32_t pad;               /* ignored */
    double ms;                 /* out: mean milliseconds per pass, -1 when skipped */
    int64_t workspace_bytes;   /* out: the candidate's workspace */
    int64_t table_bytes;       /* out: the candidate's tables */
} snd_tune_candidate;

snd_status snd_autotune(const snd_plan_desc *desc, snd_tune_candidate *cands, int32_t ncand, const void *d_in,
                        int64_t in_pitch, void *d_out, int64_t out_pitch, void *d_workspace, int64_t workspace_bytes,
                        void *d_tables, int64_t table_bytes, int32_t reps, int32_t *h_best, void *stream);

/* ---------------------------------------------------------------------------------------
 * Streaming (chunked input with device-resident history).
 *
 * The paper processes a continuous observation chunk by chunk, consecutive chunks overlapping
 * by the largest delay (Methods, "Pipeline overview"), and its neuromorphic mapping keeps a
 * history ring per neuron (Methods, "Hardware mapping and power modelling", Eq. hist_mem).
 * Here each admitted beam keeps, in a caller-owned device
 * buffer, a ring of the last max_delay + n_out input samples of every channel, where n_out of
 * the beam's plan is the longest chunk the beam accepts.  After S input samples have arrived
 * in total, output samples t < S - max_delay exist; a push appends one chunk to the ring and
 * computes exactly the output samples that became complete, each equal (bit for bit) to the
 * plain snd_execute over the concatenated input.  Only the input is kept, not the neuron
 * rows: the first stage recomputes the short spread of each leaf row from the ring.
 *
 * The plan's first stage must be the input-anchored kernel (the default schedule; plans
 * built with generic_kernels = 1 or without a materialised level are rejected with
 * UNSUPPORTED), and its tables must be uploaded before the beam's first push (STATE).
 * --------------------------------------------------------------------------------------- */
typedef struct snd_stream_s *snd_stream;

/* Device bytes of one beam's history for this plan (ring of nchan x (max_delay + n_out)
 * input samples, rows padded to 256 bytes).  BITS input keeps one bit per sample, the ring
 * length rounded up to a whole number of 32-bit words. */
snd_status snd_stream_history_bytes(snd_plan plan, int64_t *bytes);

/* Device bytes a beam of this plan is charged against the stream's budget: its history ring
 * (snd_stream_history_bytes) plus its share of a batched push's workspace (the plan's
 * workspace_bytes rounded up to 256), so that the beams a budget admits can also be pushed
 * together. */
snd_status snd_stream_admission_bytes(snd_plan plan, int64_t *bytes);

/* New stream that admits beams while the sum of their admission bytes
 * (snd_stream_admission_bytes) stays within hbm_budget_bytes (> 0).  Host object only. */
snd_status snd_stream_create(int64_t hbm_budget_bytes, snd_stream *out);
snd_status snd_stream_destroy(snd_stream s);

/* Admit beam_id (>= 0, not yet admitted) with plan and its history buffer d_history
 * (>= snd_stream_history_bytes bytes, 256-byte aligned, owned by the caller, kept until
 * evict).  CAPACITY (beam not admitted) when the budget would be exceeded by the beam's
 * snd_stream_admission_bytes.  Admission touches no device memory.  The beam starts
 * empty; its first push may carry any chunk index.  The plan must outlive the beam. */
snd_status snd_stream_admit(snd_stream s, int32_t beam_id, snd_plan plan, void *d_history, int64_t bytes);

/* Remove a beam and release its share of the budget (its buffer returns to the caller). */
snd_status snd_stream_evict(snd_stream s, int32_t beam_id);

/* One chunk of one beam in a push.  Inputs: beam_id, chunk_idx (must follow the beam's
 * previous chunk index by one), chunk_len (1 .. n_out of the beam's plan), d_chunk
 * [nchan][chunk_pitch] in the plan's input dtype (BITS: chunk_len and chunk_pitch counted in
 * bits, the pitch a multiple of 32 and d_chunk 4-byte aligned; bit i of word w of a row is
 * sample 32 w + i of the chunk, as snd_encode_bits writes), d_out [ndm][out_pitch] in the plan's output
 * dtype with out_pitch >= n_out.  Outputs: out_t0 = output time of column 0 of d_out,
 * out_n = output samples written (0 while the first max_delay samples fill the history),
 * status = SND_OK or SND_ERR_GAP. */
typedef struct {
    int32_t beam_id;
    int32_t status;
    int64_t chunk_idx;
    int64_t chunk_len;
    const void *d_chunk;
    int64_t chunk_pitch;
    void *d_out;
    int64_t out_pitch;
    int64_t out_t0;
    int64_t out_n;
} snd_stream_item;

/* Append one chunk to each of n beams (distinct beam ids) and compute their new output
 * samples, asynchronously on stream, beams in the given order.  d_workspace: at least the
 * largest workspace_bytes of the beams' plans, 256-byte aligned, reused beam after beam.
 * All items are validated before any work (INVALID, STATE for an unknown beam).  A chunk
 * index that does not follow the beam's previous one resets that beam's history, the chunk
 * starts a new history, the item's status is SND_ERR_GAP and so is the return value (the
 * other items are processed normally).  Calls on one stream object must not overlap. */
snd_status snd_stream_push(snd_stream s, int32_t n, snd_stream_item *items, void *d_workspace,
                           int64_t workspace_bytes, void *stream);

/* The same push with the beams' stage launches batched: one grid per (stage, kernel class)
 * across all items (see snd_batch_execute).  d_workspace holds one share per item, in item
 * order, each the item plan's workspace_bytes rounded up to 256; d_records is a 256-byte
 * aligned device buffer.  snd_stream_batch_bytes gives both sizes for a set of beams.  The
 * outputs equal those of snd_stream_push. */
snd_status snd_stream_push_batched(snd_stream s, int32_t n, snd_stream_item *items, void *d_workspace,
                                   int64_t workspace_bytes, void *d_records, int64_t records_bytes, void *stream);
snd_status snd_stream_batch_bytes(snd_stream s, int32_t n, const int32_t *beam_ids, int64_t *workspace_bytes,
                                  int64_t *records_bytes);

/* State of one beam: input samples received, the next expected chunk index (-1 = any),
 * output samples emitted. */
snd_status snd_stream_beam_state(snd_stream s, int32_t beam_id, int64_t *received, int64_t *next_chunk,
                                 int64_t *emitted);

/* Budget, bytes in use and number of admitted beams. */
snd_status snd_stream_usage(snd_stream s, int64_t *budget, int64_t *used, int32_t *n_beams);

/* Checkpoint of one beam: a 64-byte header (state and ring shape) followed by the ring.
 * snd_stream_export_bytes gives the size; export copies to host memory and synchronises the
 * stream; import restores into an admitted beam whose plan has the same ring shape and
 * synchronises the stream.  Import rejects (INVALID, nothing restored) a header of another
 * ring shape, a truncated buffer, and a state the beam cannot be in: either nothing received
 * (emitted 0, next chunk -1), or S >= 1 samples received with emitted = max(0, S - max_delay)
 * and next chunk >= 1. */
snd_status snd_stream_export_bytes(snd_stream s, int32_t beam_id, int64_t *bytes);
snd_status snd_stream_export(snd_stream s, int32_t beam_id, void *h_buf, int64_t bytes, void *stream);
snd_status snd_stream_import(snd_stream s, int32_t beam_id, const void *h_buf, int64_t bytes, void *stream);

/* Thread-local message describing the last failure in this thread ("" if none). */
const char *snd_last_error(void);

/* Library version string. */
const char *snd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SND_H */
