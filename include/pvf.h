/*
 * pvf.h -- C ABI of the MI355X (gfx950) PVFinder inference library.
 *
 * The library runs the hybrid PVFinder hot path of arXiv:2602.19959 on one
 * GPU: per-track FC network and histogram (Section 2, FC stage), the UNet CNN
 * over the histogram (Section 2, CNN stage), and heuristic peak finding
 * (Section 2), taking per-event structure-of-arrays track features in and
 * giving vertex z positions and probabilities out.
 *
 * Execution contract (Section 3, "Allen Integration and Translation Layer"):
 *  - a frozen tensor specification at initialisation (batch capacity,
 *    channel count, sequence length, data type), validated once;
 *  - one caller-owned device arena bound at initialisation and reused by
 *    every call; nothing is allocated on the device after pvf_init;
 *  - every kernel runs on the one stream given at initialisation; the
 *    library never uses the null stream and never synchronises in
 *    pvf_execute;
 *  - non-owning views: the caller owns every device buffer it passes;
 *  - a status code per call and a status word per event, so an event that
 *    fails validation is bypassed (no vertices) without disturbing the rest
 *    of the batch.
 *
 * No function throws; every function is callable from C.  No HIP, PyTorch or
 * C++ type appears in a signature: streams are passed as `void *` holding a
 * hipStream_t, device buffers as plain pointers.
 */
#ifndef PVF_H
#define PVF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PVF_ABI_VERSION 1u
#define PVF_N_FEATURES 9

/* Call-level status (Section 3: the Status enum).  Whatever the host can
 * check before enqueueing work yields one of these, and then nothing is
 * enqueued. */
typedef enum {
    PVF_OK = 0,
    PVF_ERR_INVALID_ARGUMENT = 1,  /* null pointer, negative count, bad enum   */
    PVF_ERR_SHAPE = 2,             /* spec geometry the kernels cannot run    */
    PVF_ERR_CAPACITY = 3,          /* batch larger than the frozen spec       */
    PVF_ERR_ARENA_TOO_SMALL = 4,   /* arena smaller than pvf_arena_bytes      */
    PVF_ERR_WEIGHTS = 5,           /* blob malformed or shape != spec          */
    PVF_ERR_UNSUPPORTED_DTYPE = 6, /* compute dtype not built                 */
    PVF_ERR_DEVICE = 7,            /* a HIP runtime call failed               */
    PVF_ERR_ALIGNMENT = 8,         /* a buffer is not aligned as documented   */
    PVF_ERR_SCRATCH_TOO_SMALL = 9  /* batch does not fit PVF_SCRATCH_BYTES     */
} pvf_status;

/* Per-event status bits written to pvf_vertices.d_event_status.  Bypass
 * bits (TOO_MANY_TRACKS, BAD_INPUT) give that event 0 vertices; the other
 * events' results are unchanged by a bypassed event. */
enum {
    PVF_EV_OK = 0,
    PVF_EV_TOO_MANY_TRACKS = 1,  /* bypass: more tracks than max_tracks_per_event */
    PVF_EV_BAD_INPUT = 2,        /* bypass: offsets decreasing or out of range    */
    PVF_EV_PEAKS_TRUNCATED = 4,  /* more vertices than max_peaks_per_event        */
    PVF_EV_TRACKS_DROPPED = 8    /* some tracks outside the z window or with a
                                    non-finite feature were left out          */
};

/* Arithmetic type of the UNet convolutions (FP32 accumulation throughout).
 * FP32 is the deployed precision of the paper (Section 2, Fig. 1); BF16 and
 * FP16 follow its mixed-precision roadmap (Section 5); FP8 (OCP e4m3) needs
 * calibration scales (pvf_init_fp8). */
typedef enum { PVF_FP32 = 0, PVF_BF16 = 1, PVF_FP16 = 2, PVF_FP8_E4M3 = 3 } pvf_dtype;

/* The frozen tensor specification ("TensorSpec", Section 3).  Fill it with
 * pvf_spec_default and change what differs. */
typedef struct pvf_spec {
    uint32_t abi_version;          /* PVF_ABI_VERSION                           */
    int32_t  max_events;           /* batch capacity (events per call)          */
    int32_t  max_tracks_per_event; /* larger events are bypassed                */
    int32_t  max_peaks_per_event;  /* vertex slots per event (<= n_bins / 2)    */
    int64_t  max_tracks_total;     /* tracks per call, <= INT32_MAX             */
    int32_t  compute_dtype;        /* pvf_dtype                                 */
    int32_t  n_levels;             /* UNet levels (4)                           */
    int32_t  base_channels;        /* channels of level 0: 32, or 64 (the paper's
                                      deployed width); level l has
                                      base_channels << l                        */
    int32_t  n_bins;               /* histogram bins per event (4000)           */
    int32_t  bins_per_interval;    /* bins per spatial interval (100)           */
    int32_t  half_window;          /* peak integration half-width in bins (5)   */
    double   z_min_mm;             /* lower edge of the histogram (-100 mm)     */
    double   bin_width_mm;         /* bin width (0.1 mm)                        */
    double   peak_min;             /* a vertex needs p > peak_min (0.01)        */
    double   integral_min;         /* and a window sum > integral_min (0.2)     */
    double   boundary_mm;          /* Section 3 variant: a track closer than this
                                      to an edge shared with another interval also
                                      feeds that interval, in its frame (0 = one
                                      interval per track); at most half an interval */
    int32_t  unet_layout;          /* pvf_layout: one UNet sequence per event (0),
                                      or per interval (1, the [intervals, C, bins]
                                      batching of Section 3)                    */
    int32_t  reserved;             /* 0                                         */
} pvf_spec;

/* UNet input layout (Section 3 reads the FC output as [B, C, L] with B the
 * spatial intervals).  PVF_LAYOUT_EVENT runs the UNet over all n_bins of an
 * event; PVF_LAYOUT_INTERVAL runs it on each interval's bins_per_interval
 * bins alone (zero padding at interval edges), which needs bins_per_interval
 * divisible by 2^(n_levels-1), e.g. 3 levels for 100 bins. */
typedef enum pvf_layout { PVF_LAYOUT_EVENT = 0, PVF_LAYOUT_INTERVAL = 1 } pvf_layout;

/* Input view: one batch of events in structure-of-arrays form (Section 3:
 * the trigger's SoA buffers, reinterpreted without copies).
 * d_event_offsets: device int32 [n_events + 1]; event e owns tracks
 *   offsets[e] .. offsets[e+1]-1; offsets[0] is expected to be 0.
 * d_feat[k]: device float32 plane k of n_tracks_total values, feature order
 *   z, x, y, c1, c2, c3, s1, s2, s3 (mm for positions).  4-byte aligned.
 * Counts are host values. */
typedef struct pvf_tracks {
    int32_t        n_events;
    int64_t        n_tracks_total;
    const int32_t *d_event_offsets;
    const float   *d_feat[PVF_N_FEATURES];
} pvf_tracks;

/* Output view (Section 3, Extract phase: results left on the device for
 * downstream consumers).  Every array is device memory owned by the caller,
 * laid out per event with stride max_peaks_per_event for the vertex arrays:
 *   d_n_vertices    int32  [n_events]
 *   d_z             double [n_events][max_peaks]   vertex z (mm), ascending
 *   d_peak_prob     float  [n_events][max_peaks]   p at the vertex bin
 *   d_integral      double [n_events][max_peaks]   sum of p over the window
 *   d_event_status  int32  [n_events]               PVF_EV_* bits
 *   d_prob_hist     float  [n_events][n_bins] or NULL: per-bin probability
 *   d_bin           int32  [n_events][max_peaks] or NULL: bin of each vertex
 * Slots past d_n_vertices[e] are left unwritten. */
typedef struct pvf_vertices {
    int32_t *d_n_vertices;
    double  *d_z;
    float   *d_peak_prob;
    double  *d_integral;
    int32_t *d_event_status;
    float   *d_prob_hist;
    int32_t *d_bin;
} pvf_vertices;

typedef struct pvf_engine pvf_engine;

/* Defaults: the 4000-bin, 4-level, 32..256-channel network in FP32, 1000
 * events per call, 1500 tracks per event, 2000 vertex slots per event,
 * 0.1 mm bins from -100 mm, thresholds 0.01 and 0.2 over +-5 bins. */
void pvf_spec_default(pvf_spec *spec);

/* Bytes of device arena the engine needs for `spec` (weights, activations
 * and per-event scratch).  Host-only; touches no device. */
pvf_status pvf_arena_bytes(const pvf_spec *spec, size_t *out_bytes);

/* Create an engine (Section 3: init takes the stream and the workspace).
 * weights_blob: host bytes in the "PVFW" layout (network shape, fixed
 *   constants, then every tensor in forward order); copied, not kept.
 * d_arena: device memory of at least pvf_arena_bytes, 256-byte aligned,
 *   owned by the caller, used exclusively by this engine until
 *   pvf_destroy.
 * stream: a hipStream_t cast to void*; NULL is rejected (no null stream).
 * The only call that synchronises (once, on `stream`, after uploading the
 * packed weights and clearing the arena).  On error *out is NULL. */
pvf_status pvf_init(const pvf_spec *spec, const void *weights_blob, size_t blob_bytes,
                    void *d_arena, size_t arena_bytes, void *stream, pvf_engine **out);

/* FP8 engine (spec.compute_dtype = PVF_FP8_E4M3).  amax: host floats, the
 * calibration table that pvf_calibrate measured on a higher-precision engine
 * of the same network, n_amax of them.  Each stored FP8 tensor then holds
 * x / a_c with a_c = amax_c / 448; each convolution and each layer of the
 * track network folds its input scales into its weights and quantises every
 * output column with its own scale (per-output-channel).  pvf_init with an
 * FP8 spec returns PVF_ERR_INVALID_ARGUMENT (the scales are needed). */
pvf_status pvf_init_fp8(const pvf_spec *spec, const void *weights_blob, size_t blob_bytes, const float *amax,
                        size_t n_amax, void *d_arena, size_t arena_bytes, void *stream, pvf_engine **out);

/* Calibration for FP8 (set-up call, synchronises nothing but clears d_amax
 * on the stream): runs the batch like pvf_execute on an FP32/BF16/FP16
 * engine and writes into d_amax (device floats) per-channel absolute maxima:
 * first of every stored UNet activation, in launch order, then of every
 * track-network layer input (9 features, then 20 channels per hidden
 * layer).  n must equal pvf_calibration_size(eng).  Not for graph capture. */
int64_t pvf_calibration_size(const pvf_engine *eng);
pvf_status pvf_calibrate(pvf_engine *eng, const pvf_tracks *tracks, const pvf_vertices *out, float *d_amax,
                         int64_t n);

/* Enqueue the whole path for one batch on the engine's stream and return
 * at once (Section 3, Execute phase).  No allocation, no synchronisation.
 * n_events == 0 enqueues nothing.  Results are visible once the stream
 * reaches the enqueued work.  Host-detectable errors return before
 * anything is enqueued. */
pvf_status pvf_execute(pvf_engine *eng, const pvf_tracks *tracks, const pvf_vertices *out);

/* Same as pvf_execute on another stream (a hipStream_t as void*).  Calls
 * that overlap in time must use different engines (each engine has one
 * arena). */
pvf_status pvf_execute_on(pvf_engine *eng, const pvf_tracks *tracks, const pvf_vertices *out,
                          void *stream);

/* Bytes of the library's fixed per-device scratch (64 MiB). */
#define PVF_SCRATCH_BYTES (64u << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * path and kernels as pvf_execute, with the same results bit for bit, but
 * every per-batch buffer (histogram rows, activations, the probability rows
 * when d_prob_hist is NULL, flags, the track work queue) lives in a fixed
 * scratch array that the library holds on each device until the process
 * ends, instead of in the engine's arena; of the arena, the call reads only
 * the weights.  Calls nothing that allocates.
 * Limit: the batch's per-batch buffers must fit PVF_SCRATCH_BYTES (about
 * 7.1 MiB per event for the default FP32 network, 3.6 MiB in BF16/FP16,
 * 1.8 MiB in FP8: 8, 17 and 35 events); a larger batch returns
 * PVF_ERR_SCRATCH_TOO_SMALL and enqueues nothing.  The other checks are
 * those of pvf_execute.
 * Sharing: every engine on a device uses that device's one scratch, and it
 * keeps the last call's contents (each call clears what it needs zeroed, on
 * the stream, before its kernels).  Calls that overlap in time on one
 * device race and corrupt each other's results: order them on one stream,
 * or with events.  pvf_debug_tensor views only pvf_execute calls.
 * PVF_ERR_DEVICE if the scratch's device address could not be obtained. */
pvf_status pvf_execute_scratch(pvf_engine *eng, const pvf_tracks *tracks, const pvf_vertices *out);

/* Release the engine's host state.  The arena is the caller's to free. */
pvf_status pvf_destroy(pvf_engine *eng);

/* Static English text of a status code. */
const char *pvf_status_string(pvf_status s);

/* ---- scheduling and graphs ------------------------------------------------ */

/* Track-stage schedule.  persistent = 1 (default): a counting-sort kernel
 * orders the batch's events by descending track count and a fixed grid of
 * blocks (as many as fit on the device at once: four per compute unit for
 * histograms of up to 48 intervals, two for longer ones) takes them from a
 * device work queue, so heavy-tailed batches do not end on their largest
 * events; with up to 48 intervals the queue is skipped, and one block runs
 * per event, when the batch fits on the device at once.  persistent = 0: one
 * block per event.  Results are identical either way. */
pvf_status pvf_set_track_schedule(pvf_engine *eng, int persistent);

/* Capture the whole path for this batch view (its pointers and counts are
 * frozen into the graph) into one HIP graph owned by the engine, replacing
 * any earlier one.  Nothing runs during capture.  Refill the same input
 * buffers and call pvf_graph_launch to run it: one launch on the engine's
 * stream instead of one per kernel. */
pvf_status pvf_graph_capture(pvf_engine *eng, const pvf_tracks *tracks, const pvf_vertices *out);

/* Replay the captured graph on the engine's stream (asynchronous).
 * PVF_ERR_INVALID_ARGUMENT if nothing was captured. */
pvf_status pvf_graph_launch(pvf_engine *eng);

/* ---- instrumentation (not on the hot path) ---------------------------- */

/* Number of launch slots of one pvf_execute for this engine.  One slot,
 * enc0.c1 (the first convolution), enqueues nothing when enc0.c2's tile
 * variant computes the first convolution in its own staging (the default in
 * every precision); its kernel name then reads "first_conv (in enc0.c2)" and
 * its profiled time is zero.  Likewise, in BF16, FP16 and FP8, the
 * transposed-conv slots up0 .. up(n_levels - 3) enqueue nothing when the
 * decoder conv before each (dec1.c2, dec2.c2, ...) has a tile variant holding
 * all its output channels (the default): that conv then runs the transposed
 * conv in its epilogue, and its kernel name reads "transposed conv (in
 * dec1.c2)".  And
 * in BF16, FP16 and FP8 with 32 level-0 channels, the dec0.c1 slot enqueues
 * nothing when the head launch ("dec0.c2+head") takes a tile variant that
 * computes dec0.c1 in the same kernel (the default); its name then reads
 * "conv (in dec0.c2+head)". */
int pvf_launch_count(const pvf_engine *eng);

/* Name of launch i (e.g. "track", "enc0.c2", "up1", "peaks"); NULL if out
 * of range.  Static storage. */
const char *pvf_launch_name(const pvf_engine *eng, int i);

/* Kernel that launch i runs, as it appears in a profiler's kernel name
 * (e.g. "conv_mfma_f32<4, 2, 4, 4, 5, 0>", "track_stage"); NULL if out of
 * range.  Owned by the engine; valid until the next pvf_set_launch_variant,
 * pvf_autotune or pvf_set_track_schedule on it. */
const char *pvf_launch_kernel(const pvf_engine *eng, int i);

/* Tile-shape variants (Section 5 of the paper: launch-geometry tuning).
 * A UNet convolution launch can run any of several tile shapes; every
 * shape accumulates each output in the same order, so the choice changes
 * speed only, never a bit of the results.  Launches without variants report
 * a count of 0 and variant -1. */
int pvf_launch_variant_count(const pvf_engine *eng, int i);
int pvf_launch_variant(const pvf_engine *eng, int i);
/* PVF_ERR_INVALID_ARGUMENT if launch i has no variants or v does not fit
 * its shape. */
pvf_status pvf_set_launch_variant(pvf_engine *eng, int i, int v);

/* Autotuner: runs the batch `tracks` (reps + 1 times per variant) on the
 * engine's stream, timing every launch with HIP events, and keeps the
 * fastest variant of each convolution launch (enc0.c2 is charged the first
 * convolution too, fused or not).  A set-up call: it synchronises the stream
 * and overwrites `out`.  Not for the hot path. */
pvf_status pvf_autotune(pvf_engine *eng, const pvf_tracks *tracks, const pvf_vertices *out, int reps);

/* on != 0: create one HIP event per launch boundary now, and from then on
 * record them around every launch that pvf_execute enqueues.  on == 0:
 * stop recording and destroy them.  Recording adds no synchronisation. */
pvf_status pvf_profile_enable(pvf_engine *eng, int on);

/* After the caller has synchronised the stream: elapsed milliseconds of
 * each launch of the most recent profiled pvf_execute, into ms[0..n). */
pvf_status pvf_profile_read(pvf_engine *eng, float *ms, int n);

/* Debug view of one internal activation of the most recent call, for
 * per-layer parity checks: copies tensor `name` ("hist", "enc0.c1", ...,
 * "dec0.c1", "prob"), for the first n_events events, into d_dst as float32
 * [n_events][C][L] (channels first), on the engine's stream.  Returns
 * PVF_ERR_INVALID_ARGUMENT for an unknown name, for "decL.c2" when that
 * conv runs the following transposed conv in its epilogue, and for
 * "dec0.c1" when the head launch computes it (those outputs are then never
 * stored); *out_count receives the number of floats
 * (C * L * n_events), also when d_dst is NULL. */
pvf_status pvf_debug_tensor(pvf_engine *eng, const char *name, int32_t n_events, float *d_dst,
                            int64_t *out_count);

#ifdef __cplusplus
}
#endif

#endif /* PVF_H */
