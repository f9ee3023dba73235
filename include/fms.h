/*
 * fms.h - C ABI of the MI355X (gfx950) Faster Mean-shift library.
 *
 * The library clusters L2-normalised per-pixel embeddings with cosine,
 * flat-kernel mean shift (Eq. 8-11 of "Faster Mean-shift: GPU-accelerated
 * clustering for cosine embedding-based cell segmentation and tracking",
 * arXiv 2007.14283), iterating a batch of seeds in parallel with early stopping
 * (Sec. 3.2.3) under the online seed optimisation policy (Eq. 14, Eq. 19,
 * Sec. 3.2.4), then prunes the modes and assigns every foreground pixel to
 * its most similar mode (Alg. 2).
 *
 * Conventions shared by every entry point
 *   - Buffers marked "device" live in the memory of the handle's GPU; buffers
 *     marked "host" live in ordinary host memory.  The caller owns every input
 *     and output buffer; the library owns only the workspace inside a handle,
 *     which grows on demand and is released by fms_destroy.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     All device work is enqueued on it.  fms_cluster and fms_shift_seeds make
 *     host decisions between GPU steps (the CPU steers the seed count, Fig. 3),
 *     so they synchronise `stream` internally; their outputs are complete when
 *     they return.  fms_seed_order only enqueues.
 *   - Errors are reported by status code only: nothing throws across the ABI
 *     and nothing aborts.  On error the output contents are unspecified except
 *     where stated.
 *   - One host thread at a time per handle.  Handles are independent.
 *   - Embeddings: FP32, any D from 1 to 128, addressed through strides, so
 *     pixel-major (NHWC: pixel_stride = D, channel_stride = 1) and
 *     channel-major (NCHW: pixel_stride = 1, channel_stride = H*W) layouts are
 *     both read in place.  Pixel p = y*W + x (raster order).
 */
#ifndef FMS_H
#define FMS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fms_handle_s* fms_handle;

typedef enum {
  FMS_OK = 0,
  FMS_ERR_INVALID_ARG = -1, /* null pointer, bad size or parameter out of range */
  FMS_ERR_UNSUPPORTED = -2, /* e.g. D > 128 */
  FMS_ERR_BAD_INPUT = -3,   /* a foreground embedding is zero or not finite */
  FMS_ERR_CAPACITY = -4,    /* k_max too small; *n_modes holds the required count */
  FMS_ERR_HIP = -5          /* the HIP runtime reported an error */
} fms_status;

typedef enum {
  FMS_PREC_FP32 = 0,        /* every step's contractions on FP32 MFMA */
  FMS_PREC_BF16_REFINE = 1, /* BF16 MFMA (FP32 accumulate) for every round's
                               iteration (Eq. 8, 10, 11, Sec. 3.2.1); then each
                               converged seed takes its final refine_iters
                               iterations again on FP32 MFMA, from the centre it
                               had that many steps before it stopped, with the
                               same stopping test (at most refine_iters + 1 FP32
                               steps; a seed still moving after them is dropped
                               with the round's unconverged seeds).  The BF16
                               iteration runs one step past its early stop, and
                               the early stop is then taken on the FP32 step
                               counts.  Window counts, pruning, coverage, the
                               controller and the labels all work on those FP32
                               endpoints. */
  FMS_PREC_BF16_SPLIT = 2   /* BF16 MFMA (FP32 accumulate) on values split into a
                               high and a low BF16 part (hi = bf16(v), lo =
                               bf16(v - hi), v kept to a relative 2^-16): each
                               similarity takes three products (hi.hi, hi.lo,
                               lo.hi) and each window sum two, so a similarity is
                               off by under 5e-5 (plain BF16: 4e-3).  Every
                               iteration runs this way; no replay.  Window counts
                               are FP32 as in the other forms. */
} fms_precision;

/* Clustering parameters.  fms_default_params fills the paper's values. */
typedef struct {
  double bandwidth;   /* h in cosine distance: a vector is in a window when
                         1 - cos <= h (Eq. 9, Eq. 11).  Required, 0 < h < 2.
                         The paper uses 0.1 (Sec. 4.1 Design, Sec. 4.2). */
  double conv_tol;    /* a seed has converged when the cosine distance between
                         consecutive centres is below this; <= 0 means h/1000
                         (Sec. 3.2.1). */
  double gamma;       /* early stop: the iteration of a round ends once more than
                         gamma of its seeds have converged (Sec. 3.2.3); 0.9. */
  double big_l;       /* L: double N while N < L * N_min (Eq. 21, Sec. 3.2.4); 2. */
  double big_h;       /* H: next frame starts at N - N_min when N > H * N_min; 8. */
  double p_target;    /* P in Eq. 19; 0.99 (Sec. 3.2.2). */
  uint64_t seed;      /* key of the seed order (SplitMix64-keyed permutation). */
  int32_t n_initial;  /* N_initial = 128 (Sec. 3.2.4). */
  int32_t n_state_in; /* N carried over from the previous frame; <= 0: n_initial. */
  int32_t max_iter;   /* cap on iterations per round (not in the paper); 100. */
  int32_t max_rounds; /* cap on seed rounds per frame (not in the paper); 32. */
  int32_t precision;  /* fms_precision. */
  int32_t refine_iters; /* BF16 form: final iterations of each converged seed
                           taken again in FP32 (0 = none: BF16 endpoints);
                           0..8, larger values give FMS_ERR_UNSUPPORTED; 2. */
  int32_t timing;     /* nonzero: time every fused-step launch with HIP events on
                         `stream` and report the totals in fms_stats. */
  /* Work decomposition of the fused step (0 = the library's choice: 8 waves
   * per work group for single frames, 4 for batches): seeds per
   * group (16, 32, 64 or 128; rounded down to a size compiled for the
   * precision and D), target number of (seed group, pixel chunk) items per
   * step, cap on pixel chunks, and waves per work group (4, 8 or 16, other
   * values give FMS_ERR_UNSUPPORTED; a group's waves split its pixel chunk;
   * halved where the group's LDS would exceed 64 KiB).  They change speed
   * only: every result is the same up to the order of FP32 additions. */
  int32_t tile_seeds;
  int32_t tile_items;
  int32_t tile_chunks;
  int32_t tile_waves;
  /* Nonzero: each batch of seed iterations (the step and reduction launches
   * enqueued between two reads of the counters) is captured once per shape
   * into a HIP graph, kept in the handle and replayed; 0 (the default)
   * launches every kernel separately.  Results are identical either way.
   * Ignored when `timing` is set. */
  int32_t graphs;
} fms_params;

/* Per-call statistics (host struct). */
typedef struct {
  int64_t seed_pixel_updates; /* sum over iterations of (active seeds) * n */
  double n_min;               /* last Eq. 19 value; NaN when no mode was found */
  int32_t n_fg;               /* foreground pixels n */
  int32_t rounds;             /* seed rounds run */
  int32_t seeds_used;         /* seeds iterated */
  int32_t iterations_total;   /* iterations summed over rounds (refine steps excluded) */
  int32_t refine_steps;       /* BF16 form: FP32 replay steps run, summed over rounds */
  int32_t n_discarded;        /* seeds dropped unconverged by the early stop */
  int32_t n_uncovered;        /* foreground pixels farther than h from every mode */
  int32_t n_state_out;        /* N to carry into the next frame (Sec. 3.2.4) */
  int32_t refine_unconverged; /* BF16 form: seeds converged in BF16 that the FP32 replay
                                 did not freeze (dropped) */
  int32_t refine_step_diff;   /* BF16 form: replayed seeds the FP32 stopping test froze
                                 after a different number of steps than the BF16 one */
  int64_t refine_updates;     /* BF16 form: (active seeds) * n summed over FP32 replay steps */
  int32_t refine_gamma_cut;   /* BF16 form: replayed seeds dropped because, counted in FP32
                                 steps, they converged after the round's early stop */
  /* Fused-step kernel timing, filled when fms_params.timing is nonzero.
   * Index 0: FP32 form of the step, index 1: BF16 form. */
  double step_ms[2];          /* summed launch durations (HIP events), ms */
  int64_t step_updates[2];    /* (active seeds) * n summed over those launches */
  int32_t step_launches[2];
  int64_t step_pixels[2];     /* n summed over the frames those launches stepped
                                 (the pixel rows they read) */
} fms_stats;

/* Fill *p with the paper's defaults (bandwidth 0.1, tol h/1000, gamma 0.9,
 * N_initial 128, L 2, H 8, P 0.99) and this library's caps (max_iter 100,
 * max_rounds 32, FP32, 2 refine iterations, seed 0).  p: host, not NULL. */
void fms_default_params(fms_params* p);

/* Create a handle bound to GPU `device_ordinal`.  *out receives the handle.
 * Errors: FMS_ERR_INVALID_ARG (out NULL, bad ordinal), FMS_ERR_HIP. */
fms_status fms_create(fms_handle* out, int32_t device_ordinal);

/* Release a handle and its workspace.  NULL is accepted. */
fms_status fms_destroy(fms_handle h);

/* Cluster one frame (Alg. 2 under the online seed optimisation policy).
 *
 *  emb            device, FP32; element (pixel p, channel c) at
 *                 emb[p*pixel_stride + c*channel_stride].
 *  mask           device, height*width bytes, nonzero = foreground
 *                 (the predicted segmentation of Sec. 3.2.2); NULL = all pixels.
 *  height, width  frame size (>= 1 each); dim = D (1..128).
 *  p              host, clustering parameters.
 *  modes          device, k_max*dim FP32: unit-norm modes in acceptance order.
 *  mode_counts    device, k_max int32 window counts of the modes, or NULL.
 *  k_max          capacity of `modes` in rows.
 *  n_modes        host: number of modes written (or required, on CAPACITY).
 *  labels         device, height*width int32: -1 on background, else the index
 *                 of the most similar mode (lowest index on ties).
 *  stats          host, or NULL.
 * An all-background mask returns FMS_OK with *n_modes = 0 and all labels -1.
 * Errors: INVALID_ARG, UNSUPPORTED (dim > 128), BAD_INPUT, CAPACITY, HIP. */
fms_status fms_cluster(fms_handle h, void* stream,
                       const float* emb, int64_t pixel_stride, int64_t channel_stride,
                       const uint8_t* mask, int32_t height, int32_t width, int32_t dim,
                       const fms_params* p,
                       float* modes, int32_t* mode_counts, int32_t k_max, int32_t* n_modes,
                       int32_t* labels, fms_stats* stats);

/* One frame of a batch (host struct; the pointers are device pointers). */
typedef struct {
  const float* emb;          /* device, FP32, (pixel p, channel c) at
                                emb[p*pixel_stride + c*channel_stride] */
  int64_t pixel_stride;
  int64_t channel_stride;
  const uint8_t* mask;       /* device, height*width bytes (nonzero = foreground),
                                or NULL = all pixels */
  int32_t height, width;     /* >= 1 each */
  double bandwidth;          /* this frame's h, 0 < h < 2 */
  int32_t n_state_in;        /* this frame's N carried over from its previous
                                frame; <= 0: fms_params.n_initial */
  int32_t* labels;           /* device, height*width int32 output: -1 on
                                background, else the index of the most similar
                                of this frame's modes (lowest on ties) */
} fms_frame;

/* Cluster a batch of frames of one embedding width (Alg. 2 under the online
 * seed optimisation policy, each frame on its own).  Every launch covers all
 * frames, so many small frames cost little more than one; each frame's
 * result is the one fms_cluster returns for it alone.
 *
 *  n_frames       >= 1; frames: host array of n_frames entries.
 *  dim            D (1..128), shared by the frames.
 *  p              host; every field but bandwidth and n_state_in (taken per
 *                 frame) applies to all frames.
 *  modes          device, k_max*dim FP32: the frames' modes, packed: frame
 *                 f's are rows mode_offsets[f] .. mode_offsets[f+1]-1, in
 *                 acceptance order.
 *  mode_counts    device, k_max int32 window counts of the modes, or NULL.
 *  mode_offsets   host, n_frames+1 int32 (output); on CAPACITY
 *                 mode_offsets[n_frames] is the required total.
 *  stats          host, n_frames entries, or NULL.  The kernel-timing fields
 *                 describe the whole call and are filled in stats[0] only.
 * A round that needs more than 16384 seeds in one frame is UNSUPPORTED in a
 * batch of two or more frames.
 * Errors: INVALID_ARG, UNSUPPORTED, BAD_INPUT, CAPACITY, HIP. */
fms_status fms_cluster_batch(fms_handle h, void* stream, int32_t n_frames, const fms_frame* frames,
                             int32_t dim, const fms_params* p, float* modes, int32_t* mode_counts,
                             int32_t k_max, int32_t* mode_offsets, fms_stats* stats);

/* One round of the parallel seed iteration (Alg. 2, the loop over seeds, with
 * the early stop of Sec. 3.2.3) on an explicit seed list, for lockstep checks
 * and benchmarking of the hot loop.
 *
 *  emb, strides, mask, height, width, dim: as fms_cluster.
 *  seed_fg        device, n_seeds int32 foreground ordinals (index into the
 *                 raster-ordered list of foreground pixels), each in [0, n).
 *  p              host; bandwidth, conv_tol, gamma, max_iter, precision and
 *                 refine_iters are used.
 *  endpoints      device, n_seeds*dim FP32: final centre of each seed (for
 *                 FMS_PREC_BF16_REFINE with refine_iters > 0, the FP32
 *                 replay's centre for the seeds converged in BF16).
 *  iters          device, n_seeds int32: steps taken until it converged or
 *                 the round stopped (the BF16 iteration's count; replay steps
 *                 excluded).
 *  converged      device, n_seeds bytes: 1 = converged (for the BF16 form:
 *                 and frozen by the FP32 replay), 0 = discarded.
 *  counts         device, n_seeds int32: window count at converged endpoints,
 *                 -1 for discarded seeds; may be NULL.
 *  stats          host or NULL (seed_pixel_updates, iterations_total, n_fg
 *                 and, for the BF16 form, the refine_* fields are filled).
 * Errors: INVALID_ARG (including a seed index outside [0, n)), UNSUPPORTED,
 * BAD_INPUT, HIP. */
fms_status fms_shift_seeds(fms_handle h, void* stream,
                           const float* emb, int64_t pixel_stride, int64_t channel_stride,
                           const uint8_t* mask, int32_t height, int32_t width, int32_t dim,
                           const int32_t* seed_fg, int32_t n_seeds, const fms_params* p,
                           float* endpoints, int32_t* iters, uint8_t* converged,
                           int32_t* counts, fms_stats* stats);

/* For callers that cannot allocate memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): fms_shift_seeds, FP32
 * form, with every buffer of its work -- the compacted frame, the centres and
 * their lists, the chunk partials, the window counts, the counters and the
 * frame tables -- in one fixed device array per GPU (about 38 MiB, held from
 * the library's first use on that GPU until the process ends), never in
 * memory it allocates.  The handle supplies only its GPU and its mapped
 * counter area (both set up by fms_create); its tuning table is not used.
 *
 * Arguments, outputs and results are those of fms_shift_seeds with
 * p->precision = FMS_PREC_FP32 (same kernels and work decomposition, so the
 * same endpoints, step counts, flags and window counts).  stats: n_fg,
 * seeds_used, iterations_total, seed_pixel_updates and n_discarded are
 * filled, the rest zero (n_min NaN).
 *
 * Limits (beyond them FMS_ERR_UNSUPPORTED, nothing written to the outputs):
 * height * width <= 1,048,576; foreground pixels <= 131,072 (counted on the
 * GPU: past it the frame's rows are not kept, the outputs' contents are
 * unspecified and the call returns FMS_ERR_UNSUPPORTED at its end); n_seeds <=
 * 4096; dim <= 32; precision FP32 and timing 0; tiling requests whose chunk
 * partials exceed 32,768 rows.
 *
 * Every call on a GPU uses that GPU's one array, whatever the handle: calls
 * that overlap on one GPU (several host threads, or streams that run
 * concurrently) race and their results are undefined; the array keeps the
 * last call's contents, and each call writes everything it reads first.
 * Errors: as fms_shift_seeds, plus FMS_ERR_UNSUPPORTED for the limits above. */
fms_status fms_shift_seeds_noalloc(fms_handle h, void* stream,
                                   const float* emb, int64_t pixel_stride, int64_t channel_stride,
                                   const uint8_t* mask, int32_t height, int32_t width, int32_t dim,
                                   const int32_t* seed_fg, int32_t n_seeds, const fms_params* p,
                                   float* endpoints, int32_t* iters, uint8_t* converged,
                                   int32_t* counts, fms_stats* stats);

/* Differentiable form: `steps` (T >= 1) unrolled FP32 steps of Eq. 8-11 from
 * the given seeds, every seed taking all T steps (no freezing, no early
 * stop), for training an embedding network through the clustering.
 *
 *  emb, strides, mask, height, width, dim: as fms_cluster.
 *  seed_fg        device, n_seeds int32 foreground ordinals, each in [0, n).
 *  bandwidth      h, 0 < h < 2.
 *  y_out          device, n_seeds*dim FP32: y_T (unit rows).
 *  y_prev         device, n_seeds*dim FP32: y_{T-1}, kept for the backward.
 *  v_norm         device, n_seeds FP32: |V_T|, the norm of the last window
 *                 sum, kept for the backward.
 * Errors: INVALID_ARG (including a seed index outside [0, n) or an empty
 * foreground), UNSUPPORTED, BAD_INPUT, HIP. */
fms_status fms_unroll(fms_handle h, void* stream,
                      const float* emb, int64_t pixel_stride, int64_t channel_stride,
                      const uint8_t* mask, int32_t height, int32_t width, int32_t dim,
                      const int32_t* seed_fg, int32_t n_seeds, int32_t steps, double bandwidth,
                      float* y_out, float* y_prev, float* v_norm);

/* Gradient of a loss L(y_T) with respect to the embeddings, given
 * grad_y = dL/dy_T (device, n_seeds*dim FP32) and the forward's y_out,
 * y_prev and v_norm.  The window weights are a step function of the
 * similarity, so only the last step contributes almost everywhere:
 *   dL/de_p = (I - x_p x_p^T) sum_j [y_{T-1,j} . x_p >= 1 - h] dL/dV_j / |e_p|,
 *   dL/dV_j = (I - y_j y_j^T) dL/dy_j / |V_j|,  x_p = e_p / |e_p|.
 * The windows are recomputed from the embeddings (no kernel matrix is
 * stored).  grad_emb: device FP32 with the same strides as emb, written
 * completely (zero on the background).
 * Errors: INVALID_ARG, UNSUPPORTED, BAD_INPUT, HIP. */
fms_status fms_unroll_backward(fms_handle h, void* stream,
                               const float* emb, int64_t pixel_stride, int64_t channel_stride,
                               const uint8_t* mask, int32_t height, int32_t width, int32_t dim,
                               int32_t n_seeds, double bandwidth, const float* y_out,
                               const float* y_prev, const float* v_norm, const float* grad_y,
                               float* grad_emb);

/* One entry of the fused-step tiling table that fms_autotune fills (host
 * struct). */
typedef struct {
  int32_t precision;    /* step form: FMS_PREC_FP32 (FP32 step) or
                           FMS_PREC_BF16_REFINE (BF16 step) */
  int32_t dim_padded;   /* D class: 32, 64 or 128 */
  int32_t n_fg;         /* foreground pixels of the frame it was timed on */
  int32_t seeds;        /* active seeds it was timed at */
  int32_t tile_seeds;   /* the chosen work decomposition (see fms_params) */
  int32_t tile_items;
  int32_t tile_waves;
  float us_per_step;    /* one fused step plus its renormalising reduction, us */
  float us_default;     /* the same with the library's default decomposition */
} fms_tune_entry;

/* What fms_autotune decided (host struct). */
typedef struct {
  float ms_default;   /* median whole call on the frame without the new entries, ms */
  float ms_tuned;     /* the same with them */
  int32_t kept;       /* 1: the new entries are in the table (ms_tuned < ms_default) */
} fms_tune_report;

/* Autotuner of the fused step's work decomposition (Eq. 8, 10, 11 as run by
 * the parallel seed loop of Alg. 2).  The decomposition changes speed only:
 * results are the same up to the order of FP32 additions.
 *
 * Compacts `frame`, then for each active-seed count m in {128, 512, 2048,
 * 8192} up to the frame's foreground count n (just n when n < 128), and each
 * step form that `p->precision` runs (the BF16 step and the FP32 step of its
 * replay for FMS_PREC_BF16_REFINE; the FP32 step for FMS_PREC_FP32),
 * times every compiled decomposition (seeds per group x about 256, 512 or
 * 1024 items x 4, 8 or 16 waves) on m centres that start at the first m
 * foreground pixels: one warm-up, then the mean of 6 back-to-back pairs of
 * (fused step, renormalising reduction) between two HIP events on `stream`.
 * The fastest per (form, m) are then checked on whole calls of fms_cluster
 * on the frame (one warm-up each, then 6 alternating rounds of two calls):
 * they go into the handle's table, replacing earlier entries of the same
 * form, D class and pixel-count bucket (n within a factor of 4), only when
 * the median call is faster with them than without; otherwise those entries
 * are removed and the defaults stay.  Later single-frame calls on this handle (fms_cluster,
 * fms_shift_seeds, fms_cluster_batch of one frame) whose tile_* parameters
 * are all 0 take, for each fused-step launch, the entry of the launch's form
 * and D class in the frame's bucket whose m is nearest (in ratio) to the
 * launch's bound on active seeds; without one, the library's defaults.
 * Batches of several frames use only entries of fms_autotune_batch.
 *
 *  frame      host struct (device pointers); its bandwidth sets the windows;
 *             labels and n_state_in are ignored.
 *  p          host: precision and the other checks of fms_cluster; tile_*
 *             ignored.
 *  entries    host, capacity rows: the entries this call chose; NULL: not
 *             reported.
 *  n_entries  host, or NULL: number of entries this call chose (<= 8).
 *  report     host, or NULL: the whole-call timings and whether the entries
 *             were kept.
 * Synchronises `stream`.  Errors: INVALID_ARG (also an empty mask),
 * UNSUPPORTED, BAD_INPUT, CAPACITY (entries given with capacity below the
 * count, which *n_entries then holds; the table is updated regardless),
 * HIP. */
fms_status fms_autotune(fms_handle h, void* stream, const fms_frame* frame, int32_t dim, const fms_params* p,
                        fms_tune_entry* entries, int32_t capacity, int32_t* n_entries, fms_tune_report* report);

/* fms_autotune for batches: the same candidates, seed counts m up to 2,048
 * (each frame taking min(m, its foreground count) centres, from its first
 * foreground pixels), the mean of 2 timed pairs, every timed launch spanning
 * all n_frames >= 2 frames as the launches of fms_cluster_batch do, and the
 * whole-call check on
 * fms_cluster_batch of these frames.  The entries go into the handle's
 * table beside the single-frame ones (entries of the same form, D class and
 * bucket of the largest frame's pixel count, tuned on batches, are
 * replaced), and later fms_cluster_batch calls of several frames whose
 * tile_* parameters are all 0 use them in the same way; n_fg of an entry is
 * the largest frame's foreground count.  Arguments and errors as for
 * fms_autotune, `frames` being an array of n_frames host structs (INVALID_ARG
 * also for n_frames < 2). */
fms_status fms_autotune_batch(fms_handle h, void* stream, int32_t n_frames, const fms_frame* frames, int32_t dim,
                              const fms_params* p, fms_tune_entry* entries, int32_t capacity, int32_t* n_entries,
                              fms_tune_report* report);

/* Empty the handle's tuned table (later calls use the library's defaults). */
fms_status fms_clear_tuning(fms_handle h);

/* The seed order: order[j] = foreground ordinal at position j, j in [0, n),
 * a permutation of [0, n) keyed by `seed` (four-round Feistel network whose
 * round keys and round function come from SplitMix64, with cycle walking).
 *  order  device, n int32.  Enqueued on `stream`; does not synchronise.
 * Errors: INVALID_ARG (n < 0, order NULL with n > 0), HIP. */
fms_status fms_seed_order(fms_handle h, void* stream, int32_t n, uint64_t seed, int32_t* order);

/* Static text for a status code. */
const char* fms_status_string(fms_status s);

#ifdef __cplusplus
}
#endif

#endif /* FMS_H */
