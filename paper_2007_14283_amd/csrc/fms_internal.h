// Internal interface between the host runtime (capi.cpp) and the gfx950
// kernels (kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fms {

// Pixels per block: the unit both contractions of the fused step consume.
constexpr int kBlockPix = 32;
// Slots of the device-side counter array.
enum MetaSlot {
  META_N = 0,          // foreground count n
  META_BAD = 1,        // rows that are zero or non-finite
  META_NSEL = 2,       // seeds selected this round
  META_CURSOR = 3,     // seed-order cursor (every earlier position is used or covered)
  META_NCONV = 4,      // converged seeds this round
  META_REFINE_DIFF = 5, // BF16 form: replayed seeds whose FP32 stop came after another step count
  META_REFINE_BAD = 6, // BF16 form: converged seeds the FP32 replay did not freeze
  META_LEFT = 7,       // nonzero iff a foreground pixel is still eligible as a seed (coverage); pixels farther than h from every mode (labels)
  META_BADSEED = 8,    // seed indices outside [0, n)
  META_GSTEP = 9,      // iteration whose step first saw more than gamma converged (-1: none yet)
  META_DONE = 10,      // the round's iteration has stopped
  META_GCUT = 11,      // BF16 form: replayed seeds dropped by the FP32 early-stop count
  META_STEPS = 12,     // iterations run this round
  META_NACC = 13,      // modes being refined / modes accepted by the last pruning pass
  META_NCAND = 14,     // converged candidates of the round
  META_OVERCAP = 15,   // foreground count beyond a fixed-capacity call's rows (0: within)
  META_ACT = 16,       // two slots (16, 17): active seeds of the even / odd iterations
  META_COUNT = 24
};

// Largest candidate set the single-block rank/greedy kernels take.
constexpr int kRankMax = 16384;

// Work decomposition of the fused step (see plan_chunks in kernels.hip):
// seeds in groups of `group_seeds`, pixels in chunks of whole 32-pixel
// blocks, about `target_items` (group, chunk) items, at most `max_chunks`
// chunks, `waves` waves per work group.  Defaults: kWaves waves and
// kWaveBudget / waves items; fms_params (or fms_autotune) can override them.
constexpr int kWaves = 4;
constexpr int kWaveBudget = 2048;
constexpr int kMaxChunks = 256;
struct Tiling {
  int group_seeds;
  int target_items;
  int max_chunks;
  int waves;  // waves per work group: 4, 8 or 16
};
// Arithmetic of a fused step: FP32 MFMA; BF16 MFMA on BF16 values; BF16 MFMA
// on values split into high and low BF16 parts (see k_shift).
enum StepForm { FORM_FP32 = 0, FORM_BF16 = 1, FORM_SPLIT = 2 };
// The tiling used for a (step form, padded D) pair given the caller's
// requests (0 = default); group sizes round down to a compiled one.
Tiling make_tiling(int form, int dp, int want_seeds, int want_items, int want_chunks, int want_waves);
struct ChunkPlan {
  int groups;
  int n_chunks;
  int chunk_blocks;
};

struct FrameDesc {
  const float* emb;
  int64_t pixel_stride, channel_stride;
  const uint8_t* mask;
  int64_t n_pixels;  // H*W
  int dim;           // D
  int dp;            // D padded to 32, 64 or 128
};

// ------------------------------------------------------------------ batches
// A call works on F >= 1 frames at once.  Every row-indexed buffer
// (compacted pixels and their transposed blocks, centres and their
// compacted rows, lists, flags, counts, modes) holds frame f's rows from
// geo[f].row0 on; a frame never needs more rows there than its padded
// foreground count.  Frame f's counters are meta + f * META_COUNT and
// meta64 + f * kMeta64.  Kernels with many work groups per frame take the
// frame from blockIdx.y; kernels with one work group per frame from
// blockIdx.x.  meta64 slot 0: (active seeds) x n summed over the round's
// steps; slot 1: n summed over them (the pixel rows they read).
constexpr int kMeta64 = 4;
struct FrameGeo {
  FrameDesc desc;  // source embeddings and mask
  int64_t mblk0;   // first mask block of the frame (compaction scan)
  int64_t row0;    // first row in every row-indexed buffer (a multiple of 32)
  int64_t part0;   // first row of the chunk partials and partial counts
  int64_t elig0;   // first byte of the eligibility flags (a multiple of 16)
  int* labels;     // the frame's label map (H*W), or null
  int n;           // foreground pixels
  int n_blocks;    // 32-pixel blocks, ceil(n / 32)
  int half_bits;   // half width of the seed-order Feistel network
  float thr;       // 1 - h in FP32
  float tol;       // convergence threshold on the cosine distance
};
// Per-frame values the host sets for one round or pass.
struct RoundTab {
  int want;          // seeds to select (0: the frame sits the round out)
  int k_modes;       // modes kept before the pass; new modes start there
  int nact;          // centre count of a plain (refinement) step or list
  int words_c;       // row stride of the candidate x candidate bits
  int words_m;       // row stride of the candidate x mode bits
  int64_t bits_c0;   // first word of the frame's candidate x candidate bits
  int64_t bits_m0;   // first word of the frame's candidate x mode bits
};
// Device view of a call.  The maxima size the grids; work groups past a
// frame's own extent return.
struct Batch {
  int F;
  const FrameGeo* geo;
  const RoundTab* rt;
  int* meta;
  unsigned long long* meta64;
  int max_n;           // largest foreground count
  int max_blocks;      // largest 32-pixel block count
  int64_t max_mblk;    // largest mask block count
  // Single-frame calls carry their round table in the launch arguments
  // (rt_inline), which saves a copy to the device per round.
  int rt_inline;
  RoundTab rt0;
};
// The round table of frame f of a launch (a copy: a reference into the
// launch arguments would make the compiler copy them to scratch memory).
__host__ __device__ inline RoundTab round_tab(const Batch& b, int f) { return b.rt_inline ? b.rt0 : b.rt[f]; }
constexpr int kMaskBlockPix = 1024;
// Eligibility bytes a frame of n foreground pixels needs (whole 16-byte
// words plus one word of zero padding).
__host__ __device__ inline int64_t elig_len(int n) { return ((int64_t)n + 15) / 16 * 16 + 16; }

// Compaction and normalisation of the foreground.  Also zeroes the padding
// rows [n, n_pad) of every layout (n = meta[META_N] of the frame).
hipError_t launch_mask_count(hipStream_t s, const Batch& b, int* block_counts);
hipError_t launch_scan_blocks(hipStream_t s, const Batch& b, int* block_counts);
// x32t (may be null: FP32 steps need it) receives the dimension-major FP32
// copy, x16 (may be null) the BF16 rounding of each value, xlo (may be null;
// only with x16) the BF16 rounding of what that leaves (split form).  enorm
// (may be null) receives each row's raw norm |e_i|.  Rows at or beyond
// row_cap are not written (fixed-capacity calls).
hipError_t launch_compact(hipStream_t s, const Batch& b, int dp, const int* block_offsets, int* fg_idx, float* x32,
                          float* x32t, uint16_t* x16, uint16_t* xlo, float* enorm, int64_t row_cap = INT64_MAX);
// Single-frame calls on caller-independent fixed buffers: write the frame and
// round tables from arguments and clear the counters (one work group); after
// the mask scan, the foreground and block counts into the table (0 when the
// count exceeds row_cap, which META_OVERCAP then holds).
hipError_t launch_set_tables(hipStream_t s, const FrameGeo& g, const RoundTab& rt, FrameGeo* geo, RoundTab* rtab,
                             int* meta, unsigned long long* meta64);
hipError_t launch_geo_from_count(hipStream_t s, const Batch& b, int64_t row_cap);

// order[j] = foreground ordinal at seed-order position j; rank = its
// inverse.  Also sets every eligibility flag of the frame (1 for j < n, 0
// for the padding) and the seed cursor to 0.
hipError_t launch_seed_order(hipStream_t s, const Batch& b, const uint64_t keys[4], int* order, int* rank,
                             uint8_t* elig);
// The seed order of a single foreground of n pixels (no flags, no rank).
hipError_t launch_seed_order_plain(hipStream_t s, int n, int half_bits, const uint64_t keys[4], int* order);

// Each frame takes its round's rt.want seeds (one work group per frame).
hipError_t launch_select(hipStream_t s, const Batch& b, const int* order, uint8_t* elig, int* seed_pos,
                         int* seed_fg);
// Single frame: the given seeds' rows as the starting centres (n < 0: the
// foreground count from meta[META_N]).
hipError_t launch_init_seeds(hipStream_t s, const int* seed_fg, int m, int n, const float* x32, int dp,
                             float* y, int* meta);
// Start of a round's iteration (identity active list, counters) for at most
// cap centres per frame.  With nsel_from_rt the frame's centre count is
// rt.nact (and is written to META_NSEL), else META_NSEL.  With seed_fg (may
// be null) the centres are also loaded from the pixel rows.
hipError_t launch_round_begin(hipStream_t s, const Batch& b, int cap, bool nsel_from_rt, int* active,
                              uint8_t* state, int* iters, const int* seed_fg, const float* x32, int dp, float* y);
struct StepGeom {
  int n;             // foreground count
  int n_blocks;      // ceil(n / 32)
  int chunk_blocks;  // blocks per pixel chunk (fixed per frame)
  int n_chunks;
};
StepGeom make_geom(int n);

// Control of the iterate loop on the device.  Iteration `iter` reads its
// active count from meta[META_ACT + iter % 2] and appends the next one to
// the other slot.  The step kernel applies the early stop of Sec. 3.2.3
// first (more than gamma of the round's seeds converged, or none left
// active): it sets meta[META_DONE] and skips the iteration, and the reduce
// kernel of that iteration sees the flag.  Otherwise its first work group
// clears the other slot and counts the iteration (META_STEPS, meta64[0]).
// With extra > 0 the iteration goes on for `extra` more steps after the
// first step that saw more than gamma converged (META_GSTEP records that
// step); only an empty active list stops it sooner.
// iter < 0: a plain step whose count is meta[nact_slot], or rt.nact when
// nact_slot < 0.
struct IterCtl {
  int nact_slot;
  int iter;
  double gamma;
  int extra = 0;
};
// One fused mean-shift step for the active seeds (at most cap per frame):
// partial window sums per pixel chunk.  Centre a is y[active[a]], or y[a]
// when active is null (rows already compacted).  ev0/ev1 (may be null)
// receive the start and end of the kernel itself (hipExtLaunchKernel), not
// of the launch call.
size_t shift_partial_rows(const Tiling& t, int cap);
// form: StepForm; xrm: the row layout of that form's values (FP32 or the
// BF16 high parts); xt: the FP32 dimension-major layout (FP32 steps only,
// else ignored); xrl: the BF16 low parts (split form only, else null).
hipError_t launch_shift(hipStream_t s, const Batch& b, int form, int dp, const Tiling& t, const void* xrm,
                        const void* xt, const uint16_t* xrl, const float* y, const int* active,
                        const IterCtl& ctl, int cap, float* partial, hipEvent_t ev0 = nullptr,
                        hipEvent_t ev1 = nullptr);
// Sum partials, renormalise, convergence test and (mode 0) the next active
// list and converged count.  yc_next (mode 0, may be null) receives the new
// rows of the seeds that stay active, in next-list order.  Mode 1 is a plain
// step (no freezing, no test; a centre whose window is empty gets state 2).
// vnorm (may be null) receives |V| of each centre.  ycur (may be null) holds
// the current centre rows in list order (the rows the step read); without it
// they are read from y through the list.  ring (mode 0, may be null): ring_len
// slabs of ring_stride floats, row-indexed like y; the centre a seed starts a
// step from goes to slab (its steps so far) % ring_len.
hipError_t launch_reduce(hipStream_t s, const Batch& b, int dp, const Tiling& t, const float* partial,
                         const int* active, float* y, uint8_t* state, int* iters, int* next_active,
                         float* yc_next, const IterCtl& ctl, int cap, int mode, float* vnorm = nullptr,
                         const float* ycur = nullptr, float* ring = nullptr, int64_t ring_stride = 0,
                         int ring_len = 0);
// Window counts |{i : y[list[a]] . x_i >= thr}| of at most m centres per
// frame: form FORM_FP32 on FP32 MFMA (xrm = the FP32 rows, xrl null) or
// FORM_SPLIT on BF16 MFMA (xrm / xrl = the high / low BF16 rows).  The
// frame's count is meta[m_slot], or rt.nact when m_slot < 0.
hipError_t launch_count(hipStream_t s, const Batch& b, int form, int dp, const Tiling& t, const void* xrm,
                        const uint16_t* xrl, const float* y, const int* list, int m, int* pcount, int* counts,
                        int m_slot);
// Similarity bits of rows y[rows[j]], j < meta[rows_slot] (m bounds it):
// against columns y[cols[c]], c < meta[cols_slot] (ncols bounds it; bits at
// rt.bits_c0, row stride rt.words_c) when cols is given, and against the
// frame's modes before the pass, c < rt.k_modes (nmodes bounds it; bits at
// rt.bits_m0, stride rt.words_m) when modes is given; one launch for both.
// With `first` (cols = rows, INT_MAX-initialised), first[j] receives the
// first word of row j holding an earlier candidate's bit.
int simbits_words(int ncols);
hipError_t launch_simbits(hipStream_t s, const Batch& b, int dp, const float* y, const int* rows, int m,
                          const int* cols, int ncols, const float* modes, int nmodes, uint32_t* bits, int rows_slot,
                          int cols_slot, int* first = nullptr);
// FP32 replay of the BF16 form.  Begin (one work group per frame): the
// round's converged slots k < meta[META_NSEL] (state 1), ascending, to
// cand[i] (their number to meta[META_NCAND]); row i of yr gets the centre
// slot cand[i] had min(iters, ring_len) steps before it stopped (from the
// ring of launch_reduce); the identity list in active, states and step
// counts zero in rstate / riters, and the frame's iteration counters set as
// at a round start (the replay then iterates like a round with gamma 1).
// End: candidate i's row and state back to slot cand[i] of y / state, and
// for a frozen one its FP32 step count (the steps before the replay's
// restart plus the replay's) to iters[cand[i]]; META_REFINE_BAD counts the
// ones not frozen, META_REFINE_DIFF the frozen ones whose replay took
// another number of steps than min(iters, ring_len).
// Gamma cut (one work group per frame): with those step counts, the first
// step t at which more than gamma of the round's meta[META_NSEL] seeds had
// converged -- the early stop of Sec. 3.2.3 taken on FP32 trajectories --
// and every converged slot whose count exceeds t loses its converged state
// (counted in META_GCUT).
hipError_t launch_replay_begin(hipStream_t s, const Batch& b, int dp, int ring_len, const uint8_t* state,
                               const int* iters, const float* ring, int64_t ring_stride, int* cand, float* yr,
                               int* active, uint8_t* rstate, int* riters);
hipError_t launch_replay_end(hipStream_t s, const Batch& b, int dp, int cap, int ring_len, const int* cand,
                             int* iters, const float* yr, const uint8_t* rstate, const int* riters, float* y,
                             uint8_t* state);
hipError_t launch_gamma_cut(hipStream_t s, const Batch& b, double gamma, const int* iters, uint8_t* state);
// Pruning on the device (one work group per frame): ranking and greedy
// suppression.
// Ranking straight from the round's states: the converged slots k <
// meta[META_NSEL] by (count desc, k asc); their number to meta[META_NCAND].
// first (may be null) is set to INT_MAX for every candidate, for
// launch_simbits.
hipError_t launch_rank_converged(hipStream_t s, const Batch& b, const uint8_t* state, const int* counts, int* sorted,
                                 int* scount, int* first = nullptr);
hipError_t launch_greedy(hipStream_t s, const Batch& b, const uint32_t* bits, const float* y, const int* sorted,
                         const int* scount, int ncand_slot, int acc_slot, int dp, float* modes, int* mode_counts,
                         const int* first = nullptr);
// Single frame: append accepted candidates (indices into list) at k0.
hipError_t launch_append_modes(hipStream_t s, int dp, const float* y, const int* list, const int* counts,
                               const int* acc, int a, float* modes, int* mode_counts, int k0);
// Coverage (mode 0: against the frame's new modes [rt.k_modes, rt.k_modes +
// meta[k1_slot])) or labels (mode 1: against modes [0, rt.k_modes)); both
// write META_LEFT (nonzero iff a pixel is left to seed, resp. the number of
// pixels farther than h from every mode).  split: similarities in the split
// form's arithmetic from the BF16 high/low pixel rows xh, xl (x32 unused);
// else FP32 from x32.
hipError_t launch_assign(hipStream_t s, const Batch& b, int dp, bool split, const float* x32, const uint16_t* xh,
                         const uint16_t* xl, const float* modes, int k1_slot, int mode, uint8_t* elig,
                         const int* rank, const int* fg_idx);
// meta[slot] of every frame to rt.nact (from_rt) or to value.
// The counters of every frame (n_words 32-bit words from b.meta on) to host
// memory mapped at dst (device address): data at dst[4..], then seq at dst[0].
hipError_t launch_publish(hipStream_t s, const Batch& b, int n_words, int* dst, int seq);
hipError_t launch_set_slot(hipStream_t s, const Batch& b, int slot, bool from_rt, int value);
// Every frame's label map to -1.
hipError_t launch_fill_labels(hipStream_t s, const Batch& b, int64_t max_pixels);
// p[row0 + k] = k for k < rt.nact of each frame (max_count bounds the grid).
hipError_t launch_iota(hipStream_t s, const Batch& b, int* p, int max_count);
// Frame f's rt.k_modes modes (first dim columns) and counts to the packed
// outputs at row out_off[f] (device array).
hipError_t launch_modes_out(hipStream_t s, const Batch& b, const float* modes, const int* mode_counts, int dp,
                            int dim, const int* out_off, float* out, int* out_counts, int max_rows);
// Adjoint of the unrolled steps (single frame, FP32).
// Rows between the caller's [m][dim] layout and the padded [m_pad][dp] one.
hipError_t launch_rows_in(hipStream_t s, int m, int m_pad, int dim, int dp, const float* src, float* dst);
hipError_t launch_rows_out(hipStream_t s, int m, int dp, int dim, const float* src, float* dst);
// gv = (g - (g . y) y) / |V| per centre, padded to m_pad rows of dp.
hipError_t launch_unroll_gv(hipStream_t s, int m, int m_pad, int dim, int dp, const float* y, const float* vnorm,
                            const float* gy, float* gv);
hipError_t launch_zero_strided(hipStream_t s, int64_t n_pixels, int dim, int64_t ps, int64_t cs, float* out);
// dL/de of the frame's foreground rows from the last step's windows of the
// centres yp (m_pad rows) and their dL/dV (gv), written through the strides.
hipError_t launch_unroll_grad(hipStream_t s, const Batch& b, int dp, const float* x32, const int* fg_idx,
                              const float* enorm, const float* yp, const float* gv, int m_pad, int dim, int64_t ps,
                              int64_t cs, float* grad);
hipError_t launch_lockstep_out(hipStream_t s, int m, int dp, int dim, const float* y, const uint8_t* state,
                               const int* iters, const int* counts_in, float* endpoints, int* iters_out,
                               uint8_t* conv_out, int* counts_out);

}  // namespace fms
