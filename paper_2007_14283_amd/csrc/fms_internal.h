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
  META_REFINE_BAD = 6, // refine steps whose move stayed >= tol
  META_LEFT = 7,       // foreground pixels still eligible as seeds (coverage), or farther than h from every mode (labels)
  META_BADSEED = 8,    // seed indices outside [0, n)
  META_DONE = 10,      // the round's iteration has stopped
  META_STEPS = 12,     // iterations run this round
  META_NACC = 13,      // modes being refined / modes accepted by the last pruning pass
  META_NCAND = 14,     // converged candidates of the round
  META_ACT = 16,       // two slots (16, 17): active seeds of the even / odd iterations
  META_COUNT = 24
};

// Largest candidate set the single-block rank/greedy kernels take.
constexpr int kRankMax = 8192;

// Work decomposition of the fused step (see plan_chunks in kernels.hip):
// seeds in groups of `group_seeds`, pixels in chunks of whole 32-pixel
// blocks, about `target_items` (group, chunk) items, at most `max_chunks`
// chunks.  Defaults below; fms_params can override them.
constexpr int kTargetItems = 512;
constexpr int kMaxChunks = 256;
struct Tiling {
  int group_seeds;
  int target_items;
  int max_chunks;
};
// The tiling used for a (precision, padded D) pair given the caller's
// requests (0 = default); group sizes round down to a compiled one.
Tiling make_tiling(bool bf16, int dp, int want_seeds, int want_items, int want_chunks);
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

// Compaction and normalisation of the foreground (one pass each).
hipError_t launch_mask_count(hipStream_t s, const uint8_t* mask, int64_t n_pixels, int* block_counts,
                             int n_mask_blocks);
hipError_t launch_scan_blocks(hipStream_t s, int* block_counts, int n_mask_blocks, int* meta);
// Also zeroes the padding rows [n, n_pad) of every layout (n = meta[META_N]).
hipError_t launch_compact(hipStream_t s, const FrameDesc& f, const int* block_offsets, int n_mask_blocks,
                          int* fg_idx, float* x32, float* x32t, uint16_t* x16, uint16_t* x16t,
                          int* meta);
constexpr int kMaskBlockPix = 1024;

// order[j] = foreground ordinal at seed-order position j; rank = its inverse
// (may be null).  With elig (may be null): elig[j] = 1 for j < n and 0 up to
// elig_len, and meta[META_CURSOR] = 0.
hipError_t launch_seed_order(hipStream_t s, int n, int half_bits, const uint64_t keys[4], int* order, int* rank,
                             uint8_t* elig = nullptr, int elig_len = 0, int* meta = nullptr);

hipError_t launch_select(hipStream_t s, const int* order, uint8_t* elig, int n, int want, int* meta, int* seed_pos,
                         int* seed_fg);
hipError_t launch_init_seeds(hipStream_t s, const int* seed_fg, int m, int n, const float* x32, int dp,
                             float* y, int* meta);
// Start of a round's iteration (identity active list, counters); with
// seed_fg (may be null) the centres are also loaded from the pixel rows.
hipError_t launch_round_begin(hipStream_t s, int cap, int* active, uint8_t* state, int* iters, int* meta,
                              unsigned long long* meta64, const int* seed_fg, const float* x32, int dp, float* y);
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
// iter < 0: a plain step whose count is meta[nact_slot] (or the host count).
struct IterCtl {
  int* meta;
  unsigned long long* meta64;
  int nact_slot;
  int iter;
  int n_fg;
  double gamma;
};
// One fused mean-shift step for the active seeds (at most cap): partial
// window sums per pixel chunk.  Centre a is y[active[a]], or y[a] when
// active is null (rows already compacted).  ev0/ev1 (may be null) receive
// the start and end of the kernel itself (hipExtLaunchKernel), not of the
// launch call.
size_t shift_partial_rows(const Tiling& t, int cap);
hipError_t launch_shift(hipStream_t s, bool bf16, int dp, const Tiling& t, int n_blocks, const void* xrm,
                        const void* xt, const float* y, const int* active, const IterCtl& ctl, int cap, float thr,
                        float* partial, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// Sum partials, renormalise, convergence test and (mode 0) the next active
// list and converged count.  yc_next (mode 0, may be null) receives the new
// rows of the seeds that stay active, in next-list order.
hipError_t launch_reduce(hipStream_t s, int dp, int n_blocks, const Tiling& t, const float* partial,
                         const int* active, float* y, uint8_t* state, int* iters, int* next_active,
                         float* yc_next, const IterCtl& ctl, int cap, float tol, int mode);
// Window counts |{i : y[list[a]] . x_i >= thr}| of m centres, on FP32 MFMA
// (xrm = the FP32 rows) or BF16 MFMA (bf16: xrm = the BF16 rows; the centres
// are rounded to BF16); with m_slot >= 0 the count is meta[m_slot] (m is
// then an upper bound).
hipError_t launch_count(hipStream_t s, bool bf16, int dp, const Tiling& t, int n_blocks, int n_pix, const void* xrm,
                        const float* y, const int* list, int m, float thr, int* pcount, int* counts, const int* meta,
                        int m_slot);
// Similarity bits between the rows y[rows[0..m)] and the columns y[cols[c]]
// (or colmat[c]) for c < ncols: row stride simbits_words(ncols) words.  With
// rows_slot / cols_slot >= 0 the counts come from meta (m, ncols are then
// upper bounds that size the grid and the row stride).
int simbits_words(int ncols);
hipError_t launch_simbits(hipStream_t s, int dp, const float* y, const int* rows, int m, const int* cols,
                          const float* colmat, int ncols, float thr, uint32_t* bits, const int* meta, int rows_slot,
                          int cols_slot);
// Pruning on the device: converged list, ranking, greedy suppression.
hipError_t launch_collect(hipStream_t s, const uint8_t* state, int* cand, int* meta);
hipError_t launch_rank(hipStream_t s, const int* cand, const int* counts, const int* meta, int* sorted, int* scount);
hipError_t launch_greedy(hipStream_t s, const uint32_t* bits_c, int words_c, const uint32_t* bits_m, int words_m,
                         int k0, const float* y, const int* sorted, const int* scount, int* meta, int ncand_slot,
                         int acc_slot, int dp, float* modes, int* mode_counts);
hipError_t launch_append_modes(hipStream_t s, int dp, const float* y, const int* list, const int* counts,
                               const int* acc, int a, float* modes, int* mode_counts, int k0);
// Coverage (mode = 0) or labels (mode = 1) against modes [k0, k1); both count
// into meta[META_LEFT] (pixels left to seed, resp. farther than h from every mode).
hipError_t launch_assign(hipStream_t s, int dp, const float* x32, int n, const float* modes, int k0,
                         int k1, int k1_slot, float thr, int mode, uint8_t* elig, const int* rank, int* meta,
                         const int* fg_idx, int* labels);
hipError_t launch_fill_i32(hipStream_t s, int* p, int64_t count, int value);
hipError_t launch_iota(hipStream_t s, int* p, int count);
hipError_t launch_copy_rows(hipStream_t s, const float* src, int src_stride, float* dst, int dst_stride,
                            int rows, int cols);
hipError_t launch_lockstep_out(hipStream_t s, int m, int dp, int dim, const float* y, const uint8_t* state,
                               const int* iters, const int* counts_in, float* endpoints, int* iters_out,
                               uint8_t* conv_out, int* counts_out);

}  // namespace fms
