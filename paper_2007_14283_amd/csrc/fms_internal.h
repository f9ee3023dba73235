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
  META_NNEXT = 5,      // active seeds for the next iteration
  META_REFINE_BAD = 6, // refine steps whose move stayed >= tol
  META_LEFT = 7,       // foreground pixels neither covered nor used
  META_BADSEED = 8,    // seed indices outside [0, n)
  META_COUNT = 16
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
hipError_t launch_compact(hipStream_t s, const FrameDesc& f, const int* block_offsets, int n_mask_blocks,
                          int* fg_idx, float* x32, float* x32t, uint16_t* x16, uint16_t* x16t,
                          int* meta);
constexpr int kMaskBlockPix = 1024;

hipError_t launch_seed_order(hipStream_t s, int n, int half_bits, const uint64_t keys[4], int* order);

hipError_t launch_select(hipStream_t s, const int* order, const uint8_t* uncovered, uint8_t* used, int n,
                         int want, int* meta, int* seed_pos, int* seed_fg, const float* x32, int dp,
                         float* y);
hipError_t launch_init_seeds(hipStream_t s, const int* seed_fg, int m, int n, const float* x32, int dp,
                             float* y, int* meta);
hipError_t launch_round_init(hipStream_t s, int m, int* active, uint8_t* state, int* iters);

struct StepGeom {
  int n;             // foreground count
  int n_blocks;      // ceil(n / 32)
  int chunk_blocks;  // blocks per pixel chunk (fixed per frame)
  int n_chunks;
};
StepGeom make_geom(int n);

// One fused mean-shift step for the active seeds: partial window sums per chunk.
hipError_t launch_shift(hipStream_t s, bool bf16, int dp, const StepGeom& g, const void* xrm,
                        const void* xt, const float* y, const int* active, int n_act, float thr,
                        float* partial);
// Sum partials, renormalise, convergence test, next active list.
hipError_t launch_reduce(hipStream_t s, int dp, const StepGeom& g, const float* partial, int n_act,
                         const int* active, float* y, uint8_t* state, int* iters, float tol, int mode,
                         int* meta, int* next_active);
// Window counts of the centres listed in `list`.
hipError_t launch_count(hipStream_t s, int dp, const StepGeom& g, const float* x32, const float* y,
                        const int* list, int m, float thr, int* pcount, int* counts);
// Pairwise conflicts among candidates and against existing modes.
hipError_t launch_conflicts(hipStream_t s, int dp, const float* y, const int* list, int m,
                            const float* modes, int k, float thr, uint32_t* bits, int words,
                            uint8_t* blocked);
hipError_t launch_append_modes(hipStream_t s, int dp, const float* y, const int* list, const int* counts,
                               const int* acc, int a, float* modes, int* mode_counts, int k0);
// Coverage (mode = 0) or labels (mode = 1) against modes [k0, k1); both count
// into meta[META_LEFT] (pixels left to seed, resp. farther than h from every mode).
hipError_t launch_assign(hipStream_t s, int dp, const float* x32, int n, const float* modes, int k0,
                         int k1, float thr, int mode, uint8_t* uncovered, const uint8_t* used,
                         int* meta, const int* fg_idx, int* labels);
hipError_t launch_fill_i32(hipStream_t s, int* p, int64_t count, int value);
hipError_t launch_copy_rows(hipStream_t s, const float* src, int src_stride, float* dst, int dst_stride,
                            int rows, int cols);
hipError_t launch_lockstep_out(hipStream_t s, int m, int dp, int dim, const float* y, const uint8_t* state,
                               const int* iters, const int* counts_in, float* endpoints, int* iters_out,
                               uint8_t* conv_out, int* counts_out);

}  // namespace fms
