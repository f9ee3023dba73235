// gfx950 kernels of the Faster Mean-shift hot path.
//
// Data layout in HBM (per frame, n foreground pixels, n_pad = 32 * ceil(n/32),
// DP = D padded to 32, 64 or 128, padding rows and columns zero):
//   x32  [n_pad][DP]  FP32 unit rows, raster order of the foreground
//   x32t [n_pad/32][DP][32]  the same values, each 32-pixel block stored
//                    dimension-major, so a lane reads 8 pixels of one
//                    dimension with one 16-byte (BF16) or two (FP32) loads
//   x16, x16t        the same two layouts in BF16
//   y    [slots][DP] FP32 seed centres
//
// The fused step (Eq. 8, 10, 11): for a seed tile Y and a pixel block X it
// forms S^T = X Y^T on MFMA, thresholds it to W = [S >= 1 - h] in registers
// and accumulates V^T += X^T W^T on MFMA.  S^T is computed (pixels as rows) so
// that its accumulator layout (lane (g, r) holds rows 4g..4g+3 of column r) is
// directly the B operand of the second product once the 32 pixels of a block
// are ordered so that k-slot 8g+e of lane group g is pixel 8g+e; the first
// product therefore reads pixel sigma_t(r) = 8(r/4) + 4t + r%4 as row r of
// tile t.  S is never written to memory.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fms_internal.h"

namespace fms {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint16_t to_bf16_bits(float f) {
  return __builtin_bit_cast(uint16_t, (__bf16)f);
}

__device__ __forceinline__ float wave_sum_f(float v, int width) {
  for (int m = width >> 1; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

__device__ __forceinline__ int wave_sum_i(int v) {
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Exclusive scan over a 1024-thread block; returns the prefix, *total gets the sum.
template <int NT>
__device__ __forceinline__ int block_exclusive_scan(int v, int* total, int* sh /* >= NT/64 + 1 ints */) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int incl = v;
  for (int m = 1; m < 64; m <<= 1) {
    int o = __shfl_up(incl, m, 64);
    if (lane >= m) incl += o;
  }
  if (lane == 63) sh[wave] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int w = 0; w < NT / 64; ++w) {
      int t = sh[w];
      sh[w] = run;
      run += t;
    }
    sh[NT / 64] = run;
  }
  __syncthreads();
  int res = sh[wave] + incl - v;
  *total = sh[NT / 64];
  __syncthreads();
  return res;
}

// ------------------------------------------------------------------ compaction

__global__ __launch_bounds__(256) void k_mask_count(const uint8_t* __restrict__ mask, int64_t n_pixels,
                                                    int* __restrict__ block_counts) {
  __shared__ int red[4];
  const int64_t base = (int64_t)blockIdx.x * kMaskBlockPix + threadIdx.x * 4;
  int c = 0;
  for (int e = 0; e < 4; ++e) {
    int64_t p = base + e;
    if (p < n_pixels) c += mask ? (mask[p] != 0) : 1;
  }
  c = wave_sum_i(c);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) block_counts[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// Exclusive scan of the per-block counts in place; total into meta[META_N].
__global__ __launch_bounds__(1024) void k_scan_blocks(int* __restrict__ counts, int nb, int* __restrict__ meta) {
  __shared__ int sh[17];
  int carry = 0;
  for (int base = 0; base < nb; base += 1024) {
    int i = base + threadIdx.x;
    int v = i < nb ? counts[i] : 0;
    int tot;
    int ex = block_exclusive_scan<1024>(v, &tot, sh);
    if (i < nb) counts[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) {
    meta[META_N] = carry;
    meta[META_BAD] = 0;
  }
}

// Gather the foreground rows in raster order, normalise them and write the
// four layouts.  Each thread owns 4 consecutive pixels.
template <int DP>
__global__ __launch_bounds__(256) void k_compact(FrameDesc f, const int* __restrict__ block_offsets,
                                                 int* __restrict__ fg_idx, float* __restrict__ x32,
                                                 float* __restrict__ x32t, uint16_t* __restrict__ x16,
                                                 uint16_t* __restrict__ x16t, int* __restrict__ meta) {
  __shared__ int sh[5];
  const int64_t base = (int64_t)blockIdx.x * kMaskBlockPix + threadIdx.x * 4;
  int flags = 0, c = 0;
  for (int e = 0; e < 4; ++e) {
    int64_t p = base + e;
    bool on = p < f.n_pixels && (f.mask ? (f.mask[p] != 0) : true);
    flags |= (on ? 1 : 0) << e;
    c += on;
  }
  // Block-level exclusive scan (256 threads = 4 waves).
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int incl = c;
  for (int m = 1; m < 64; m <<= 1) {
    int o = __shfl_up(incl, m, 64);
    if (lane >= m) incl += o;
  }
  if (lane == 63) sh[wave] = incl;
  __syncthreads();
  int wpre = 0;
  for (int w = 0; w < wave; ++w) wpre += sh[w];
  int ord = block_offsets[blockIdx.x] + wpre + incl - c;
  int bad = 0;
  for (int e = 0; e < 4; ++e) {
    if (!((flags >> e) & 1)) continue;
    const int64_t p = base + e;
    const float* src = f.emb + p * f.pixel_stride;
    // Scale by a power of two first (exact), so the sum of squares neither
    // overflows nor underflows for any finite non-zero row.
    float mx = 0.f;
    bool finite = true;
    for (int d = 0; d < f.dim; ++d) {
      float v = src[(int64_t)d * f.channel_stride];
      finite = finite && __builtin_isfinite(v);
      mx = fmaxf(mx, fabsf(v));
    }
    float vals[DP];
    float inv = 0.f;
    if (finite && mx > 0.f) {
      int ex;
      frexpf(mx, &ex);
      float ss = 0.f;
      for (int d = 0; d < DP; ++d) {
        float v = d < f.dim ? ldexpf(src[(int64_t)d * f.channel_stride], -ex) : 0.f;
        vals[d] = v;
        ss = fmaf(v, v, ss);
      }
      inv = 1.0f / sqrtf(ss);
    } else {
      bad += 1;
      for (int d = 0; d < DP; ++d) vals[d] = 0.f;
    }
    fg_idx[ord] = (int)p;
    float* rowp = x32 + (int64_t)ord * DP;
    uint16_t* row16 = x16 + (int64_t)ord * DP;
    const int64_t blk = ord / kBlockPix, q = ord % kBlockPix;
    for (int d = 0; d < DP; d += 4) {
      float4 v4 = make_float4(vals[d] * inv, vals[d + 1] * inv, vals[d + 2] * inv, vals[d + 3] * inv);
      *reinterpret_cast<float4*>(rowp + d) = v4;
      x32t[(blk * DP + d + 0) * kBlockPix + q] = v4.x;
      x32t[(blk * DP + d + 1) * kBlockPix + q] = v4.y;
      x32t[(blk * DP + d + 2) * kBlockPix + q] = v4.z;
      x32t[(blk * DP + d + 3) * kBlockPix + q] = v4.w;
      uint16_t b0 = to_bf16_bits(v4.x), b1 = to_bf16_bits(v4.y), b2 = to_bf16_bits(v4.z),
               b3 = to_bf16_bits(v4.w);
      row16[d] = b0;
      row16[d + 1] = b1;
      row16[d + 2] = b2;
      row16[d + 3] = b3;
      x16t[(blk * DP + d + 0) * kBlockPix + q] = b0;
      x16t[(blk * DP + d + 1) * kBlockPix + q] = b1;
      x16t[(blk * DP + d + 2) * kBlockPix + q] = b2;
      x16t[(blk * DP + d + 3) * kBlockPix + q] = b3;
    }
    ++ord;
  }
  if (bad) atomicAdd(meta + META_BAD, bad);
}

// ------------------------------------------------------------------ seed order

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void k_seed_order(int n, int b, uint64_t k0, uint64_t k1, uint64_t k2,
                                                    uint64_t k3, int* __restrict__ order) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  const uint64_t mask = (1ull << b) - 1;
  const uint64_t keys[4] = {k0, k1, k2, k3};
  uint64_t y = (uint64_t)j;
  // Cycle walking: y stays in [0, 2^(2b)); the orbit of j < n returns below n.
  do {
    uint64_t left = y >> b, right = y & mask;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      uint64_t t = left ^ (mix64(right ^ keys[r]) & mask);
      left = right;
      right = t;
    }
    y = (left << b) | right;
  } while (y >= (uint64_t)n);
  order[j] = (int)y;
}

// ------------------------------------------------------------------ seeds

// One 1024-thread block: take the first `want` positions of the seed order
// (from the cursor on) whose pixels are uncovered and unused, mark them used
// and load their vectors as the round's starting centres.
__global__ __launch_bounds__(1024) void k_select(const int* __restrict__ order,
                                                 const uint8_t* __restrict__ uncovered,
                                                 uint8_t* __restrict__ used, int n, int want,
                                                 int* __restrict__ meta, int* __restrict__ seed_pos,
                                                 int* __restrict__ seed_fg, const float* __restrict__ x32,
                                                 int dp, float* __restrict__ y) {
  __shared__ int sh[17];
  __shared__ int s_last;
  __shared__ int s_base;
  if (threadIdx.x == 0) s_base = meta[META_CURSOR];
  __syncthreads();
  int base = s_base;
  int got = 0;
  int new_cursor = n;
  while (got < want && base < n) {
    const int pos = base + (int)threadIdx.x;
    int e = 0, o = -1;
    if (pos < n) {
      o = order[pos];
      e = uncovered[o] && !used[o];
    }
    int tot;
    int rank = block_exclusive_scan<1024>(e, &tot, sh);
    if (e && got + rank < want) {
      seed_pos[got + rank] = pos;
      seed_fg[got + rank] = o;
      if (got + rank == want - 1) s_last = pos;
    }
    __syncthreads();
    if (got + tot >= want) {
      new_cursor = s_last + 1;
      got = want;
    } else {
      got += tot;
      base += 1024;
    }
    __syncthreads();
  }
  // Mark used and load starting centres.
  for (int k = threadIdx.x; k < got * dp; k += 1024) {
    int s = k / dp, d = k - s * dp;
    int o = seed_fg[s];
    y[(int64_t)s * dp + d] = x32[(int64_t)o * dp + d];
    if (d == 0) used[o] = 1;
  }
  if (threadIdx.x == 0) {
    meta[META_NSEL] = got;
    meta[META_CURSOR] = (got < want) ? n : new_cursor;
  }
}

__global__ __launch_bounds__(256) void k_init_seeds(const int* __restrict__ seed_fg, int m, int n,
                                                    const float* __restrict__ x32, int dp,
                                                    float* __restrict__ y, int* __restrict__ meta) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= (int64_t)m * dp) return;
  const int s = (int)(k / dp), d = (int)(k - (int64_t)s * dp);
  const int o = seed_fg[s];
  if (o < 0 || o >= n) {
    if (d == 0) atomicAdd(meta + META_BADSEED, 1);
    y[k] = 0.f;
    return;
  }
  y[k] = x32[(int64_t)o * dp + d];
}

__global__ __launch_bounds__(256) void k_round_init(int m, int* __restrict__ active, uint8_t* __restrict__ state,
                                                    int* __restrict__ iters) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= m) return;
  active[k] = k;
  state[k] = 0;
  iters[k] = 0;
}

// ------------------------------------------------------------------ fused step

// FP32 form.  One wave = one work item (a group of ST x 16 seeds, one pixel
// chunk).  v_mfma_f32_16x16x4_f32: lane (g, r) feeds A[r][g] and B[g][r].
template <int DP, int ST>
__global__ __launch_bounds__(64) void k_shift_f32(const float* __restrict__ x, const float* __restrict__ xt,
                                                  const float* __restrict__ y, const int* __restrict__ active,
                                                  int n_act, int n_blocks, int chunk_blocks, int n_chunks,
                                                  float thr, float* __restrict__ partial) {
  constexpr int KJ = DP / 4;    // dims per lane group = MFMA steps of S
  constexpr int NDB = DP / 16;  // 16-dim blocks of V
  const int lane = threadIdx.x;
  const int g = lane >> 4, r = lane & 15;
  const int grp = blockIdx.x / n_chunks;
  const int chunk = blockIdx.x - grp * n_chunks;
  const int a0 = grp * ST * 16;

  float yb[ST][KJ];
#pragma unroll
  for (int s = 0; s < ST; ++s) {
    const int a = a0 + 16 * s + r;
    if (a < n_act) {
      const float4* yr = reinterpret_cast<const float4*>(y + (int64_t)active[a] * DP + g * KJ);
#pragma unroll
      for (int j = 0; j < KJ / 4; ++j) {
        float4 v = yr[j];
        yb[s][4 * j] = v.x;
        yb[s][4 * j + 1] = v.y;
        yb[s][4 * j + 2] = v.z;
        yb[s][4 * j + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int j = 0; j < KJ; ++j) yb[s][j] = 0.f;
    }
  }
  f32x4 acc[ST][NDB];
#pragma unroll
  for (int s = 0; s < ST; ++s)
#pragma unroll
    for (int db = 0; db < NDB; ++db) acc[s][db] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int b0 = chunk * chunk_blocks;
  const int b1 = min(n_blocks, b0 + chunk_blocks);
  const int rowsel0 = 8 * (r >> 2) + (r & 3);
  for (int b = b0; b < b1; ++b) {
    const float* xb = x + (int64_t)b * kBlockPix * DP;
    float xa[2][KJ];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const float4* xr = reinterpret_cast<const float4*>(xb + (rowsel0 + 4 * t) * DP + g * KJ);
#pragma unroll
      for (int j = 0; j < KJ / 4; ++j) {
        float4 v = xr[j];
        xa[t][4 * j] = v.x;
        xa[t][4 * j + 1] = v.y;
        xa[t][4 * j + 2] = v.z;
        xa[t][4 * j + 3] = v.w;
      }
    }
    float xv[NDB][8];
#pragma unroll
    for (int db = 0; db < NDB; ++db) {
      const float4* tp = reinterpret_cast<const float4*>(xt + ((int64_t)b * DP + 16 * db + r) * kBlockPix + 8 * g);
      float4 u = tp[0], v = tp[1];
      xv[db][0] = u.x; xv[db][1] = u.y; xv[db][2] = u.z; xv[db][3] = u.w;
      xv[db][4] = v.x; xv[db][5] = v.y; xv[db][6] = v.z; xv[db][7] = v.w;
    }
#pragma unroll
    for (int s = 0; s < ST; ++s) {
      f32x4 s0 = {0.f, 0.f, 0.f, 0.f}, s1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int j = 0; j < KJ; ++j) {
        s0 = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[0][j], yb[s][j], s0, 0, 0, 0);
        s1 = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[1][j], yb[s][j], s1, 0, 0, 0);
      }
      float w[8];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        w[i] = s0[i] >= thr ? 1.f : 0.f;
        w[4 + i] = s1[i] >= thr ? 1.f : 0.f;
      }
#pragma unroll
      for (int db = 0; db < NDB; ++db)
#pragma unroll
        for (int e = 0; e < 8; ++e)
          acc[s][db] = __builtin_amdgcn_mfma_f32_16x16x4f32(xv[db][e], w[e], acc[s][db], 0, 0, 0);
    }
  }
#pragma unroll
  for (int s = 0; s < ST; ++s) {
    const int a = a0 + 16 * s + r;
    if (a < n_act) {
      float* dst = partial + ((int64_t)chunk * n_act + a) * DP + 4 * g;
#pragma unroll
      for (int db = 0; db < NDB; ++db) {
        f32x4 v = acc[s][db];
        *reinterpret_cast<float4*>(dst + 16 * db) = make_float4(v[0], v[1], v[2], v[3]);
      }
    }
  }
}

// BF16 form.  v_mfma_f32_16x16x32_bf16: lane (g, r) feeds A[r][8g..8g+7] and
// B[8g..8g+7][r]; FP32 accumulate.  Centres are rounded to BF16 as they load.
template <int DP, int ST>
__global__ __launch_bounds__(64) void k_shift_bf16(const uint16_t* __restrict__ x, const uint16_t* __restrict__ xt,
                                                   const float* __restrict__ y, const int* __restrict__ active,
                                                   int n_act, int n_blocks, int chunk_blocks, int n_chunks,
                                                   float thr, float* __restrict__ partial) {
  constexpr int KS = DP / 32;   // MFMA steps of S (32 dims each)
  constexpr int KJ = DP / 4;    // dims per lane group
  constexpr int NDB = DP / 16;
  const int lane = threadIdx.x;
  const int g = lane >> 4, r = lane & 15;
  const int grp = blockIdx.x / n_chunks;
  const int chunk = blockIdx.x - grp * n_chunks;
  const int a0 = grp * ST * 16;

  bf16x8 yb[ST][KS];
#pragma unroll
  for (int s = 0; s < ST; ++s) {
    const int a = a0 + 16 * s + r;
#pragma unroll
    for (int j = 0; j < KS; ++j) {
      if (a < n_act) {
        const float4* yr = reinterpret_cast<const float4*>(y + (int64_t)active[a] * DP + g * KJ + 8 * j);
        float4 u = yr[0], v = yr[1];
        yb[s][j] = bf16x8{(__bf16)u.x, (__bf16)u.y, (__bf16)u.z, (__bf16)u.w,
                          (__bf16)v.x, (__bf16)v.y, (__bf16)v.z, (__bf16)v.w};
      } else {
        yb[s][j] = bf16x8{(__bf16)0.f, (__bf16)0.f, (__bf16)0.f, (__bf16)0.f,
                          (__bf16)0.f, (__bf16)0.f, (__bf16)0.f, (__bf16)0.f};
      }
    }
  }
  f32x4 acc[ST][NDB];
#pragma unroll
  for (int s = 0; s < ST; ++s)
#pragma unroll
    for (int db = 0; db < NDB; ++db) acc[s][db] = f32x4{0.f, 0.f, 0.f, 0.f};

  const __bf16 one = (__bf16)1.0f, zero = (__bf16)0.0f;
  const int b0 = chunk * chunk_blocks;
  const int b1 = min(n_blocks, b0 + chunk_blocks);
  const int rowsel0 = 8 * (r >> 2) + (r & 3);
  for (int b = b0; b < b1; ++b) {
    const uint16_t* xb = x + (int64_t)b * kBlockPix * DP;
    bf16x8 xa[2][KS];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int j = 0; j < KS; ++j)
        xa[t][j] = *reinterpret_cast<const bf16x8*>(xb + (rowsel0 + 4 * t) * DP + g * KJ + 8 * j);
    bf16x8 xv[NDB];
#pragma unroll
    for (int db = 0; db < NDB; ++db)
      xv[db] = *reinterpret_cast<const bf16x8*>(xt + ((int64_t)b * DP + 16 * db + r) * kBlockPix + 8 * g);
#pragma unroll
    for (int s = 0; s < ST; ++s) {
      f32x4 s0 = {0.f, 0.f, 0.f, 0.f}, s1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int j = 0; j < KS; ++j) {
        s0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa[0][j], yb[s][j], s0, 0, 0, 0);
        s1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa[1][j], yb[s][j], s1, 0, 0, 0);
      }
      bf16x8 w;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        w[i] = s0[i] >= thr ? one : zero;
        w[4 + i] = s1[i] >= thr ? one : zero;
      }
#pragma unroll
      for (int db = 0; db < NDB; ++db)
        acc[s][db] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xv[db], w, acc[s][db], 0, 0, 0);
    }
  }
#pragma unroll
  for (int s = 0; s < ST; ++s) {
    const int a = a0 + 16 * s + r;
    if (a < n_act) {
      float* dst = partial + ((int64_t)chunk * n_act + a) * DP + 4 * g;
#pragma unroll
      for (int db = 0; db < NDB; ++db) {
        f32x4 v = acc[s][db];
        *reinterpret_cast<float4*>(dst + 16 * db) = make_float4(v[0], v[1], v[2], v[3]);
      }
    }
  }
}

// Sum the chunk partials of each active seed in a fixed order, renormalise,
// test convergence (Sec. 3.2.1: cosine distance between consecutive centres
// below tol), and build the next active list.  One wave per seed.
// mode 0: iterate (freeze converged seeds).  mode 1: refine step (no freezing;
// counts moves >= tol).  mode 2: last refine step (same, and counts).
template <int DP>
__global__ __launch_bounds__(256) void k_reduce(const float* __restrict__ partial, int n_chunks, int n_act,
                                                const int* __restrict__ active, float* __restrict__ y,
                                                uint8_t* __restrict__ state, int* __restrict__ iters, float tol,
                                                int mode, int* __restrict__ meta, int* __restrict__ next_active) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int a = blockIdx.x * 4 + wave;
  if (a >= n_act) return;
  const int slot = active[a];
  constexpr int DPL = DP > 64 ? DP / 64 : 1;  // dims per lane
  float v[DPL];
  int width;
  if constexpr (DP == 32) {
    const int d = lane & 31, ph = lane >> 5;
    float acc = 0.f;
    for (int c = ph; c < n_chunks; c += 2) acc += partial[((int64_t)c * n_act + a) * DP + d];
    // Fixed pairing: even-chunk sum + odd-chunk sum, identical in both halves.
    float other = __shfl_xor(acc, 32, 64);
    v[0] = ph == 0 ? acc + other : other + acc;
    width = 32;
  } else {
#pragma unroll
    for (int q = 0; q < DPL; ++q) {
      const int d = lane + 64 * q;
      float acc = 0.f;
      for (int c = 0; c < n_chunks; ++c) acc += partial[((int64_t)c * n_act + a) * DP + d];
      v[q] = acc;
    }
    width = 64;
  }
  float ss = 0.f;
#pragma unroll
  for (int q = 0; q < DPL; ++q) ss = fmaf(v[q], v[q], ss);
  ss = wave_sum_f(ss, width);
  const float nv = sqrtf(ss);
  const bool dead = !(nv > 0.f) || !__builtin_isfinite(nv);
  const float inv = dead ? 0.f : 1.0f / nv;
  float dd = 0.f;
  float yn[DPL];
#pragma unroll
  for (int q = 0; q < DPL; ++q) {
    const int d = (DP == 32) ? (lane & 31) : lane + 64 * q;
    const float yo = y[(int64_t)slot * DP + d];
    yn[q] = v[q] * inv;
    const float df = yo - yn[q];
    dd = fmaf(df, df, dd);
  }
  // 1 - y.y' = |y - y'|^2 / 2 for unit vectors, without cancellation.
  const float delta = 0.5f * wave_sum_f(dd, width);
  if (!dead) {
#pragma unroll
    for (int q = 0; q < DPL; ++q) {
      const int d = (DP == 32) ? (lane & 31) : lane + 64 * q;
      if (DP != 32 || lane < 32) y[(int64_t)slot * DP + d] = yn[q];
    }
  }
  if (lane == 0) {
    if (mode == 0) {
      iters[slot] += 1;
      if (dead) {
        state[slot] = 2;
      } else if (delta < tol) {
        state[slot] = 1;
        atomicAdd(meta + META_NCONV, 1);
      } else {
        next_active[atomicAdd(meta + META_NNEXT, 1)] = slot;
      }
    } else {
      if (dead) state[slot] = 2;
      if (mode == 2 && (dead || !(delta < tol))) atomicAdd(meta + META_REFINE_BAD, 1);
    }
  }
}

// Window counts |{i : y . x_i >= thr}| for the centres in `list`, FP32 MFMA.
template <int DP, int ST>
__global__ __launch_bounds__(64) void k_count(const float* __restrict__ x, const float* __restrict__ y,
                                              const int* __restrict__ list, int m, int n, int n_blocks,
                                              int chunk_blocks, int n_chunks, float thr, int* __restrict__ pcount) {
  constexpr int KJ = DP / 4;
  const int lane = threadIdx.x;
  const int g = lane >> 4, r = lane & 15;
  const int grp = blockIdx.x / n_chunks;
  const int chunk = blockIdx.x - grp * n_chunks;
  const int a0 = grp * ST * 16;
  float yb[ST][KJ];
#pragma unroll
  for (int s = 0; s < ST; ++s) {
    const int a = a0 + 16 * s + r;
#pragma unroll
    for (int j = 0; j < KJ; ++j) yb[s][j] = a < m ? y[(int64_t)list[a] * DP + g * KJ + j] : 0.f;
  }
  int cnt[ST];
#pragma unroll
  for (int s = 0; s < ST; ++s) cnt[s] = 0;
  const int b0 = chunk * chunk_blocks;
  const int b1 = min(n_blocks, b0 + chunk_blocks);
  const int rowsel0 = 8 * (r >> 2) + (r & 3);
  for (int b = b0; b < b1; ++b) {
    const float* xb = x + (int64_t)b * kBlockPix * DP;
    float xa[2][KJ];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int j = 0; j < KJ; ++j) xa[t][j] = xb[(rowsel0 + 4 * t) * DP + g * KJ + j];
    const int pbase = b * kBlockPix + 8 * g;
#pragma unroll
    for (int s = 0; s < ST; ++s) {
      f32x4 s0 = {0.f, 0.f, 0.f, 0.f}, s1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int j = 0; j < KJ; ++j) {
        s0 = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[0][j], yb[s][j], s0, 0, 0, 0);
        s1 = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[1][j], yb[s][j], s1, 0, 0, 0);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        cnt[s] += (s0[i] >= thr && pbase + i < n) ? 1 : 0;
        cnt[s] += (s1[i] >= thr && pbase + 4 + i < n) ? 1 : 0;
      }
    }
  }
#pragma unroll
  for (int s = 0; s < ST; ++s) {
    int c = cnt[s];
    c += __shfl_xor(c, 16, 64);
    c += __shfl_xor(c, 32, 64);
    const int a = a0 + 16 * s + r;
    if (g == 0 && a < m) pcount[(int64_t)chunk * m + a] = c;
  }
}

__global__ __launch_bounds__(256) void k_sum_counts(const int* __restrict__ pcount, int m, int n_chunks,
                                                    int* __restrict__ counts) {
  const int a = blockIdx.x * 256 + threadIdx.x;
  if (a >= m) return;
  int c = 0;
  for (int k = 0; k < n_chunks; ++k) c += pcount[(int64_t)k * m + a];
  counts[a] = c;
}

// Conflict bits: bit k of row j is set when candidate j and candidate k are
// inside each other's window; blocked[j] when an existing mode is.
template <int DP>
__global__ __launch_bounds__(256) void k_conflicts(const float* __restrict__ y, const int* __restrict__ list, int m,
                                                   const float* __restrict__ modes, int k, float thr,
                                                   uint32_t* __restrict__ bits, int words,
                                                   uint8_t* __restrict__ blocked) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t nbits = (int64_t)m * words;
  if (t < nbits) {
    const int j = (int)(t / words), w = (int)(t - (int64_t)j * words);
    const float* yj = y + (int64_t)list[j] * DP;
    uint32_t word = 0;
    for (int b = 0; b < 32; ++b) {
      const int c = 32 * w + b;
      if (c >= m) break;
      const float* yc = y + (int64_t)list[c] * DP;
      float s = 0.f;
      for (int d = 0; d < DP; ++d) s = fmaf(yj[d], yc[d], s);
      if (s >= thr) word |= 1u << b;
    }
    bits[t] = word;
  } else if (t < nbits + m) {
    const int j = (int)(t - nbits);
    const float* yj = y + (int64_t)list[j] * DP;
    uint8_t bl = 0;
    for (int q = 0; q < k && !bl; ++q) {
      float s = 0.f;
      for (int d = 0; d < DP; ++d) s = fmaf(yj[d], modes[(int64_t)q * DP + d], s);
      if (s >= thr) bl = 1;
    }
    blocked[j] = bl;
  }
}

// Append accepted candidates (indices into `list`) to the mode set.
__global__ __launch_bounds__(256) void k_append_modes(int dp, const float* __restrict__ y,
                                                      const int* __restrict__ list, const int* __restrict__ counts,
                                                      const int* __restrict__ acc, int a, float* __restrict__ modes,
                                                      int* __restrict__ mode_counts, int k0) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= a * dp) return;
  const int q = t / dp, d = t - q * dp;
  const int cand = acc[q];
  modes[(int64_t)(k0 + q) * dp + d] = y[(int64_t)list[cand] * dp + d];
  if (d == 0) mode_counts[k0 + q] = counts[cand];
}

// Coverage (mode 0): clear `uncovered` for pixels within h of a mode in
// [k0, k1) and count pixels still uncovered and unused.  Labels (mode 1):
// most similar mode in [k0, k1), lowest index on ties.
template <int DP>
__global__ __launch_bounds__(256) void k_assign(const float* __restrict__ x, int n, const float* __restrict__ modes,
                                                int k0, int k1, float thr, int mode, uint8_t* __restrict__ uncovered,
                                                const uint8_t* __restrict__ used, int* __restrict__ meta,
                                                const int* __restrict__ fg_idx, int* __restrict__ labels) {
  constexpr int KT = 64;
  __shared__ float sm[KT * DP];
  const int i = blockIdx.x * 256 + threadIdx.x;
  float xi[DP];
#pragma unroll
  for (int d = 0; d < DP; d += 4) {
    float4 v = i < n ? *reinterpret_cast<const float4*>(x + (int64_t)i * DP + d) : make_float4(0.f, 0.f, 0.f, 0.f);
    xi[d] = v.x; xi[d + 1] = v.y; xi[d + 2] = v.z; xi[d + 3] = v.w;
  }
  float best = -INFINITY;
  int arg = -1;
  for (int kb = k0; kb < k1; kb += KT) {
    const int cnt = min(KT, k1 - kb);
    __syncthreads();
    for (int e = threadIdx.x; e < cnt * DP; e += 256) sm[e] = modes[(int64_t)kb * DP + e];
    __syncthreads();
    for (int q = 0; q < cnt; ++q) {
      float s = 0.f;
#pragma unroll
      for (int d = 0; d < DP; ++d) s = fmaf(xi[d], sm[q * DP + d], s);
      if (s > best) {
        best = s;
        arg = kb + q;
      }
    }
  }
  if (mode == 0) {
    int left = 0;
    if (i < n) {
      uint8_t u = uncovered[i];
      if (u && best >= thr) {
        uncovered[i] = 0;
        u = 0;
      }
      left = (u && !used[i]) ? 1 : 0;
    }
    left = wave_sum_i(left);
    if ((threadIdx.x & 63) == 0 && left) atomicAdd(meta + META_LEFT, left);
  } else {
    int far = 0;
    if (i < n) {
      labels[fg_idx[i]] = arg;
      far = best < thr ? 1 : 0;
    }
    far = wave_sum_i(far);
    if ((threadIdx.x & 63) == 0 && far) atomicAdd(meta + META_LEFT, far);
  }
}

__global__ __launch_bounds__(256) void k_fill_i32(int* __restrict__ p, int64_t count, int value) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < count) p[i] = value;
}

__global__ __launch_bounds__(256) void k_copy_rows(const float* __restrict__ src, int src_stride,
                                                   float* __restrict__ dst, int dst_stride, int rows, int cols) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)rows * cols) return;
  const int64_t rr = t / cols, c = t - rr * cols;
  dst[rr * dst_stride + c] = src[rr * src_stride + c];
}

__global__ __launch_bounds__(256) void k_lockstep_out(int m, int dp, int dim, const float* __restrict__ y,
                                                      const uint8_t* __restrict__ state,
                                                      const int* __restrict__ iters,
                                                      const int* __restrict__ counts_in,
                                                      float* __restrict__ endpoints, int* __restrict__ iters_out,
                                                      uint8_t* __restrict__ conv_out, int* __restrict__ counts_out) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)m * dim) return;
  const int s = (int)(t / dim), d = (int)(t - (int64_t)s * dim);
  endpoints[t] = y[(int64_t)s * dp + d];
  if (d == 0) {
    iters_out[s] = iters[s];
    conv_out[s] = state[s] == 1 ? 1 : 0;
    if (counts_out) counts_out[s] = state[s] == 1 ? counts_in[s] : -1;
  }
}

// ------------------------------------------------------------------ launchers

static inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

hipError_t launch_mask_count(hipStream_t s, const uint8_t* mask, int64_t n_pixels, int* block_counts,
                             int n_mask_blocks) {
  hipLaunchKernelGGL(k_mask_count, dim3(n_mask_blocks), dim3(256), 0, s, mask, n_pixels, block_counts);
  return hipGetLastError();
}

hipError_t launch_scan_blocks(hipStream_t s, int* block_counts, int n_mask_blocks, int* meta) {
  hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, s, block_counts, n_mask_blocks, meta);
  return hipGetLastError();
}

hipError_t launch_compact(hipStream_t s, const FrameDesc& f, const int* block_offsets, int n_mask_blocks,
                          int* fg_idx, float* x32, float* x32t, uint16_t* x16, uint16_t* x16t, int* meta) {
  switch (f.dp) {
    case 32:
      hipLaunchKernelGGL(k_compact<32>, dim3(n_mask_blocks), dim3(256), 0, s, f, block_offsets, fg_idx, x32, x32t,
                         x16, x16t, meta);
      break;
    case 64:
      hipLaunchKernelGGL(k_compact<64>, dim3(n_mask_blocks), dim3(256), 0, s, f, block_offsets, fg_idx, x32, x32t,
                         x16, x16t, meta);
      break;
    case 128:
      hipLaunchKernelGGL(k_compact<128>, dim3(n_mask_blocks), dim3(256), 0, s, f, block_offsets, fg_idx, x32,
                         x32t, x16, x16t, meta);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_seed_order(hipStream_t s, int n, int half_bits, const uint64_t keys[4], int* order) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_seed_order, dim3(cdiv(n, 256)), dim3(256), 0, s, n, half_bits, keys[0], keys[1], keys[2],
                     keys[3], order);
  return hipGetLastError();
}

hipError_t launch_select(hipStream_t s, const int* order, const uint8_t* uncovered, uint8_t* used, int n, int want,
                         int* meta, int* seed_pos, int* seed_fg, const float* x32, int dp, float* y) {
  hipLaunchKernelGGL(k_select, dim3(1), dim3(1024), 0, s, order, uncovered, used, n, want, meta, seed_pos, seed_fg,
                     x32, dp, y);
  return hipGetLastError();
}

hipError_t launch_init_seeds(hipStream_t s, const int* seed_fg, int m, int n, const float* x32, int dp, float* y,
                             int* meta) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_init_seeds, dim3(cdiv((int64_t)m * dp, 256)), dim3(256), 0, s, seed_fg, m, n, x32, dp, y,
                     meta);
  return hipGetLastError();
}

hipError_t launch_round_init(hipStream_t s, int m, int* active, uint8_t* state, int* iters) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_round_init, dim3(cdiv(m, 256)), dim3(256), 0, s, m, active, state, iters);
  return hipGetLastError();
}

StepGeom make_geom(int n) {
  StepGeom g;
  g.n = n;
  g.n_blocks = (n + kBlockPix - 1) / kBlockPix;
  const int target_chunks = 64;
  g.chunk_blocks = g.n_blocks > 0 ? (g.n_blocks + target_chunks - 1) / target_chunks : 1;
  g.n_chunks = g.n_blocks > 0 ? (g.n_blocks + g.chunk_blocks - 1) / g.chunk_blocks : 0;
  return g;
}

// Seed tiles per wave: enough work items to cover the chip, as few as that
// allows (each wave re-reads its pixel chunk once per 16-seed tile group).
static int pick_st(int n_act, int n_chunks, int dp) {
  const int max_st = dp >= 128 ? 2 : 4;
  for (int st = max_st; st > 1; st >>= 1) {
    const int64_t items = (int64_t)cdiv(n_act, 16 * st) * n_chunks;
    if (items >= 1024) return st;
  }
  return 1;
}

#define FMS_SHIFT_CASE(KERNEL, T, DPV, STV)                                                                   \
  hipLaunchKernelGGL((KERNEL<DPV, STV>), dim3(items), dim3(64), 0, s, static_cast<const T*>(xrm),           \
                     static_cast<const T*>(xt), y, active, n_act, g.n_blocks, g.chunk_blocks, g.n_chunks, thr, \
                     partial)

hipError_t launch_shift(hipStream_t s, bool bf16, int dp, const StepGeom& g, const void* xrm, const void* xt,
                        const float* y, const int* active, int n_act, float thr, float* partial) {
  if (n_act <= 0 || g.n_chunks <= 0) return hipSuccess;
  const int st = pick_st(n_act, g.n_chunks, dp);
  const unsigned items = cdiv(n_act, 16 * st) * g.n_chunks;
  const int key = (bf16 ? 1000 : 0) + dp * 10 + st;
  switch (key) {
    case 321: FMS_SHIFT_CASE(k_shift_f32, float, 32, 1); break;
    case 322: FMS_SHIFT_CASE(k_shift_f32, float, 32, 2); break;
    case 324: FMS_SHIFT_CASE(k_shift_f32, float, 32, 4); break;
    case 641: FMS_SHIFT_CASE(k_shift_f32, float, 64, 1); break;
    case 642: FMS_SHIFT_CASE(k_shift_f32, float, 64, 2); break;
    case 644: FMS_SHIFT_CASE(k_shift_f32, float, 64, 4); break;
    case 1281: FMS_SHIFT_CASE(k_shift_f32, float, 128, 1); break;
    case 1282: FMS_SHIFT_CASE(k_shift_f32, float, 128, 2); break;
    case 1321: FMS_SHIFT_CASE(k_shift_bf16, uint16_t, 32, 1); break;
    case 1322: FMS_SHIFT_CASE(k_shift_bf16, uint16_t, 32, 2); break;
    case 1324: FMS_SHIFT_CASE(k_shift_bf16, uint16_t, 32, 4); break;
    case 1641: FMS_SHIFT_CASE(k_shift_bf16, uint16_t, 64, 1); break;
    case 1642: FMS_SHIFT_CASE(k_shift_bf16, uint16_t, 64, 2); break;
    case 1644: FMS_SHIFT_CASE(k_shift_bf16, uint16_t, 64, 4); break;
    case 2281: FMS_SHIFT_CASE(k_shift_bf16, uint16_t, 128, 1); break;
    case 2282: FMS_SHIFT_CASE(k_shift_bf16, uint16_t, 128, 2); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
#undef FMS_SHIFT_CASE

hipError_t launch_reduce(hipStream_t s, int dp, const StepGeom& g, const float* partial, int n_act, const int* active,
                         float* y, uint8_t* state, int* iters, float tol, int mode, int* meta, int* next_active) {
  if (n_act <= 0) return hipSuccess;
  const dim3 grid(cdiv(n_act, 4)), block(256);
  switch (dp) {
    case 32:
      hipLaunchKernelGGL(k_reduce<32>, grid, block, 0, s, partial, g.n_chunks, n_act, active, y, state, iters, tol,
                         mode, meta, next_active);
      break;
    case 64:
      hipLaunchKernelGGL(k_reduce<64>, grid, block, 0, s, partial, g.n_chunks, n_act, active, y, state, iters, tol,
                         mode, meta, next_active);
      break;
    case 128:
      hipLaunchKernelGGL(k_reduce<128>, grid, block, 0, s, partial, g.n_chunks, n_act, active, y, state, iters, tol,
                         mode, meta, next_active);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_count(hipStream_t s, int dp, const StepGeom& g, const float* x32, const float* y, const int* list,
                        int m, float thr, int* pcount, int* counts) {
  if (m <= 0 || g.n_chunks <= 0) return hipSuccess;
  const unsigned items = cdiv(m, 32) * g.n_chunks;
  switch (dp) {
    case 32:
      hipLaunchKernelGGL((k_count<32, 2>), dim3(items), dim3(64), 0, s, x32, y, list, m, g.n, g.n_blocks,
                         g.chunk_blocks, g.n_chunks, thr, pcount);
      break;
    case 64:
      hipLaunchKernelGGL((k_count<64, 2>), dim3(items), dim3(64), 0, s, x32, y, list, m, g.n, g.n_blocks,
                         g.chunk_blocks, g.n_chunks, thr, pcount);
      break;
    case 128:
      hipLaunchKernelGGL((k_count<128, 2>), dim3(items), dim3(64), 0, s, x32, y, list, m, g.n, g.n_blocks,
                         g.chunk_blocks, g.n_chunks, thr, pcount);
      break;
    default:
      return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_counts, dim3(cdiv(m, 256)), dim3(256), 0, s, pcount, m, g.n_chunks, counts);
  return hipGetLastError();
}

hipError_t launch_conflicts(hipStream_t s, int dp, const float* y, const int* list, int m, const float* modes, int k,
                            float thr, uint32_t* bits, int words, uint8_t* blocked) {
  if (m <= 0) return hipSuccess;
  const dim3 grid(cdiv((int64_t)m * words + m, 256)), block(256);
  switch (dp) {
    case 32:
      hipLaunchKernelGGL(k_conflicts<32>, grid, block, 0, s, y, list, m, modes, k, thr, bits, words, blocked);
      break;
    case 64:
      hipLaunchKernelGGL(k_conflicts<64>, grid, block, 0, s, y, list, m, modes, k, thr, bits, words, blocked);
      break;
    case 128:
      hipLaunchKernelGGL(k_conflicts<128>, grid, block, 0, s, y, list, m, modes, k, thr, bits, words, blocked);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_append_modes(hipStream_t s, int dp, const float* y, const int* list, const int* counts,
                               const int* acc, int a, float* modes, int* mode_counts, int k0) {
  if (a <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_append_modes, dim3(cdiv((int64_t)a * dp, 256)), dim3(256), 0, s, dp, y, list, counts, acc, a,
                     modes, mode_counts, k0);
  return hipGetLastError();
}

hipError_t launch_assign(hipStream_t s, int dp, const float* x32, int n, const float* modes, int k0, int k1, float thr,
                         int mode, uint8_t* uncovered, const uint8_t* used, int* meta, const int* fg_idx,
                         int* labels) {
  if (n <= 0) return hipSuccess;
  const dim3 grid(cdiv(n, 256)), block(256);
  switch (dp) {
    case 32:
      hipLaunchKernelGGL(k_assign<32>, grid, block, 0, s, x32, n, modes, k0, k1, thr, mode, uncovered, used, meta,
                         fg_idx, labels);
      break;
    case 64:
      hipLaunchKernelGGL(k_assign<64>, grid, block, 0, s, x32, n, modes, k0, k1, thr, mode, uncovered, used, meta,
                         fg_idx, labels);
      break;
    case 128:
      hipLaunchKernelGGL(k_assign<128>, grid, block, 0, s, x32, n, modes, k0, k1, thr, mode, uncovered, used, meta,
                         fg_idx, labels);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fill_i32(hipStream_t s, int* p, int64_t count, int value) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(cdiv(count, 256)), dim3(256), 0, s, p, count, value);
  return hipGetLastError();
}

hipError_t launch_copy_rows(hipStream_t s, const float* src, int src_stride, float* dst, int dst_stride, int rows,
                            int cols) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_rows, dim3(cdiv((int64_t)rows * cols, 256)), dim3(256), 0, s, src, src_stride, dst,
                     dst_stride, rows, cols);
  return hipGetLastError();
}

hipError_t launch_lockstep_out(hipStream_t s, int m, int dp, int dim, const float* y, const uint8_t* state,
                               const int* iters, const int* counts_in, float* endpoints, int* iters_out,
                               uint8_t* conv_out, int* counts_out) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lockstep_out, dim3(cdiv((int64_t)m * dim, 256)), dim3(256), 0, s, m, dp, dim, y, state, iters,
                     counts_in, endpoints, iters_out, conv_out, counts_out);
  return hipGetLastError();
}

}  // namespace fms
