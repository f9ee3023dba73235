// gfx950 kernels of the Faster Mean-shift hot path.
//
// Data layout in HBM (per frame, n foreground pixels, n_pad = 32 * ceil(n/32),
// DP = D padded to 32, 64 or 128, padding rows and columns zero):
//   x32  [n_pad][DP]  FP32 unit rows, raster order of the foreground
//   x32t [n_pad/32][DP][32]  the same values, each 32-pixel block stored
//                    dimension-major, so a lane reads 8 pixels of one
//                    dimension with two 16-byte loads (FP32 steps only)
//   x16, x16l [n_pad][DP]  BF16 rows: the high part bf16(x) and the low part
//                    bf16(x - hi) (low part for the split form only); BF16
//                    steps transpose each block in LDS instead of reading a
//                    second layout
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
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <climits>
#include <type_traits>

#include "fms_internal.h"

namespace fms {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

// Bit pattern of a float taken by value.  (Bit-casting an element of an
// ext_vector_type in place reads the vector's first element instead.)
__device__ __forceinline__ uint32_t fbits(float f) { return __builtin_bit_cast(uint32_t, f); }

__device__ __forceinline__ uint16_t to_bf16_bits(float f) {
  return __builtin_bit_cast(uint16_t, (__bf16)f);
}
// Low BF16 part of f given its high part (bits hi): round(f - hi).  With the
// high part, it holds f to a relative 2^-16.
__device__ __forceinline__ uint16_t low_bf16_bits(float f, uint16_t hi) {
  return to_bf16_bits(f - __uint_as_float((uint32_t)hi << 16));
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

__global__ __launch_bounds__(256) void k_mask_count(const FrameGeo* __restrict__ geo, int* __restrict__ block_counts) {
  __shared__ int red[4];
  const FrameGeo& g = geo[blockIdx.y];
  const uint8_t* mask = g.desc.mask;
  const int64_t n_pixels = g.desc.n_pixels;
  if ((int64_t)blockIdx.x * kMaskBlockPix >= n_pixels) return;
  block_counts += g.mblk0;
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

// Exclusive scan of a frame's per-block counts in place; total into
// meta[META_N] (one work group per frame).
__global__ __launch_bounds__(1024) void k_scan_blocks(const FrameGeo* __restrict__ geo, int* __restrict__ counts,
                                                      int* __restrict__ meta) {
  __shared__ int sh[17];
  const FrameGeo& g = geo[blockIdx.x];
  const int nb = (int)((g.desc.n_pixels + kMaskBlockPix - 1) / kMaskBlockPix);
  counts += g.mblk0;
  meta += (int64_t)blockIdx.x * META_COUNT;
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
// row layouts (FP32, and the BF16 high and low parts when asked; k_transpose
// then writes the FP32 dimension-major copy when FP32 steps need it).  A
// work group takes kMaskBlockPix pixels: each thread owns 4
// consecutive pixels for the mask scan, the foreground pixels of the block go
// to an LDS list in raster order, and then 8 lanes take each listed pixel
// (lane q holds dimensions KD*q .. KD*q+KD-1), so a row is read and written
// with consecutive addresses whatever the strides.
template <int DP>
__global__ __launch_bounds__(256) void k_compact(const FrameGeo* __restrict__ geo,
                                                 const int* __restrict__ block_offsets, int* __restrict__ fg_idx,
                                                 float* __restrict__ x32, uint16_t* __restrict__ x16,
                                                 uint16_t* __restrict__ xlo, float* __restrict__ enorm,
                                                 int* __restrict__ meta, int64_t row_cap) {
  constexpr int KD = DP / 8;  // dimensions per lane
  __shared__ int sh[5];
  __shared__ int lp[kMaskBlockPix];
  const FrameGeo& gf = geo[blockIdx.y];
  const FrameDesc f = gf.desc;
  if ((int64_t)blockIdx.x * kMaskBlockPix >= f.n_pixels) return;
  block_offsets += gf.mblk0;
  fg_idx += gf.row0;
  if (enorm) enorm += gf.row0;
  x32 += gf.row0 * DP;
  if (x16) x16 += gf.row0 * DP;
  if (xlo) xlo += gf.row0 * DP;
  meta += (int64_t)blockIdx.y * META_COUNT;
  const int64_t blk0 = (int64_t)blockIdx.x * kMaskBlockPix;
  const int64_t base = blk0 + threadIdx.x * 4;
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
  const int total = sh[0] + sh[1] + sh[2] + sh[3];
  int local = wpre + incl - c;
  for (int e = 0; e < 4; ++e)
    if ((flags >> e) & 1) lp[local++] = (int)(threadIdx.x * 4 + e);
  const int ord0 = block_offsets[blockIdx.x];
  __syncthreads();
  int bad = 0;
  const int q = lane & 7;
  // U pixels per 8-lane group per pass, their loads issued together (one
  // pixel at a time leaves a work group waiting on one load chain after
  // another).  Positions past the list or past row_cap load the group's
  // first pixel again and are not written.
  constexpr int U = 4;
  // Pixel-major rows of whole 16-byte words (the usual H x W x D layout with
  // D a multiple of 4) are read with 16-byte loads.
  const bool vec = f.channel_stride == 1 && f.pixel_stride % 4 == 0 && f.dim % 4 == 0 &&
                   (reinterpret_cast<uintptr_t>(f.emb) & 15) == 0;
  for (int k0 = (int)threadIdx.x / 8; k0 < total; k0 += 32 * U) {
    float v[U][KD];
    int64_t pix[U];
    bool live[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + 32 * u;
      live[u] = k < total && ord0 + k < row_cap;  // beyond the layouts' rows: the caller reports it
      pix[u] = blk0 + lp[live[u] ? k : k0];
      const float* src = f.emb + pix[u] * f.pixel_stride;
      if (vec) {
#pragma unroll
        for (int j = 0; j < KD; j += 4) {
          const int d = KD * q + j;
          const float4 w = d < f.dim ? *reinterpret_cast<const float4*>(src + d) : make_float4(0.f, 0.f, 0.f, 0.f);
          v[u][j] = w.x;
          v[u][j + 1] = w.y;
          v[u][j + 2] = w.z;
          v[u][j + 3] = w.w;
        }
      } else {
#pragma unroll
        for (int j = 0; j < KD; ++j) {
          const int d = KD * q + j;
          v[u][j] = d < f.dim ? src[(int64_t)d * f.channel_stride] : 0.f;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int ord = ord0 + k0 + 32 * u;
      float mx = 0.f;
      bool finite = true;
#pragma unroll
      for (int j = 0; j < KD; ++j) {
        finite = finite && __builtin_isfinite(v[u][j]);
        mx = fmaxf(mx, fabsf(v[u][j]));
      }
      // The 8 lanes of the pixel agree on the largest magnitude and on
      // finiteness; the row is scaled by a power of two first (exact), so the
      // sum of squares neither overflows nor underflows.
#pragma unroll
      for (int m = 1; m < 8; m <<= 1) {
        mx = fmaxf(mx, __shfl_xor(mx, m, 64));
        finite = (__shfl_xor(finite ? 1 : 0, m, 64) != 0) && finite;
      }
      const bool ok = finite && mx > 0.f;
      int ex = 0;
      if (ok) frexpf(mx, &ex);
      float ss = 0.f;
#pragma unroll
      for (int j = 0; j < KD; ++j) {
        v[u][j] = ok ? ldexpf(v[u][j], -ex) : 0.f;
        ss = fmaf(v[u][j], v[u][j], ss);
      }
#pragma unroll
      for (int m = 1; m < 8; m <<= 1) ss += __shfl_xor(ss, m, 64);
      if (!live[u]) continue;
      const float inv = ok ? 1.0f / sqrtf(ss) : 0.f;
      if (q == 0) {
        bad += ok ? 0 : 1;
        fg_idx[ord] = (int)pix[u];
        if (enorm) enorm[ord] = ok ? ldexpf(sqrtf(ss), ex) : 0.f;  // |e| of the raw row
      }
      float* rowp = x32 + (int64_t)ord * DP + KD * q;
#pragma unroll
      for (int j = 0; j < KD; j += 4) {
        const float4 v4 = make_float4(v[u][j] * inv, v[u][j + 1] * inv, v[u][j + 2] * inv, v[u][j + 3] * inv);
        *reinterpret_cast<float4*>(rowp + j) = v4;
        if (!x16) continue;
        const int d = KD * q + j;
        const uint16_t b0 = to_bf16_bits(v4.x), b1 = to_bf16_bits(v4.y), b2 = to_bf16_bits(v4.z),
                       b3 = to_bf16_bits(v4.w);
        *reinterpret_cast<uint2*>(x16 + (int64_t)ord * DP + d) =
            make_uint2((uint32_t)b0 | ((uint32_t)b1 << 16), (uint32_t)b2 | ((uint32_t)b3 << 16));
        if (!xlo) continue;
        // Low parts: the BF16 rounding of what the high part leaves.
        const uint16_t l0 = low_bf16_bits(v4.x, b0), l1 = low_bf16_bits(v4.y, b1), l2 = low_bf16_bits(v4.z, b2),
                       l3 = low_bf16_bits(v4.w, b3);
        *reinterpret_cast<uint2*>(xlo + (int64_t)ord * DP + d) =
            make_uint2((uint32_t)l0 | ((uint32_t)l1 << 16), (uint32_t)l2 | ((uint32_t)l3 << 16));
      }
    }
  }
  bad = wave_sum_i(bad);
  bad = lane == 0 ? bad : 0;
  if (bad) atomicAdd(meta + META_BAD, bad);
  // The rows from n up to the next multiple of 32 are padding: zero in every
  // row layout (and so in the transposed ones), so they add nothing to any
  // sum.
  if (blockIdx.x == 0 && meta[META_N] < row_cap) {
    const int n = meta[META_N];
    const int pad = (kBlockPix - n % kBlockPix) % kBlockPix;
    for (int e = threadIdx.x; e < pad * DP; e += 256) {
      const int64_t row = n + e / DP, d = e % DP;
      x32[row * DP + d] = 0.f;
      if (x16) x16[row * DP + d] = 0;
      if (xlo) xlo[row * DP + d] = 0;
    }
  }
}

// The FP32 dimension-major copy of every 32-pixel block (x32t), from the
// rows k_compact wrote: one wave per block stages the block's 32 x DP values
// in LDS with 16-byte row loads and writes the transposed block, a
// contiguous 32 * DP values, with 16-byte stores.  The block count follows
// meta[META_N] (nothing when it exceeds row_cap).
template <int DP>
__global__ __launch_bounds__(64) void k_transpose(const FrameGeo* __restrict__ geo, const float* __restrict__ x32,
                                                  float* __restrict__ x32t, const int* __restrict__ meta,
                                                  int64_t row_cap) {
  constexpr int E = kBlockPix * DP;  // values per block
  __shared__ float tile[kBlockPix][DP + 1];
  const FrameGeo& gf = geo[blockIdx.y];
  const int n = meta[(int64_t)blockIdx.y * META_COUNT + META_N];
  if (n > row_cap) return;
  const int blk = (int)blockIdx.x;
  if (blk * kBlockPix >= n) return;
  const int64_t base = (gf.row0 + (int64_t)blk * kBlockPix) * DP;  // same offset in every layout
  const int lane = threadIdx.x;
#pragma unroll
  for (int i = 0; i < E / 256; ++i) {
    const int e = 4 * lane + 256 * i;
    const float4 u = *reinterpret_cast<const float4*>(x32 + base + e);
    const int r = e / DP, c = e % DP;
    tile[r][c] = u.x;
    tile[r][c + 1] = u.y;
    tile[r][c + 2] = u.z;
    tile[r][c + 3] = u.w;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < E / 256; ++i) {
    const int o = 4 * lane + 256 * i;  // transposed index: dimension o / 32, pixels o % 32 .. + 3
    const int d = o / kBlockPix, p = o % kBlockPix;
    const float4 v = make_float4(tile[p][d], tile[p + 1][d], tile[p + 2][d], tile[p + 3][d]);
    *reinterpret_cast<float4*>(x32t + base + o) = v;
  }
}

// ------------------------------------------------------------------ seed order

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void k_seed_order(const FrameGeo* __restrict__ geo, int n, int b, uint64_t k0,
                                                    uint64_t k1, uint64_t k2, uint64_t k3, int* __restrict__ order,
                                                    int* __restrict__ rank, uint8_t* __restrict__ elig,
                                                    int* __restrict__ meta) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (geo) {
    // Start of a frame's seeding: every position eligible, the tail padding
    // not, the cursor at 0.
    const FrameGeo& g = geo[blockIdx.y];
    n = g.n;
    b = g.half_bits;
    order += g.row0;
    rank += g.row0;
    elig += g.elig0;
    meta += (int64_t)blockIdx.y * META_COUNT;
    if (j < elig_len(n)) elig[j] = j < n ? 1 : 0;
    if (j == 0) meta[META_CURSOR] = 0;
  }
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
  if (geo) rank[y] = j;
}

// ------------------------------------------------------------------ seeds

// One 1024-thread block: take the first `want` positions of the seed order
// (from the cursor on) that are still eligible (elig[pos] = 1: the pixel is
// neither covered by a mode nor used as a seed) and clear them; their
// vectors are loaded by the round's first kernel.  Each pass reads RUN = 16
// consecutive eligibility bytes per thread in 16-byte loads (16384 positions
// per pass; 64 per thread measured slower on the 512x512 frame, whose first
// rounds need one pass).  Positions before the cursor are all ineligible, so
// a pass may start at the cursor rounded down to RUN; `elig` is zero-padded
// to a multiple of 16, and a 16-byte word is read only when it starts below
// n.
__global__ __launch_bounds__(1024) void k_select(Batch bt, const int* __restrict__ order, uint8_t* __restrict__ elig,
                                                 int* __restrict__ seed_pos, int* __restrict__ seed_fg) {
  constexpr int RUN = 16;
  __shared__ int sh[17];
  __shared__ int s_last;
  __shared__ int s_base;
  const FrameGeo& g = bt.geo[blockIdx.x];
  const int n = g.n, want = round_tab(bt, blockIdx.x).want;
  order += g.row0;
  elig += g.elig0;
  seed_pos += g.row0;
  seed_fg += g.row0;
  int* meta = bt.meta + (int64_t)blockIdx.x * META_COUNT;
  if (threadIdx.x == 0) s_base = meta[META_CURSOR] & ~(RUN - 1);
  __syncthreads();
  int base = s_base;
  int got = 0;
  int new_cursor = n;
  while (got < want && base < n) {
    const int p0 = base + (int)threadIdx.x * RUN;
    uint32_t ew[RUN / 4];
#pragma unroll
    for (int w = 0; w < RUN / 16; ++w) {
      uint4 e4 = make_uint4(0u, 0u, 0u, 0u);
      if (p0 + 16 * w < n) e4 = *reinterpret_cast<const uint4*>(elig + p0 + 16 * w);
      ew[4 * w] = e4.x;
      ew[4 * w + 1] = e4.y;
      ew[4 * w + 2] = e4.z;
      ew[4 * w + 3] = e4.w;
    }
    int cnt = 0;
#pragma unroll
    for (int w = 0; w < RUN / 4; ++w) cnt += __popc(ew[w]);
    int tot;
    int rank = block_exclusive_scan<1024>(cnt, &tot, sh);
    if (cnt && got + rank < want) {
#pragma unroll
      for (int k = 0; k < RUN; ++k) {
        if ((ew[k >> 2] >> (8 * (k & 3))) & 1u) {
          const int q = got + rank;
          if (q < want) {
            const int pos = p0 + k;
            seed_pos[q] = pos;
            seed_fg[q] = order[pos];
            elig[pos] = 0;
            if (q == want - 1) s_last = pos;
          }
          ++rank;
        }
      }
    }
    __syncthreads();
    if (got + tot >= want) {
      new_cursor = s_last + 1;
      got = want;
    } else {
      got += tot;
      base += 1024 * RUN;
    }
    __syncthreads();
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
  if (n < 0) n = meta[META_N];
  const int s = (int)(k / dp), d = (int)(k - (int64_t)s * dp);
  const int o = seed_fg[s];
  if (o < 0 || o >= n) {
    if (d == 0) atomicAdd(meta + META_BADSEED, 1);
    y[k] = 0.f;
    return;
  }
  y[k] = x32[(int64_t)o * dp + d];
}


// Tables and counters of a single-frame call whose buffers the caller does
// not allocate: the frame's table and round table are written from kernel
// arguments (no host staging), and its counters are cleared with stores.
__global__ __launch_bounds__(64) void k_set_tables(FrameGeo g, RoundTab rt, FrameGeo* __restrict__ geo,
                                                  RoundTab* __restrict__ rtab, int* __restrict__ meta,
                                                  unsigned long long* __restrict__ meta64) {
  if (threadIdx.x == 0) {
    *geo = g;
    *rtab = rt;
  }
  for (int i = threadIdx.x; i < META_COUNT; i += 64) meta[i] = 0;
  for (int i = threadIdx.x; i < kMeta64; i += 64) meta64[i] = 0ull;
}

// After the mask scan of such a call: the frame's foreground count and block
// count into its table.  A count above row_cap (the rows the layouts hold)
// leaves the frame empty for every later kernel: the table and META_N take
// 0 and META_OVERCAP the count.
__global__ __launch_bounds__(64) void k_geo_from_count(Batch bt, int64_t row_cap) {
  if (threadIdx.x != 0) return;
  FrameGeo* g = const_cast<FrameGeo*>(bt.geo);
  int* meta = bt.meta;
  const int n = meta[META_N];
  const int m = n <= row_cap ? n : 0;
  if (m != n) {
    meta[META_OVERCAP] = n;
    meta[META_N] = 0;
  }
  g->n = m;
  g->n_blocks = (m + kBlockPix - 1) / kBlockPix;
}

// ------------------------------------------------------------------ fused step

// Eight BF16 values of one dimension for eight consecutive pixels, read from
// a block staged in LDS pixel-major with ds_read_b64_tr_b16 (two reads of
// four).  Within each 16-lane group, lane i of such a read receives element
// i % 4 of the 8 bytes that lanes 4e + i / 4 (e = 0..3) address; so when lane
// r of group g addresses row p0 + (r >> 2), columns c0 + 4 (r & 3) .. + 3,
// it receives rows p0 .. p0 + 3 of column c0 + r.
__device__ __forceinline__ bf16x8 lds_tr_b16x8(const uint16_t* p0, const uint16_t* p1) {
#if defined(__HIP_DEVICE_COMPILE__)
  typedef short s16x4 __attribute__((ext_vector_type(4)));
  typedef short s16x8 __attribute__((ext_vector_type(8)));
  const s16x4 a = __builtin_amdgcn_ds_read_tr16_b64_v4i16((s16x4*)p0);
  const s16x4 b = __builtin_amdgcn_ds_read_tr16_b64_v4i16((s16x4*)p1);
  const s16x8 v = __builtin_shufflevector(a, b, 0, 1, 2, 3, 4, 5, 6, 7);
  return __builtin_bit_cast(bf16x8, v);
#else
  (void)p0;
  (void)p1;
  return bf16x8{};
#endif
}

// Work plan of one fused step: seeds in groups of 16*ST, pixels in chunks of
// whole 32-pixel blocks, about target_items (group, chunk) items in total.
// The kernels derive it from the active count held on the device; the host
// uses the same function with upper bounds to size the partial buffer.
// The grid holds target_items work groups, so up to a quarter of that many
// groups the chunk count rounds down: every item then runs in the grid's one
// pass, where rounding up would leave a few items for a second pass that
// the rest of the grid waits for.  Beyond, rounding down would idle up to
// half the grid, and the count rounds up.
__host__ __device__ inline ChunkPlan plan_chunks(int n_act, const Tiling& t, int n_blocks) {
  ChunkPlan cp;
  const int groups = n_act > 0 ? (n_act + t.group_seeds - 1) / t.group_seeds : 1;
  int want = 4 * groups <= t.target_items ? t.target_items / groups : (t.target_items + groups - 1) / groups;
  int lim = n_blocks < t.max_chunks ? n_blocks : t.max_chunks;
  if (lim < 1) lim = 1;
  int nc = want < 1 ? 1 : (want > lim ? lim : want);
  const int cb = n_blocks > 0 ? (n_blocks + nc - 1) / nc : 1;
  nc = n_blocks > 0 ? (n_blocks + cb - 1) / cb : 1;
  cp.groups = groups;
  cp.n_chunks = nc;
  cp.chunk_blocks = cb;
  return cp;
}

// Blocks per wave from which a step's waves load their pixel blocks
// unconditionally (see shift_body).
constexpr int kDeepBlocks = 8;

// The fused mean-shift step (Eq. 8, 10, 11) for the active seeds.
//
// Work group = WV waves = one item: a group of 16*ST seeds and one pixel
// chunk.  The waves share the seeds and take every WV-th block of the chunk
// (a wide group leaves each wave few blocks, so few dependent loads); their
// window sums are added in LDS by a fixed-order tree and written as the
// item's partial sum.  Items are spread over the XCDs so that the work groups of
// one XCD walk through neighbouring items (same chunk, different seed groups)
// and share that chunk in their L2.
//
// The MFMA accumulator of S^T starts at -thr, so S - thr comes out of the
// matrix core and the window test is a sign test.  FP32 form:
// v_mfma_f32_16x16x4_f32 (lane (g, r) feeds A[r][g], B[g][r]).  BF16 form:
// v_mfma_f32_16x16x32_bf16 (lane (g, r) feeds A[r][8g..8g+7], B[8g..8g+7][r]),
// FP32 accumulation; the 0/1 weights of two pixels are packed into one BF16
// pair with one v_perm_b32 (sign bytes) and one bit-select.
//
// SPLIT form (with BF16): every value v -- pixel vectors and centres -- is
// held as a high and a low BF16 part, hi = bf16(v), lo = bf16(v - hi), which
// together keep v to a relative 2^-16.  S^T takes three products per tile
// (hi.hi + hi.lo + lo.hi; lo.lo is below 2^-16) and V^T two (the 0/1 weights
// are exact in BF16), all on BF16 MFMA with FP32 accumulation: a similarity
// is off by at most 3 * 2^-16 (under 5e-5) for unit vectors, against 2^-8 for
// the plain BF16 form.
//
// COUNT form: the same S^T tiles, no second product; each item writes the
// per-seed number of its pixels inside the window (window counts at the
// centres, used to rank candidate modes).
template <bool BF16, bool SPLIT, bool COUNT, int DP, int ST, int WV>
__device__ __forceinline__ void shift_body(const void* __restrict__ xrm_, const void* __restrict__ xt_,
                                           const uint16_t* __restrict__ xrl, const float* __restrict__ y,
                                           const int* __restrict__ active, int n_act,
                                           const Tiling& tl, int n_blocks, int n_pix, float thr,
                                           float* __restrict__ partial, int* __restrict__ pcount, int wg, int nwg) {
  constexpr int KJ = DP / 4;     // dimensions held per lane group
  constexpr int KS = BF16 ? DP / 32 : DP / 4;  // MFMA steps of S per 16x16 tile
  constexpr int NDB = DP / 16;   // 16-dimension blocks of V
  // Register buffers of pixel blocks: up to PD - 1 blocks are in flight while
  // one computes.  Sixteen-wave groups (128 registers per lane) and the
  // largest seed groups keep two.
  constexpr int PD = (DP == 32 && WV < 16) ? ((BF16 && !SPLIT) ? (ST >= 8 ? 3 : 4) : (ST >= 8 ? 2 : 3)) : 2;
  typedef typename std::conditional<BF16, uint16_t, float>::type T;
  typedef typename std::conditional<BF16, bf16x8, float>::type AOp;
  const T* __restrict__ xrm = static_cast<const T*>(xrm_);
  const T* __restrict__ xt = static_cast<const T*>(xt_);

  const ChunkPlan cp = plan_chunks(n_act, tl, n_blocks);
  const int items = cp.groups * cp.n_chunks;

  // BF16 steps read only the row layout: each wave stages its block (high,
  // and low parts for the split form) pixel-major in its own LDS area and
  // reads the dimension-major operand of V back with transposing reads.  The
  // staging areas share LDS with the waves' tree sum, which starts after a
  // barrier.  A staged row's 16-byte chunks are permuted, chunk q of pixel p
  // stored at q ^ swz(p), swz(p) = 2 ((p >> 3) mod DP/16): a transposing
  // read then spreads its 16 rows (4 per 8-pixel group) over all banks, and
  // so does a row store (at D = 32).
  constexpr bool STAGE = BF16 && !COUNT;
  constexpr int STAGE_ELEMS = kBlockPix * DP;
  constexpr int STAGE_BYTES = STAGE ? WV * (SPLIT ? 2 : 1) * STAGE_ELEMS * 2 : 0;
  typedef f32x4 RedT[COUNT ? 1 : WV / 2][ST][COUNT ? 1 : NDB][64];
  constexpr int LDS_BYTES = STAGE_BYTES > (int)sizeof(RedT) ? STAGE_BYTES : (int)sizeof(RedT);
  __shared__ __align__(16) unsigned char lds_raw[LDS_BYTES];
  RedT& red = *reinterpret_cast<RedT*>(lds_raw);
  __shared__ int redc[COUNT ? WV - 1 : 1][ST][16];
  // The wave index is uniform within a wave: in a scalar register, the
  // block loop's tests are scalar branches.
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint16_t* const stage = reinterpret_cast<uint16_t*>(lds_raw) + (STAGE ? wave * (SPLIT ? 2 : 1) * STAGE_ELEMS : 0);
  auto swz = [](int p) { return 2 * ((p >> 3) & (DP / 16 - 1)); };
  const int g = lane >> 4, r = lane & 15;
  const int rowsel0 = 8 * (r >> 2) + (r & 3);
  const f32x4 cinit = {-thr, -thr, -thr, -thr};

  // nwg is a multiple of 8: work group wg runs on XCD wg % 8 (round-robin
  // dispatch), and each XCD owns one contiguous eighth of the items.
  const int xcd = wg & 7, per = nwg >> 3;
  const int lo = (int)((int64_t)items * xcd / 8), hi = (int)((int64_t)items * (xcd + 1) / 8);
  for (int it = lo + (wg >> 3); it < hi; it += per) {
    const int chunk = it / cp.groups, grp = it - chunk * cp.groups;
    const int b0 = chunk * cp.chunk_blocks;
    const int b1 = min(n_blocks, b0 + cp.chunk_blocks);
    // Register operands of one block, in PD buffers: rows for S (two 16-pixel
    // tiles) and, for FP32 steps, the dimension-major copy for V.
    AOp xa[PD][2][KS];
    float xv[BF16 ? 1 : PD][NDB][8];
    // Low parts of the split form (unused otherwise).
    bf16x8 xal[PD][2][SPLIT ? KS : 1];
    auto load = [&](int buf, int b) {
      if constexpr (BF16) {
        const int64_t o = (int64_t)b * kBlockPix * DP;
        const uint16_t* xb = reinterpret_cast<const uint16_t*>(xrm) + o;
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
          for (int j = 0; j < KS; ++j) {
            xa[buf][t][j] = *reinterpret_cast<const bf16x8*>(xb + (rowsel0 + 4 * t) * DP + g * KJ + 8 * j);
            if constexpr (SPLIT)
              xal[buf][t][j] = *reinterpret_cast<const bf16x8*>(xrl + o + (rowsel0 + 4 * t) * DP + g * KJ + 8 * j);
          }
      } else {
        const float* xb = reinterpret_cast<const float*>(xrm) + (int64_t)b * kBlockPix * DP;
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const float4* xr = reinterpret_cast<const float4*>(xb + (rowsel0 + 4 * t) * DP + g * KJ);
#pragma unroll
          for (int j = 0; j < KJ / 4; ++j) {
            float4 u = xr[j];
            xa[buf][t][4 * j] = u.x;
            xa[buf][t][4 * j + 1] = u.y;
            xa[buf][t][4 * j + 2] = u.z;
            xa[buf][t][4 * j + 3] = u.w;
          }
        }
#pragma unroll
        for (int db = 0; db < (COUNT ? 0 : NDB); ++db) {
          const float4* tp = reinterpret_cast<const float4*>(reinterpret_cast<const float*>(xt) +
                                                             ((int64_t)b * DP + 16 * db + r) * kBlockPix + 8 * g);
          float4 u = tp[0], v = tp[1];
          xv[buf][db][0] = u.x; xv[buf][db][1] = u.y; xv[buf][db][2] = u.z; xv[buf][db][3] = u.w;
          xv[buf][db][4] = v.x; xv[buf][db][5] = v.y; xv[buf][db][6] = v.z; xv[buf][db][7] = v.w;
        }
      }
    };
    int b = b0 + wave;
    const int a0 = grp * 16 * ST;
    // Seed operands (B of S^T = X Y^T); low parts for the split form.
    AOp yb[ST][KS];
    bf16x8 ybl[ST][SPLIT ? KS : 1];
    // Every lane loads: positions past the active count take the last
    // active seed (n_act >= 1 here) and are zeroed after the loads, so no
    // load sits behind a branch and all of them are in flight together (a
    // branch per load makes the wave wait for each in turn).
    auto load_seeds = [&]() {
      int idx[ST];
#pragma unroll
      for (int s = 0; s < ST; ++s) {
        const int a = min(a0 + 16 * s + r, n_act - 1);
        idx[s] = active ? active[a] : a;
      }
      float4 raw[ST][KJ / 4];
#pragma unroll
      for (int s = 0; s < ST; ++s) {
        const float4* yr = reinterpret_cast<const float4*>(y + (int64_t)idx[s] * DP + g * KJ);
#pragma unroll
        for (int j = 0; j < KJ / 4; ++j) raw[s][j] = yr[j];
      }
#pragma unroll
      for (int s = 0; s < ST; ++s) {
        const bool ok = a0 + 16 * s + r < n_act;
        float e[KJ];
#pragma unroll
        for (int j = 0; j < KJ / 4; ++j) {
          e[4 * j] = ok ? raw[s][j].x : 0.f;
          e[4 * j + 1] = ok ? raw[s][j].y : 0.f;
          e[4 * j + 2] = ok ? raw[s][j].z : 0.f;
          e[4 * j + 3] = ok ? raw[s][j].w : 0.f;
        }
        if constexpr (BF16) {
#pragma unroll
          for (int j = 0; j < KS; ++j) {
            __bf16 hi[8], lo[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
              hi[i] = (__bf16)e[8 * j + i];
              lo[i] = (__bf16)(e[8 * j + i] - (float)hi[i]);
            }
            yb[s][j] = bf16x8{hi[0], hi[1], hi[2], hi[3], hi[4], hi[5], hi[6], hi[7]};
            if constexpr (SPLIT) ybl[s][j] = bf16x8{lo[0], lo[1], lo[2], lo[3], lo[4], lo[5], lo[6], lo[7]};
          }
        } else {
#pragma unroll
          for (int i = 0; i < KJ; ++i) yb[s][i] = e[i];
        }
      }
    };
    f32x4 acc[ST][NDB];
    int cnt[ST];
#pragma unroll
    for (int s = 0; s < ST; ++s) {
      cnt[s] = 0;
#pragma unroll
      for (int db = 0; db < NDB; ++db) acc[s][db] = f32x4{0.f, 0.f, 0.f, 0.f};
    }

    auto compute = [&](int buf, int b) {
      // BF16: the block's rows go to this wave's staging area (pixel p of the
      // block at row p); lane (g, r) reads back dimension 16 db + r of pixels
      // 8g .. 8g+7, the A operand of V^T = X^T W^T.  The reads are issued
      // before S's products, which hide them.
      bf16x8 xvt[STAGE ? NDB : 1], xvtl[STAGE && SPLIT ? NDB : 1];
      if constexpr (STAGE) {
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
          for (int j = 0; j < KS; ++j) {
            const int p = rowsel0 + 4 * t;
            const int o = p * DP + 8 * (((g * KJ) / 8 + j) ^ swz(p));
            *reinterpret_cast<bf16x8*>(stage + o) = xa[buf][t][j];
            if constexpr (SPLIT) *reinterpret_cast<bf16x8*>(stage + STAGE_ELEMS + o) = xal[buf][t][j];
          }
#pragma unroll
        for (int db = 0; db < NDB; ++db) {
          // Rows 8g + (r >> 2) and 4 further (same permutation), columns
          // 16 db + 4 (r & 3) .. + 3: half r & 1 of chunk 2 db + (r & 3) / 2.
          const int p0 = 8 * g + (r >> 2);
          const int o0 = p0 * DP + 8 * ((2 * db + ((r & 3) >> 1)) ^ swz(p0)) + 4 * (r & 1);
          xvt[db] = lds_tr_b16x8(stage + o0, stage + o0 + 4 * DP);
          if constexpr (SPLIT)
            xvtl[db] = lds_tr_b16x8(stage + STAGE_ELEMS + o0, stage + STAGE_ELEMS + o0 + 4 * DP);
        }
      }
#pragma unroll
      for (int s = 0; s < ST; ++s) {
        f32x4 s0 = cinit, s1 = cinit;
#pragma unroll
        for (int j = 0; j < KS; ++j) {
          if constexpr (BF16) {
            if constexpr (SPLIT) {
              // Small cross terms first, then the main product.
              s0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xal[buf][0][j], yb[s][j], s0, 0, 0, 0);
              s1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xal[buf][1][j], yb[s][j], s1, 0, 0, 0);
              s0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa[buf][0][j], ybl[s][j], s0, 0, 0, 0);
              s1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa[buf][1][j], ybl[s][j], s1, 0, 0, 0);
            }
            s0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa[buf][0][j], yb[s][j], s0, 0, 0, 0);
            s1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa[buf][1][j], yb[s][j], s1, 0, 0, 0);
          } else {
            s0 = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[buf][0][j], yb[s][j], s0, 0, 0, 0);
            s1 = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[buf][1][j], yb[s][j], s1, 0, 0, 0);
          }
        }
        if constexpr (COUNT) {
          if ((int64_t)(b + 1) * kBlockPix <= n_pix) {
            // Every pixel of the block is real: the lane's eight results lose
            // their negative ones, counted from the sign bits (v_perm
            // selectors 9 and 11 give 0xff for a negative low or high source
            // dword, 12 gives 0), four to a popcount.
            const uint32_t n0 = __builtin_amdgcn_perm(fbits(s0[1]), fbits(s0[0]), 0x0C0C0B09u) |
                                __builtin_amdgcn_perm(fbits(s0[3]), fbits(s0[2]), 0x0B090C0Cu);
            const uint32_t n1 = __builtin_amdgcn_perm(fbits(s1[1]), fbits(s1[0]), 0x0C0C0B09u) |
                                __builtin_amdgcn_perm(fbits(s1[3]), fbits(s1[2]), 0x0B090C0Cu);
            cnt[s] += 8 - __builtin_popcount(n0 & 0x01010101u) - __builtin_popcount(n1 & 0x01010101u);
          } else {
            const int pbase = b * kBlockPix + 8 * g;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              cnt[s] += ((fbits(s0[i]) >> 31) == 0u && pbase + i < n_pix) ? 1 : 0;
              cnt[s] += ((fbits(s1[i]) >> 31) == 0u && pbase + 4 + i < n_pix) ? 1 : 0;
            }
          }
        } else if constexpr (BF16) {
          // Pixels 8g..8g+3 come from tile 0, 8g+4..8g+7 from tile 1.
          uint32_t m0 = __builtin_amdgcn_perm(fbits(s0[1]), fbits(s0[0]),
                                              0x0B0B0909u);
          uint32_t m1 = __builtin_amdgcn_perm(fbits(s0[3]), fbits(s0[2]),
                                              0x0B0B0909u);
          uint32_t m2 = __builtin_amdgcn_perm(fbits(s1[1]), fbits(s1[0]),
                                              0x0B0B0909u);
          uint32_t m3 = __builtin_amdgcn_perm(fbits(s1[3]), fbits(s1[2]),
                                              0x0B0B0909u);
          typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
          const uint32_t one2 = 0x3F803F80u;  // two BF16 ones
          u32x4 wp = {~m0 & one2, ~m1 & one2, ~m2 & one2, ~m3 & one2};
          const bf16x8 w = __builtin_bit_cast(bf16x8, wp);
#pragma unroll
          for (int db = 0; db < NDB; ++db) {
            if constexpr (SPLIT)
              acc[s][db] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xvtl[db], w, acc[s][db], 0, 0, 0);
            acc[s][db] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xvt[db], w, acc[s][db], 0, 0, 0);
          }
        } else {
          float w[8];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            w[i] = (fbits(s0[i]) >> 31) ? 0.f : 1.f;
            w[4 + i] = (fbits(s1[i]) >> 31) ? 0.f : 1.f;
          }
#pragma unroll
          for (int db = 0; db < NDB; ++db)
#pragma unroll
            for (int e = 0; e < 8; ++e)
              acc[s][db] = __builtin_amdgcn_mfma_f32_16x16x4f32(xv[buf][db][e], w[e], acc[s][db], 0, 0, 0);
        }
      }
    };
    // The first pixel blocks are requested before the seeds, so the loads
    // overlap instead of queueing behind each other.  A wave with at least
    // kDeepBlocks blocks loads unconditionally, past its last block from that
    // block again (a cache hit): the compiler then knows how many loads are
    // younger than a block's and waits for that block alone, keeping PD - 1
    // blocks in flight.  Conditional loads make it wait for every load in
    // flight, which short runs of blocks tolerate better than the extra
    // loads, and so do eight-wave groups of FP32 and split steps (two waves
    // per SIMD, whose products per block hide more); four-wave groups (one
    // wave per SIMD) and plain BF16 steps gain.
    constexpr bool DEEP = WV == 4 || (BF16 && !SPLIT && !COUNT && WV == 8);
    const int nbw = b < b1 ? (b1 - 1 - b) / WV + 1 : 0;
    if (DEEP && nbw >= kDeepBlocks) {
      const int bl = b + (nbw - 1) * WV;
#pragma unroll
      for (int k = 0; k < PD - 1; ++k) load(k, min(b + k * WV, bl));
      load_seeds();
      // Whole rounds of PD blocks run without a test, so the scheduler can
      // overlap one block's products with the next one's.
      for (; b + (PD - 1) * WV < b1; b += PD * WV) {
#pragma unroll
        for (int u = 0; u < PD; ++u) {
          load((u + PD - 1) % PD, min(b + (u + PD - 1) * WV, bl));
          compute(u, b + u * WV);
        }
      }
      // Fewer than PD blocks are left, all of them loaded.
#pragma unroll
      for (int u = 0; u < PD - 1; ++u)
        if (b + u * WV < b1) compute(u, b + u * WV);
    } else {
#pragma unroll
      for (int k = 0; k < PD - 1; ++k)
        if (b + k * WV < b1) load(k, b + k * WV);
      load_seeds();
      for (; b < b1; b += PD * WV) {
#pragma unroll
        for (int u = 0; u < PD; ++u) {
          if (b + (u + PD - 1) * WV < b1) load((u + PD - 1) % PD, b + (u + PD - 1) * WV);
          if (b + u * WV < b1) compute(u, b + u * WV);
        }
      }
    }
    if constexpr (COUNT) {
      // Counts of seed r are spread over the four lane groups, then the waves.
#pragma unroll
      for (int s = 0; s < ST; ++s) {
        int c = cnt[s];
        c += __shfl_xor(c, 16, 64);
        c += __shfl_xor(c, 32, 64);
        if (wave > 0 && g == 0) redc[wave - 1][s][r] = c;
        cnt[s] = c;
      }
      __syncthreads();
      if (wave == 0 && g == 0) {
#pragma unroll
        for (int s = 0; s < ST; ++s) {
          const int a = a0 + 16 * s + r;
          int c = cnt[s];
#pragma unroll
          for (int w = 0; w < WV - 1; ++w) c += redc[w][s][r];
          if (a < n_act) pcount[(int64_t)chunk * n_act + a] = c;
        }
      }
      __syncthreads();
      continue;
    }
    // Fixed-order tree sum of the waves' window sums (each round the upper
    // half of the remaining waves hands its sums to the lower half), then one
    // partial per item.  Every wave is done with its staging area first.
    if constexpr (!COUNT) {
      if constexpr (STAGE) __syncthreads();
#pragma unroll
      for (int half = WV / 2; half >= 1; half >>= 1) {
        if (wave >= half && wave < 2 * half) {
#pragma unroll
          for (int s = 0; s < ST; ++s)
#pragma unroll
            for (int db = 0; db < NDB; ++db) red[wave - half][s][db][lane] = acc[s][db];
        }
        __syncthreads();
        if (wave < half) {
#pragma unroll
          for (int s = 0; s < ST; ++s)
#pragma unroll
            for (int db = 0; db < NDB; ++db) acc[s][db] += red[wave][s][db][lane];
        }
        __syncthreads();
      }
      if (wave == 0) {
#pragma unroll
        for (int s = 0; s < ST; ++s) {
          const int a = a0 + 16 * s + r;
#pragma unroll
          for (int db = 0; db < NDB; ++db) {
            const f32x4 v = acc[s][db];
            if (a < n_act)
              *reinterpret_cast<float4*>(partial + ((int64_t)chunk * n_act + a) * DP + 16 * db + 4 * g) =
                  make_float4(v[0], v[1], v[2], v[3]);
          }
        }
      }
    }
  }
}

template <bool BF16, bool SPLIT, bool COUNT, int DP, int ST, int WV>
__global__ __launch_bounds__(64 * WV) void k_shift(Batch bt, const void* __restrict__ xrm_, const void* __restrict__ xt_,
                                               const uint16_t* __restrict__ xrl,
                                               const float* __restrict__ y, const int* __restrict__ active,
                                               IterCtl ctl, Tiling tl, float* __restrict__ partial,
                                               int* __restrict__ pcount) {
  typedef typename std::conditional<BF16, uint16_t, float>::type T;
  const int f = blockIdx.y;
  const FrameGeo& g = bt.geo[f];
  int* meta = bt.meta + (int64_t)f * META_COUNT;
  const T* xrm = static_cast<const T*>(xrm_) + g.row0 * DP;
  const T* xt = xt_ ? static_cast<const T*>(xt_) + g.row0 * DP : nullptr;
  if (SPLIT) {
    xrl += g.row0 * DP;
  }
  y += g.row0 * DP;
  if (active) active += g.row0;
  if (partial) partial += g.part0 * DP;
  if (pcount) pcount += g.part0;
  int n_act;
  if (ctl.iter >= 0) {
    // Every counter is read before the one test (a single round trip; a
    // test per counter would wait for each).
    const int done = meta[META_DONE];
    const int act0 = meta[META_ACT], act1 = meta[META_ACT + 1];
    n_act = (ctl.iter & 1) ? act1 : act0;
    const int n_conv = meta[META_NCONV];
    const int n_sel = meta[META_NSEL];
    const int gstep = meta[META_GSTEP];
    const bool first = blockIdx.x == 0 && threadIdx.x == 0;
    // Same test, in the same precision, as the host's between batches.  A
    // step that is the first to see more than gamma converged records
    // itself; every work group of it counts 0 steps past that point whether
    // or not it sees the record, so they all decide alike.
    const bool over = (double)n_conv > ctl.gamma * (double)n_sel;
    const int past = (over && gstep >= 0) ? ctl.iter - gstep : 0;
    if ((done != 0) | (n_act <= 0) | (over & (past >= ctl.extra))) {
      // Setting the flag again when it is set is harmless.
      if (first) meta[META_DONE] = 1;
      return;
    }
    if (first && over && gstep < 0) meta[META_GSTEP] = ctl.iter;
    if (first) {
      meta[META_ACT + ((ctl.iter + 1) & 1)] = 0;
      meta[META_STEPS] += 1;
      bt.meta64[(int64_t)f * kMeta64] += (unsigned long long)n_act * (unsigned long long)g.n;
      bt.meta64[(int64_t)f * kMeta64 + 1] += (unsigned long long)g.n;
    }
  } else {
    n_act = ctl.nact_slot >= 0 ? meta[ctl.nact_slot] : round_tab(bt, f).nact;
  }
  if (n_act <= 0) return;
  shift_body<BF16, SPLIT, COUNT, DP, ST, WV>(xrm, xt, xrl, y, active, n_act, tl, g.n_blocks, g.n, g.thr,
                                             partial, pcount, (int)blockIdx.x, (int)gridDim.x);
}

// Sum the chunk partials of each active seed in a fixed order, renormalise,
// test convergence (Sec. 3.2.1: cosine distance between consecutive centres
// below tol), and build the next active list.
//
// Threads are laid out (seed, phase, 4-dimension slice): a seed's DP/4 slices
// times P phases, P the smallest power of two with at most 8 chunks per
// phase, so every thread issues at most 8 float4 loads at once.  Phases are
// added in order in LDS; norms and moves are reduced over the seed's slice
// lanes with a fixed butterfly.  Work groups loop over tiles of seeds.
//   mode 0: iterate, freezing converged seeds: next active list and
//           converged count (the early stop is taken by the next step).
//           With a ring (BF16 form), the centre a step starts from is also
//           kept in ring slab iters % ring_len, so that the last ring_len
//           centres of every seed's trajectory are at hand when it stops.
//   mode 1: plain step (no freezing, no test).
// Reduce/renormalise/converge the active seeds' tiles owned by work group wg
// of nwg.  Returns (in every thread) this group's number of newly converged
// seeds (mode 0).  next_ctr receives the appends to next_active.
template <int DP>
__device__ __forceinline__ int reduce_body(const float* __restrict__ partial, const int* __restrict__ active,
                                           const float* __restrict__ ycur, float* __restrict__ y,
                                           uint8_t* __restrict__ state,
                                           int* __restrict__ iters, int* __restrict__ next_active,
                                           float* __restrict__ yc_next, float* __restrict__ vnorm,
                                           int* __restrict__ next_ctr, float* __restrict__ ring,
                                           int64_t ring_stride, int ring_len, int n_act,
                                           const Tiling& tl, int n_blocks, float tol, int mode, int wg, int nwg) {
  constexpr int Q = DP / 4;  // float4 slices per row
  __shared__ float4 part[256];
  __shared__ int s_conv;
  __shared__ int s_wn[4], s_wb[4];
  const ChunkPlan cp = plan_chunks(n_act, tl, n_blocks);
  const int nc = cp.n_chunks;
  int P = 1;
  while (P * 8 < nc && Q * P * 2 <= 256) P <<= 1;
  const int tpr = Q * P;       // threads per seed
  const int spw = 256 / tpr;   // seeds per work group tile
  const int tiles = (n_act + spw - 1) / spw;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int sl = tid / tpr, rest = tid - sl * tpr, q = rest % Q, ph = rest / Q;
  if (tid == 0) s_conv = 0;
  __syncthreads();
  const int64_t cstride = (int64_t)n_act * DP;
  for (int tile = wg; tile < tiles; tile += nwg) {
    const int a = tile * spw + sl;
    const bool live_seed = a < n_act && sl < spw;
    const bool owner = live_seed && ph == 0;
    // The centre's slot and its current row do not depend on the partials:
    // request them first (the row from the compacted copy in list order when
    // there is one, so that it does not wait for the slot).
    const int slot = owner ? active[a] : 0;
    // Steps this seed has taken so far (read before the head lane adds one;
    // a seed's Q owner lanes are in one wave).
    const int it0 = (ring && owner) ? iters[slot] : 0;
    float4 yo = make_float4(0.f, 0.f, 0.f, 0.f);
    if (owner)
      yo = *reinterpret_cast<const float4*>(ycur ? ycur + (int64_t)a * DP + 4 * q : y + (int64_t)slot * DP + 4 * q);
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    if (live_seed) {
      const float4* src = reinterpret_cast<const float4*>(partial + (int64_t)a * DP + 4 * q);
      for (int c0 = ph; c0 < nc; c0 += 8 * P) {
        float4 t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int c = c0 + u * P;
          t[u] = c < nc ? src[(int64_t)c * (cstride / 4)] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          acc.x += t[u].x;
          acc.y += t[u].y;
          acc.z += t[u].z;
          acc.w += t[u].w;
        }
      }
    }
    part[tid] = acc;
    __syncthreads();
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (owner) {
      for (int pp = 0; pp < P; ++pp) {
        const float4 u = part[sl * tpr + pp * Q + q];
        v.x += u.x;
        v.y += u.y;
        v.z += u.z;
        v.w += u.w;
      }
    }
    // The Q owner lanes of a seed are consecutive and aligned within a wave.
    float ss = v.x * v.x + v.y * v.y + v.z * v.z + v.w * v.w;
    for (int m = Q / 2; m >= 1; m >>= 1) ss += __shfl_xor(ss, m, 64);
    const float nv = sqrtf(ss);
    const bool dead = !(nv > 0.f) || !__builtin_isfinite(nv);
    const float inv = dead ? 0.f : 1.0f / nv;
    const float4 yn = make_float4(v.x * inv, v.y * inv, v.z * inv, v.w * inv);
    float dd = (yo.x - yn.x) * (yo.x - yn.x) + (yo.y - yn.y) * (yo.y - yn.y) + (yo.z - yn.z) * (yo.z - yn.z) +
               (yo.w - yn.w) * (yo.w - yn.w);
    for (int m = Q / 2; m >= 1; m >>= 1) dd += __shfl_xor(dd, m, 64);
    // 1 - y.y' = |y - y'|^2 / 2 for unit vectors, without cancellation.
    const float delta = 0.5f * dd;
    if (owner && !dead) *reinterpret_cast<float4*>(y + (int64_t)slot * DP + 4 * q) = yn;
    const bool head = owner && q == 0;
    if (vnorm && head) vnorm[slot] = nv;
    if (mode == 0) {
      const bool conv = head && !dead && delta < tol;
      const bool next = head && !dead && !(delta < tol);
      if (ring && owner && !dead)
        *reinterpret_cast<float4*>(ring + (int64_t)(it0 % ring_len) * ring_stride + (int64_t)slot * DP + 4 * q) = yo;
      if (head) {
        iters[slot] += 1;
        if (dead) state[slot] = 2;
        if (conv) state[slot] = 1;
      }
      // List append: one counter update per work group (updates of one
      // address from every wave queue behind each other), each wave's place
      // after the waves before it; converged count per wave into LDS.
      const unsigned long long bn = __ballot(next);
      const unsigned long long bc = __ballot(conv);
      if (lane == 0) s_wn[wave] = __popcll(bn);
      __syncthreads();
      if (tid == 0) {
        int tot = 0;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          s_wb[w] = tot;
          tot += s_wn[w];
        }
        const int b0 = tot ? atomicAdd(next_ctr, tot) : 0;
#pragma unroll
        for (int w = 0; w < 4; ++w) s_wb[w] += b0;
      }
      __syncthreads();
      const int pos = s_wb[wave] + __popcll(bn & ((1ull << lane) - 1ull));
      if (next) next_active[pos] = slot;
      if (yc_next) {
        // The seed's owner lanes copy its new row to its place in the
        // compacted rows of the next iteration (position from the head lane).
        const int hpos = __shfl(pos, lane - q, 64);
        const int hnext = __shfl(next ? 1 : 0, lane - q, 64);
        if (owner && hnext) *reinterpret_cast<float4*>(yc_next + (int64_t)hpos * DP + 4 * q) = yn;
      }
      if (lane == 0 && bc) atomicAdd(&s_conv, __popcll(bc));
    } else if (head) {
      if (dead) state[slot] = 2;
    }
    __syncthreads();
  }
  return s_conv;
}

template <int DP>
__global__ __launch_bounds__(256) void k_reduce(Batch bt, const float* __restrict__ partial,
                                                const int* __restrict__ active, const float* __restrict__ ycur,
                                                float* __restrict__ y, uint8_t* __restrict__ state,
                                                int* __restrict__ iters, int* __restrict__ next_active,
                                                float* __restrict__ yc_next, float* __restrict__ vnorm, IterCtl ctl,
                                                Tiling tl, int mode, float* __restrict__ ring, int64_t ring_stride,
                                                int ring_len) {
  const int f = blockIdx.y;
  const FrameGeo& g = bt.geo[f];
  int* meta = bt.meta + (int64_t)f * META_COUNT;
  partial += g.part0 * DP;
  active += g.row0;
  if (ycur) ycur += g.row0 * DP;
  y += g.row0 * DP;
  state += g.row0;
  iters += g.row0;
  if (next_active) next_active += g.row0;
  if (yc_next) yc_next += g.row0 * DP;
  if (vnorm) vnorm += g.row0;
  if (ring) ring += g.row0 * DP;
  int n_act;
  int* next_ctr = nullptr;
  if (ctl.iter >= 0) {
    // The counters are read before the one test (a single round trip); a
    // reduction of no seeds has nothing to do either.
    const int done = meta[META_DONE];
    const int act0 = meta[META_ACT], act1 = meta[META_ACT + 1];
    n_act = (ctl.iter & 1) ? act1 : act0;
    if ((done != 0) | (n_act <= 0)) return;
    next_ctr = meta + META_ACT + ((ctl.iter + 1) & 1);
  } else {
    n_act = ctl.nact_slot >= 0 ? meta[ctl.nact_slot] : round_tab(bt, f).nact;
  }
  const int conv = reduce_body<DP>(partial, active, ycur, y, state, iters, next_active, yc_next, vnorm, next_ctr,
                                   ring, ring_stride, ring_len, n_act, tl, g.n_blocks, g.tol, mode, (int)blockIdx.x,
                                   (int)gridDim.x);
  if (mode == 0 && threadIdx.x == 0 && conv) atomicAdd(meta + META_NCONV, conv);
}

// Sum the per-chunk window counts of each centre (one wave per centre).
__global__ __launch_bounds__(256) void k_reduce_counts(Batch bt, const int* __restrict__ pcount, Tiling tl, int m_slot,
                                                       int* __restrict__ counts) {
  const int f = blockIdx.y;
  const FrameGeo& g = bt.geo[f];
  const int m = m_slot >= 0 ? bt.meta[(int64_t)f * META_COUNT + m_slot] : round_tab(bt, f).nact;
  pcount += g.part0;
  counts += g.row0;
  const int n_chunks = plan_chunks(m, tl, g.n_blocks).n_chunks;
  const int a = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (a >= m) return;
  int c = 0;
  for (int k = lane; k < n_chunks; k += 64) c += pcount[(int64_t)k * m + a];
  c = wave_sum_i(c);
  if (lane == 0) counts[a] = c;
}

// Start of a round: the selected seeds become the active list.  With
// seed_fg, centre k also starts at pixel row seed_fg[k] of x32.
template <int DP>
__global__ __launch_bounds__(256) void k_round_begin(Batch bt, int cap, int nsel_from_rt, int* __restrict__ active,
                                                     uint8_t* __restrict__ state, int* __restrict__ iters,
                                                     const int* __restrict__ seed_fg, const float* __restrict__ x32,
                                                     float* __restrict__ y) {
  const int f = blockIdx.y;
  const FrameGeo& g = bt.geo[f];
  int* meta = bt.meta + (int64_t)f * META_COUNT;
  unsigned long long* meta64 = bt.meta64 + (int64_t)f * kMeta64;
  active += g.row0;
  state += g.row0;
  iters += g.row0;
  y += g.row0 * DP;
  x32 += g.row0 * DP;
  if (seed_fg) seed_fg += g.row0;
  const int m = nsel_from_rt ? round_tab(bt, f).nact : meta[META_NSEL];
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k < m && k < cap) {
    active[k] = k;
    state[k] = 0;
    iters[k] = 0;
    if (seed_fg) {
      const float4* src = reinterpret_cast<const float4*>(x32 + (int64_t)seed_fg[k] * DP);
      float4* dst = reinterpret_cast<float4*>(y + (int64_t)k * DP);
#pragma unroll
      for (int q = 0; q < DP / 4; ++q) dst[q] = src[q];
    }
  }
  if (k == 0) {
    if (nsel_from_rt) meta[META_NSEL] = m;
    meta[META_ACT] = m;
    meta[META_ACT + 1] = 0;
    meta[META_NCONV] = 0;
    meta[META_LEFT] = 0;  // the round's coverage counts the pixels left to seed
    meta[META_DONE] = m > 0 ? 0 : 1;
    meta[META_STEPS] = 0;
    meta[META_GSTEP] = -1;
    meta64[0] = 0;
    meta64[1] = 0;
  }
}

// Similarity bits: bit c of row j is set when row vector j and column
// vector c are inside each other's window (dot >= thr).  Rows are
// y[rows[j]]; the columns of the first `split` work groups are y[cols[c]]
// (bits at tab.bits_c0, tab.words_c words per row), those of the rest the
// frame's modes (bits at tab.bits_m0, tab.words_m words per row).  A wave
// owns 64 columns and 16 rows; each lane keeps its column vector in
// registers and reads the row vectors, staged in LDS per work group, as
// broadcasts.  Row strides are multiples of 2 words.  With `first` (candidate columns = the rows, in rank
// order), first[j] is lowered to the first word of row j holding a column
// c < j that is set (it must start at INT_MAX).
template <int DP>
__global__ __launch_bounds__(256) void k_simbits(Batch bt, const float* __restrict__ y, const int* __restrict__ rows,
                                                 const int* __restrict__ cols_, const float* __restrict__ colmat_,
                                                 uint32_t* __restrict__ bits, int rows_slot, int cols_slot, int split,
                                                 int* __restrict__ first) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int f = blockIdx.y;
  const bool mode_part = (int)blockIdx.x >= split;
  const int bx = mode_part ? (int)blockIdx.x - split : (int)blockIdx.x;
  const int* cols = mode_part ? nullptr : cols_;
  const float* colmat = mode_part ? colmat_ : nullptr;
  const FrameGeo& g = bt.geo[f];
  const RoundTab tab = round_tab(bt, f);
  const int* meta = bt.meta + (int64_t)f * META_COUNT;
  const int m = meta[rows_slot];
  const int ncols = cols ? meta[cols_slot] : tab.k_modes;
  const int words = cols ? tab.words_c : tab.words_m;
  const float thr = g.thr;
  y += g.row0 * DP;
  rows += g.row0;
  if (cols) cols += g.row0;
  if (colmat) colmat += g.row0 * DP;
  if (first) first += g.row0;
  bits += cols ? tab.bits_c0 : tab.bits_m0;
  const int col_tiles = words / 2;
  if (col_tiles == 0 || bx >= col_tiles * ((m + 63) / 64)) return;
  const int ct = bx % col_tiles, rt = bx / col_tiles;
  const int c = ct * 64 + lane;
  float xc[DP];
  if (c < ncols) {
    const float* src = cols ? y + (int64_t)cols[c] * DP : colmat + (int64_t)c * DP;
#pragma unroll
    for (int d = 0; d < DP; d += 4) {
      float4 u = *reinterpret_cast<const float4*>(src + d);
      xc[d] = u.x; xc[d + 1] = u.y; xc[d + 2] = u.z; xc[d + 3] = u.w;
    }
  } else {
#pragma unroll
    for (int d = 0; d < DP; ++d) xc[d] = 0.f;
  }
  // The tile's 64 row vectors are staged in LDS with one round of loads
  // (read back as broadcasts), instead of one dependent load per row.
  __shared__ __align__(16) float rs[64 * DP];
  for (int e = threadIdx.x; e < 16 * DP; e += 256) {
    const int q = e / (DP / 4), d4 = e - q * (DP / 4);
    const int j = rt * 64 + q;
    const float4 u = j < m ? *reinterpret_cast<const float4*>(y + (int64_t)rows[j] * DP + 4 * d4)
                           : make_float4(0.f, 0.f, 0.f, 0.f);
    *reinterpret_cast<float4*>(&rs[q * DP + 4 * d4]) = u;
  }
  __syncthreads();
  const int j0 = rt * 64 + wave * 16;
  for (int jj = 0; jj < 16; ++jj) {
    const int j = j0 + jj;
    if (j >= m) break;
    const float* rv = &rs[(wave * 16 + jj) * DP];
    float dot = 0.f;
#pragma unroll
    for (int d = 0; d < DP; ++d) dot = fmaf(rv[d], xc[d], dot);
    const unsigned long long bal = __ballot(c < ncols && dot >= thr);
    if (lane == 0) {
      bits[(int64_t)j * words + 2 * ct] = (uint32_t)bal;
      bits[(int64_t)j * words + 2 * ct + 1] = (uint32_t)(bal >> 32);
      if (first && cols) {
        // The columns of this tile before column j.
        const int before = j - ct * 64;
        const unsigned long long early =
            before <= 0 ? 0ull : (before >= 64 ? bal : bal & ((1ull << before) - 1ull));
        if (early) atomicMin(first + j, 2 * ct + ((uint32_t)early ? 0 : 1));
      }
    }
  }
}

// ------------------------------------------------------------------ pruning on the device

// ------------------------------------------------------------------ FP32 replay (BF16 form)
//
// The BF16 form takes the last ring_len iterations of every converged seed
// again in FP32 (Eq. 8, 10, 11 with the Sec. 3.2.1 stopping test): the
// membership decisions and the window sum that give the seed its mode are
// then FP32 ones.  k_replay_begin lists the round's converged slots in
// ascending order (cand[i], i < meta[META_NCAND]), puts each one's restart
// centre -- the centre it had min(iters, ring_len) steps before it stopped,
// kept in the ring by the BF16 reduction -- at row i of yr, and sets the
// replay's identity list, states, step counts and iteration counters as a
// round start does.  One 1024-thread work group per frame.
template <int DP>
__global__ __launch_bounds__(1024) void k_replay_begin(Batch bt, int ring_len, const uint8_t* __restrict__ state,
                                                       const int* __restrict__ iters, const float* __restrict__ ring,
                                                       int64_t ring_stride, int* __restrict__ cand,
                                                       float* __restrict__ yr, int* __restrict__ active,
                                                       uint8_t* __restrict__ rstate, int* __restrict__ riters) {
  __shared__ int sh[17];
  const int f = blockIdx.x;
  const FrameGeo& g = bt.geo[f];
  int* meta = bt.meta + (int64_t)f * META_COUNT;
  state += g.row0;
  iters += g.row0;
  ring += g.row0 * DP;
  cand += g.row0;
  yr += g.row0 * DP;
  active += g.row0;
  rstate += g.row0;
  riters += g.row0;
  const int m = meta[META_NSEL];
  int base = 0;
  for (int k0 = 0; k0 < m; k0 += 1024) {
    const int k = k0 + (int)threadIdx.x;
    const int c = (k < m && state[k] == 1) ? 1 : 0;
    int tot;
    const int r = block_exclusive_scan<1024>(c, &tot, sh);
    if (c) {
      const int i = base + r;
      const int t = max(iters[k], 1);
      const int back = min(t, ring_len);
      const float4* src = reinterpret_cast<const float4*>(ring + (int64_t)((t - back) % ring_len) * ring_stride +
                                                          (int64_t)k * DP);
      float4* dst = reinterpret_cast<float4*>(yr + (int64_t)i * DP);
#pragma unroll
      for (int q = 0; q < DP / 4; ++q) dst[q] = src[q];
      cand[i] = k;
      active[i] = i;
      rstate[i] = 0;
      riters[i] = 0;
    }
    base += tot;
  }
  if (threadIdx.x == 0) {
    meta[META_NCAND] = base;
    meta[META_ACT] = base;
    meta[META_ACT + 1] = 0;
    meta[META_NCONV] = 0;
    meta[META_DONE] = base > 0 ? 0 : 1;
    meta[META_STEPS] = 0;
    meta[META_REFINE_BAD] = 0;
    meta[META_REFINE_DIFF] = 0;
    meta[META_GSTEP] = -1;
    meta[META_GCUT] = 0;
    bt.meta64[(int64_t)f * kMeta64] = 0;
    bt.meta64[(int64_t)f * kMeta64 + 1] = 0;
  }
}

// End of the replay: candidate i's FP32 centre and state go back to its slot
// (state 1 only when the replay froze it; a seed still moving is dropped
// with the round's unconverged ones), and a frozen one's step count becomes
// its FP32 trajectory's: the BF16 steps before the restart plus the
// replay's.  META_REFINE_BAD counts the candidates the replay did not
// freeze, META_REFINE_DIFF the frozen ones whose FP32 stop came after a
// different number of steps than the BF16 one.
template <int DP>
__global__ __launch_bounds__(256) void k_replay_end(Batch bt, int cap, int ring_len, const int* __restrict__ cand,
                                                    int* __restrict__ iters, const float* __restrict__ yr,
                                                    const uint8_t* __restrict__ rstate,
                                                    const int* __restrict__ riters, float* __restrict__ y,
                                                    uint8_t* __restrict__ state) {
  const int f = blockIdx.y;
  const FrameGeo& g = bt.geo[f];
  int* meta = bt.meta + (int64_t)f * META_COUNT;
  const int m = meta[META_NCAND];
  const int i = blockIdx.x * 256 + threadIdx.x;
  const bool live = i < m && i < cap;
  bool bad = false, diff = false;
  if (live) {
    const int k = cand[g.row0 + i];
    const uint8_t st = rstate[g.row0 + i];
    const float4* src = reinterpret_cast<const float4*>(yr + (g.row0 + i) * DP);
    float4* dst = reinterpret_cast<float4*>(y + (g.row0 + k) * DP);
#pragma unroll
    for (int q = 0; q < DP / 4; ++q) dst[q] = src[q];
    state[g.row0 + k] = st;
    bad = st != 1;
    const int t = max(iters[g.row0 + k], 1);
    const int back = min(t, ring_len);
    const int rit = riters[g.row0 + i];
    diff = st == 1 && rit != back;
    if (st == 1) iters[g.row0 + k] = t - back + rit;
  }
  const unsigned long long bb = __ballot(bad), bd = __ballot(diff);
  if ((threadIdx.x & 63) == 0) {
    if (bb) atomicAdd(meta + META_REFINE_BAD, __popcll(bb));
    if (bd) atomicAdd(meta + META_REFINE_DIFF, __popcll(bd));
  }
}

// The early stop of Sec. 3.2.3 on the FP32 step counts of the replay: the
// first step t after which more than gamma of the round's seeds had
// converged; converged slots whose count exceeds t are dropped, as the
// plain iteration would have stopped before they converged.  Counts above
// kCutSteps share the histogram's last bin (they can only be cut or kept
// together).  One 1024-thread work group per frame.
constexpr int kCutSteps = 1024;
__global__ __launch_bounds__(1024) void k_gamma_cut(Batch bt, double gamma, const int* __restrict__ iters,
                                                    uint8_t* __restrict__ state) {
  __shared__ int hist[kCutSteps + 1];
  __shared__ int s_cut, s_drop;
  const FrameGeo& g = bt.geo[blockIdx.x];
  int* meta = bt.meta + (int64_t)blockIdx.x * META_COUNT;
  iters += g.row0;
  state += g.row0;
  const int m = meta[META_NSEL];
  for (int t = threadIdx.x; t <= kCutSteps; t += 1024) hist[t] = 0;
  if (threadIdx.x == 0) s_drop = 0;
  __syncthreads();
  for (int k = threadIdx.x; k < m; k += 1024)
    if (state[k] == 1) atomicAdd(&hist[min(max(iters[k], 0), kCutSteps)], 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    int cut = INT_MAX, run = 0;
    for (int t = 0; t <= kCutSteps; ++t) {
      run += hist[t];
      if ((double)run > gamma * (double)m) {
        cut = t;
        break;
      }
    }
    s_cut = cut;
  }
  __syncthreads();
  const int cut = s_cut;
  int drop = 0;
  if (cut < kCutSteps)
    for (int k = threadIdx.x; k < m; k += 1024)
      if (state[k] == 1 && iters[k] > cut) {
        state[k] = 0;
        ++drop;
      }
  if (drop) atomicAdd(&s_drop, drop);
  __syncthreads();
  if (threadIdx.x == 0) meta[META_GCUT] = s_drop;
}

// Rank the converged slots k < meta[META_NSEL] (state[k] == 1) of the round
// by window count (descending), then by slot (ascending, = seed position):
// sorted[r] = k_r, scount[r] = counts[k_r]; their number goes to
// meta[META_NCAND].  Bitonic sort of 64-bit keys, the other slots' keys
// sorting last; NSEL <= kRankMax.  Up to 1,024 keys sit one per thread and
// exchange within a wave by shuffles (strides below 64) and through LDS
// otherwise, so a sort of 512 keys passes 6 barriers instead of 45; larger
// sets sort in LDS.
__global__ __launch_bounds__(1024) void k_rank_converged(Batch bt, const uint8_t* __restrict__ state,
                                                         const int* __restrict__ counts, int* __restrict__ sorted,
                                                         int* __restrict__ scount, int* __restrict__ first) {
  __shared__ unsigned long long key[kRankMax];
  __shared__ int s_nc;
  const FrameGeo& g = bt.geo[blockIdx.x];
  int* meta = bt.meta + (int64_t)blockIdx.x * META_COUNT;
  state += g.row0;
  counts += g.row0;
  sorted += g.row0;
  scount += g.row0;
  const int m = meta[META_NSEL];
  if (threadIdx.x == 0) s_nc = 0;
  __syncthreads();
  int np = 1;
  while (np < m) np <<= 1;
  int mine = 0;
  for (int i = threadIdx.x; i < np; i += 1024) {
    const bool c = i < m && state[i] == 1;
    mine += c ? 1 : 0;
    key[i] = c ? ((unsigned long long)(uint32_t)(0x7FFFFFFF - counts[i]) << 32) | (uint32_t)i : ~0ull;
  }
  mine = wave_sum_i(mine);
  if ((threadIdx.x & 63) == 0 && mine) atomicAdd(&s_nc, mine);
  __syncthreads();
  if (np <= 1024) {
    // Threads at or past np hold the largest key and only meet each other.
    const int i = threadIdx.x;
    unsigned long long k = i < np ? key[i] : ~0ull;
    for (int size = 2; size <= np; size <<= 1) {
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        unsigned long long o;
        if (stride >= 64) {
          key[i] = k;
          __syncthreads();
          o = key[i ^ stride];
          __syncthreads();
        } else {
          const uint32_t lo = __shfl_xor((uint32_t)k, stride, 64);
          const uint32_t hi = __shfl_xor((uint32_t)(k >> 32), stride, 64);
          o = ((unsigned long long)hi << 32) | lo;
        }
        const bool up = (i & size) == 0, lower = (i & stride) == 0;
        k = (lower == up) ? (k < o ? k : o) : (k < o ? o : k);
      }
    }
    key[i] = k;
    __syncthreads();
  } else {
    for (int size = 2; size <= np; size <<= 1) {
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        for (int i = threadIdx.x; i < np; i += 1024) {
          const int j = i ^ stride;
          if (j > i) {
            const bool up = (i & size) == 0;
            const unsigned long long a = key[i], b = key[j];
            if ((a > b) == up) {
              key[i] = b;
              key[j] = a;
            }
          }
        }
        __syncthreads();
      }
    }
  }
  const int nc = s_nc;
  if (first) first += g.row0;
  for (int r = threadIdx.x; r < nc; r += 1024) {
    const int k = (int)(key[r] & 0xFFFFFFFFull);
    sorted[r] = k;
    scount[r] = counts[k];
    if (first) first[r] = INT_MAX;
  }
  if (threadIdx.x == 0) meta[META_NCAND] = nc;
}

// Greedy suppression (Alg. 2 "Prune modes") over candidates already in rank
// order: candidate r is accepted when no existing mode is within its window
// (row r of bits_m is empty) and no accepted candidate r' < r is (bit r' of
// row r of bits_c).  Decided in parallel passes: an undecided r is rejected
// as soon as an earlier accepted candidate conflicts with it and accepted
// once every earlier conflicting candidate is rejected; each pass decides at
// least the first undecided candidate, and every decision equals the
// sequential one whatever order the passes observe.  A candidate scans its
// row upwards from a cursor and stops at the first undecided conflict; the
// next pass resumes there, so a row is read about once in all.  With
// `first` (the first word of each row with an earlier conflict, INT_MAX for
// none) the scan starts there instead of at word 0.  The accepted rows are
// appended to the mode set at k0; their number goes to meta[acc_slot].
__global__ __launch_bounds__(1024) void k_greedy(Batch bt, const uint32_t* __restrict__ bits,
                                                 const float* __restrict__ y, const int* __restrict__ sorted,
                                                 const int* __restrict__ scount, int ncand_slot, int acc_slot, int dp,
                                                 float* __restrict__ modes, int* __restrict__ mode_counts,
                                                 const int* __restrict__ first) {
  __shared__ uint8_t st[kRankMax];
  __shared__ uint16_t cur[kRankMax];
  __shared__ int s_open;
  __shared__ int sh[17];
  const FrameGeo& g = bt.geo[blockIdx.x];
  const RoundTab tab = round_tab(bt, blockIdx.x);
  int* meta = bt.meta + (int64_t)blockIdx.x * META_COUNT;
  const uint32_t* bits_c = bits + tab.bits_c0;
  const uint32_t* bits_m = bits + tab.bits_m0;
  const int words_c = tab.words_c, words_m = tab.words_m, k0 = tab.k_modes;
  y += g.row0 * dp;
  sorted += g.row0;
  scount += g.row0;
  modes += g.row0 * dp;
  mode_counts += g.row0;
  if (first) first += g.row0;
  const int nc = meta[ncand_slot];
  for (int r = threadIdx.x; r < nc; r += 1024) {
    const int f0 = first ? first[r] : 0;
    cur[r] = (uint16_t)(f0 == INT_MAX ? (r >> 5) + 1 : f0);
    uint8_t v = 0;
    if (k0 > 0) {
      const uint32_t* rm = bits_m + (int64_t)r * words_m;
      for (int w = 0; w < words_m; ++w)
        if (rm[w]) {
          v = 2;
          break;
        }
    }
    st[r] = v;
  }
  __syncthreads();
  for (;;) {
    if (threadIdx.x == 0) s_open = 0;
    __syncthreads();
    for (int r = threadIdx.x; r < nc; r += 1024) {
      if (reinterpret_cast<volatile uint8_t*>(st)[r] != 0) continue;
      const uint32_t* row = bits_c + (int64_t)r * words_c;
      bool rejected = false, waiting = false;
      const int wend = r >> 5;
      int w = cur[r];
      for (; w <= wend; ++w) {
        uint32_t b = row[w];
        if (w == wend) b &= (r & 31) ? ((1u << (r & 31)) - 1u) : 0u;
        while (b) {
          const int k = (w << 5) + __ffs(b) - 1;
          b &= b - 1;
          const uint8_t sk = reinterpret_cast<volatile uint8_t*>(st)[k];
          if (sk == 1) {
            rejected = true;
            break;
          }
          if (sk == 0) {
            waiting = true;
            break;
          }
        }
        if (rejected || waiting) break;
      }
      if (rejected) {
        reinterpret_cast<volatile uint8_t*>(st)[r] = 2;
      } else if (!waiting) {
        reinterpret_cast<volatile uint8_t*>(st)[r] = 1;
      } else {
        cur[r] = (uint16_t)w;
        atomicAdd(&s_open, 1);
      }
    }
    __syncthreads();
    const int open = s_open;
    __syncthreads();
    if (open == 0) break;
  }
  // Append the accepted candidates in rank order.
  int base = 0;
  for (int r0 = 0; r0 < nc; r0 += 1024) {
    const int r = r0 + (int)threadIdx.x;
    const int acc = (r < nc && st[r] == 1) ? 1 : 0;
    int tot;
    const int q = base + block_exclusive_scan<1024>(acc, &tot, sh);
    if (acc) {
      const float* src = y + (int64_t)sorted[r] * dp;
      float* dst = modes + (int64_t)(k0 + q) * dp;
      for (int d = 0; d < dp; ++d) dst[d] = src[d];
      mode_counts[k0 + q] = scount[r];
    }
    base += tot;
  }
  if (threadIdx.x == 0) meta[acc_slot] = base;
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

// Coverage (mode 0): pixels within h of a new mode, [rt.k_modes,
// rt.k_modes + meta[k1_slot]), stop being eligible seeds (elig[rank[i]] =
// 0); count the pixels still eligible.  Labels (mode 1): most similar mode
// in [0, rt.k_modes), lowest index on ties; count the pixels farther than h
// from every mode.
//
// The similarities come from v_mfma_f32_16x16x4_f32 with modes as rows and
// pixels as columns: lane (g, r) feeds mode row r and pixel column r with
// dimension g*KJ + j at step j, and receives the similarities of modes
// 4g..4g+3 of the tile with its pixel r.  Each lane keeps the best of the
// modes it sees (ascending, first of equals), then the four lane groups
// combine (larger similarity, else lower index).  A wave owns PT 16-pixel
// tiles; the work group stages up to KT modes at a time in LDS.
//
// SPLIT (the split form's arithmetic): the pixels come as their BF16 high and
// low parts (x16, x16l) and the modes split into the same; each similarity
// takes hi.hi + hi.lo + lo.hi on v_mfma_f32_16x16x32_bf16 (lane (g, r) feeds
// dimensions 8g..8g+7 of mode r and of pixel r per 32-dimension step), with
// the same output layout, so a similarity is within 3 * 2^-16 of exact, as in
// the split form's steps.  The modes are split once, as they are staged, into
// two BF16 LDS tiles.
template <int DP, bool SPLIT>
__global__ __launch_bounds__(256) void k_assign(Batch bt, const float* __restrict__ x,
                                                const uint16_t* __restrict__ xh, const uint16_t* __restrict__ xl,
                                                const float* __restrict__ modes, int k1_slot, int mode,
                                                uint8_t* __restrict__ elig, const int* __restrict__ rank,
                                                const int* __restrict__ fg_idx) {
  constexpr int KJ = DP / 4;
  constexpr int KS = DP / 32;  // 32-dimension steps of the split form
  constexpr int PT = DP == 32 ? 4 : (DP == 64 ? 2 : 1);
  constexpr int KT = 64;
  constexpr int LD = DP + 4;   // padded FP32 LDS row
  constexpr int LDB = DP + 8;  // padded BF16 LDS row (16-byte aligned)
  constexpr int SM_BYTES = SPLIT ? 2 * KT * LDB * 2 : KT * LD * 4;
  const int f = blockIdx.y;
  const FrameGeo& g = bt.geo[f];
  const int n = g.n;
  if ((int)blockIdx.x * 64 * PT >= n) return;
  int* meta = bt.meta + (int64_t)f * META_COUNT;
  const int k0 = mode == 0 ? round_tab(bt, f).k_modes : 0;
  const int k1 = mode == 0 ? k0 + meta[k1_slot] : round_tab(bt, f).k_modes;
  const float thr = g.thr;
  int* labels = g.labels;
  if (SPLIT) {
    xh += g.row0 * DP;
    xl += g.row0 * DP;
  } else {
    x += g.row0 * DP;
  }
  modes += g.row0 * DP;
  if (elig) elig += g.elig0;
  if (rank) rank += g.row0;
  if (fg_idx) fg_idx += g.row0;
  __shared__ __align__(16) unsigned char smraw[SM_BYTES];
  float* sm = reinterpret_cast<float*>(smraw);
  __bf16* smh = reinterpret_cast<__bf16*>(smraw);
  __bf16* sml = smh + KT * LDB;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int gq = lane >> 4, r = lane & 15;
  const int p0 = (int)blockIdx.x * 64 * PT + wave * 16 * PT;
  float xb[PT][SPLIT ? 1 : KJ];
  bf16x8 xbh[PT][SPLIT ? KS : 1], xbl[PT][SPLIT ? KS : 1];
#pragma unroll
  for (int t = 0; t < PT; ++t) {
    const int i = p0 + 16 * t + r;
    if constexpr (SPLIT) {
      const bf16x8 z = {};
#pragma unroll
      for (int j = 0; j < KS; ++j) {
        xbh[t][j] = i < n ? *reinterpret_cast<const bf16x8*>(xh + (int64_t)i * DP + 8 * gq + 32 * j) : z;
        xbl[t][j] = i < n ? *reinterpret_cast<const bf16x8*>(xl + (int64_t)i * DP + 8 * gq + 32 * j) : z;
      }
    } else {
#pragma unroll
      for (int j = 0; j < KJ; j += 4) {
        const float4 v = i < n ? *reinterpret_cast<const float4*>(x + (int64_t)i * DP + gq * KJ + j)
                               : make_float4(0.f, 0.f, 0.f, 0.f);
        xb[t][j] = v.x;
        xb[t][j + 1] = v.y;
        xb[t][j + 2] = v.z;
        xb[t][j + 3] = v.w;
      }
    }
  }
  float best[PT];
  int arg[PT];
#pragma unroll
  for (int t = 0; t < PT; ++t) {
    best[t] = -INFINITY;
    arg[t] = -1;
  }
  for (int kb = k0; kb < k1; kb += KT) {
    const int cnt = min(KT, k1 - kb);
    const int rows = (cnt + 15) & ~15;
    __syncthreads();
    for (int e = threadIdx.x; e < rows * DP; e += 256) {
      const int q = e / DP, d = e - q * DP;
      const float v = q < cnt ? modes[(int64_t)(kb + q) * DP + d] : 0.f;
      if constexpr (SPLIT) {
        const __bf16 h = (__bf16)v;
        smh[q * LDB + d] = h;
        sml[q * LDB + d] = (__bf16)(v - (float)h);
      } else {
        sm[q * LD + d] = v;
      }
    }
    __syncthreads();
    for (int mt = 0; mt < rows; mt += 16) {
      float a[SPLIT ? 1 : KJ];
      bf16x8 ah[SPLIT ? KS : 1], al[SPLIT ? KS : 1];
      if constexpr (SPLIT) {
#pragma unroll
        for (int j = 0; j < KS; ++j) {
          ah[j] = *reinterpret_cast<const bf16x8*>(&smh[(mt + r) * LDB + 8 * gq + 32 * j]);
          al[j] = *reinterpret_cast<const bf16x8*>(&sml[(mt + r) * LDB + 8 * gq + 32 * j]);
        }
      } else {
#pragma unroll
        for (int j = 0; j < KJ; j += 4) {
          const float4 v = *reinterpret_cast<const float4*>(&sm[(mt + r) * LD + gq * KJ + j]);
          a[j] = v.x;
          a[j + 1] = v.y;
          a[j + 2] = v.z;
          a[j + 3] = v.w;
        }
      }
#pragma unroll
      for (int t = 0; t < PT; ++t) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        if constexpr (SPLIT) {
#pragma unroll
          for (int j = 0; j < KS; ++j) {
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[j], xbh[t][j], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[j], xbl[t][j], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[j], xbh[t][j], acc, 0, 0, 0);
          }
        } else {
#pragma unroll
          for (int j = 0; j < KJ; ++j) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[j], xb[t][j], acc, 0, 0, 0);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int idx = kb + mt + 4 * gq + e;
          if (mt + 4 * gq + e < cnt && acc[e] > best[t]) {
            best[t] = acc[e];
            arg[t] = idx;
          }
        }
      }
    }
  }
  int tally = 0;
#pragma unroll
  for (int t = 0; t < PT; ++t) {
#pragma unroll
    for (int off = 16; off <= 32; off <<= 1) {
      const float ob = __shfl_xor(best[t], off, 64);
      const int oa = __shfl_xor(arg[t], off, 64);
      if (ob > best[t] || (ob == best[t] && oa < arg[t])) {
        best[t] = ob;
        arg[t] = oa;
      }
    }
    const int i = p0 + 16 * t + r;
    if (gq == 0 && i < n) {
      if (mode == 0) {
        const int pos = rank[i];
        uint8_t e = elig[pos];
        if (e && best[t] >= thr) {
          elig[pos] = 0;
          e = 0;
        }
        tally += e ? 1 : 0;
      } else {
        if (labels) labels[fg_idx[i]] = arg[t];
        tally += best[t] < thr ? 1 : 0;
      }
    }
  }
  // One counter update per work group.  Coverage only tells whether any
  // pixel is left to seed, so it stores a flag instead of adding (updates of
  // one address from every work group queue behind each other); labels add
  // the exact count.
  __shared__ int s_tally[4];
  tally = wave_sum_i(tally);
  if (lane == 0) s_tally[wave] = tally;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int t = s_tally[0] + s_tally[1] + s_tally[2] + s_tally[3];
    if (t > 0) {
      if (mode == 0)
        meta[META_LEFT] = 1;
      else
        atomicAdd(meta + META_LEFT, t);
    }
  }
}

__global__ __launch_bounds__(256) void k_iota(Batch bt, int* __restrict__ p) {
  const int f = blockIdx.y;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < round_tab(bt, f).nact) p[bt.geo[f].row0 + i] = i;
}

// meta[slot] of every frame from rt.nact (from_rt) or to `value`.
__global__ __launch_bounds__(256) void k_set_slot(Batch bt, int slot, int from_rt, int value) {
  const int f = blockIdx.x * 256 + threadIdx.x;
  if (f < bt.F) bt.meta[(int64_t)f * META_COUNT + slot] = from_rt ? round_tab(bt, f).nact : value;
}

// Copy every frame's counters (n_words 32-bit words from bt.meta, which the
// 64-bit counters follow) into host memory at dst[4..], then, after a
// system-scope fence, write `seq` to dst[0]: the host polls dst[0] instead of
// waiting on an event.  One work group.
__global__ __launch_bounds__(256) void k_publish(Batch bt, int n_words, int* __restrict__ dst, int seq) {
  volatile int* out = dst;
  for (int i = threadIdx.x; i < n_words; i += 256) out[4 + i] = bt.meta[i];
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) {
    out[0] = seq;
    __threadfence_system();
  }
}

__global__ __launch_bounds__(256) void k_fill_labels(Batch bt) {
  const FrameGeo& g = bt.geo[blockIdx.y];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g.labels && i < g.desc.n_pixels) g.labels[i] = -1;
}


__global__ __launch_bounds__(256) void k_modes_out(Batch bt, const float* __restrict__ modes,
                                                   const int* __restrict__ mode_counts, int dp, int dim,
                                                   const int* __restrict__ out_off, float* __restrict__ out,
                                                   int* __restrict__ out_counts) {
  const int f = blockIdx.y;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int k = round_tab(bt, f).k_modes;
  if (t >= (int64_t)k * dim) return;
  const int64_t r = t / dim, d = t - r * dim;
  const int64_t src = bt.geo[f].row0 + r, dst = (int64_t)out_off[f] + r;
  out[dst * dim + d] = modes[src * dp + d];
  if (d == 0 && out_counts) out_counts[dst] = mode_counts[src];
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

// ------------------------------------------------------------------ adjoint of the unrolled steps

// Rows of m centres between the caller's [m][dim] layout and the padded
// [m_pad][DP] one (zero padding; rows m..m_pad-1 zero).
__global__ __launch_bounds__(256) void k_rows_in(int m, int m_pad, int dim, int dp, const float* __restrict__ src,
                                                 float* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)m_pad * dp) return;
  const int64_t r = t / dp, d = t - r * dp;
  dst[t] = (r < m && d < dim) ? src[r * dim + d] : 0.f;
}

__global__ __launch_bounds__(256) void k_rows_out(int m, int dp, int dim, const float* __restrict__ src,
                                                  float* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)m * dim) return;
  const int64_t r = t / dim, d = t - r * dim;
  dst[t] = src[r * dp + d];
}

// dL/dV of the last step per centre (one wave per centre):
// gv = (g - (g . y) y) / |V|, the adjoint of the renormalisation y = V / |V|.
// Rows m..m_pad-1 are zero.
template <int DP>
__global__ __launch_bounds__(256) void k_unroll_gv(int m, int m_pad, int dim, const float* __restrict__ y,
                                                   const float* __restrict__ vnorm, const float* __restrict__ gy,
                                                   float* __restrict__ gv) {
  constexpr int PER = DP / 64 > 0 ? DP / 64 : 1;  // dimensions per lane
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (j >= m_pad) return;
  float yv[PER], gvv[PER];
  float dot = 0.f;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int d = lane + 64 * k;
    const bool on = j < m && d < dim;
    yv[k] = on ? y[(int64_t)j * dim + d] : 0.f;
    gvv[k] = on ? gy[(int64_t)j * dim + d] : 0.f;
    dot = fmaf(yv[k], gvv[k], dot);
  }
  for (int o = 32; o >= 1; o >>= 1) dot += __shfl_xor(dot, o, 64);
  const float inv = j < m ? 1.0f / vnorm[j] : 0.f;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int d = lane + 64 * k;
    if (d < DP) gv[(int64_t)j * DP + d] = (gvv[k] - dot * yv[k]) * inv;
  }
}

// Zero a strided [n_pixels][dim] tensor (element (p, c) at p*ps + c*cs).
__global__ __launch_bounds__(256) void k_zero_strided(int64_t n_pixels, int dim, int64_t ps, int64_t cs,
                                                      float* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= n_pixels * dim) return;
  const int64_t p = t / dim, c = t - p * dim;
  out[p * ps + c * cs] = 0.f;
}

// Gradient of the loss with respect to the raw embeddings, for the last of
// the unrolled steps (the only one whose derivative is not zero almost
// everywhere):
//   dL/dx_i = sum_j [yp_j . x_i >= thr] gv_j,   dL/de_i = (I - x_i x_i^T) dL/dx_i / |e_i|.
// S = Yp X^T and G^T = GV^T W are chained on v_mfma_f32_16x16x4_f32 without
// storing W: the S accumulator of lane (g, r) holds seeds 4g..4g+3 of pixel
// r, which is exactly the B operand of the k-steps i = 0..3 of the second
// product when k-step i pairs lane group g with seed 4g + i.  A wave owns PT
// tiles of 16 pixels and loops over all seed tiles; no cross-wave
// reduction.  yp and gv are padded to a multiple of 16 rows with zeros.
template <int DP, int PT>
__global__ __launch_bounds__(256) void k_unroll_grad(Batch bt, const float* __restrict__ x32,
                                                     const int* __restrict__ fg_idx, const float* __restrict__ enorm,
                                                     const float* __restrict__ yp, const float* __restrict__ gv,
                                                     int m_pad, int dim, int64_t ps, int64_t cs,
                                                     float* __restrict__ grad) {
  constexpr int KS = DP / 4;    // k-steps of S (4 dimensions each)
  constexpr int NDB = DP / 16;  // 16-dimension blocks of G^T
  const FrameGeo& g0 = bt.geo[0];
  const int n = g0.n;
  const float thr = g0.thr;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, r = lane & 15;
  const int tile0 = ((int)blockIdx.x * 4 + wave) * PT;  // first 16-pixel tile of this wave
  if (tile0 * 16 >= n) return;
  // B operands of S: x[pixel r][4k + g].
  float xb[PT][KS];
  f32x4 acc[PT][NDB];
#pragma unroll
  for (int p = 0; p < PT; ++p) {
    const int row = (tile0 + p) * 16 + r;
#pragma unroll
    for (int k = 0; k < KS; ++k) xb[p][k] = row < n ? x32[(int64_t)row * DP + 4 * k + g] : 0.f;
#pragma unroll
    for (int db = 0; db < NDB; ++db) acc[p][db] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  const f32x4 cinit = {-thr, -thr, -thr, -thr};
  for (int s0 = 0; s0 < m_pad; s0 += 16) {
    // A operands: yp[seed s0 + r][4k + g]; gv[seed s0 + 4g + i][16 db + r].
    float ya[KS];
#pragma unroll
    for (int k = 0; k < KS; ++k) ya[k] = yp[(int64_t)(s0 + r) * DP + 4 * k + g];
    float ga[4][NDB];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int db = 0; db < NDB; ++db) ga[i][db] = gv[(int64_t)(s0 + 4 * g + i) * DP + 16 * db + r];
#pragma unroll
    for (int p = 0; p < PT; ++p) {
      f32x4 sc = cinit;
#pragma unroll
      for (int k = 0; k < KS; ++k) sc = __builtin_amdgcn_mfma_f32_16x16x4f32(ya[k], xb[p][k], sc, 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float w = (fbits(sc[i]) >> 31) ? 0.f : 1.f;
#pragma unroll
        for (int db = 0; db < NDB; ++db)
          acc[p][db] = __builtin_amdgcn_mfma_f32_16x16x4f32(ga[i][db], w, acc[p][db], 0, 0, 0);
      }
    }
  }
  // Epilogue: lane (g, r) holds dL/dx[pixel r][16 db + 4 g + i].
#pragma unroll
  for (int p = 0; p < PT; ++p) {
    const int row = (tile0 + p) * 16 + r;
    const bool live = row < n;
    float xv[NDB][4];
    float dot = 0.f;
#pragma unroll
    for (int db = 0; db < NDB; ++db) {
      const float4 u = live ? *reinterpret_cast<const float4*>(x32 + (int64_t)row * DP + 16 * db + 4 * g)
                            : make_float4(0.f, 0.f, 0.f, 0.f);
      xv[db][0] = u.x; xv[db][1] = u.y; xv[db][2] = u.z; xv[db][3] = u.w;
#pragma unroll
      for (int i = 0; i < 4; ++i) dot = fmaf(acc[p][db][i], xv[db][i], dot);
    }
    dot += __shfl_xor(dot, 16, 64);
    dot += __shfl_xor(dot, 32, 64);
    if (!live) continue;
    const float inv = 1.0f / enorm[row];
    const int64_t pix = fg_idx[row];
#pragma unroll
    for (int db = 0; db < NDB; ++db)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int c = 16 * db + 4 * g + i;
        if (c < dim) grad[pix * ps + (int64_t)c * cs] = (acc[p][db][i] - dot * xv[db][i]) * inv;
      }
  }
}

static inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

hipError_t launch_mask_count(hipStream_t s, const Batch& b, int* block_counts) {
  if (b.max_mblk <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mask_count, dim3((unsigned)b.max_mblk, b.F), dim3(256), 0, s, b.geo, block_counts);
  return hipGetLastError();
}

hipError_t launch_scan_blocks(hipStream_t s, const Batch& b, int* block_counts) {
  hipLaunchKernelGGL(k_scan_blocks, dim3(b.F), dim3(1024), 0, s, b.geo, block_counts, b.meta);
  return hipGetLastError();
}

hipError_t launch_compact(hipStream_t s, const Batch& b, int dp, const int* block_offsets, int* fg_idx, float* x32,
                          float* x32t, uint16_t* x16, uint16_t* xlo, float* enorm, int64_t row_cap) {
  if (xlo && !x16) return hipErrorInvalidValue;
  if (b.max_mblk <= 0) return hipSuccess;
  const dim3 grid((unsigned)b.max_mblk, b.F);
  switch (dp) {
    case 32:
      hipLaunchKernelGGL(k_compact<32>, grid, dim3(256), 0, s, b.geo, block_offsets, fg_idx, x32, x16, xlo, enorm,
                         b.meta, row_cap);
      break;
    case 64:
      hipLaunchKernelGGL(k_compact<64>, grid, dim3(256), 0, s, b.geo, block_offsets, fg_idx, x32, x16, xlo, enorm,
                         b.meta, row_cap);
      break;
    case 128:
      hipLaunchKernelGGL(k_compact<128>, grid, dim3(256), 0, s, b.geo, block_offsets, fg_idx, x32, x16, xlo, enorm,
                         b.meta, row_cap);
      break;
    default:
      return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || b.max_blocks <= 0 || !x32t) return e;
  // The transposed copy, one wave per 32-pixel block of the largest frame.
  const dim3 tgrid((unsigned)b.max_blocks, b.F);
  switch (dp) {
    case 32:
      hipLaunchKernelGGL(k_transpose<32>, tgrid, dim3(64), 0, s, b.geo, x32, x32t, b.meta, row_cap);
      break;
    case 64:
      hipLaunchKernelGGL(k_transpose<64>, tgrid, dim3(64), 0, s, b.geo, x32, x32t, b.meta, row_cap);
      break;
    default:
      hipLaunchKernelGGL(k_transpose<128>, tgrid, dim3(64), 0, s, b.geo, x32, x32t, b.meta, row_cap);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_seed_order(hipStream_t s, const Batch& b, const uint64_t keys[4], int* order, int* rank,
                             uint8_t* elig) {
  if (b.max_n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_seed_order, dim3(cdiv(elig_len(b.max_n), 256), b.F), dim3(256), 0, s, b.geo, 0, 0, keys[0],
                     keys[1], keys[2], keys[3], order, rank, elig, b.meta);
  return hipGetLastError();
}

hipError_t launch_seed_order_plain(hipStream_t s, int n, int half_bits, const uint64_t keys[4], int* order) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_seed_order, dim3(cdiv(n, 256)), dim3(256), 0, s, nullptr, n, half_bits, keys[0], keys[1],
                     keys[2], keys[3], order, nullptr, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t launch_select(hipStream_t s, const Batch& b, const int* order, uint8_t* elig, int* seed_pos,
                         int* seed_fg) {
  hipLaunchKernelGGL(k_select, dim3(b.F), dim3(1024), 0, s, b, order, elig, seed_pos, seed_fg);
  return hipGetLastError();
}

hipError_t launch_set_tables(hipStream_t s, const FrameGeo& g, const RoundTab& rt, FrameGeo* geo, RoundTab* rtab,
                             int* meta, unsigned long long* meta64) {
  hipLaunchKernelGGL(k_set_tables, dim3(1), dim3(64), 0, s, g, rt, geo, rtab, meta, meta64);
  return hipGetLastError();
}

hipError_t launch_geo_from_count(hipStream_t s, const Batch& b, int64_t row_cap) {
  hipLaunchKernelGGL(k_geo_from_count, dim3(1), dim3(64), 0, s, b, row_cap);
  return hipGetLastError();
}

hipError_t launch_init_seeds(hipStream_t s, const int* seed_fg, int m, int n, const float* x32, int dp, float* y,
                             int* meta) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_init_seeds, dim3(cdiv((int64_t)m * dp, 256)), dim3(256), 0, s, seed_fg, m, n, x32, dp, y,
                     meta);
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

// Seed groups of the fused step: enough seeds per pixel read to keep the loads
// well below the matrix-core rate, few enough registers for several waves per
// SIMD.  Compiled group sizes per (form, padded D):
//   FP32:       D 32 -> 16, 32, 64; D 64 -> 16, 32; D 128 -> 16.
//   BF16:       D 32 -> 32, 64, 128; D 64 -> 16, 32, 64; D 128 -> 16, 32.
//   split BF16: D 32 -> 32, 64; D 64 -> 16, 32; D 128 -> 16.
// Fused-step shapes compiled with WV waves per group.  Four waves: every
// shape.  Eight or sixteen: DP = 32 only, where a wave's operands fit the
// registers a wave of a 512- or 1024-lane group may hold without scratch (FP32
// groups of more than 16 seeds do not at sixteen waves, nor split-BF16 groups
// of any size), and the wave tree's LDS (WV/2 slots of ST x DP/16 accumulator
// tiles of 1 KiB) fits in 64 KiB.
constexpr bool shift_shape_ok(int form, bool count, int dp, int st, int wv) {
  if (wv == 4) return true;
  if ((wv != 8 && wv != 16) || dp != 32) return false;
  // Sixteen waves leave 128 registers per lane: not enough for the split
  // form or the larger FP32 / BF16 groups without spilling; eight leave 256,
  // not enough for 128-seed split groups.
  if (wv == 16 && (form == FORM_SPLIT || (form == FORM_FP32 && st >= 2) || (form == FORM_BF16 && st >= 4)))
    return false;
  if (wv == 8 && form == FORM_SPLIT && st >= 8 && !count) return false;
  return count || (wv / 2) * st * (dp / 16) * 1024 <= 65536;
}

static int max_group(int form, int dp) {
  if (form != FORM_FP32 && dp <= 32) return 128;
  if (form == FORM_BF16) return dp <= 64 ? 64 : 32;
  return dp <= 32 ? 64 : (dp <= 64 ? 32 : 16);
}
static int min_group(int form, int dp) { return (form != FORM_FP32 && dp <= 32) ? 32 : 16; }

Tiling make_tiling(int form, int dp, int want_seeds, int want_items, int want_chunks, int want_waves) {
  Tiling t;
  // Defaults from sweeps on the 512x512, D = 32 frame and the 64-frame batch:
  // 32-seed groups (larger ones for many centres, chosen by the caller), four
  // waves per group (the caller asks for eight on single frames) and
  // kWaveBudget / waves items, <= 256 chunks.
  int def = dp <= 64 ? 32 : 16;
  int g = want_seeds > 0 ? want_seeds : def;
  int gs = min_group(form, dp);
  while (gs * 2 <= g && gs * 2 <= max_group(form, dp)) gs *= 2;
  t.group_seeds = gs;
  t.max_chunks = want_chunks > 0 ? std::max(1, std::min(want_chunks, 4096)) : kMaxChunks;
  // Waves per group: 4, 8 or 16, halved until the shape is compiled.
  int wv = want_waves > 0 ? want_waves : kWaves;
  wv = wv >= 16 ? 16 : (wv >= 8 ? 8 : 4);
  while (wv > 4 && !shift_shape_ok(form, false, dp, gs / 16, wv)) wv /= 2;
  t.waves = wv;
  t.target_items = want_items > 0 ? std::max(8, std::min(want_items, 1 << 16)) : kWaveBudget / wv;
  return t;
}

size_t shift_partial_rows(const Tiling& t, int cap) {
  const int64_t a = std::min<int64_t>((int64_t)t.max_chunks * cap, (int64_t)t.target_items * t.group_seeds + cap);
  return (size_t)std::max<int64_t>(a, 1);
}

// Work groups of a fused-step launch for at most `cap` active seeds: enough
// for the items of any active count up to cap (groups * chunks never exceeds
// groups(cap) * min(n_blocks, max_chunks)), at most target_items; beyond
// that the work groups loop over the items.
static unsigned shift_grid(int cap, const Tiling& t, int n_blocks) {
  const int groups = cap > 0 ? (cap + t.group_seeds - 1) / t.group_seeds : 1;
  const int lim = std::max(1, std::min(n_blocks, t.max_chunks));
  int64_t items = (int64_t)groups * lim;
  if (items > t.target_items) items = t.target_items;
  unsigned grid = (unsigned)((items + 7) / 8 * 8);
  return grid < 8 ? 8 : grid;
}

template <int FORM, bool CNT, int DPV, int STV, int WV>
static hipError_t shift_launch_one(hipStream_t s, dim3 grid, const Batch& b, const void* xrm, const void* xt,
                                   const uint16_t* xrl, const float* y, const int* active,
                                   const IterCtl& ctl, const Tiling& t, float* partial, int* pcount, hipEvent_t ev0,
                                   hipEvent_t ev1) {
  if constexpr (!shift_shape_ok(FORM, CNT, DPV, STV, WV)) {
    return hipErrorInvalidValue;
  } else {
    constexpr bool BFV = FORM != FORM_FP32, SPV = FORM == FORM_SPLIT;
    if (ev0 || ev1)
      hipExtLaunchKernelGGL((k_shift<BFV, SPV, CNT, DPV, STV, WV>), grid, dim3(64 * WV), 0, s, ev0, ev1, 0, b, xrm, xt,
                            xrl, y, active, ctl, t, partial, pcount);
    else
      hipLaunchKernelGGL((k_shift<BFV, SPV, CNT, DPV, STV, WV>), grid, dim3(64 * WV), 0, s, b, xrm, xt, xrl, y,
                         active, ctl, t, partial, pcount);
    return hipGetLastError();
  }
}

template <int FORM, bool CNT, int DPV, int STV>
static hipError_t shift_launch_waves(hipStream_t s, dim3 grid, const Batch& b, const void* xrm, const void* xt,
                                     const uint16_t* xrl, const float* y, const int* active,
                                     const IterCtl& ctl, const Tiling& t, float* partial, int* pcount, hipEvent_t ev0,
                                     hipEvent_t ev1) {
  switch (t.waves) {
    case 4:
      return shift_launch_one<FORM, CNT, DPV, STV, 4>(s, grid, b, xrm, xt, xrl, y, active, ctl, t, partial,
                                                      pcount, ev0, ev1);
    case 8:
      return shift_launch_one<FORM, CNT, DPV, STV, 8>(s, grid, b, xrm, xt, xrl, y, active, ctl, t, partial,
                                                      pcount, ev0, ev1);
    case 16:
      return shift_launch_one<FORM, CNT, DPV, STV, 16>(s, grid, b, xrm, xt, xrl, y, active, ctl, t, partial,
                                                       pcount, ev0, ev1);
    default: return hipErrorInvalidValue;
  }
}

static hipError_t shift_dispatch(hipStream_t s, const Batch& b, int form, bool count, int dp, const Tiling& t,
                                 const void* xrm, const void* xt, const uint16_t* xrl,
                                 const float* y, const int* active, const IterCtl& ctl, int cap, float* partial,
                                 int* pcount, hipEvent_t ev0, hipEvent_t ev1) {
  if (cap <= 0 || b.max_blocks <= 0) {
    // Nothing to launch; the events still mark this point of the stream.
    hipError_t e = ev0 ? hipEventRecord(ev0, s) : hipSuccess;
    if (e == hipSuccess && ev1) e = hipEventRecord(ev1, s);
    return e;
  }
  if (form == FORM_SPLIT && !xrl) return hipErrorInvalidValue;
  if (form == FORM_FP32 && !count && !xt) return hipErrorInvalidValue;
  const dim3 grid(shift_grid(cap, t, b.max_blocks), b.F);
  const int key = form * 1000000 + (count ? 100000 : 0) + dp * 100 + t.group_seeds / 16;
// Fused steps: every (form, padded D, seed tiles per group) shape above.
// Window counts: FP32, and split BF16 for the split form (its similarities
// are within 5e-5 of exact, as in its iteration); the plain BF16 form counts
// in FP32.
#define FMS_SHIFT_SHAPES(X)                                                                                   \
  X(FORM_FP32, 32, 1) X(FORM_FP32, 32, 2) X(FORM_FP32, 32, 4) X(FORM_FP32, 64, 1) X(FORM_FP32, 64, 2)        \
  X(FORM_FP32, 128, 1) X(FORM_BF16, 32, 2) X(FORM_BF16, 32, 4) X(FORM_BF16, 32, 8) X(FORM_BF16, 64, 1)      \
  X(FORM_BF16, 64, 2) X(FORM_BF16, 64, 4) X(FORM_BF16, 128, 1) X(FORM_BF16, 128, 2) X(FORM_SPLIT, 32, 2)    \
  X(FORM_SPLIT, 32, 4) X(FORM_SPLIT, 32, 8) X(FORM_SPLIT, 64, 1) X(FORM_SPLIT, 64, 2) X(FORM_SPLIT, 128, 1)
#define FMS_COUNT_SHAPES(X) X(FORM_FP32, 32, 1) X(FORM_FP32, 32, 2) X(FORM_FP32, 32, 4) X(FORM_FP32, 64, 1) \
  X(FORM_FP32, 64, 2) X(FORM_FP32, 128, 1) X(FORM_SPLIT, 32, 2) X(FORM_SPLIT, 32, 4) X(FORM_SPLIT, 32, 8)      \
  X(FORM_SPLIT, 64, 1) X(FORM_SPLIT, 64, 2) X(FORM_SPLIT, 128, 1)
#define FMS_SHIFT_CASE(FV, DPV, STV)                                                                          \
  case FV * 1000000 + DPV * 100 + STV:                                                                        \
    return shift_launch_waves<FV, false, DPV, STV>(s, grid, b, xrm, xt, xrl, y, active, ctl, t, partial, \
                                                   pcount, ev0, ev1);
#define FMS_COUNT_CASE(FV, DPV, STV)                                                                          \
  case FV * 1000000 + 100000 + DPV * 100 + STV:                                                               \
    return shift_launch_waves<FV, true, DPV, STV>(s, grid, b, xrm, xt, xrl, y, active, ctl, t, partial,  \
                                                  pcount, ev0, ev1);
  switch (key) {
    FMS_SHIFT_SHAPES(FMS_SHIFT_CASE)
    FMS_COUNT_SHAPES(FMS_COUNT_CASE)
    default: return hipErrorInvalidValue;
  }
#undef FMS_SHIFT_CASE
#undef FMS_COUNT_CASE
#undef FMS_SHIFT_SHAPES
#undef FMS_COUNT_SHAPES
}

hipError_t launch_shift(hipStream_t s, const Batch& b, int form, int dp, const Tiling& t, const void* xrm,
                        const void* xt, const uint16_t* xrl, const float* y, const int* active,
                        const IterCtl& ctl, int cap, float* partial, hipEvent_t ev0, hipEvent_t ev1) {
  return shift_dispatch(s, b, form, false, dp, t, xrm, xt, xrl, y, active, ctl, cap, partial, nullptr, ev0,
                        ev1);
}

hipError_t launch_reduce(hipStream_t s, const Batch& b, int dp, const Tiling& t, const float* partial,
                         const int* active, float* y, uint8_t* state, int* iters, int* next_active,
                         float* yc_next, const IterCtl& ctl, int cap, int mode, float* vnorm, const float* ycur,
                         float* ring, int64_t ring_stride, int ring_len) {
  if (ring && ring_len < 1) return hipErrorInvalidValue;
  if (cap <= 0) return hipSuccess;
  // Enough work groups for the seed tiles of the largest active count; they
  // loop when the active count shrinks and tiles get smaller.
  const ChunkPlan cp = plan_chunks(cap, t, b.max_blocks);
  int P = 1;
  while (P * 8 < cp.n_chunks && (dp / 4) * P * 2 <= 256) P <<= 1;
  const int spw = std::max(1, 256 / ((dp / 4) * P));
  const dim3 grid(cdiv(cap, spw), b.F), block(256);
#define FMS_REDUCE_CASE(DPV)                                                                                      \
  hipLaunchKernelGGL(k_reduce<DPV>, grid, block, 0, s, b, partial, active, ycur, y, state, iters, next_active,     \
                     yc_next, vnorm, ctl, t, mode, ring, ring_stride, ring_len)
  switch (dp) {
    case 32: FMS_REDUCE_CASE(32); break;
    case 64: FMS_REDUCE_CASE(64); break;
    case 128: FMS_REDUCE_CASE(128); break;
    default: return hipErrorInvalidValue;
  }
#undef FMS_REDUCE_CASE
  return hipGetLastError();
}

hipError_t launch_count(hipStream_t s, const Batch& b, int form, int dp, const Tiling& t, const void* xrm,
                        const uint16_t* xrl, const float* y, const int* list, int m, int* pcount, int* counts,
                        int m_slot) {
  if (m <= 0 || b.max_blocks <= 0) return hipSuccess;
  if (form == FORM_BF16) return hipErrorInvalidValue;
  const IterCtl ctl{m_slot, -1, 0.0};
  hipError_t e = shift_dispatch(s, b, form, true, dp, t, xrm, nullptr, xrl, y, list, ctl, m, nullptr, pcount,
                                nullptr, nullptr);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_counts, dim3(cdiv(m, 4), b.F), dim3(256), 0, s, b, pcount, t, m_slot, counts);
  return hipGetLastError();
}

hipError_t launch_replay_begin(hipStream_t s, const Batch& b, int dp, int ring_len, const uint8_t* state,
                               const int* iters, const float* ring, int64_t ring_stride, int* cand, float* yr,
                               int* active, uint8_t* rstate, int* riters) {
  if (ring_len < 1) return hipErrorInvalidValue;
  switch (dp) {
#define FMS_RB_CASE(DPV)                                                                                     \
  case DPV:                                                                                                  \
    hipLaunchKernelGGL(k_replay_begin<DPV>, dim3(b.F), dim3(1024), 0, s, b, ring_len, state, iters, ring,    \
                       ring_stride, cand, yr, active, rstate, riters);                                       \
    break;
    FMS_RB_CASE(32)
    FMS_RB_CASE(64)
    FMS_RB_CASE(128)
#undef FMS_RB_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_gamma_cut(hipStream_t s, const Batch& b, double gamma, const int* iters, uint8_t* state) {
  hipLaunchKernelGGL(k_gamma_cut, dim3(b.F), dim3(1024), 0, s, b, gamma, iters, state);
  return hipGetLastError();
}

hipError_t launch_replay_end(hipStream_t s, const Batch& b, int dp, int cap, int ring_len, const int* cand,
                             int* iters, const float* yr, const uint8_t* rstate, const int* riters, float* y,
                             uint8_t* state) {
  if (cap <= 0) return hipSuccess;
  const dim3 grid(cdiv(cap, 256), b.F), block(256);
  switch (dp) {
#define FMS_RE_CASE(DPV)                                                                                     \
  case DPV:                                                                                                  \
    hipLaunchKernelGGL(k_replay_end<DPV>, grid, block, 0, s, b, cap, ring_len, cand, iters, yr, rstate,       \
                       riters, y, state);                                                                    \
    break;
    FMS_RE_CASE(32)
    FMS_RE_CASE(64)
    FMS_RE_CASE(128)
#undef FMS_RE_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_rank_converged(hipStream_t s, const Batch& b, const uint8_t* state, const int* counts, int* sorted,
                                int* scount, int* first) {
  hipLaunchKernelGGL(k_rank_converged, dim3(b.F), dim3(1024), 0, s, b, state, counts, sorted, scount, first);
  return hipGetLastError();
}

hipError_t launch_greedy(hipStream_t s, const Batch& b, const uint32_t* bits, const float* y, const int* sorted,
                         const int* scount, int ncand_slot, int acc_slot, int dp, float* modes, int* mode_counts,
                         const int* first) {
  hipLaunchKernelGGL(k_greedy, dim3(b.F), dim3(1024), 0, s, b, bits, y, sorted, scount, ncand_slot, acc_slot, dp,
                     modes, mode_counts, first);
  return hipGetLastError();
}

int simbits_words(int ncols) { return std::max(2, ((ncols + 63) / 64) * 2); }

hipError_t launch_simbits(hipStream_t s, const Batch& b, int dp, const float* y, const int* rows, int m,
                          const int* cols, int ncols, const float* modes, int nmodes, uint32_t* bits, int rows_slot,
                          int cols_slot, int* first) {
  if (m <= 0) return hipSuccess;
  const unsigned part_c = cols && ncols > 0 ? (unsigned)((simbits_words(ncols) / 2) * cdiv(m, 64)) : 0u;
  const unsigned part_m = modes && nmodes > 0 ? (unsigned)((simbits_words(nmodes) / 2) * cdiv(m, 64)) : 0u;
  if (part_c + part_m == 0) return hipSuccess;
  const dim3 grid(part_c + part_m, b.F);
  const int split = (int)part_c;
#define FMS_SIM_CASE(DPV)                                                                                     \
  hipLaunchKernelGGL(k_simbits<DPV>, grid, dim3(256), 0, s, b, y, rows, cols, modes, bits, rows_slot, cols_slot, \
                     split, first)
  switch (dp) {
    case 32: FMS_SIM_CASE(32); break;
    case 64: FMS_SIM_CASE(64); break;
    case 128: FMS_SIM_CASE(128); break;
    default: return hipErrorInvalidValue;
  }
#undef FMS_SIM_CASE
  return hipGetLastError();
}

hipError_t launch_round_begin(hipStream_t s, const Batch& b, int cap, bool nsel_from_rt, int* active,
                              uint8_t* state, int* iters, const int* seed_fg, const float* x32, int dp, float* y) {
  const dim3 grid(cdiv(std::max(cap, 1), 256), b.F), block(256);
  const int fr = nsel_from_rt ? 1 : 0;
  switch (dp) {
    case 32:
      hipLaunchKernelGGL(k_round_begin<32>, grid, block, 0, s, b, cap, fr, active, state, iters, seed_fg, x32, y);
      break;
    case 64:
      hipLaunchKernelGGL(k_round_begin<64>, grid, block, 0, s, b, cap, fr, active, state, iters, seed_fg, x32, y);
      break;
    case 128:
      hipLaunchKernelGGL(k_round_begin<128>, grid, block, 0, s, b, cap, fr, active, state, iters, seed_fg, x32, y);
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

hipError_t launch_assign(hipStream_t s, const Batch& b, int dp, bool split, const float* x32, const uint16_t* xh,
                         const uint16_t* xl, const float* modes, int k1_slot, int mode, uint8_t* elig,
                         const int* rank, const int* fg_idx) {
  if (b.max_n <= 0) return hipSuccess;
  if (split && (!xh || !xl)) return hipErrorInvalidValue;
  if (!split && !x32) return hipErrorInvalidValue;
  // Pixels per work group: 4 waves x PT 16-pixel tiles (PT = 4, 2, 1).
  const int pix = dp == 32 ? 256 : (dp == 64 ? 128 : 64);
  const dim3 grid(cdiv(b.max_n, pix), b.F), block(256);
#define FMS_ASSIGN(D, S) \
  hipLaunchKernelGGL((k_assign<D, S>), grid, block, 0, s, b, x32, xh, xl, modes, k1_slot, mode, elig, rank, fg_idx)
  switch (dp) {
    case 32:
      if (split) FMS_ASSIGN(32, true); else FMS_ASSIGN(32, false);
      break;
    case 64:
      if (split) FMS_ASSIGN(64, true); else FMS_ASSIGN(64, false);
      break;
    case 128:
      if (split) FMS_ASSIGN(128, true); else FMS_ASSIGN(128, false);
      break;
    default:
      return hipErrorInvalidValue;
  }
#undef FMS_ASSIGN
  return hipGetLastError();
}

hipError_t launch_publish(hipStream_t s, const Batch& b, int n_words, int* dst, int seq) {
  hipLaunchKernelGGL(k_publish, dim3(1), dim3(256), 0, s, b, n_words, dst, seq);
  return hipGetLastError();
}

hipError_t launch_set_slot(hipStream_t s, const Batch& b, int slot, bool from_rt, int value) {
  hipLaunchKernelGGL(k_set_slot, dim3(cdiv(b.F, 256)), dim3(256), 0, s, b, slot, from_rt ? 1 : 0, value);
  return hipGetLastError();
}

hipError_t launch_fill_labels(hipStream_t s, const Batch& b, int64_t max_pixels) {
  if (max_pixels <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_labels, dim3(cdiv(max_pixels, 256), b.F), dim3(256), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_iota(hipStream_t s, const Batch& b, int* p, int max_count) {
  if (max_count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_iota, dim3(cdiv(max_count, 256), b.F), dim3(256), 0, s, b, p);
  return hipGetLastError();
}

hipError_t launch_modes_out(hipStream_t s, const Batch& b, const float* modes, const int* mode_counts, int dp,
                            int dim, const int* out_off, float* out, int* out_counts, int max_rows) {
  if (max_rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_modes_out, dim3(cdiv((int64_t)max_rows * dim, 256), b.F), dim3(256), 0, s, b, modes,
                     mode_counts, dp, dim, out_off, out, out_counts);
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

hipError_t launch_rows_in(hipStream_t s, int m, int m_pad, int dim, int dp, const float* src, float* dst) {
  if (m_pad <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rows_in, dim3(cdiv((int64_t)m_pad * dp, 256)), dim3(256), 0, s, m, m_pad, dim, dp, src, dst);
  return hipGetLastError();
}

hipError_t launch_rows_out(hipStream_t s, int m, int dp, int dim, const float* src, float* dst) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rows_out, dim3(cdiv((int64_t)m * dim, 256)), dim3(256), 0, s, m, dp, dim, src, dst);
  return hipGetLastError();
}

hipError_t launch_unroll_gv(hipStream_t s, int m, int m_pad, int dim, int dp, const float* y, const float* vnorm,
                            const float* gy, float* gv) {
  if (m_pad <= 0) return hipSuccess;
  const dim3 grid(cdiv(m_pad, 4)), block(256);
  switch (dp) {
    case 32: hipLaunchKernelGGL(k_unroll_gv<32>, grid, block, 0, s, m, m_pad, dim, y, vnorm, gy, gv); break;
    case 64: hipLaunchKernelGGL(k_unroll_gv<64>, grid, block, 0, s, m, m_pad, dim, y, vnorm, gy, gv); break;
    case 128: hipLaunchKernelGGL(k_unroll_gv<128>, grid, block, 0, s, m, m_pad, dim, y, vnorm, gy, gv); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_zero_strided(hipStream_t s, int64_t n_pixels, int dim, int64_t ps, int64_t cs, float* out) {
  if (n_pixels <= 0 || dim <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_strided, dim3(cdiv(n_pixels * dim, 256)), dim3(256), 0, s, n_pixels, dim, ps, cs, out);
  return hipGetLastError();
}

hipError_t launch_unroll_grad(hipStream_t s, const Batch& b, int dp, const float* x32, const int* fg_idx,
                              const float* enorm, const float* yp, const float* gv, int m_pad, int dim, int64_t ps,
                              int64_t cs, float* grad) {
  if (b.max_n <= 0 || m_pad <= 0) return hipSuccess;
  const int tiles = (b.max_n + 15) / 16;
  switch (dp) {
    case 32:
      hipLaunchKernelGGL((k_unroll_grad<32, 4>), dim3(cdiv(tiles, 16)), dim3(256), 0, s, b, x32, fg_idx, enorm, yp, gv,
                         m_pad, dim, ps, cs, grad);
      break;
    case 64:
      hipLaunchKernelGGL((k_unroll_grad<64, 2>), dim3(cdiv(tiles, 8)), dim3(256), 0, s, b, x32, fg_idx, enorm, yp, gv,
                         m_pad, dim, ps, cs, grad);
      break;
    case 128:
      hipLaunchKernelGGL((k_unroll_grad<128, 1>), dim3(cdiv(tiles, 4)), dim3(256), 0, s, b, x32, fg_idx, enorm, yp,
                         gv, m_pad, dim, ps, cs, grad);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace fms
