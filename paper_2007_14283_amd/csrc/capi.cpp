// Host runtime of the Faster Mean-shift library: handle and workspace, frame
// preparation, the round loop of the online seed optimisation policy
// (Sec. 3.2.2-3.2.4) and the C ABI declared in include/fms.h.
//
// The CPU steers the seed count and the GPU iterates the seeds (Fig. 3): the
// host reads a few counters back after each batch of GPU steps and after
// each round, and decides what to launch next.  Every call works on a batch
// of F >= 1 frames: each launch covers all of them (the frame is the second
// grid dimension), each frame keeps its own counters and OSOP state, and the
// rounds of the frames run in lockstep.  A single-frame call is a batch of
// one.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>

#include "fms.h"
#include "fms_internal.h"

namespace {

using fms::kMeta64;
using fms::META_BAD;
using fms::META_BADSEED;
using fms::META_COUNT;
using fms::META_LEFT;
using fms::META_N;
using fms::META_NACC;
using fms::META_NCAND;
using fms::META_NCONV;
using fms::META_NSEL;
using fms::META_REFINE_BAD;
using fms::META_REFINE_DIFF;
using fms::META_STEPS;

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  hipError_t ensure(size_t bytes) {
    if (bytes <= cap) return hipSuccess;
    if (p) {
      hipError_t e = hipFree(p);
      p = nullptr;
      cap = 0;
      if (e != hipSuccess) return e;
    }
    size_t want = std::max<size_t>(bytes + bytes / 4, 4096);
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
    cap = want;
    return hipSuccess;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

// Pinned host buffer that grows on demand (contents are not kept).
struct PinBuf {
  void* p = nullptr;
  size_t cap = 0;
  // An enqueued copy still reads or writes this buffer (cleared by a wait).
  bool busy = false;
  hipError_t ensure(size_t bytes, unsigned flags = hipHostMallocDefault) {
    if (bytes <= cap) return hipSuccess;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
    const size_t want = std::max<size_t>(bytes + bytes / 4, 4096);
    hipError_t e = hipHostMalloc(&p, want, flags);
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
    cap = want;
    return hipSuccess;
  }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

// SplitMix64 (Steele, Lea and Flood 2014): the seed order's round keys are
// the first four outputs for the user's seed.
uint64_t splitmix_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

void round_keys(uint64_t seed, uint64_t keys[4]) {
  uint64_t st = seed;
  for (int r = 0; r < 4; ++r) {
    st += 0x9E3779B97F4A7C15ull;
    keys[r] = splitmix_mix(st);
  }
}

int half_bits(int64_t n) {
  int k = 0;
  while ((int64_t(1) << k) < n) ++k;
  return std::max(1, (k + 1) / 2);
}

// Eq. 19 with the guards of the controller: no value without an instance, one
// seed when r / I >= 1.
bool eq19_n_min(double p_target, int64_t n_inst, double r, double* out) {
  if (n_inst <= 0) return false;
  const double ratio = r / double(n_inst);
  if (ratio >= 1.0) {
    *out = 1.0;
    return true;
  }
  *out = std::log(1.0 - std::exp(std::log(p_target) / double(n_inst))) / std::log(1.0 - ratio);
  return true;
}

int pad_dim(int dim) { return dim <= 32 ? 32 : (dim <= 64 ? 64 : 128); }

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

// Launches with at least kBigGroupMin centres per frame use seed groups of
// kBigGroup, and plain BF16 launches with at least kHugeGroupMin use
// kHugeGroup (where compiled): on the 512x512, D = 32 workload a fused step
// plus its reduction over 512 centres takes 16.6 us with 64-seed groups
// against 19.4 with 32, and over 8192 BF16 centres 82 us with 128-seed
// groups against 121 with 64 (larger groups reuse each pixel tile for more
// seeds; there a step's pixel loads, not its MFMA work, bound it).
constexpr int kBigGroup = 64;
constexpr int kBigGroupMin = 512;
constexpr int kHugeGroup = 128;
constexpr int kHugeGroupMin = 2048;

}  // namespace

// A fused-step decomposition chosen by fms_autotune for one step form, D
// class, pixel-count bucket and active-seed count.
struct TunedTiling {
  int form;    // fms::StepForm
  bool batch;  // tuned on launches over several frames (fms_autotune_batch)
  int dp;
  int nb;
  int m;
  fms::Tiling t;
  fms_tune_entry e;
};

// Everything the launches of one batch of seed iterations depend on: a
// captured graph replays only for an equal key.  Only the parity of the
// iteration number reaches the kernels, and whether the batch starts the
// round (its first step reads the centres in place).
struct IterKey {
  const void* ptr[16] = {};
  int64_t val[16] = {};
  double gamma = 0.0;
  bool operator==(const IterKey& o) const {
    return std::memcmp(ptr, o.ptr, sizeof(ptr)) == 0 && std::memcmp(val, o.val, sizeof(val)) == 0 &&
           gamma == o.gamma;
  }
};
struct CachedGraph {
  IterKey key;
  hipGraphExec_t exec = nullptr;
};

struct fms_handle_s {
  int device = 0;
  // Device address of the no-allocation entry point's fixed buffer on this
  // handle's GPU (hipGetSymbolAddress at fms_create).
  unsigned char* na_scratch = nullptr;
  // Decompositions chosen by fms_autotune (empty: the library's defaults).
  std::vector<TunedTiling> tuned;
  // Pixel data of the call's frames; every row-indexed buffer holds frame f
  // from row geo[f].row0 on.
  DevBuf blk, fg_idx, x32, x32t, x16, x16l, order, rank, elig, enorm;
  // Centres of a round, their lists and flags, window counts and ranking.
  DevBuf y, yc0, yc1, active, next_active, state, iters, seed_pos, seed_fg, ident, cand, counts, sorted, scount;
  DevBuf pcount, partial;
  // BF16 form: the last centres of every seed's trajectory (ring slabs) and
  // the FP32 replay's centres, states and step counts.
  DevBuf ring, yr, rstate, riters;
  // Similarity bits of the pruning passes (all frames), accepted list.
  DevBuf bits, acc;
  // Modes found so far (rows of frame f from geo[f].row0 on).
  DevBuf modes, mode_counts;
  // Per-frame counters (F * META_COUNT ints, then F * kMeta64 64-bit words,
  // so that one copy brings both to the host) and tables.
  DevBuf meta, geo, rt, out_off;
  // Event pairs for timing fused-step launches (created on first use).
  std::vector<hipEvent_t> events;
  hipError_t ensure_events(size_t count) {
    while (events.size() < count) {
      hipEvent_t e;
      hipError_t err = hipEventCreate(&e);
      if (err != hipSuccess) return err;
      events.push_back(e);
    }
    return hipSuccess;
  }
  // Host waits go through an event without timing (cheaper to wait on than a
  // whole-stream synchronisation).  A wait also frees the pinned tables for
  // the next upload.
  hipEvent_t sync_ev = nullptr;
  // Captured iteration batches (fms_params.graphs) and the stream they are
  // captured on (created on first use; the caller's stream may be the null
  // stream, which cannot be captured).
  std::vector<CachedGraph> graphs;
  hipStream_t cap_st = nullptr;
  void drop_graphs() {
    for (CachedGraph& g : graphs) (void)hipGraphExecDestroy(g.exec);
    graphs.clear();
  }
  hipError_t wait(hipStream_t st) {
    hipError_t e = hipEventRecord(sync_ev, st);
    if (e == hipSuccess) e = hipEventSynchronize(sync_ev);
    if (e == hipSuccess)
      clear_busy();
    return e;
  }
  void clear_busy() {
    for (PinBuf* b : {&hgeo, &hrt, &hoff, &hstage}) b->busy = false;
  }
  bool any_busy() const { return hgeo.busy || hrt.busy || hoff.busy || hstage.busy; }
  // Pinned host staging: frame tables, output offsets, a general area.  A
  // buffer is rewritten on the host only once no enqueued copy uses it.
  PinBuf hgeo, hrt, hoff, hstage;
  // Counters published by k_publish into coherent host memory mapped for the
  // device (dpub): a sequence word at [0], then from word 4 on F * META_COUNT
  // ints and F * kMeta64 64-bit words.
  PinBuf hpub;
  int* dpub = nullptr;
  int pub_seq = 0;
  hipError_t ensure_pub(size_t bytes) {
    if (bytes <= hpub.cap && dpub) return hipSuccess;
    hipError_t e = hpub.ensure(bytes, hipHostMallocCoherent | hipHostMallocMapped);
    if (e == hipSuccess) {
      std::memset(hpub.p, 0, hpub.cap);
      pub_seq = 0;
      e = hipHostGetDevicePointer(reinterpret_cast<void**>(&dpub), hpub.p, 0);
    }
    if (e != hipSuccess) dpub = nullptr;
    return e;
  }
  const int* hm(int f) const { return hpub.as<int>() + 4 + size_t(f) * META_COUNT; }
  unsigned long long hm64(int f, int F, int slot = 0) const {
    const unsigned long long* q =
        reinterpret_cast<const unsigned long long*>(hpub.as<int>() + 4 + size_t(F) * META_COUNT);
    return q[size_t(f) * kMeta64 + slot];
  }
};

namespace {

#define HIP_TRY(expr)                         \
  do {                                        \
    hipError_t _e = (expr);                   \
    if (_e != hipSuccess) return FMS_ERR_HIP; \
  } while (0)

#define FMS_TRY(expr)                    \
  do {                                   \
    fms_status _s = (expr);              \
    if (_s != FMS_OK) return _s;         \
  } while (0)

// Host state of one frame of a call.
struct FrameHost {
  fms::FrameGeo g{};  // what the kernels see
  int n_pad = 0;
  double r = 0.0;     // foreground fraction n / (H*W)
  // OSOP state (Sec. 3.2.4).
  int64_t n_seeds = 0, n_used = 0;
  int k_modes = 0;
  bool live = false;
  bool have_nmin = false;
  double nmin = 0.0;
  fms::RoundTab rt{};
  fms_stats sx{};
};

// Fused-step launches of a call, timed with kernel-bound events.
struct Timing {
  double step_ms[2] = {0.0, 0.0};
  int64_t step_updates[2] = {0, 0};
  int64_t step_pixels[2] = {0, 0};
  int step_launches[2] = {0, 0};
};

struct Call {
  hipStream_t st = nullptr;
  int F = 0, dim = 0, dp = 32;
  int form = fms::FORM_FP32;  // arithmetic of the round's iteration (fms::StepForm)
  bool bf16 = false;          // the plain BF16 form with its FP32 replay
  std::vector<FrameHost> fr;
  fms::Tiling tile{}, tile_fp32{}, tile_big{}, tile_fp32_big{}, tile_huge{};
  // The handle's tuned decompositions when the call leaves the tiling to the
  // library, and the pixel-count bucket of its largest frame.
  const std::vector<TunedTiling>* tuned = nullptr;
  int nb = 0;
  fms::Batch b{};
  int64_t max_pixels = 0;
  Timing tm;
  bool graphs = false;  // capture and replay iteration batches
  // BF16 form: iterations of each converged seed taken again in FP32
  // (fms_params.refine_iters; 0 = none), and the stride of one ring slab.
  int ring_len = 0;
  int64_t ring_stride = 0;
};

// Most FP32 replay iterations of the BF16 form (ring slabs kept per seed).
constexpr int kMaxRefine = 8;

fms_status check_params(const fms_params* p) {
  if (!p) return FMS_ERR_INVALID_ARG;
  if (!(p->gamma >= 0.0 && p->gamma <= 1.0)) return FMS_ERR_INVALID_ARG;
  if (!(p->big_l > 0.0) || !(p->big_h > 0.0)) return FMS_ERR_INVALID_ARG;
  if (!(p->p_target > 0.0 && p->p_target < 1.0)) return FMS_ERR_INVALID_ARG;
  if (!std::isfinite(p->conv_tol)) return FMS_ERR_INVALID_ARG;
  if (p->n_initial < 1 || p->max_iter < 1 || p->max_rounds < 1 || p->refine_iters < 0) return FMS_ERR_INVALID_ARG;
  if (p->refine_iters > kMaxRefine) return FMS_ERR_UNSUPPORTED;
  if (p->precision != FMS_PREC_FP32 && p->precision != FMS_PREC_BF16_REFINE && p->precision != FMS_PREC_BF16_SPLIT)
    return FMS_ERR_INVALID_ARG;
  if (p->tile_seeds < 0 || p->tile_items < 0 || p->tile_chunks < 0) return FMS_ERR_INVALID_ARG;
  if (p->tile_waves != 0 && p->tile_waves != 4 && p->tile_waves != 8 && p->tile_waves != 16)
    return FMS_ERR_UNSUPPORTED;
  return FMS_OK;
}

fms_status check_frame(const fms_frame& f, int32_t dim) {
  if (!f.emb || f.height < 1 || f.width < 1 || f.pixel_stride < 0 || f.channel_stride < 0)
    return FMS_ERR_INVALID_ARG;
  if (dim < 1) return FMS_ERR_INVALID_ARG;
  if (dim > 128) return FMS_ERR_UNSUPPORTED;
  if (int64_t(f.height) * int64_t(f.width) > int64_t(std::numeric_limits<int32_t>::max())) return FMS_ERR_UNSUPPORTED;
  if (!(f.bandwidth > 0.0 && f.bandwidth < 2.0)) return FMS_ERR_INVALID_ARG;
  return FMS_OK;
}

double tol_of(const fms_params* p, double h) { return p->conv_tol > 0.0 ? p->conv_tol : h / 1000.0; }

// Pixel-count bucket: n within a factor of 4.
int n_bucket(int64_t n) {
  int b = 0;
  while (n >= 4) {
    n >>= 2;
    ++b;
  }
  return b;
}

// Default tiling of a launch of step form `form` with at most `bound`
// centres per frame (the call's own form, or FP32).
const fms::Tiling& default_tiling(const Call& c, int form, int bound) {
  if (form == fms::FORM_FP32) return bound >= kBigGroupMin ? c.tile_fp32_big : c.tile_fp32;
  if (form == fms::FORM_BF16 && bound >= kHugeGroupMin) return c.tile_huge;
  return bound >= kBigGroupMin ? c.tile_big : c.tile;
}

// Arithmetic of the window counts: the split form counts in its own
// arithmetic, the others in FP32.
int count_form(const Call& c) { return c.form == fms::FORM_SPLIT ? fms::FORM_SPLIT : fms::FORM_FP32; }

// Tiling of a window-count launch.  The autotuner times shift launches only,
// so count launches keep the defaults (their integer counts do not depend on
// the decomposition).
const fms::Tiling& count_tiling(const Call& c, int bound) { return default_tiling(c, count_form(c), bound); }

// Window counts of at most m centres y[list[..]] per frame (see launch_count)
// in the call's count arithmetic.
hipError_t count_windows(fms_handle h, const Call& c, const float* y, const int* list, int m, int* counts,
                         int m_slot) {
  const bool split = count_form(c) == fms::FORM_SPLIT;
  return fms::launch_count(c.st, c.b, count_form(c), c.dp, count_tiling(c, m), split ? h->x16.p : h->x32.p,
                           split ? h->x16l.as<uint16_t>() : nullptr, y, list, m, h->pcount.as<int>(), counts, m_slot);
}

// Tiling of a fused-step launch with at most `bound` centres per frame: the
// tuned entry of the form, D class and bucket whose seed count is nearest in
// ratio, else the defaults.
const fms::Tiling& pick_tiling(const Call& c, int form, int bound) {
  if (c.tuned) {
    const TunedTiling* best = nullptr;
    double bd = 0.0;
    for (const TunedTiling& t : *c.tuned) {
      if (t.form != form || t.batch != (c.F > 1) || t.dp != c.dp || t.nb != c.nb) continue;
      const double d = std::fabs(std::log(double(std::max(bound, 1)) / double(t.m)));
      if (!best || d < bd) {
        best = &t;
        bd = d;
      }
    }
    if (best) return best->t;
  }
  return default_tiling(c, form, bound);
}

// Waves per work group of single-frame calls when the caller fixes none.
// With the chunk plan filling one grid pass, eight waves (and the item
// target that goes with them) run whole frames 2-3% (512x512) and 2-6%
// (1024x1024) faster than four; batched launches, which spread over all
// frames, stay at four, where eight were 4-5% slower.
constexpr int kSingleFrameWaves = 8;

// Batched calls, whose launches spread over every frame, default to
// kBatchItems items per step, and the split form to 64-seed groups at every
// active count: the 64-frame batch (split form) ran 1,829 frames/s with both
// against 1,618 with the single-frame defaults (512 items, 32-seed groups
// below kBigGroupMin centres), 1,733 with the items alone and 1,657 with
// the groups alone.
constexpr int kBatchItems = 256;
constexpr int kBatchSplitGroup = 64;

void set_tiling(Call& c, const fms_params* p) {
  const bool batch = c.F > 1;
  const int wv = p->tile_waves > 0 ? p->tile_waves : (batch ? 0 : kSingleFrameWaves);
  const int items = p->tile_items > 0 ? p->tile_items : (batch ? kBatchItems : 0);
  const int seeds =
      p->tile_seeds > 0 ? p->tile_seeds : (batch && c.form == fms::FORM_SPLIT ? kBatchSplitGroup : 0);
  c.tile = fms::make_tiling(c.form, c.dp, seeds, items, p->tile_chunks, wv);
  c.tile_fp32 = fms::make_tiling(fms::FORM_FP32, c.dp, p->tile_seeds, items, p->tile_chunks, wv);
  // A caller-fixed group size holds for every launch.
  const int big = p->tile_seeds > 0 ? p->tile_seeds : kBigGroup;
  c.tile_big = fms::make_tiling(c.form, c.dp, big, items, p->tile_chunks, wv);
  c.tile_fp32_big = fms::make_tiling(fms::FORM_FP32, c.dp, big, items, p->tile_chunks, wv);
  const int huge = p->tile_seeds > 0 ? p->tile_seeds : kHugeGroup;
  c.tile_huge = fms::make_tiling(fms::FORM_BF16, c.dp, huge, items, p->tile_chunks, wv);
}

// Chunk-partial rows a frame of `cap` centres needs under any tiling.
int64_t partial_rows(const Call& c, int cap) {
  size_t r = std::max({fms::shift_partial_rows(c.tile, cap), fms::shift_partial_rows(c.tile_fp32, cap),
                       fms::shift_partial_rows(c.tile_big, cap), fms::shift_partial_rows(c.tile_fp32_big, cap),
                       fms::shift_partial_rows(c.tile_huge, cap)});
  if (c.tuned)
    for (const TunedTiling& t : *c.tuned)
      if (t.dp == c.dp) r = std::max(r, fms::shift_partial_rows(t.t, cap));
  return (int64_t)r;
}

// Upload the frame tables.  The pinned copy is rewritten only after the
// previous upload has completed.
fms_status upload_geo(fms_handle h, Call& c) {
  if (h->hgeo.busy) HIP_TRY(h->wait(c.st));
  fms::FrameGeo* hg = h->hgeo.as<fms::FrameGeo>();
  for (int f = 0; f < c.F; ++f) hg[f] = c.fr[f].g;
  HIP_TRY(hipMemcpyAsync(h->geo.p, hg, size_t(c.F) * sizeof(fms::FrameGeo), hipMemcpyHostToDevice, c.st));
  h->hgeo.busy = true;
  return FMS_OK;
}

fms_status upload_rt(fms_handle h, Call& c) {
  if (c.b.rt_inline) {
    c.b.rt0 = c.fr[0].rt;
    return FMS_OK;
  }
  if (h->hrt.busy) HIP_TRY(h->wait(c.st));
  fms::RoundTab* hr = h->hrt.as<fms::RoundTab>();
  for (int f = 0; f < c.F; ++f) hr[f] = c.fr[f].rt;
  HIP_TRY(hipMemcpyAsync(h->rt.p, hr, size_t(c.F) * sizeof(fms::RoundTab), hipMemcpyHostToDevice, c.st));
  h->hrt.busy = true;
  return FMS_OK;
}

// Staging upload of n ints to device memory (waits first if a copy still
// uses the staging area).
fms_status upload_ints(fms_handle h, Call& c, void* dst, const int* src, size_t n) {
  if (h->hstage.busy) HIP_TRY(h->wait(c.st));
  HIP_TRY(h->hstage.ensure(n * sizeof(int) + 256));
  std::memcpy(h->hstage.p, src, n * sizeof(int));
  HIP_TRY(hipMemcpyAsync(dst, h->hstage.p, n * sizeof(int), hipMemcpyHostToDevice, c.st));
  h->hstage.busy = true;
  return FMS_OK;
}

// Bytes of the counters of F frames: META_COUNT ints per frame, then kMeta64
// 64-bit words per frame (META_COUNT * 4 is a multiple of 8).
size_t meta_bytes(int F) {
  static_assert((META_COUNT * sizeof(int)) % sizeof(unsigned long long) == 0, "64-bit counters misaligned");
  return size_t(F) * (META_COUNT * sizeof(int) + kMeta64 * sizeof(unsigned long long));
}

// All frames' counters to the host: k_publish writes them into mapped host
// memory and then a sequence number, which the host polls (a round trip
// about 4 us shorter than a copy and an event wait on MI355X).
fms_status read_meta_begin(fms_handle h, Call& c, int* seq) {
  *seq = ++h->pub_seq;
  HIP_TRY(fms::launch_publish(c.st, c.b, int(meta_bytes(c.F) / sizeof(int)), h->dpub, *seq));
  return FMS_OK;
}

// Wait until the counters carrying `seq` are on the host; by then everything
// enqueued before that publish has completed.  After two seconds of polling
// it synchronises the stream instead (which also reports a failed stream).
fms_status read_meta_end(fms_handle h, Call& c, int seq) {
  const int* flag = h->hpub.as<int>();
  const auto t0 = std::chrono::steady_clock::now();
  for (uint64_t i = 0; __atomic_load_n(flag, __ATOMIC_ACQUIRE) != seq; ++i) {
    __builtin_ia32_pause();
    if ((i & 4095) == 4095 && std::chrono::steady_clock::now() - t0 > std::chrono::seconds(2)) {
      HIP_TRY(hipStreamSynchronize(c.st));
      if (__atomic_load_n(flag, __ATOMIC_ACQUIRE) != seq) return FMS_ERR_HIP;
      break;
    }
  }
  h->clear_busy();
  return FMS_OK;
}

fms_status read_meta(fms_handle h, Call& c) {
  int seq = 0;
  FMS_TRY(read_meta_begin(h, c, &seq));
  return read_meta_end(h, c, seq);
}

// BF16 form: ring slabs and replay buffers for R rows per buffer (the rows of
// every row-indexed centre buffer).
fms_status ensure_replay(fms_handle h, Call& c, size_t R) {
  if (c.ring_len <= 0) return FMS_OK;
  const size_t dp = size_t(c.dp);
  c.ring_stride = int64_t(R * dp);
  HIP_TRY(h->ring.ensure(size_t(c.ring_len) * R * dp * sizeof(float)));
  HIP_TRY(h->yr.ensure(R * dp * sizeof(float)));
  HIP_TRY(h->riters.ensure(R * sizeof(int)));
  HIP_TRY(h->rstate.ensure(R));
  return FMS_OK;
}

// Compact the foreground of every frame, normalise it and write the layouts;
// set every frame's label map to -1.  The frames' n, rows and tables are
// set; the caller checks META_BAD at its next read of the counters (no
// kernel indexes by embedding values, so the work enqueued meanwhile is
// merely wasted).
fms_status setup_call(fms_handle h, Call& c, const fms_frame* frames, const fms_params* p) {
  const int F = c.F;
  HIP_TRY(h->geo.ensure(size_t(F) * sizeof(fms::FrameGeo)));
  HIP_TRY(h->rt.ensure(size_t(F) * sizeof(fms::RoundTab)));
  HIP_TRY(h->out_off.ensure(size_t(F + 1) * sizeof(int)));
  HIP_TRY(h->meta.ensure(meta_bytes(F)));
  if (h->any_busy()) HIP_TRY(h->wait(c.st));
  HIP_TRY(h->ensure_pub(16 + meta_bytes(F)));
  HIP_TRY(h->hgeo.ensure(size_t(F) * sizeof(fms::FrameGeo)));
  HIP_TRY(h->hrt.ensure(size_t(F) * sizeof(fms::RoundTab)));
  HIP_TRY(h->hoff.ensure(size_t(F + 1) * sizeof(int)));
  c.fr.assign(size_t(F), FrameHost{});
  c.b = fms::Batch{};
  c.b.F = F;
  c.b.geo = h->geo.as<fms::FrameGeo>();
  c.b.rt = h->rt.as<fms::RoundTab>();
  c.b.meta = h->meta.as<int>();
  c.b.meta64 = reinterpret_cast<unsigned long long*>(h->meta.as<int>() + size_t(F) * META_COUNT);
  // A single frame's round table goes with every launch, except under graph
  // capture, whose replays keep the arguments they were captured with.
  c.b.rt_inline = (F == 1 && !c.graphs) ? 1 : 0;
  int64_t mblk = 0;
  for (int f = 0; f < F; ++f) {
    const fms_frame& in = frames[f];
    FrameHost& fh = c.fr[f];
    const int64_t P = int64_t(in.height) * int64_t(in.width);
    fh.g.desc = fms::FrameDesc{in.emb, in.pixel_stride, in.channel_stride, in.mask, P, c.dim, c.dp};
    fh.g.mblk0 = mblk;
    fh.g.labels = in.labels;
    fh.g.thr = float(1.0 - in.bandwidth);
    fh.g.tol = float(tol_of(p, in.bandwidth));
    const int64_t nmb = (P + fms::kMaskBlockPix - 1) / fms::kMaskBlockPix;
    mblk += nmb;
    c.b.max_mblk = std::max(c.b.max_mblk, nmb);
    c.max_pixels = std::max(c.max_pixels, P);
    fh.sx.n_min = std::numeric_limits<double>::quiet_NaN();
    fh.n_seeds = in.n_state_in > 0 ? in.n_state_in : p->n_initial;
  }
  HIP_TRY(h->blk.ensure(size_t(std::max<int64_t>(mblk, 1)) * sizeof(int)));
  FMS_TRY(upload_geo(h, c));
  HIP_TRY(hipMemsetAsync(h->meta.p, 0, meta_bytes(F), c.st));
  HIP_TRY(fms::launch_mask_count(c.st, c.b, h->blk.as<int>()));
  HIP_TRY(fms::launch_scan_blocks(c.st, c.b, h->blk.as<int>()));
  FMS_TRY(read_meta(h, c));
  // Frame regions: rows (pixels, centres, modes), chunk partials, flags.
  int64_t rows = 0, part = 0, elig = 0;
  for (int f = 0; f < F; ++f) {
    FrameHost& fh = c.fr[f];
    const int n = h->hm(f)[META_N];
    fh.g.n = n;
    fh.n_pad = ((n + fms::kBlockPix - 1) / fms::kBlockPix) * fms::kBlockPix;
    fh.g.n_blocks = fh.n_pad / fms::kBlockPix;
    fh.g.half_bits = half_bits(n);
    fh.g.row0 = rows;
    fh.g.part0 = part;
    fh.g.elig0 = elig;
    fh.r = double(n) / double(fh.g.desc.n_pixels);
    fh.sx.n_fg = n;
    rows += fh.n_pad;
    part += n > 0 ? partial_rows(c, n) : 0;
    elig += fms::elig_len(n);
    c.b.max_n = std::max(c.b.max_n, n);
    c.nb = n_bucket(c.b.max_n);
    c.b.max_blocks = std::max(c.b.max_blocks, fh.g.n_blocks);
  }
  const size_t R = size_t(std::max<int64_t>(rows, fms::kBlockPix)), dp = size_t(c.dp);
  HIP_TRY(h->fg_idx.ensure(R * sizeof(int)));
  HIP_TRY(h->enorm.ensure(R * sizeof(float)));
  // Layouts: FP32 rows always (seeds, labels); the FP32 dimension-major copy
  // where FP32 steps run (the FP32 form and the BF16 form's replay); BF16
  // rows for the BF16 forms, whose steps transpose blocks in LDS.
  const bool fp32_steps = c.form != fms::FORM_SPLIT;
  HIP_TRY(h->x32.ensure(R * dp * sizeof(float)));
  if (fp32_steps) HIP_TRY(h->x32t.ensure(R * dp * sizeof(float)));
  if (c.form != fms::FORM_FP32) HIP_TRY(h->x16.ensure(R * dp * sizeof(uint16_t)));
  if (c.form == fms::FORM_SPLIT) HIP_TRY(h->x16l.ensure(R * dp * sizeof(uint16_t)));
  for (DevBuf* b : {&h->y, &h->yc0, &h->yc1, &h->modes}) HIP_TRY(b->ensure(R * dp * sizeof(float)));
  FMS_TRY(ensure_replay(h, c, R));
  for (DevBuf* b : {&h->order, &h->rank, &h->active, &h->next_active, &h->iters, &h->seed_pos, &h->seed_fg,
                    &h->ident, &h->cand, &h->counts, &h->sorted, &h->scount, &h->mode_counts})
    HIP_TRY(b->ensure(R * sizeof(int)));
  HIP_TRY(h->state.ensure(R));
  HIP_TRY(h->elig.ensure(size_t(std::max<int64_t>(elig, 16))));
  const size_t PR = size_t(std::max<int64_t>(part, 1));
  HIP_TRY(h->pcount.ensure(PR * sizeof(int)));
  HIP_TRY(h->partial.ensure(PR * dp * sizeof(float)));
  FMS_TRY(upload_geo(h, c));
  HIP_TRY(fms::launch_fill_labels(c.st, c.b, c.max_pixels));
  if (c.b.max_n > 0)
    HIP_TRY(fms::launch_compact(c.st, c.b, c.dp, h->blk.as<int>(), h->fg_idx.as<int>(), h->x32.as<float>(),
                                fp32_steps ? h->x32t.as<float>() : nullptr,
                                c.form != fms::FORM_FP32 ? h->x16.as<uint16_t>() : nullptr,
                                c.form == fms::FORM_SPLIT ? h->x16l.as<uint16_t>() : nullptr, h->enorm.as<float>()));
  return FMS_OK;
}

// Launch the graph captured for `key` on stream st, capturing it first (the
// launches `record` makes on the stream it is given) when the handle has
// none.  The cache is emptied when it reaches 64 graphs.
template <typename Record>
hipError_t run_graph(fms_handle h, hipStream_t st, const IterKey& key, Record&& record) {
  for (const CachedGraph& g : h->graphs)
    if (g.key == key) return hipGraphLaunch(g.exec, st);
  if (!h->cap_st) {
    const hipError_t e = hipStreamCreateWithFlags(&h->cap_st, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
  }
  hipError_t e = hipStreamBeginCapture(h->cap_st, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  const hipError_t er = record(h->cap_st);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(h->cap_st, &graph);
  if (er != hipSuccess || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return er != hipSuccess ? er : e;
  }
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return e;
  if (h->graphs.size() >= 64) h->drop_graphs();
  h->graphs.push_back(CachedGraph{key, exec});
  return hipGraphLaunch(exec, st);
}

// Iterate every frame's centres y[row0 .. row0 + NSEL) (Alg. 2, the parallel
// seed loop) until more than gamma of them converged (Sec. 3.2.3), none is
// active, or max_iter steps; each frame stops on its own counters.  With
// seed_fg the centres first load from those pixel rows; with nsel_from_rt a
// frame's centre count is rt.nact.  The active count, the early-stop test and
// the done flag live on the device; the host enqueues iterations in batches
// and reads the counters back between batches.  cap: most centres of any
// frame.  extra: steps a frame goes on after its first step that saw more
// than gamma converged (IterCtl::extra).  On return h->hm(f) holds every
// frame's counters.
fms_status run_iterations(fms_handle h, Call& c, float* ybuf, int cap, double gamma, int max_iter, int form,
                          bool timing, const int* seed_fg, bool nsel_from_rt, int extra = 0) {
  const fms::Batch& b = c.b;
  const bool bf16 = form != fms::FORM_FP32;  // a BF16 MFMA step
  const void* xrm = bf16 ? h->x16.p : h->x32.p;
  const void* xt = bf16 ? nullptr : h->x32t.p;
  const uint16_t* xrl = form == fms::FORM_SPLIT ? h->x16l.as<uint16_t>() : nullptr;
  const int pk = bf16 ? 1 : 0;
  // The plain BF16 form keeps the last centres of each trajectory for the
  // replay.
  float* ring = form == fms::FORM_BF16 && c.ring_len > 0 ? h->ring.as<float>() : nullptr;
  HIP_TRY(fms::launch_round_begin(c.st, b, cap, nsel_from_rt, h->active.as<int>(), h->state.as<uint8_t>(),
                                  h->iters.as<int>(), seed_fg, h->x32.as<float>(), c.dp, ybuf));
  int* lists[2] = {h->active.as<int>(), h->next_active.as<int>()};
  float* yc[2] = {h->yc0.as<float>(), h->yc1.as<float>()};
  // Batch sizes: most rounds of the 512x512 workload stop within 3 to 9
  // iterations; 3, 6, 8 measured best among the schedules tried.
  static constexpr int kSched[] = {3, 6, 8};
  int t = 0, nbatch = 0;
  int bound = cap;  // active centres of any frame in the next iteration, at most
  // Iteration t: the step, then the reduction that renormalises, freezes and
  // compacts.  Iteration 0 reads the centres in place (the active list is
  // the identity); later iterations read the rows the previous reduce
  // compacted in active-list order.
  auto iterate_on = [&](hipStream_t st, const fms::Tiling& tl, int it, hipEvent_t e0, hipEvent_t e1) -> hipError_t {
    const fms::IterCtl ctl{-1, it, gamma, extra};
    const float* yin = it == 0 ? ybuf : yc[it & 1];
    hipError_t e = fms::launch_shift(st, b, form, c.dp, tl, xrm, xt, xrl, yin, nullptr, ctl, cap,
                                     h->partial.as<float>(), e0, e1);
    if (e == hipSuccess)
      e = fms::launch_reduce(st, b, c.dp, tl, h->partial.as<float>(), lists[it & 1], ybuf, h->state.as<uint8_t>(),
                             h->iters.as<int>(), lists[(it + 1) & 1], yc[(it + 1) & 1], ctl, cap, 0, nullptr, yin,
                             ring, c.ring_stride, c.ring_len);
    return e;
  };
  auto iterate = [&](const fms::Tiling& tl, int it, hipEvent_t e0, hipEvent_t e1) -> hipError_t {
    return iterate_on(c.st, tl, it, e0, e1);
  };
  // Iterations t .. t + n - 1 as one replayed graph.
  auto iterate_graph = [&](const fms::Tiling& tl, int t0, int n) -> hipError_t {
    IterKey k;
    const void* ptrs[] = {xrm, xt, ybuf, yc[0], yc[1], lists[0], lists[1], h->partial.p, h->state.p, h->iters.p,
                          b.geo, b.rt, b.meta, b.meta64, ring, xrl};
    std::memcpy(k.ptr, ptrs, sizeof(ptrs));
    // The kernels see the iteration's parity and whether it starts the round;
    // with extra steps the early stop also counts from absolute iterations.
    const int64_t it_key = extra > 0 ? t0 : (t0 & 1) + 2 * (t0 == 0);
    const int64_t vals[] = {form, c.dp, tl.group_seeds, tl.target_items, tl.max_chunks, tl.waves, cap, n,
                            it_key, b.F, b.max_n, b.max_blocks, b.max_mblk, c.ring_stride, c.ring_len, extra};
    std::memcpy(k.val, vals, sizeof(vals));
    k.gamma = gamma;
    return run_graph(h, c.st, k, [&](hipStream_t st) -> hipError_t {
      for (int i = 0; i < n; ++i) {
        const hipError_t e = iterate_on(st, tl, t0 + i, nullptr, nullptr);
        if (e != hipSuccess) return e;
      }
      return hipSuccess;
    });
  };
  while (t < max_iter) {
    const int nb = std::min(kSched[std::min(nbatch, 2)], max_iter - t);
    ++nbatch;
    if (timing) HIP_TRY(h->ensure_events(2 * size_t(nb)));
    const fms::Tiling& tl = pick_tiling(c, form, bound);
    if (c.graphs) {
      HIP_TRY(iterate_graph(tl, t, nb));
      t += nb;
    } else {
      for (int i = 0; i < nb; ++i, ++t)
        HIP_TRY(iterate(tl, t, timing ? h->events[2 * i] : nullptr, timing ? h->events[2 * i + 1] : nullptr));
    }
    // The counters after this batch go to the host while the GPU runs one
    // more iteration behind them (without timing): a round that goes on
    // keeps the GPU busy during the host's decision, and one that stopped
    // costs one launch pair that returns at its head.
    int seq = 0;
    FMS_TRY(read_meta_begin(h, c, &seq));
    const bool spec = !timing && t < max_iter;
    if (spec) HIP_TRY(iterate(tl, t, nullptr, nullptr));
    FMS_TRY(read_meta_end(h, c, seq));
    if (timing) {
      for (int i = 0; i < nb; ++i) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, h->events[2 * i], h->events[2 * i + 1]));
        c.tm.step_ms[pk] += ms;
        c.tm.step_launches[pk] += 1;
      }
    }
    // The early stop of each frame's next iteration, as its step kernel
    // takes it (the speculative iteration, when there is one).
    bool all_done = true;
    bound = 0;
    for (int f = 0; f < c.F; ++f) {
      const int* hm = h->hm(f);
      const int act = hm[fms::META_ACT + (t & 1)];
      const bool over = (double)hm[META_NCONV] > gamma * (double)hm[META_NSEL];
      const int gstep = hm[fms::META_GSTEP];
      const int past = (over && gstep >= 0) ? t - gstep : 0;
      const bool done = hm[fms::META_DONE] || act <= 0 || (over && past >= extra);
      if (!done) {
        all_done = false;
        bound = std::max(bound, act);
      }
    }
    if (all_done) break;
    if (spec) ++t;
  }
  if (timing)
    for (int f = 0; f < c.F; ++f) {
      c.tm.step_updates[pk] += int64_t(h->hm64(f, c.F));
      c.tm.step_pixels[pk] += int64_t(h->hm64(f, c.F, 1));
    }
  return FMS_OK;
}

// Steps the BF16 iteration goes on after it first sees more than gamma of a
// round's seeds converged: BF16 and FP32 trajectories may converge a step
// apart, and the early stop is then taken again on FP32 step counts (see
// run_replay), which needs the seeds that converge one step later too.
constexpr int kReplayExtra = 1;
int replay_extra(const Call& c) { return c.ring_len > 0 ? kReplayExtra : 0; }

// BF16 form, after a round's BF16 iteration: the converged seeds of every
// frame take their last c.ring_len iterations again in FP32 (Eq. 8, 10, 11
// and the stopping test of Sec. 3.2.1), from the centre each one had that
// many steps before it stopped.  The replay iterates like a round (FP32
// steps with freezing, no early stop), ring_len + 1 steps at most, with no
// host read; a seed the replay has not frozen by then is dropped like the
// round's unconverged seeds.  The replayed centres, states and step counts
// go back to the round's slots, and the early stop of Sec. 3.2.3 is taken
// again on those FP32 step counts (a seed converging after that step is
// dropped), so the counts, pruning and coverage that follow see the FP32
// iteration's endpoints.  The frames' META_STEPS, meta64[0],
// META_REFINE_BAD, META_REFINE_DIFF and META_GCUT then hold the replay's
// figures.  cap: most seeds of any frame in the round.
fms_status run_replay(fms_handle h, Call& c, int cap, double gamma, bool timing) {
  if (c.ring_len <= 0 || cap <= 0) return FMS_OK;
  const fms::Batch& b = c.b;
  HIP_TRY(fms::launch_replay_begin(c.st, b, c.dp, c.ring_len, h->state.as<uint8_t>(), h->iters.as<int>(),
                                   h->ring.as<float>(), c.ring_stride, h->cand.as<int>(), h->yr.as<float>(),
                                   h->active.as<int>(), h->rstate.as<uint8_t>(), h->riters.as<int>()));
  const fms::Tiling& tl = pick_tiling(c, fms::FORM_FP32, cap);
  int* lists[2] = {h->active.as<int>(), h->next_active.as<int>()};
  float* yc[2] = {h->yc0.as<float>(), h->yc1.as<float>()};
  float* yr = h->yr.as<float>();
  const int steps = c.ring_len + 1;
  if (timing) HIP_TRY(h->ensure_events(2 * size_t(steps)));
  for (int it = 0; it < steps; ++it) {
    // gamma = 1: more than all of the round's seeds can never have
    // converged, so only an empty active list stops the replay early.
    const fms::IterCtl ctl{-1, it, 1.0};
    const float* yin = it == 0 ? yr : yc[it & 1];
    // Step it reads its centres in list order (in place through the identity
    // list at it = 0, then the rows the previous reduction compacted).
    HIP_TRY(fms::launch_shift(c.st, b, fms::FORM_FP32, c.dp, tl, h->x32.p, h->x32t.p, nullptr, yin, nullptr,
                              ctl, cap,
                              h->partial.as<float>(), timing ? h->events[2 * it] : nullptr,
                              timing ? h->events[2 * it + 1] : nullptr));
    HIP_TRY(fms::launch_reduce(c.st, b, c.dp, tl, h->partial.as<float>(), lists[it & 1], yr,
                               h->rstate.as<uint8_t>(), h->riters.as<int>(), lists[(it + 1) & 1], yc[(it + 1) & 1],
                               ctl, cap, 0, nullptr, yin));
  }
  HIP_TRY(fms::launch_replay_end(c.st, b, c.dp, cap, c.ring_len, h->cand.as<int>(), h->iters.as<int>(), yr,
                                 h->rstate.as<uint8_t>(), h->riters.as<int>(), h->y.as<float>(),
                                 h->state.as<uint8_t>()));
  HIP_TRY(fms::launch_gamma_cut(c.st, b, gamma, h->iters.as<int>(), h->state.as<uint8_t>()));
  if (timing) {
    // Timed calls only: wait here so the events can be read.
    HIP_TRY(h->wait(c.st));
    for (int it = 0; it < steps; ++it) {
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, h->events[2 * it], h->events[2 * it + 1]));
      c.tm.step_ms[0] += ms;
      c.tm.step_launches[0] += 1;
    }
  }
  return FMS_OK;
}

// The replay's figures of frame f (counters on the host) into its stats.
void add_replay_stats(fms_handle h, Call& c, int f, Timing* tm) {
  FrameHost& fh = c.fr[f];
  const int* hm = h->hm(f);
  const int64_t upd = int64_t(h->hm64(f, c.F));
  fh.sx.refine_steps += hm[META_STEPS];
  fh.sx.refine_updates += upd;
  fh.sx.refine_unconverged += hm[META_REFINE_BAD];
  fh.sx.refine_step_diff += hm[META_REFINE_DIFF];
  fh.sx.refine_gamma_cut += hm[fms::META_GCUT];
  if (tm) {
    tm->step_updates[0] += upd;
    tm->step_pixels[0] += int64_t(h->hm64(f, c.F, 1));
  }
}

// Bit-matrix layout of a device pruning pass: frame f's candidate x
// candidate rows (rt.want rows of simbits_words(rt.want) words) and, with
// modes, candidate x mode rows (simbits_words(rt.k_modes) words).  Returns
// the words needed.
int64_t layout_bits(Call& c, bool with_modes) {
  int64_t w = 0;
  for (FrameHost& fh : c.fr) {
    const int m = fh.rt.want;
    fh.rt.words_c = fms::simbits_words(m);
    fh.rt.words_m = with_modes ? fms::simbits_words(fh.rt.k_modes) : 0;
    fh.rt.bits_c0 = w;
    w += int64_t(m) * fh.rt.words_c;
    fh.rt.bits_m0 = w;
    w += int64_t(m) * fh.rt.words_m;
  }
  return std::max<int64_t>(w, 2);
}

// Greedy pruning (Alg. 2) on the host: visit candidates in `order`, accept
// one when it is not within the window of an existing mode (a nonzero row of
// bits_m) and not within the window of a candidate accepted before it.
std::vector<int> greedy_accept(const std::vector<int>& order, const int* counts, const uint32_t* bits_c, int words_c,
                               const uint32_t* bits_m, int words_m) {
  (void)counts;
  std::vector<uint32_t> taken(size_t(std::max(words_c, 1)), 0u);
  std::vector<int> acc;
  for (int a : order) {
    if (bits_m) {
      const uint32_t* rm = bits_m + size_t(a) * words_m;
      bool blocked = false;
      for (int w = 0; w < words_m && !blocked; ++w) blocked = rm[w] != 0;
      if (blocked) continue;
    }
    const uint32_t* row = bits_c + size_t(a) * words_c;
    bool clash = false;
    for (int w = 0; w < words_c && !clash; ++w) clash = (row[w] & taken[w]) != 0;
    if (clash) continue;
    taken[a >> 5] |= 1u << (a & 31);
    acc.push_back(a);
  }
  return acc;
}

// Converged slots of a single frame's round, ascending (state == 1).
fms_status host_converged(fms_handle h, Call& c, std::vector<int>& conv) {
  const int msel = h->hm(0)[META_NSEL];
  conv.clear();
  if (msel <= 0) return FMS_OK;
  if (h->hstage.busy) HIP_TRY(h->wait(c.st));
  HIP_TRY(h->hstage.ensure(size_t(msel) + 256));
  HIP_TRY(hipMemcpyAsync(h->hstage.p, h->state.p, size_t(msel), hipMemcpyDeviceToHost, c.st));
  HIP_TRY(h->wait(c.st));
  const uint8_t* hs = h->hstage.as<uint8_t>();
  for (int k = 0; k < msel; ++k)
    if (hs[k] == 1) conv.push_back(k);
  return FMS_OK;
}

// Single frame with more candidates than the device ranking takes: window
// counts and similarity bits of the converged candidates against each other
// and the modes kept so far go to the host in one copy; greedy acceptance
// on the host by (count desc, slot asc); the accepted rows are appended to
// the modes and their number put in META_NACC.
fms_status host_prune(fms_handle h, Call& c, const std::vector<int>& conv) {
  FrameHost& fh = c.fr[0];
  const int nc = int(conv.size());
  if (nc == 0) {
    HIP_TRY(fms::launch_set_slot(c.st, c.b, META_NACC, false, 0));
    return FMS_OK;
  }
  const int k = fh.k_modes;
  fh.rt.want = nc;
  fh.rt.k_modes = k;
  const int64_t words = layout_bits(c, k > 0);
  const size_t nb_n = ((size_t(nc) * sizeof(int) + 255) / 256) * 256;
  const size_t bytes = nb_n + size_t(words) * sizeof(uint32_t);
  HIP_TRY(h->bits.ensure(bytes));
  FMS_TRY(upload_ints(h, c, h->cand.p, conv.data(), size_t(nc)));
  FMS_TRY(upload_rt(h, c));
  HIP_TRY(fms::launch_set_slot(c.st, c.b, META_NCAND, false, nc));
  int* counts = h->bits.as<int>();
  uint32_t* bits = reinterpret_cast<uint32_t*>(h->bits.as<uint8_t>() + nb_n);
  HIP_TRY(count_windows(h, c, h->y.as<float>(), h->cand.as<int>(), nc, counts, META_NCAND));
  HIP_TRY(fms::launch_simbits(c.st, c.b, c.dp, h->y.as<float>(), h->cand.as<int>(), nc, h->cand.as<int>(), nc,
                              h->modes.as<float>(), k, bits, META_NCAND, META_NCAND));
  if (h->hstage.busy) HIP_TRY(h->wait(c.st));
  HIP_TRY(h->hstage.ensure(bytes + 256));
  HIP_TRY(hipMemcpyAsync(h->hstage.p, h->bits.p, bytes, hipMemcpyDeviceToHost, c.st));
  HIP_TRY(h->wait(c.st));
  const int* hc = h->hstage.as<int>();
  const uint32_t* hb = reinterpret_cast<const uint32_t*>(h->hstage.as<uint8_t>() + nb_n);
  std::vector<int> ord(static_cast<size_t>(nc));
  for (int a = 0; a < nc; ++a) ord[a] = a;
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return hc[a] > hc[b]; });
  std::vector<int> acc = greedy_accept(ord, hc, hb + fh.rt.bits_c0, fh.rt.words_c,
                                       k > 0 ? hb + fh.rt.bits_m0 : nullptr, fh.rt.words_m);
  const int na = int(acc.size());
  if (na > 0) {
    HIP_TRY(h->acc.ensure(size_t(na) * sizeof(int)));
    FMS_TRY(upload_ints(h, c, h->acc.p, acc.data(), size_t(na)));
    HIP_TRY(fms::launch_append_modes(c.st, c.dp, h->y.as<float>(), h->cand.as<int>(), counts, h->acc.as<int>(), na,
                                     h->modes.as<float>(), h->mode_counts.as<int>(), k));
  }
  HIP_TRY(fms::launch_set_slot(c.st, c.b, META_NACC, false, na));
  return FMS_OK;
}

// Every frame's modes (rt.k_modes uploaded) to the packed outputs at rows
// off[f].
fms_status write_modes(fms_handle h, Call& c, float* modes_out, int32_t* counts_out, const int* off) {
  int kmax = 0;
  for (const FrameHost& fh : c.fr) kmax = std::max(kmax, fh.k_modes);
  if (kmax == 0) return FMS_OK;
  if (h->hoff.busy) HIP_TRY(h->wait(c.st));
  std::memcpy(h->hoff.p, off, size_t(c.F) * sizeof(int));
  HIP_TRY(hipMemcpyAsync(h->out_off.p, h->hoff.p, size_t(c.F) * sizeof(int), hipMemcpyHostToDevice, c.st));
  h->hoff.busy = true;
  HIP_TRY(fms::launch_modes_out(c.st, c.b, h->modes.as<float>(), h->mode_counts.as<int>(), c.dp, c.dim,
                                h->out_off.as<int>(), modes_out, counts_out, kmax));
  return FMS_OK;
}

// Where fms_cluster_batch wants the modes: packed rows, frame f from
// offsets[f]; written only when the total fits k_max.
struct ModeOutputs {
  float* modes;
  int32_t* counts;
  int32_t k_max;
  std::vector<int> offsets;  // F + 1 entries, filled by cluster_frames
  int64_t total;
};

// The OSOP round loop (Sec. 3.2.4) over the frames of a call, then the
// labels.  Modes stay in h->modes; on return rt.k_modes of every frame
// (uploaded) is its final mode count.
fms_status cluster_frames(fms_handle h, Call& c, const fms_params* p, ModeOutputs& out) {
  const int F = c.F;
  const bool timing = p->timing != 0;
  // Coverage and labels take the split form's arithmetic in that form, FP32
  // otherwise (BF16 iterations end in FP32 replays).
  const bool split = c.form == fms::FORM_SPLIT;
  if (c.b.max_n > 0) {
    uint64_t keys[4];
    round_keys(p->seed, keys);
    HIP_TRY(
        fms::launch_seed_order(c.st, c.b, keys, h->order.as<int>(), h->rank.as<int>(), h->elig.as<uint8_t>()));
  }
  for (FrameHost& fh : c.fr) fh.live = fh.g.n > 0;
  bool checked_bad = false;
  for (int round = 0; round < p->max_rounds; ++round) {
    // Seeds of this round per frame: N - N_used fresh ones.
    int cap = 0;
    for (FrameHost& fh : c.fr) {
      fh.rt = fms::RoundTab{};
      fh.rt.k_modes = fh.k_modes;
      if (!fh.live) continue;
      const int64_t want64 = std::min<int64_t>(fh.n_seeds - fh.n_used, fh.g.n);
      if (want64 <= 0) {
        fh.live = false;
        continue;
      }
      fh.rt.want = int(want64);
      cap = std::max(cap, fh.rt.want);
    }
    if (cap == 0) break;
    const bool on_device = cap <= fms::kRankMax;
    if (!on_device && F > 1) return FMS_ERR_UNSUPPORTED;
    if (on_device) HIP_TRY(h->bits.ensure(size_t(layout_bits(c, true)) * sizeof(uint32_t)));
    FMS_TRY(upload_rt(h, c));
    HIP_TRY(fms::launch_select(c.st, c.b, h->order.as<int>(), h->elig.as<uint8_t>(), h->seed_pos.as<int>(),
                               h->seed_fg.as<int>()));
    FMS_TRY(run_iterations(h, c, h->y.as<float>(), cap, p->gamma, p->max_iter, c.form, timing, h->seed_fg.as<int>(),
                           false, replay_extra(c)));
    // BF16 form: the converged seeds' last iterations again in FP32 and the
    // early stop taken on their FP32 step counts, so that everything from
    // here on works on FP32 endpoints.
    FMS_TRY(run_replay(h, c, cap, p->gamma, timing));
    if (!checked_bad) {
      for (int f = 0; f < F; ++f)
        if (h->hm(f)[META_BAD] != 0) return FMS_ERR_BAD_INPUT;
      checked_bad = true;
    }
    std::vector<int> msel(static_cast<size_t>(F)), steps(static_cast<size_t>(F));
    std::vector<unsigned long long> upd(static_cast<size_t>(F));
    for (int f = 0; f < F; ++f) {
      msel[f] = h->hm(f)[META_NSEL];
      steps[f] = h->hm(f)[META_STEPS];
      upd[f] = h->hm64(f, F);
    }
    int host_cand = 0;
    if (on_device) {
      // Prune (Alg. 2): window counts at the converged endpoints (FP32, or the
      // split form's own arithmetic), ranking by count (descending) then seed
      // position, greedy suppression against the modes kept so far and the
      // candidates accepted before.
      // Counts at every slot of the round (the list is the identity); the
      // ranking keeps the converged ones.
      HIP_TRY(count_windows(h, c, h->y.as<float>(), nullptr, cap, h->counts.as<int>(), META_NSEL));
      // The candidate list buffer is free in a round: it holds each
      // candidate's first word with an earlier conflict for the greedy pass.
      int* first = h->cand.as<int>();
      HIP_TRY(fms::launch_rank_converged(c.st, c.b, h->state.as<uint8_t>(), h->counts.as<int>(), h->sorted.as<int>(),
                                         h->scount.as<int>(), first));
      int kmax = 0;
      for (const FrameHost& fh : c.fr) kmax = std::max(kmax, fh.rt.want > 0 ? fh.k_modes : 0);
      HIP_TRY(fms::launch_simbits(c.st, c.b, c.dp, h->y.as<float>(), h->sorted.as<int>(), cap, h->sorted.as<int>(),
                                  cap, h->modes.as<float>(), kmax, h->bits.as<uint32_t>(), META_NCAND, META_NCAND,
                                  first));
      HIP_TRY(fms::launch_greedy(c.st, c.b, h->bits.as<uint32_t>(), h->y.as<float>(), h->sorted.as<int>(),
                                 h->scount.as<int>(), META_NCAND, META_NACC, c.dp, h->modes.as<float>(),
                                 h->mode_counts.as<int>(), first));
    } else {
      std::vector<int> conv;
      FMS_TRY(host_converged(h, c, conv));
      FMS_TRY(host_prune(h, c, conv));
      host_cand = int(conv.size());
    }
    // Coverage by the new modes, and the pool left to seed; then one read of
    // the counters.
    HIP_TRY(fms::launch_assign(c.st, c.b, c.dp, split, h->x32.as<float>(), h->x16.as<uint16_t>(),
                               h->x16l.as<uint16_t>(), h->modes.as<float>(), META_NACC, 0, h->elig.as<uint8_t>(),
                               h->rank.as<int>(), nullptr));
    FMS_TRY(read_meta(h, c));
    for (int f = 0; f < F; ++f) {
      FrameHost& fh = c.fr[f];
      if (!fh.live) continue;
      const int* hm = h->hm(f);
      const int m = msel[f];
      if (m == 0) {
        fh.live = false;
        continue;
      }
      if (c.ring_len > 0) add_replay_stats(h, c, f, timing ? &c.tm : nullptr);
      fh.n_used += m;
      fh.sx.rounds += 1;
      fh.sx.seeds_used += m;
      fh.sx.iterations_total += steps[f];
      fh.sx.seed_pixel_updates += int64_t(upd[f]);
      fh.sx.n_discarded += m - (on_device ? hm[META_NCAND] : host_cand);
      fh.k_modes += hm[META_NACC];
      const bool left = hm[META_LEFT] > 0;
      // Controller (Sec. 3.2.4).
      bool go_on = false;
      fh.have_nmin = eq19_n_min(p->p_target, fh.k_modes, fh.r, &fh.nmin);
      if (left && (!fh.have_nmin || double(fh.n_seeds) < p->big_l * fh.nmin)) {
        fh.n_seeds *= 2;
        go_on = true;
      }
      fh.live = go_on;
    }
  }

  // Labels (Alg. 2): most similar mode, lowest index on ties; count pixels
  // farther than h from every mode.
  for (FrameHost& fh : c.fr) {
    fh.rt = fms::RoundTab{};
    fh.rt.k_modes = fh.k_modes;
  }
  FMS_TRY(upload_rt(h, c));
  HIP_TRY(fms::launch_set_slot(c.st, c.b, META_LEFT, false, 0));
  HIP_TRY(fms::launch_assign(c.st, c.b, c.dp, split, h->x32.as<float>(), h->x16.as<uint16_t>(),
                             h->x16l.as<uint16_t>(), h->modes.as<float>(), -1, 1, nullptr, nullptr,
                             h->fg_idx.as<int>()));
  // The packed modes go out before the last read of the counters, so the
  // call ends with one wait.
  out.offsets.assign(size_t(F) + 1, 0);
  out.total = 0;
  for (int f = 0; f < F; ++f) {
    out.offsets[size_t(f)] = int(std::min<int64_t>(out.total, std::numeric_limits<int32_t>::max()));
    out.total += c.fr[f].k_modes;
  }
  out.offsets[size_t(F)] = int(std::min<int64_t>(out.total, std::numeric_limits<int32_t>::max()));
  if (out.total <= out.k_max) FMS_TRY(write_modes(h, c, out.modes, out.counts, out.offsets.data()));
  FMS_TRY(read_meta(h, c));
  for (int f = 0; f < F; ++f) {
    FrameHost& fh = c.fr[f];
    fh.sx.n_uncovered = fh.g.n > 0 ? h->hm(f)[META_LEFT] : 0;
    fh.sx.n_min = fh.have_nmin ? fh.nmin : std::numeric_limits<double>::quiet_NaN();
    int64_t next = fh.n_seeds;
    if (fh.have_nmin && double(fh.n_seeds) > p->big_h * fh.nmin) next = fh.n_seeds - int64_t(std::ceil(fh.nmin));
    fh.sx.n_state_out = int32_t(std::min<int64_t>(next, std::numeric_limits<int32_t>::max()));
  }
  return FMS_OK;
}


void fill_stats(const Call& c, fms_stats* stats) {
  if (!stats) return;
  for (int f = 0; f < c.F; ++f) stats[f] = c.fr[f].sx;
  // Kernel timing covers the whole call; it is reported with the first frame.
  for (int k = 0; k < 2; ++k) {
    stats[0].step_ms[k] = c.tm.step_ms[k];
    stats[0].step_updates[k] = c.tm.step_updates[k];
    stats[0].step_pixels[k] = c.tm.step_pixels[k];
    stats[0].step_launches[k] = c.tm.step_launches[k];
  }
}

fms_status begin_call(fms_handle h, void* stream, int32_t n_frames, const fms_frame* frames, int32_t dim,
                      const fms_params* p, Call& c) {
  if (!h || n_frames < 1 || !frames) return FMS_ERR_INVALID_ARG;
  for (int f = 0; f < n_frames; ++f) FMS_TRY(check_frame(frames[f], dim));
  FMS_TRY(check_params(p));
  c.st = static_cast<hipStream_t>(stream);
  c.F = n_frames;
  c.dim = dim;
  c.dp = pad_dim(dim);
  c.bf16 = p->precision == FMS_PREC_BF16_REFINE;
  c.form = p->precision == FMS_PREC_BF16_REFINE ? fms::FORM_BF16
           : p->precision == FMS_PREC_BF16_SPLIT ? fms::FORM_SPLIT
                                                  : fms::FORM_FP32;
  c.graphs = p->graphs != 0 && p->timing == 0;
  c.ring_len = c.bf16 ? p->refine_iters : 0;
  set_tiling(c, p);
  // The tuned table (single-frame entries for one frame, batch entries for
  // several) applies when the call leaves the tiling to the library.
  if (p->tile_seeds == 0 && p->tile_items == 0 && p->tile_chunks == 0 && p->tile_waves == 0 && !h->tuned.empty())
    c.tuned = &h->tuned;
  return setup_call(h, c, frames, p);
}

// A single-frame FP32 call with the library's defaults and bandwidth h.
fms_status begin_single(fms_handle h, void* stream, const fms_frame& fr, int32_t dim, Call& c) {
  fms_params p;
  fms_default_params(&p);
  p.bandwidth = fr.bandwidth;
  return begin_call(h, stream, 1, &fr, dim, &p, c);
}

// Widen the (single) frame's centre region and partials for m centres.
fms_status ensure_centres(fms_handle h, Call& c, int m) {
  const size_t R = size_t(std::max(m, c.fr[0].n_pad)) + fms::kBlockPix, dp = size_t(c.dp);
  for (DevBuf* b : {&h->y, &h->yc0, &h->yc1}) HIP_TRY(b->ensure(R * dp * sizeof(float)));
  for (DevBuf* b : {&h->active, &h->next_active, &h->iters, &h->ident, &h->cand, &h->counts})
    HIP_TRY(b->ensure(R * sizeof(int)));
  HIP_TRY(h->state.ensure(R));
  FMS_TRY(ensure_replay(h, c, R));
  const size_t PR = size_t(partial_rows(c, std::max(m, c.fr[0].g.n)));
  HIP_TRY(h->pcount.ensure(PR * sizeof(int)));
  HIP_TRY(h->partial.ensure(PR * dp * sizeof(float)));
  return FMS_OK;
}

fms_frame frame_of(const float* emb, int64_t ps, int64_t cs, const uint8_t* mask, int32_t height, int32_t width,
                   double bandwidth, int32_t n_state_in, int32_t* labels) {
  fms_frame f;
  f.emb = emb;
  f.pixel_stride = ps;
  f.channel_stride = cs;
  f.mask = mask;
  f.height = height;
  f.width = width;
  f.bandwidth = bandwidth;
  f.n_state_in = n_state_in;
  f.labels = labels;
  return f;
}

// ------------------------------------------------------------------ no-allocation lockstep
//
// fms_shift_seeds_noalloc runs fms_shift_seeds' FP32 path on one fixed
// device array per GPU instead of the handle's growable workspace: the
// frame's layouts, the centres and their lists, the chunk partials, the
// window counts, the counters and the frame tables all live in `scratch`.
// Capacity: H * W <= kNaMaxPixels, foreground <= kNaMaxFg, seeds <=
// kNaMaxSeeds, D <= 32, chunk partials <= kNaPartialRows rows.
constexpr int64_t kNaMaxPixels = int64_t(1) << 20;
constexpr int kNaMaxFg = 1 << 17;
constexpr int kNaMaxSeeds = 4096;
constexpr int kNaDp = 32;
constexpr int64_t kNaPartialRows = 32768;
constexpr int kNaCentreRows = kNaMaxSeeds + fms::kBlockPix;

constexpr size_t na_align(size_t b) { return (b + 255) / 256 * 256; }
// Byte offsets of the regions of `scratch`.
struct NaLayout {
  static constexpr size_t blk = 0;
  static constexpr size_t fg_idx = blk + na_align(sizeof(int) * size_t(kNaMaxPixels / fms::kMaskBlockPix));
  static constexpr size_t x32 = fg_idx + na_align(sizeof(int) * size_t(kNaMaxFg));
  static constexpr size_t x32t = x32 + na_align(sizeof(float) * size_t(kNaMaxFg) * kNaDp);
  static constexpr size_t y = x32t + na_align(sizeof(float) * size_t(kNaMaxFg) * kNaDp);
  static constexpr size_t yc0 = y + na_align(sizeof(float) * size_t(kNaCentreRows) * kNaDp);
  static constexpr size_t yc1 = yc0 + na_align(sizeof(float) * size_t(kNaCentreRows) * kNaDp);
  static constexpr size_t active = yc1 + na_align(sizeof(float) * size_t(kNaCentreRows) * kNaDp);
  static constexpr size_t next_active = active + na_align(sizeof(int) * size_t(kNaCentreRows));
  static constexpr size_t iters = next_active + na_align(sizeof(int) * size_t(kNaCentreRows));
  static constexpr size_t ident = iters + na_align(sizeof(int) * size_t(kNaCentreRows));
  static constexpr size_t counts = ident + na_align(sizeof(int) * size_t(kNaCentreRows));
  static constexpr size_t state = counts + na_align(sizeof(int) * size_t(kNaCentreRows));
  static constexpr size_t pcount = state + na_align(size_t(kNaCentreRows));
  static constexpr size_t partial = pcount + na_align(sizeof(int) * size_t(kNaPartialRows));
  static constexpr size_t meta = partial + na_align(sizeof(float) * size_t(kNaPartialRows) * kNaDp);
  static constexpr size_t geo = meta + na_align(sizeof(int) * META_COUNT + sizeof(unsigned long long) * fms::kMeta64);
  static constexpr size_t rt = geo + na_align(sizeof(fms::FrameGeo));
  static constexpr size_t bytes = rt + na_align(sizeof(fms::RoundTab));
};

}  // namespace

// The fixed buffer of fms_shift_seeds_noalloc (about 38 MiB), one copy per
// GPU for the life of the process.  Host code never uses this name as an
// address: fms_create looks up each GPU's copy with hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[NaLayout::bytes];

namespace {

fms_status shift_seeds_noalloc(fms_handle h, void* stream, const float* emb, int64_t pixel_stride,
                               int64_t channel_stride, const uint8_t* mask, int32_t height, int32_t width,
                               int32_t dim, const int32_t* seed_fg, int32_t n_seeds, const fms_params* p,
                               float* endpoints, int32_t* iters, uint8_t* converged, int32_t* counts,
                               fms_stats* stats) {
  if (!h || !p) return FMS_ERR_INVALID_ARG;
  if (n_seeds < 0 || (n_seeds > 0 && (!seed_fg || !endpoints || !iters || !converged))) return FMS_ERR_INVALID_ARG;
  FMS_TRY(check_params(p));
  const fms_frame fr = frame_of(emb, pixel_stride, channel_stride, mask, height, width, p->bandwidth, 0, nullptr);
  FMS_TRY(check_frame(fr, dim));
  if (p->precision != FMS_PREC_FP32 || p->timing != 0) return FMS_ERR_UNSUPPORTED;
  const int64_t P = int64_t(height) * int64_t(width);
  if (dim > kNaDp || P > kNaMaxPixels || n_seeds > kNaMaxSeeds) return FMS_ERR_UNSUPPORTED;
  if (!h->na_scratch || !h->dpub || h->hpub.cap < 16 + meta_bytes(1)) return FMS_ERR_HIP;
  DeviceGuard guard(h->device);
  Call c;
  c.st = static_cast<hipStream_t>(stream);
  c.F = 1;
  c.dim = dim;
  c.dp = kNaDp;
  c.form = fms::FORM_FP32;
  set_tiling(c, p);  // the handle's tuning table is not used
  const int m = n_seeds;
  // Chunk partials of the FP32 tilings the steps and the window counts take.
  if (m > 0 && int64_t(std::max(fms::shift_partial_rows(c.tile_fp32, m),
                                fms::shift_partial_rows(c.tile_fp32_big, m))) > kNaPartialRows)
    return FMS_ERR_UNSUPPORTED;
  unsigned char* base = h->na_scratch;
  int* blk = reinterpret_cast<int*>(base + NaLayout::blk);
  int* fg_idx = reinterpret_cast<int*>(base + NaLayout::fg_idx);
  float* x32 = reinterpret_cast<float*>(base + NaLayout::x32);
  float* x32t = reinterpret_cast<float*>(base + NaLayout::x32t);
  float* y = reinterpret_cast<float*>(base + NaLayout::y);
  float* yc[2] = {reinterpret_cast<float*>(base + NaLayout::yc0), reinterpret_cast<float*>(base + NaLayout::yc1)};
  int* lists[2] = {reinterpret_cast<int*>(base + NaLayout::active), reinterpret_cast<int*>(base + NaLayout::next_active)};
  int* its = reinterpret_cast<int*>(base + NaLayout::iters);
  int* ident = reinterpret_cast<int*>(base + NaLayout::ident);
  int* cnt = reinterpret_cast<int*>(base + NaLayout::counts);
  uint8_t* state = base + NaLayout::state;
  int* pcount = reinterpret_cast<int*>(base + NaLayout::pcount);
  float* partial = reinterpret_cast<float*>(base + NaLayout::partial);
  int* meta = reinterpret_cast<int*>(base + NaLayout::meta);
  auto* geo = reinterpret_cast<fms::FrameGeo*>(base + NaLayout::geo);
  auto* rtab = reinterpret_cast<fms::RoundTab*>(base + NaLayout::rt);
  c.b.F = 1;
  c.b.geo = geo;
  c.b.rt = rtab;
  c.b.meta = meta;
  c.b.meta64 = reinterpret_cast<unsigned long long*>(meta + META_COUNT);
  c.b.max_n = kNaMaxFg;
  c.b.max_blocks = kNaMaxFg / fms::kBlockPix;
  c.b.max_mblk = (P + fms::kMaskBlockPix - 1) / fms::kMaskBlockPix;
  c.fr.assign(1, FrameHost{});
  fms::FrameGeo g{};
  g.desc = fms::FrameDesc{emb, pixel_stride, channel_stride, mask, P, dim, kNaDp};
  g.thr = float(1.0 - p->bandwidth);
  g.tol = float(tol_of(p, p->bandwidth));
  fms::RoundTab rt{};
  rt.nact = m;
  // Tables and counters, compaction (rows beyond the capacity are neither
  // written nor used), seeds, the round's start.
  HIP_TRY(fms::launch_set_tables(c.st, g, rt, geo, rtab, meta, c.b.meta64));
  HIP_TRY(fms::launch_mask_count(c.st, c.b, blk));
  HIP_TRY(fms::launch_scan_blocks(c.st, c.b, blk));
  HIP_TRY(fms::launch_compact(c.st, c.b, kNaDp, blk, fg_idx, x32, x32t, nullptr, nullptr, nullptr,
                              kNaMaxFg));
  HIP_TRY(fms::launch_geo_from_count(c.st, c.b, kNaMaxFg));
  if (m > 0) {
    HIP_TRY(fms::launch_init_seeds(c.st, seed_fg, m, -1, x32, kNaDp, y, meta));
    HIP_TRY(fms::launch_round_begin(c.st, c.b, m, true, lists[0], state, its, nullptr, x32, kNaDp, y));
    // The iteration (Alg. 2, the parallel seed loop; Sec. 3.2.1 and 3.2.3),
    // enqueued in batches with a read of the counters between them.
    static constexpr int kSched[] = {3, 6, 8};
    int t = 0, nbatch = 0, bound = m;
    while (t < p->max_iter) {
      const int nb = std::min(kSched[std::min(nbatch, 2)], p->max_iter - t);
      ++nbatch;
      const fms::Tiling& tl = pick_tiling(c, fms::FORM_FP32, bound);
      for (int i = 0; i < nb; ++i, ++t) {
        const fms::IterCtl ctl{-1, t, p->gamma, 0};
        const float* yin = t == 0 ? y : yc[t & 1];
        HIP_TRY(fms::launch_shift(c.st, c.b, fms::FORM_FP32, kNaDp, tl, x32, x32t, nullptr, yin, nullptr,
                                  ctl, m, partial));
        HIP_TRY(fms::launch_reduce(c.st, c.b, kNaDp, tl, partial, lists[t & 1], y, state, its, lists[(t + 1) & 1],
                                   yc[(t + 1) & 1], ctl, m, 0, nullptr, yin));
      }
      FMS_TRY(read_meta(h, c));
      const int* hm = h->hm(0);
      const bool over = double(hm[META_NCONV]) > p->gamma * double(hm[META_NSEL]);
      if (hm[fms::META_DONE] || hm[fms::META_ACT + (t & 1)] <= 0 || over) break;
      bound = hm[fms::META_ACT + (t & 1)];
    }
    // Window counts at every slot (kept for the converged seeds), outputs.
    HIP_TRY(fms::launch_iota(c.st, c.b, ident, m));
    HIP_TRY(fms::launch_count(c.st, c.b, fms::FORM_FP32, kNaDp, count_tiling(c, m), x32, nullptr, y, ident, m, pcount,
                              cnt, -1));
    HIP_TRY(fms::launch_lockstep_out(c.st, m, kNaDp, dim, y, state, its, cnt, endpoints, iters, converged, counts));
  }
  FMS_TRY(read_meta(h, c));
  const int* hm = h->hm(0);
  if (hm[fms::META_OVERCAP] != 0) return FMS_ERR_UNSUPPORTED;
  if (hm[META_N] == 0 && m > 0) return FMS_ERR_INVALID_ARG;
  if (hm[fms::META_BAD] != 0) return FMS_ERR_BAD_INPUT;
  if (hm[fms::META_BADSEED] != 0) return FMS_ERR_INVALID_ARG;
  if (stats) {
    fms_stats& sx = stats[0];
    std::memset(&sx, 0, sizeof(sx));
    sx.n_min = std::numeric_limits<double>::quiet_NaN();
    sx.n_fg = hm[META_N];
    sx.seeds_used = m;
    if (m > 0) {
      sx.iterations_total = hm[META_STEPS];
      sx.seed_pixel_updates = int64_t(h->hm64(0, 1));
      sx.n_discarded = m - hm[META_NCONV];
    }
  }
  return FMS_OK;
}

}  // namespace

extern "C" {

void fms_default_params(fms_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->bandwidth = 0.1;
  p->conv_tol = 0.0;
  p->gamma = 0.9;
  p->big_l = 2.0;
  p->big_h = 8.0;
  p->p_target = 0.99;
  p->seed = 0;
  p->n_initial = 128;
  p->n_state_in = 0;
  p->max_iter = 100;
  p->max_rounds = 32;
  p->precision = FMS_PREC_FP32;
  p->refine_iters = 2;
}

const char* fms_status_string(fms_status s) {
  switch (s) {
    case FMS_OK: return "ok";
    case FMS_ERR_INVALID_ARG: return "invalid argument";
    case FMS_ERR_UNSUPPORTED: return "unsupported configuration";
    case FMS_ERR_BAD_INPUT: return "a foreground embedding is zero or not finite";
    case FMS_ERR_CAPACITY: return "mode buffer too small";
    case FMS_ERR_HIP: return "HIP runtime error";
  }
  return "unknown status";
}

fms_status fms_create(fms_handle* out, int32_t device_ordinal) {
  if (!out) return FMS_ERR_INVALID_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess) return FMS_ERR_HIP;
  if (device_ordinal < 0 || device_ordinal >= count) return FMS_ERR_INVALID_ARG;
  DeviceGuard guard(device_ordinal);
  fms_handle h = new (std::nothrow) fms_handle_s();
  if (!h) return FMS_ERR_HIP;
  h->device = device_ordinal;
  if (hipEventCreateWithFlags(&h->sync_ev, hipEventDisableTiming) != hipSuccess) {
    fms_destroy(h);
    return FMS_ERR_HIP;
  }
  // This GPU's copy of the no-allocation entry point's buffer, and the mapped
  // counter area every call reads (sized for one frame here, so that entry
  // point never allocates).
  void* sp = nullptr;
  if (hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)) != hipSuccess || !sp ||
      h->ensure_pub(16 + meta_bytes(1)) != hipSuccess) {
    fms_destroy(h);
    return FMS_ERR_HIP;
  }
  h->na_scratch = static_cast<unsigned char*>(sp);
  *out = h;
  return FMS_OK;
}

fms_status fms_destroy(fms_handle h) {
  if (!h) return FMS_OK;
  DeviceGuard guard(h->device);
  (void)hipDeviceSynchronize();
  DevBuf* bufs[] = {&h->blk,    &h->fg_idx,  &h->x32,        &h->x32t,    &h->x16,
                    &h->order,  &h->rank,    &h->elig,       &h->y,       &h->yc0,         &h->yc1,
                    &h->active, &h->next_active, &h->state,  &h->iters,   &h->seed_pos,    &h->seed_fg,
                    &h->ident,  &h->cand,    &h->counts,     &h->sorted,  &h->scount,      &h->pcount,
                    &h->partial, &h->bits,   &h->acc,        &h->modes,   &h->mode_counts, &h->meta,
                    &h->geo,     &h->rt,         &h->out_off, &h->enorm, &h->x16l,
                    &h->ring,    &h->yr,         &h->rstate,  &h->riters};
  for (DevBuf* b : bufs) b->release();
  for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
  if (h->sync_ev) (void)hipEventDestroy(h->sync_ev);
  h->drop_graphs();
  if (h->cap_st) (void)hipStreamDestroy(h->cap_st);
  for (PinBuf* b : {&h->hpub, &h->hgeo, &h->hrt, &h->hoff, &h->hstage}) b->release();
  delete h;
  return FMS_OK;
}

fms_status fms_seed_order(fms_handle h, void* stream, int32_t n, uint64_t seed, int32_t* order) {
  if (!h || n < 0 || (n > 0 && !order)) return FMS_ERR_INVALID_ARG;
  if (n == 0) return FMS_OK;
  DeviceGuard guard(h->device);
  uint64_t keys[4];
  round_keys(seed, keys);
  HIP_TRY(fms::launch_seed_order_plain(static_cast<hipStream_t>(stream), n, half_bits(n), keys, order));
  return FMS_OK;
}

fms_status fms_cluster_batch(fms_handle h, void* stream, int32_t n_frames, const fms_frame* frames, int32_t dim,
                             const fms_params* p, float* modes, int32_t* mode_counts, int32_t k_max,
                             int32_t* mode_offsets, fms_stats* stats) {
  if (!h || !frames || n_frames < 1 || !mode_offsets || k_max < 0 || (k_max > 0 && !modes))
    return FMS_ERR_INVALID_ARG;
  for (int f = 0; f < n_frames; ++f)
    if (!frames[f].labels) return FMS_ERR_INVALID_ARG;
  DeviceGuard guard(h->device);
  Call c;
  FMS_TRY(begin_call(h, stream, n_frames, frames, dim, p, c));
  ModeOutputs out{modes, mode_counts, k_max, {}, 0};
  FMS_TRY(cluster_frames(h, c, p, out));
  for (int f = 0; f <= c.F; ++f) mode_offsets[f] = int32_t(out.offsets[size_t(f)]);
  fill_stats(c, stats);
  if (out.total > k_max) return FMS_ERR_CAPACITY;
  return FMS_OK;
}

fms_status fms_cluster(fms_handle h, void* stream, const float* emb, int64_t pixel_stride, int64_t channel_stride,
                       const uint8_t* mask, int32_t height, int32_t width, int32_t dim, const fms_params* p,
                       float* modes_out, int32_t* mode_counts_out, int32_t k_max, int32_t* n_modes, int32_t* labels,
                       fms_stats* stats) {
  if (!h || !p || !n_modes || !labels || k_max < 0 || (k_max > 0 && !modes_out)) return FMS_ERR_INVALID_ARG;
  const fms_frame fr =
      frame_of(emb, pixel_stride, channel_stride, mask, height, width, p->bandwidth, p->n_state_in, labels);
  int32_t off[2] = {0, 0};
  const fms_status stt = fms_cluster_batch(h, stream, 1, &fr, dim, p, modes_out, mode_counts_out, k_max, off, stats);
  if (stt == FMS_OK || stt == FMS_ERR_CAPACITY) *n_modes = off[1];
  return stt;
}

fms_status fms_shift_seeds(fms_handle h, void* stream, const float* emb, int64_t pixel_stride, int64_t channel_stride,
                           const uint8_t* mask, int32_t height, int32_t width, int32_t dim, const int32_t* seed_fg,
                           int32_t n_seeds, const fms_params* p, float* endpoints, int32_t* iters, uint8_t* converged,
                           int32_t* counts, fms_stats* stats) {
  if (!h || !p) return FMS_ERR_INVALID_ARG;
  if (n_seeds < 0 || (n_seeds > 0 && (!seed_fg || !endpoints || !iters || !converged))) return FMS_ERR_INVALID_ARG;
  DeviceGuard guard(h->device);
  const fms_frame fr = frame_of(emb, pixel_stride, channel_stride, mask, height, width, p->bandwidth, 0, nullptr);
  Call c;
  FMS_TRY(begin_call(h, stream, 1, &fr, dim, p, c));
  FrameHost& fh = c.fr[0];
  if (n_seeds == 0) {
    HIP_TRY(h->wait(c.st));
    fill_stats(c, stats);
    return FMS_OK;
  }
  if (fh.g.n == 0) return FMS_ERR_INVALID_ARG;
  const int m = n_seeds;
  // More seeds than foreground pixels: widen the (single) frame's centre
  // region and its chunk partials.
  if (m > fh.g.n) FMS_TRY(ensure_centres(h, c, m));
  HIP_TRY(fms::launch_init_seeds(c.st, seed_fg, m, fh.g.n, h->x32.as<float>(), c.dp, h->y.as<float>(),
                                 h->meta.as<int>()));
  fh.rt = fms::RoundTab{};
  fh.rt.nact = m;
  FMS_TRY(upload_rt(h, c));
  FMS_TRY(read_meta(h, c));
  if (h->hm(0)[META_BAD] != 0) return FMS_ERR_BAD_INPUT;
  if (h->hm(0)[META_BADSEED] != 0) return FMS_ERR_INVALID_ARG;
  const bool timing = p->timing != 0;
  FMS_TRY(run_iterations(h, c, h->y.as<float>(), m, p->gamma, p->max_iter, c.form, timing, nullptr, true,
                         replay_extra(c)));
  fh.sx.iterations_total = h->hm(0)[META_STEPS];
  fh.sx.seed_pixel_updates = int64_t(h->hm64(0, 1));
  if (c.ring_len > 0) {
    // The converged seeds' last iterations again in FP32 and the early stop
    // on their FP32 step counts; the outputs are the replay's endpoints,
    // step counts and converged flags.
    FMS_TRY(run_replay(h, c, m, p->gamma, timing));
    FMS_TRY(read_meta(h, c));
    add_replay_stats(h, c, 0, timing ? &c.tm : nullptr);
  }
  std::vector<int> conv;
  FMS_TRY(host_converged(h, c, conv));
  const int nc = int(conv.size());
  // Window counts of every slot (the output keeps them for converged seeds).
  fh.rt.nact = m;
  FMS_TRY(upload_rt(h, c));
  HIP_TRY(fms::launch_iota(c.st, c.b, h->ident.as<int>(), m));
  HIP_TRY(count_windows(h, c, h->y.as<float>(), h->ident.as<int>(), m, h->counts.as<int>(), -1));
  HIP_TRY(fms::launch_lockstep_out(c.st, m, c.dp, dim, h->y.as<float>(), h->state.as<uint8_t>(), h->iters.as<int>(),
                                   h->counts.as<int>(), endpoints, iters, converged, counts));
  HIP_TRY(h->wait(c.st));
  fh.sx.seeds_used = m;
  fh.sx.n_discarded = m - nc;
  fill_stats(c, stats);
  return FMS_OK;
}

fms_status fms_shift_seeds_noalloc(fms_handle h, void* stream, const float* emb, int64_t pixel_stride,
                                   int64_t channel_stride, const uint8_t* mask, int32_t height, int32_t width,
                                   int32_t dim, const int32_t* seed_fg, int32_t n_seeds, const fms_params* p,
                                   float* endpoints, int32_t* iters, uint8_t* converged, int32_t* counts,
                                   fms_stats* stats) {
  return shift_seeds_noalloc(h, stream, emb, pixel_stride, channel_stride, mask, height, width, dim, seed_fg, n_seeds,
                             p, endpoints, iters, converged, counts, stats);
}

// The tuner of fms_autotune (one frame) and fms_autotune_batch (several
// frames, every launch spanning all of them, as in fms_cluster_batch).
fms_status autotune_frames(fms_handle h, void* stream, int32_t n_frames, const fms_frame* frames, int32_t dim,
                           const fms_params* p, fms_tune_entry* entries, int32_t capacity, int32_t* n_entries,
                           fms_tune_report* report) {
  if (!h || n_frames < 1 || !frames || !p || capacity < 0 || (capacity > 0 && !entries)) return FMS_ERR_INVALID_ARG;
  DeviceGuard guard(h->device);
  fms_params q = *p;
  q.tile_seeds = q.tile_items = q.tile_chunks = q.tile_waves = 0;
  q.timing = 0;
  q.graphs = 0;
  const bool batch = n_frames > 1;
  std::vector<fms_frame> frs(frames, frames + n_frames);
  for (fms_frame& fr : frs) {
    fr.labels = nullptr;
    fr.n_state_in = 0;
  }
  Call c;
  FMS_TRY(begin_call(h, stream, n_frames, frs.data(), dim, &q, c));
  c.tuned = nullptr;
  const int n = c.b.max_n;
  FMS_TRY(read_meta(h, c));
  for (int f = 0; f < n_frames; ++f)
    if (h->hm(f)[META_BAD] != 0) return FMS_ERR_BAD_INPUT;
  if (n == 0) return FMS_ERR_INVALID_ARG;
  // Seed counts per frame (a frame takes at most its foreground count); a
  // batch stops at 2,048 (its steps at 8,192 seeds per frame take seconds in
  // FP32, and larger launches take the nearest entry).
  std::vector<int> ms;
  for (int m : {128, 512, 2048, 8192})
    if (m <= n && (!batch || m <= 2048)) ms.push_back(m);
  if (ms.empty()) ms.push_back(n);
  const int mmax = ms.back();
  auto m_of = [&](int f, int m) { return std::min(m, c.fr[f].g.n); };
  if (!batch) FMS_TRY(ensure_centres(h, c, mmax));
  // Candidates of each step form the precision runs (the plain BF16 form's
  // replay runs FP32 steps): every compiled (group, items, waves) shape.
  std::vector<int> forms{c.form};
  if (c.form == fms::FORM_BF16 && c.ring_len > 0) forms.push_back(fms::FORM_FP32);
  std::vector<std::vector<fms::Tiling>> cand(forms.size());
  for (size_t fi = 0; fi < forms.size(); ++fi) {
    for (int gs : {16, 32, 64, 128})
      for (int items : {256, 512, 1024})
        for (int wv : {4, 8, 16}) {
          const fms::Tiling t = fms::make_tiling(forms[fi], c.dp, gs, items, 0, wv);
          if (t.group_seeds != gs || t.waves != wv) continue;  // rounded to another shape
          cand[fi].push_back(t);
        }
  }
  // Chunk partials: each frame's region holds the largest any candidate
  // (or the defaults) needs at the frame's most centres.
  size_t prows = 0;
  for (int f = 0; f < n_frames; ++f) {
    FrameHost& fh = c.fr[f];
    const int cap_f = batch ? m_of(f, mmax) : mmax;
    size_t r = size_t(partial_rows(c, cap_f));
    for (const auto& cf : cand)
      for (const fms::Tiling& t : cf) r = std::max(r, fms::shift_partial_rows(t, cap_f));
    fh.g.part0 = int64_t(prows);
    prows += r;
  }
  if (batch) FMS_TRY(upload_geo(h, c));
  HIP_TRY(h->pcount.ensure(prows * sizeof(int)));
  HIP_TRY(h->partial.ensure(prows * size_t(c.dp) * sizeof(float)));
  HIP_TRY(h->ensure_events(2));
  // The identity list of the timed centres: k_iota writes rt.nact entries,
  // so the counts go to the device first.
  for (int f = 0; f < n_frames; ++f) {
    c.fr[f].rt = fms::RoundTab{};
    c.fr[f].rt.nact = batch ? m_of(f, mmax) : mmax;
  }
  FMS_TRY(upload_rt(h, c));
  HIP_TRY(fms::launch_iota(c.st, c.b, h->ident.as<int>(), mmax));
  int* ident = h->ident.as<int>();
  float* y = h->y.as<float>();
  // One warm-up, then the mean of kReps (fused step, reduction) pairs (two
  // for a batch, whose launches are long).
  const int kReps = batch ? 2 : 6;
  auto time_one = [&](const fms::Tiling& t, int form, int m, float* us) -> fms_status {
    const bool bf16 = form != fms::FORM_FP32;
    const void* xrm = bf16 ? h->x16.p : h->x32.p;
    const void* xt = bf16 ? nullptr : h->x32t.p;
    const uint16_t* xrl = form == fms::FORM_SPLIT ? h->x16l.as<uint16_t>() : nullptr;
    for (int f = 0; f < n_frames; ++f) {
      const int64_t r0 = c.fr[f].g.row0;
      HIP_TRY(fms::launch_init_seeds(c.st, ident + r0, batch ? m_of(f, m) : m, c.fr[f].g.n,
                                     h->x32.as<float>() + r0 * c.dp, c.dp, y + r0 * c.dp,
                                     h->meta.as<int>() + int64_t(f) * META_COUNT));
    }
    const fms::IterCtl ctl{-1, -1, 1.0};
    for (int r = 0; r <= kReps; ++r) {
      if (r == 1) HIP_TRY(hipEventRecord(h->events[0], c.st));
      HIP_TRY(fms::launch_shift(c.st, c.b, form, c.dp, t, xrm, xt, xrl, y, ident, ctl, m,
                                h->partial.as<float>(), nullptr, nullptr));
      HIP_TRY(fms::launch_reduce(c.st, c.b, c.dp, t, h->partial.as<float>(), ident, y, h->state.as<uint8_t>(),
                                 h->iters.as<int>(), nullptr, nullptr, ctl, m, 1));
    }
    HIP_TRY(hipEventRecord(h->events[1], c.st));
    HIP_TRY(hipEventSynchronize(h->events[1]));
    float ms_ = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms_, h->events[0], h->events[1]));
    *us = 1000.f * ms_ / kReps;
    return FMS_OK;
  };
  std::vector<TunedTiling> found;
  for (size_t fi = 0; fi < forms.size(); ++fi) {
    const int form = forms[fi];
    for (int m : ms) {
      for (int f = 0; f < n_frames; ++f) {
        c.fr[f].rt = fms::RoundTab{};
        c.fr[f].rt.nact = batch ? m_of(f, m) : m;
      }
      FMS_TRY(upload_rt(h, c));
      float us_def = 0.f;
      FMS_TRY(time_one(pick_tiling(c, form, m), form, m, &us_def));
      TunedTiling best{};
      bool have = false;
      for (const fms::Tiling& t : cand[fi]) {
        float us = 0.f;
        FMS_TRY(time_one(t, form, m, &us));
        if (!have || us < best.e.us_per_step) {
          have = true;
          best.t = t;
          best.e.us_per_step = us;
        }
      }
      best.form = form;
      best.batch = batch;
      best.dp = c.dp;
      best.nb = c.nb;
      best.m = m;
      best.e.precision = form == fms::FORM_BF16 ? FMS_PREC_BF16_REFINE
                         : form == fms::FORM_SPLIT ? FMS_PREC_BF16_SPLIT
                                                   : FMS_PREC_FP32;
      best.e.dim_padded = c.dp;
      best.e.n_fg = n;
      best.e.seeds = m;
      best.e.tile_seeds = best.t.group_seeds;
      best.e.tile_items = best.t.target_items;
      best.e.tile_waves = best.t.waves;
      best.e.us_default = us_def;
      found.push_back(best);
    }
  }
  // The table without entries of the same forms, D class and bucket, and
  // with the new ones.
  std::vector<TunedTiling> without, with;
  for (const TunedTiling& t : h->tuned) {
    bool same = false;
    for (const TunedTiling& u : found)
      same = same || (t.form == u.form && t.batch == u.batch && t.dp == u.dp && t.nb == u.nb);
    if (!same) without.push_back(t);
  }
  with = without;
  for (const TunedTiling& u : found) with.push_back(u);
  // Whole calls on the frame with each table, alternating (one warm-up call
  // each, then kCallReps rounds of two calls); the new entries stay only
  // when the median call is faster with them.
  constexpr int kCallReps = 6;
  std::vector<double> call_ms[2];
  auto call = [&](const std::vector<TunedTiling>& table) -> fms_status {
    h->tuned = table;
    Call cc;
    FMS_TRY(begin_call(h, stream, n_frames, frs.data(), dim, &q, cc));
    ModeOutputs none{nullptr, nullptr, 0, {}, 0};
    return cluster_frames(h, cc, &q, none);
  };
  for (int v = 0; v < 2; ++v) FMS_TRY(call(v ? with : without));
  for (int r = 0; r < kCallReps; ++r)
    for (int k = 0; k < 2; ++k) {
      const int v = (r & 1) ? 1 - k : k;
      const auto t0 = std::chrono::steady_clock::now();
      FMS_TRY(call(v ? with : without));
      FMS_TRY(call(v ? with : without));
      call_ms[v].push_back(std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() / 2);
    }
  for (auto& m : call_ms) std::sort(m.begin(), m.end());
  const double ms_default = call_ms[0][kCallReps / 2], ms_tuned = call_ms[1][kCallReps / 2];
  const bool kept = ms_tuned < ms_default;
  h->tuned = kept ? with : without;
  if (report) {
    report->ms_default = float(ms_default);
    report->ms_tuned = float(ms_tuned);
    report->kept = kept ? 1 : 0;
  }
  const int cnt = int(found.size());
  if (n_entries) *n_entries = cnt;
  if (!entries) return FMS_OK;
  if (capacity < cnt) return FMS_ERR_CAPACITY;
  for (int i = 0; i < cnt; ++i) entries[i] = found[size_t(i)].e;
  return FMS_OK;
}

fms_status fms_autotune(fms_handle h, void* stream, const fms_frame* frame, int32_t dim, const fms_params* p,
                        fms_tune_entry* entries, int32_t capacity, int32_t* n_entries, fms_tune_report* report) {
  return autotune_frames(h, stream, 1, frame, dim, p, entries, capacity, n_entries, report);
}

fms_status fms_autotune_batch(fms_handle h, void* stream, int32_t n_frames, const fms_frame* frames, int32_t dim,
                              const fms_params* p, fms_tune_entry* entries, int32_t capacity, int32_t* n_entries,
                              fms_tune_report* report) {
  if (n_frames < 2) return FMS_ERR_INVALID_ARG;
  return autotune_frames(h, stream, n_frames, frames, dim, p, entries, capacity, n_entries, report);
}

fms_status fms_clear_tuning(fms_handle h) {
  if (!h) return FMS_ERR_INVALID_ARG;
  h->tuned.clear();
  return FMS_OK;
}

fms_status fms_unroll(fms_handle h, void* stream, const float* emb, int64_t pixel_stride, int64_t channel_stride,
                      const uint8_t* mask, int32_t height, int32_t width, int32_t dim, const int32_t* seed_fg,
                      int32_t n_seeds, int32_t steps, double bandwidth, float* y_out, float* y_prev,
                      float* v_norm) {
  if (!h || n_seeds < 1 || steps < 1 || !seed_fg || !y_out || !y_prev || !v_norm) return FMS_ERR_INVALID_ARG;
  DeviceGuard guard(h->device);
  const fms_frame fr = frame_of(emb, pixel_stride, channel_stride, mask, height, width, bandwidth, 0, nullptr);
  Call c;
  FMS_TRY(begin_single(h, stream, fr, dim, c));
  FrameHost& fh = c.fr[0];
  if (fh.g.n == 0) return FMS_ERR_INVALID_ARG;
  const int m = n_seeds;
  FMS_TRY(ensure_centres(h, c, m));
  HIP_TRY(fms::launch_init_seeds(c.st, seed_fg, m, fh.g.n, h->x32.as<float>(), c.dp, h->y.as<float>(),
                                 h->meta.as<int>()));
  fh.rt = fms::RoundTab{};
  fh.rt.nact = m;
  FMS_TRY(upload_rt(h, c));
  HIP_TRY(fms::launch_iota(c.st, c.b, h->ident.as<int>(), m));
  FMS_TRY(read_meta(h, c));
  if (h->hm(0)[META_BAD] != 0) return FMS_ERR_BAD_INPUT;
  if (h->hm(0)[META_BADSEED] != 0) return FMS_ERR_INVALID_ARG;
  // `steps` plain FP32 steps (no freezing, no early stop); y_{T-1} is kept
  // and the last step also reports |V_T|.
  const fms::Tiling& tl = pick_tiling(c, fms::FORM_FP32, m);
  const fms::IterCtl ctl{-1, -1, 1.0};
  float* y = h->y.as<float>();
  for (int t = 0; t < steps; ++t) {
    if (t + 1 == steps) HIP_TRY(fms::launch_rows_out(c.st, m, c.dp, dim, y, y_prev));
    HIP_TRY(fms::launch_shift(c.st, c.b, fms::FORM_FP32, c.dp, tl, h->x32.p, h->x32t.p, nullptr, y,
                              h->ident.as<int>(), ctl, m, h->partial.as<float>()));
    HIP_TRY(fms::launch_reduce(c.st, c.b, c.dp, tl, h->partial.as<float>(), h->ident.as<int>(), y,
                               h->state.as<uint8_t>(), h->iters.as<int>(), nullptr, nullptr, ctl, m, 1,
                               t + 1 == steps ? v_norm : nullptr));
  }
  HIP_TRY(fms::launch_rows_out(c.st, m, c.dp, dim, y, y_out));
  HIP_TRY(h->wait(c.st));
  return FMS_OK;
}

fms_status fms_unroll_backward(fms_handle h, void* stream, const float* emb, int64_t pixel_stride,
                               int64_t channel_stride, const uint8_t* mask, int32_t height, int32_t width, int32_t dim,
                               int32_t n_seeds, double bandwidth, const float* y_out, const float* y_prev,
                               const float* v_norm, const float* grad_y, float* grad_emb) {
  if (!h || n_seeds < 1 || !y_out || !y_prev || !v_norm || !grad_y || !grad_emb) return FMS_ERR_INVALID_ARG;
  DeviceGuard guard(h->device);
  const fms_frame fr = frame_of(emb, pixel_stride, channel_stride, mask, height, width, bandwidth, 0, nullptr);
  Call c;
  FMS_TRY(begin_single(h, stream, fr, dim, c));
  const int m = n_seeds;
  const int m_pad = (m + 15) / 16 * 16;
  FMS_TRY(ensure_centres(h, c, m_pad));
  float* yp = h->yc0.as<float>();
  float* gv = h->yc1.as<float>();
  HIP_TRY(fms::launch_rows_in(c.st, m, m_pad, dim, c.dp, y_prev, yp));
  HIP_TRY(fms::launch_unroll_gv(c.st, m, m_pad, dim, c.dp, y_out, v_norm, grad_y, gv));
  HIP_TRY(fms::launch_zero_strided(c.st, c.fr[0].g.desc.n_pixels, dim, pixel_stride, channel_stride, grad_emb));
  HIP_TRY(fms::launch_unroll_grad(c.st, c.b, c.dp, h->x32.as<float>(), h->fg_idx.as<int>(), h->enorm.as<float>(), yp,
                                  gv, m_pad, dim, pixel_stride, channel_stride, grad_emb));
  FMS_TRY(read_meta(h, c));
  if (h->hm(0)[META_BAD] != 0) return FMS_ERR_BAD_INPUT;
  return FMS_OK;
}

}  // extern "C"
