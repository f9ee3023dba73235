// Host runtime of the Faster Mean-shift library: handle and workspace, frame
// preparation, the round loop of the online seed optimisation policy
// (Sec. 3.2.2-3.2.4) and the C ABI declared in include/fms.h.
//
// The CPU steers the seed count and the GPU iterates the seeds (Fig. 3): the
// host reads a few counters back after each GPU step (iteration, round) and
// decides what to launch next.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>

#include "fms.h"
#include "fms_internal.h"

namespace {

using fms::META_BAD;
using fms::META_BADSEED;
using fms::META_COUNT;
using fms::META_CURSOR;
using fms::META_LEFT;
using fms::META_N;
using fms::META_NCONV;
using fms::META_NSEL;
using fms::META_REFINE_BAD;

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
  // Grow like ensure(), keeping the first `keep` bytes (the old buffer is
  // copied on `st` and freed once the copy has finished).
  hipError_t grow_keep(size_t bytes, size_t keep, hipStream_t st) {
    if (bytes <= cap) return hipSuccess;
    size_t want = std::max<size_t>(bytes + bytes / 2, 4096);
    void* np = nullptr;
    hipError_t e = hipMalloc(&np, want);
    if (e != hipSuccess) return e;
    if (p && keep > 0) {
      e = hipMemcpyAsync(np, p, std::min(keep, cap), hipMemcpyDeviceToDevice, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) {
        (void)hipFree(np);
        return e;
      }
    }
    if (p) (void)hipFree(p);
    p = np;
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

}  // namespace

struct fms_handle_s {
  int device = 0;
  // Frame data.
  DevBuf blk, fg_idx, x32, x32t, x16, x16t, order, rank, elig;
  // Round data.
  DevBuf y, yc0, yc1, active, next_active, state, iters, seed_pos, seed_fg, ident, cand, counts, pcount, partial;
  DevBuf bits, blocked, acc, sorted, scount;
  // Modes found so far.
  DevBuf modes, mode_counts;
  DevBuf meta, meta64;
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
  // Host waits go through an event without timing (cheaper to wait on than
  // a whole-stream synchronisation).
  hipEvent_t sync_ev = nullptr;
  hipError_t wait(hipStream_t st) {
    hipError_t e = hipEventRecord(sync_ev, st);
    return e == hipSuccess ? hipEventSynchronize(sync_ev) : e;
  }
  // Pinned host staging.
  int* hmeta = nullptr;
  void* hstage = nullptr;
  size_t hstage_cap = 0;

  hipError_t stage(size_t bytes) {
    if (bytes <= hstage_cap) return hipSuccess;
    if (hstage) (void)hipHostFree(hstage);
    hstage = nullptr;
    hstage_cap = 0;
    size_t want = std::max<size_t>(bytes + bytes / 4, 1 << 16);
    hipError_t e = hipHostMalloc(&hstage, want, hipHostMallocDefault);
    if (e != hipSuccess) {
      hstage = nullptr;
      return e;
    }
    hstage_cap = want;
    return hipSuccess;
  }
};

namespace {

#define HIP_TRY(expr)                       \
  do {                                      \
    hipError_t _e = (expr);                 \
    if (_e != hipSuccess) return FMS_ERR_HIP; \
  } while (0)

// Launches with at least kBigGroupMin centres use seed groups of kBigGroup
// (where compiled): on the 512x512, D = 32 workload a 64-seed group is about
// 20% faster than a 32-seed one from 1,024 centres on, and no slower at 256.
constexpr int kBigGroup = 64;
constexpr int kBigGroupMin = 512;

struct Frame {
  fms::FrameDesc desc;
  int n = 0;
  int dp = 32;
  int n_pad = 0;
  fms::StepGeom geom{};
  fms::Tiling tile{};       // the precision of the call
  fms::Tiling tile_fp32{};  // FP32 steps (refinement) and window counts
  // The same with larger seed groups, for launches with many centres (fewer
  // re-reads of the pixels per centre).
  fms::Tiling tile_big{};
  fms::Tiling tile_fp32_big{};
};

fms_status check_params(const fms_params* p) {
  if (!p) return FMS_ERR_INVALID_ARG;
  if (!(p->bandwidth > 0.0 && p->bandwidth < 2.0)) return FMS_ERR_INVALID_ARG;
  if (!(p->gamma >= 0.0 && p->gamma <= 1.0)) return FMS_ERR_INVALID_ARG;
  if (!(p->big_l > 0.0) || !(p->big_h > 0.0)) return FMS_ERR_INVALID_ARG;
  if (!(p->p_target > 0.0 && p->p_target < 1.0)) return FMS_ERR_INVALID_ARG;
  if (!std::isfinite(p->conv_tol)) return FMS_ERR_INVALID_ARG;
  if (p->n_initial < 1 || p->max_iter < 1 || p->max_rounds < 1 || p->refine_iters < 0) return FMS_ERR_INVALID_ARG;
  if (p->precision != FMS_PREC_FP32 && p->precision != FMS_PREC_BF16_REFINE) return FMS_ERR_INVALID_ARG;
  if (p->tile_seeds < 0 || p->tile_items < 0 || p->tile_chunks < 0) return FMS_ERR_INVALID_ARG;
  return FMS_OK;
}

fms_status check_frame_args(fms_handle h, const float* emb, int64_t ps, int64_t cs, int32_t height, int32_t width,
                            int32_t dim) {
  if (!h || !emb) return FMS_ERR_INVALID_ARG;
  if (height < 1 || width < 1 || ps < 0 || cs < 0) return FMS_ERR_INVALID_ARG;
  if (dim < 1) return FMS_ERR_INVALID_ARG;
  if (dim > 128) return FMS_ERR_UNSUPPORTED;
  if (int64_t(height) * int64_t(width) > int64_t(std::numeric_limits<int32_t>::max())) return FMS_ERR_UNSUPPORTED;
  return FMS_OK;
}

// Compact the foreground, normalise it and write the four layouts.
fms_status prepare_frame(fms_handle h, hipStream_t st, const float* emb, int64_t ps, int64_t cs, const uint8_t* mask,
                         int32_t height, int32_t width, int32_t dim, bool bf16, Frame& fr) {
  const int64_t P = int64_t(height) * int64_t(width);
  const int nmb = int((P + fms::kMaskBlockPix - 1) / fms::kMaskBlockPix);
  fr.dp = pad_dim(dim);
  fr.desc = fms::FrameDesc{emb, ps, cs, mask, P, dim, fr.dp};
  HIP_TRY(h->blk.ensure(size_t(nmb) * sizeof(int)));
  HIP_TRY(h->meta.ensure(META_COUNT * sizeof(int)));
  HIP_TRY(hipMemsetAsync(h->meta.p, 0, META_COUNT * sizeof(int), st));
  HIP_TRY(fms::launch_mask_count(st, mask, P, h->blk.as<int>(), nmb));
  HIP_TRY(fms::launch_scan_blocks(st, h->blk.as<int>(), nmb, h->meta.as<int>()));
  HIP_TRY(hipMemcpyAsync(h->hmeta, h->meta.p, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(h->wait(st));
  fr.n = h->hmeta[META_N];
  fr.n_pad = ((fr.n + fms::kBlockPix - 1) / fms::kBlockPix) * fms::kBlockPix;
  fr.geom = fms::make_geom(fr.n);
  if (fr.n == 0) return FMS_OK;
  const size_t rows = size_t(fr.n_pad);
  const size_t dp = size_t(fr.dp);
  HIP_TRY(h->fg_idx.ensure(rows * sizeof(int)));
  HIP_TRY(h->x32.ensure(rows * dp * sizeof(float)));
  HIP_TRY(h->x32t.ensure(rows * dp * sizeof(float)));
  if (bf16) {
    HIP_TRY(h->x16.ensure(rows * dp * sizeof(uint16_t)));
    HIP_TRY(h->x16t.ensure(rows * dp * sizeof(uint16_t)));
  }
  HIP_TRY(fms::launch_compact(st, fr.desc, h->blk.as<int>(), nmb, h->fg_idx.as<int>(), h->x32.as<float>(),
                              h->x32t.as<float>(), bf16 ? h->x16.as<uint16_t>() : nullptr,
                              bf16 ? h->x16t.as<uint16_t>() : nullptr, h->meta.as<int>()));
  // meta[META_BAD] counts zero or non-finite rows.  The caller checks it at
  // its next read of the counters (no kernel indexes by embedding values, so
  // the work enqueued meanwhile is merely wasted).
  return FMS_OK;
}

void set_tiling(Frame& fr, const fms_params* p) {
  const bool bf16 = p->precision == FMS_PREC_BF16_REFINE;
  fr.tile = fms::make_tiling(bf16, fr.dp, p->tile_seeds, p->tile_items, p->tile_chunks);
  fr.tile_fp32 = fms::make_tiling(false, fr.dp, p->tile_seeds, p->tile_items, p->tile_chunks);
  // A caller-fixed group size holds for every launch.
  const int big = p->tile_seeds > 0 ? p->tile_seeds : kBigGroup;
  fr.tile_big = fms::make_tiling(bf16, fr.dp, big, p->tile_items, p->tile_chunks);
  fr.tile_fp32_big = fms::make_tiling(false, fr.dp, big, p->tile_items, p->tile_chunks);
}

// Tiling of a fused-step launch with at most `bound` centres.
const fms::Tiling& pick_tiling(const Frame& fr, bool bf16, int bound) {
  if (bound >= kBigGroupMin) return bf16 ? fr.tile_big : fr.tile_fp32_big;
  return bf16 ? fr.tile : fr.tile_fp32;
}

fms_status ensure_round(fms_handle h, const Frame& fr, int m, bool bf16) {
  HIP_TRY(h->stage(size_t(std::max(m, 1)) * sizeof(int) + 256));
  const size_t mm = size_t(std::max(m, 1));
  const size_t dp = size_t(fr.dp);
  HIP_TRY(h->y.ensure(mm * dp * sizeof(float)));
  HIP_TRY(h->yc0.ensure(mm * dp * sizeof(float)));
  HIP_TRY(h->yc1.ensure(mm * dp * sizeof(float)));
  HIP_TRY(h->active.ensure(mm * sizeof(int)));
  HIP_TRY(h->next_active.ensure(mm * sizeof(int)));
  HIP_TRY(h->state.ensure(mm));
  HIP_TRY(h->iters.ensure(mm * sizeof(int)));
  HIP_TRY(h->seed_pos.ensure(mm * sizeof(int)));
  HIP_TRY(h->seed_fg.ensure(mm * sizeof(int)));
  HIP_TRY(h->ident.ensure(mm * sizeof(int)));
  HIP_TRY(h->cand.ensure(mm * sizeof(int)));
  HIP_TRY(h->counts.ensure(mm * sizeof(int)));
  HIP_TRY(h->sorted.ensure(mm * sizeof(int)));
  HIP_TRY(h->scount.ensure(mm * sizeof(int)));
  (void)bf16;
  const int im = int(mm);
  const size_t rows = std::max({fms::shift_partial_rows(fr.tile, im), fms::shift_partial_rows(fr.tile_fp32, im),
                                fms::shift_partial_rows(fr.tile_big, im), fms::shift_partial_rows(fr.tile_fp32_big, im)});
  HIP_TRY(h->pcount.ensure(rows * sizeof(int)));
  HIP_TRY(h->partial.ensure(rows * dp * sizeof(float)));
  return FMS_OK;
}

// Device transfer area of one pruning pass (counts, candidate x candidate
// bits, candidate x mode bits) and the host staging that receives it in one
// copy.  Sized before any copy is enqueued, never reallocated mid-flight.
struct Xfer {
  int* counts;
  uint32_t* bits_c;
  uint32_t* bits_m;
  int words_c, words_m;
  size_t bytes;
};

fms_status ensure_xfer(fms_handle h, int nc, int k, Xfer& x) {
  x.words_c = fms::simbits_words(nc);
  x.words_m = fms::simbits_words(k);
  const size_t nb_c = size_t(nc) * x.words_c * sizeof(uint32_t);
  const size_t nb_m = size_t(nc) * x.words_m * sizeof(uint32_t);
  const size_t nb_n = ((size_t(nc) * sizeof(int) + 255) / 256) * 256;
  x.bytes = nb_n + nb_c + nb_m;
  HIP_TRY(h->bits.ensure(x.bytes));
  HIP_TRY(h->stage(x.bytes + 256));
  uint8_t* base = static_cast<uint8_t*>(h->bits.p);
  x.counts = reinterpret_cast<int*>(base);
  x.bits_c = reinterpret_cast<uint32_t*>(base + nb_n);
  x.bits_m = reinterpret_cast<uint32_t*>(base + nb_n + nb_c);
  return FMS_OK;
}

// Host view of an Xfer after its copy.
struct XferHost {
  const int* counts;
  const uint32_t* bits_c;
  const uint32_t* bits_m;
};

XferHost xfer_host(fms_handle h, const Xfer& x, int nc) {
  const uint8_t* hb = static_cast<const uint8_t*>(h->hstage);
  const size_t nb_n = ((size_t(nc) * sizeof(int) + 255) / 256) * 256;
  const size_t nb_c = size_t(nc) * x.words_c * sizeof(uint32_t);
  return XferHost{reinterpret_cast<const int*>(hb), reinterpret_cast<const uint32_t*>(hb + nb_n),
                  reinterpret_cast<const uint32_t*>(hb + nb_n + nb_c)};
}

struct RoundOut {
  int steps = 0;
  int64_t updates = 0;
  int refine_steps = 0;
  int refine_bad = 0;
  int64_t refine_updates = 0;
  double step_ms[2] = {0.0, 0.0};
  int64_t step_updates[2] = {0, 0};
  int step_launches[2] = {0, 0};
  std::vector<int> conv;  // converged slots, ascending
};

void add_timing(fms_stats& sx, const RoundOut& ro) {
  for (int k = 0; k < 2; ++k) {
    sx.step_ms[k] += ro.step_ms[k];
    sx.step_updates[k] += ro.step_updates[k];
    sx.step_launches[k] += ro.step_launches[k];
  }
}

// Iterate the seeds whose centres are in y[0..m) (Alg. 2, the parallel seed
// loop) until more than gamma of them converged (Sec. 3.2.3), none is
// active, or max_iter steps.  With seed_fg the centres first load from those
// pixel rows.  The active count, the early-stop test and the done flag live
// on the device; the host enqueues iterations in batches and reads the flag
// back between batches.  The converged slots end up in out.conv (ascending)
// and in h->cand.
fms_status run_iterations_on(fms_handle h, hipStream_t st, const Frame& fr, float* ybuf, int cap,
                             const fms_params* p, float thr, float tol, RoundOut& out, bool host_list,
                             const int* seed_fg = nullptr) {
  const int m = cap;  // upper bound; the round's seed count is meta[META_NSEL]
  int* meta = h->meta.as<int>();
  unsigned long long* meta64 = h->meta64.as<unsigned long long>();
  const bool bf16 = p->precision == FMS_PREC_BF16_REFINE;
  const void* xrm = bf16 ? h->x16.p : h->x32.p;
  const void* xt = bf16 ? h->x16t.p : h->x32t.p;
  const int pk = bf16 ? 1 : 0;
  const bool timing = p->timing != 0;
  HIP_TRY(fms::launch_round_begin(st, m, h->active.as<int>(), h->state.as<uint8_t>(), h->iters.as<int>(), meta,
                                  meta64, seed_fg, h->x32.as<float>(), fr.dp, ybuf));
  int* lists[2] = {h->active.as<int>(), h->next_active.as<int>()};
  float* yc[2] = {h->yc0.as<float>(), h->yc1.as<float>()};
  // Iterations go out in batches; the host reads the counters back after
  // each batch and stops enqueueing at the early stop.  Launches queued past
  // the stop find the done flag and return at once.
  // Batch sizes: most rounds of the 512x512 workload stop within 3 to 9
  // iterations; 3, 6, 8 measured best among the schedules tried.
  static constexpr int kSched[] = {3, 6, 8};
  int t = 0, nbatch = 0;
  int bound = m;  // active centres of the next iteration, at most
  while (t < p->max_iter) {
    const int want_nb = kSched[std::min(nbatch, 2)];
    ++nbatch;
    const int nb = std::min(want_nb, p->max_iter - t);
    if (timing) HIP_TRY(h->ensure_events(2 * size_t(nb)));
    const fms::Tiling& tl = pick_tiling(fr, bf16, bound);
    for (int i = 0; i < nb; ++i, ++t) {
      const fms::IterCtl ctl{meta, meta64, -1, t, fr.n, p->gamma};
      // Iteration 0 reads the centres in place (the active list is the
      // identity); later iterations read the rows the previous reduce
      // compacted in active-list order.
      const float* yin = t == 0 ? ybuf : yc[t & 1];
      HIP_TRY(fms::launch_shift(st, bf16, fr.dp, tl, fr.geom.n_blocks, xrm, xt, yin, nullptr, ctl, m, thr,
                                h->partial.as<float>(), timing ? h->events[2 * i] : nullptr,
                                timing ? h->events[2 * i + 1] : nullptr));
      HIP_TRY(fms::launch_reduce(st, fr.dp, fr.geom.n_blocks, tl, h->partial.as<float>(), lists[t & 1], ybuf,
                                 h->state.as<uint8_t>(), h->iters.as<int>(), lists[(t + 1) & 1], yc[(t + 1) & 1],
                                 ctl, m, tol, 0));
    }
    HIP_TRY(hipMemcpyAsync(h->hmeta, meta, META_COUNT * sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(h->wait(st));
    if (timing) {
      for (int i = 0; i < nb; ++i) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, h->events[2 * i], h->events[2 * i + 1]));
        out.step_ms[pk] += ms;
        out.step_launches[pk] += 1;
      }
    }
    // The early stop of the next iteration, as its step kernel takes it.
    const int* hm = h->hmeta;
    bound = hm[fms::META_ACT + (t & 1)];
    if (hm[fms::META_DONE] || bound <= 0 || (double)hm[fms::META_NCONV] > p->gamma * (double)hm[fms::META_NSEL])
      break;
  }
  out.steps = h->hmeta[fms::META_STEPS];
  out.conv.clear();
  if (!host_list) return FMS_OK;  // the caller collects on the device and reads the counters later
  // Converged slots, in slot (= seed-order) order, and the update count.
  const int msel = h->hmeta[fms::META_NSEL];
  uint8_t* hs = static_cast<uint8_t*>(h->hstage);
  HIP_TRY(hipMemcpyAsync(hs, h->state.p, size_t(msel), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(hs + ((size_t(m) + 15) / 16) * 16, meta64, sizeof(unsigned long long),
                         hipMemcpyDeviceToHost, st));
  HIP_TRY(h->wait(st));
  unsigned long long upd = 0;
  std::memcpy(&upd, hs + ((size_t(m) + 15) / 16) * 16, sizeof(upd));
  out.updates = int64_t(upd);
  if (timing) out.step_updates[pk] += out.updates;
  for (int k = 0; k < msel; ++k)
    if (hs[k] == 1) out.conv.push_back(k);
  const int nc = int(out.conv.size());
  if (nc > 0) {
    std::memcpy(h->hstage, out.conv.data(), size_t(nc) * sizeof(int));
    HIP_TRY(hipMemcpyAsync(h->cand.p, h->hstage, size_t(nc) * sizeof(int), hipMemcpyHostToDevice, st));
    HIP_TRY(h->wait(st));
  }
  return FMS_OK;
}

fms_status run_iterations(fms_handle h, hipStream_t st, const Frame& fr, int m, const fms_params* p, float thr,
                          float tol, RoundOut& out, bool host_list, const int* seed_fg = nullptr) {
  return run_iterations_on(h, st, fr, h->y.as<float>(), m, p, thr, tol, out, host_list, seed_fg);
}

// FP32 refinement (BF16 form) of the `a` centres y[list[0..a)]: `steps`
// steps without freezing.  With `early_stop`, the centres then keep iterating
// with freezing under the early stop of Sec. 3.2.3 (until more than gamma of
// them have converged, or max_steps in total); out_keep receives, per centre,
// 1 when it converged and 0 when it was still moving and is dropped, like an
// unconverged seed.  Without it, the centres whose last step moved >= tol
// are counted.
fms_status run_refine(fms_handle h, hipStream_t st, const Frame& fr, float* y, const int* list, int a, int steps,
                      int max_steps, float thr, float tol, double gamma, bool early_stop, bool timing,
                      RoundOut& out, std::vector<uint8_t>* out_keep) {
  if (a <= 0 || steps <= 0) return FMS_OK;
  int* meta = h->meta.as<int>();
  const fms::Tiling& tl = pick_tiling(fr, false, a);
  h->hmeta[fms::META_NACC] = a;
  HIP_TRY(hipMemcpyAsync(meta + fms::META_NACC, h->hmeta + fms::META_NACC, sizeof(int), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemsetAsync(meta + fms::META_REFINE_BAD, 0, sizeof(int), st));
  if (timing) HIP_TRY(h->ensure_events(2 * size_t(steps)));
  for (int r = 0; r < steps; ++r) {
    const fms::IterCtl ctl{meta, nullptr, fms::META_NACC, -1, fr.n, 1.0};
    HIP_TRY(fms::launch_shift(st, false, fr.dp, tl, fr.geom.n_blocks, h->x32.p, h->x32t.p, y, list, ctl, a, thr,
                              h->partial.as<float>(), timing ? h->events[2 * r] : nullptr,
                              timing ? h->events[2 * r + 1] : nullptr));
    HIP_TRY(fms::launch_reduce(st, fr.dp, fr.geom.n_blocks, tl, h->partial.as<float>(), list, y,
                               h->state.as<uint8_t>(), h->iters.as<int>(), nullptr, nullptr, ctl, a, tol,
                               r + 1 == steps ? 2 : 1));
    out.refine_steps += 1;
    out.refine_updates += int64_t(a) * int64_t(fr.n);
  }
  HIP_TRY(hipMemcpyAsync(h->hmeta + fms::META_REFINE_BAD, meta + fms::META_REFINE_BAD, sizeof(int),
                         hipMemcpyDeviceToHost, st));
  HIP_TRY(h->wait(st));
  if (timing) {
    for (int r = 0; r < steps; ++r) {
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, h->events[2 * r], h->events[2 * r + 1]));
      out.step_ms[0] += ms;
      out.step_updates[0] += int64_t(a) * int64_t(fr.n);
      out.step_launches[0] += 1;
    }
  }
  const int moving = h->hmeta[fms::META_REFINE_BAD];
  if (!early_stop) {
    out.refine_bad += moving;
    return FMS_OK;
  }
  out_keep->assign(size_t(a), 1);
  if (moving == 0) return FMS_OK;
  // Continue with freezing; the list maps iteration slots to the centres.
  RoundOut ro;
  h->hmeta[fms::META_NSEL] = a;
  HIP_TRY(hipMemcpyAsync(meta + fms::META_NSEL, h->hmeta + fms::META_NSEL, sizeof(int), hipMemcpyHostToDevice, st));
  fms_params q{};
  q.gamma = gamma;
  q.max_iter = std::max(max_steps - steps, 1);
  q.precision = FMS_PREC_FP32;
  q.timing = timing ? 1 : 0;
  q.tile_seeds = tl.group_seeds;
  q.tile_items = tl.target_items;
  q.tile_chunks = tl.max_chunks;
  fms_status stt = run_iterations_on(h, st, fr, y, a, &q, thr, tol, ro, true);
  if (stt != FMS_OK) return stt;
  out.refine_steps += ro.steps;
  out.refine_updates += ro.updates;
  for (int k = 0; k < 2; ++k) {
    out.step_ms[k] += ro.step_ms[k];
    out.step_updates[k] += ro.step_updates[k];
    out.step_launches[k] += ro.step_launches[k];
  }
  std::fill(out_keep->begin(), out_keep->end(), uint8_t(0));
  for (int k : ro.conv) (*out_keep)[size_t(k)] = 1;
  out.refine_bad += a - int(ro.conv.size());
  return FMS_OK;
}

// Greedy pruning (Alg. 2): visit candidates in `order`, accept one when it is
// not within the window of an existing mode (a nonzero row of bits_m) and not
// within the window of a candidate accepted before it (bits_c).
std::vector<int> greedy_accept(const std::vector<int>& order, const XferHost& xh, const Xfer& x, bool have_modes) {
  std::vector<uint32_t> taken(size_t(std::max(x.words_c, 1)), 0u);
  std::vector<int> acc;
  for (int a : order) {
    if (have_modes) {
      const uint32_t* rm = xh.bits_m + size_t(a) * x.words_m;
      bool blocked = false;
      for (int w = 0; w < x.words_m && !blocked; ++w) blocked = rm[w] != 0;
      if (blocked) continue;
    }
    const uint32_t* row = xh.bits_c + size_t(a) * x.words_c;
    bool clash = false;
    for (int w = 0; w < x.words_c && !clash; ++w) clash = (row[w] & taken[w]) != 0;
    if (clash) continue;
    taken[a >> 5] |= 1u << (a & 31);
    acc.push_back(a);
  }
  return acc;
}

// Similarity bits of the nc centres y[list[..]] among themselves and against
// modes[0..k), with their window counts when `counts` is requested, copied to
// the host in one transfer.
fms_status prune_inputs(fms_handle h, hipStream_t st, const Frame& fr, const float* y, const int* list, int nc, int k,
                        float thr, bool with_counts, Xfer& x, XferHost& xh) {
  fms_status stt = ensure_xfer(h, nc, k, x);
  if (stt != FMS_OK) return stt;
  if (with_counts)
    HIP_TRY(fms::launch_count(st, false, fr.dp, pick_tiling(fr, false, nc), fr.geom.n_blocks, fr.n, h->x32.p, y,
                              list, nc, thr,
                              h->pcount.as<int>(), x.counts, nullptr, -1));
  HIP_TRY(fms::launch_simbits(st, fr.dp, y, list, nc, list, nullptr, nc, thr, x.bits_c, nullptr, -1, -1));
  if (k > 0)
    HIP_TRY(fms::launch_simbits(st, fr.dp, y, list, nc, nullptr, h->modes.as<float>(), k, thr, x.bits_m, nullptr, -1,
                                -1));
  HIP_TRY(hipMemcpyAsync(h->hstage, h->bits.p, x.bytes, hipMemcpyDeviceToHost, st));
  HIP_TRY(h->wait(st));
  xh = xfer_host(h, x, nc);
  return FMS_OK;
}

fms_status grow_modes(fms_handle h, hipStream_t st, const Frame& fr, int k_modes, int extra) {
  // The mode set persists across rounds: grow it without losing rows.
  HIP_TRY(h->modes.grow_keep(size_t(k_modes + extra) * fr.dp * sizeof(float), size_t(k_modes) * fr.dp * sizeof(float),
                             st));
  HIP_TRY(h->mode_counts.grow_keep(size_t(k_modes + extra) * sizeof(int), size_t(k_modes) * sizeof(int), st));
  return FMS_OK;
}

double tol_of(const fms_params* p) { return p->conv_tol > 0.0 ? p->conv_tol : p->bandwidth / 1000.0; }

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
  p->refine_iters = 3;
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
  if (hipHostMalloc(reinterpret_cast<void**>(&h->hmeta), (META_COUNT + 4) * sizeof(int), hipHostMallocDefault) !=
          hipSuccess ||
      hipEventCreateWithFlags(&h->sync_ev, hipEventDisableTiming) != hipSuccess ||

      h->meta.ensure(META_COUNT * sizeof(int)) != hipSuccess ||
      h->meta64.ensure(4 * sizeof(unsigned long long)) != hipSuccess) {
    fms_destroy(h);
    return FMS_ERR_HIP;
  }
  *out = h;
  return FMS_OK;
}

fms_status fms_destroy(fms_handle h) {
  if (!h) return FMS_OK;
  DeviceGuard guard(h->device);
  (void)hipDeviceSynchronize();
  DevBuf* bufs[] = {&h->blk,   &h->fg_idx, &h->x32,     &h->x32t,        &h->x16,     &h->x16t,     &h->order,
                    &h->rank, &h->elig, &h->y, &h->yc0, &h->yc1, &h->active, &h->next_active, &h->state, &h->iters,
                    &h->seed_pos, &h->seed_fg, &h->ident, &h->cand, &h->counts, &h->pcount, &h->partial,
                    &h->bits, &h->blocked, &h->acc, &h->sorted, &h->scount, &h->modes, &h->mode_counts, &h->meta, &h->meta64};
  for (DevBuf* b : bufs) b->release();
  for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
  if (h->hmeta) (void)hipHostFree(h->hmeta);
  if (h->sync_ev) (void)hipEventDestroy(h->sync_ev);
  if (h->hstage) (void)hipHostFree(h->hstage);
  delete h;
  return FMS_OK;
}

fms_status fms_seed_order(fms_handle h, void* stream, int32_t n, uint64_t seed, int32_t* order) {
  if (!h || n < 0 || (n > 0 && !order)) return FMS_ERR_INVALID_ARG;
  if (n == 0) return FMS_OK;
  DeviceGuard guard(h->device);
  uint64_t keys[4];
  round_keys(seed, keys);
  HIP_TRY(fms::launch_seed_order(static_cast<hipStream_t>(stream), n, half_bits(n), keys, order, nullptr));
  return FMS_OK;
}

fms_status fms_cluster(fms_handle h, void* stream, const float* emb, int64_t pixel_stride, int64_t channel_stride,
                       const uint8_t* mask, int32_t height, int32_t width, int32_t dim, const fms_params* p,
                       float* modes_out, int32_t* mode_counts_out, int32_t k_max, int32_t* n_modes, int32_t* labels,
                       fms_stats* stats) {
  fms_status stt = check_frame_args(h, emb, pixel_stride, channel_stride, height, width, dim);
  if (stt != FMS_OK) return stt;
  stt = check_params(p);
  if (stt != FMS_OK) return stt;
  if (!n_modes || !labels || k_max < 0 || (k_max > 0 && !modes_out)) return FMS_ERR_INVALID_ARG;
  DeviceGuard guard(h->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t P = int64_t(height) * int64_t(width);
  fms_stats sx;
  std::memset(&sx, 0, sizeof(sx));
  sx.n_min = std::numeric_limits<double>::quiet_NaN();
  int64_t n_seeds = p->n_state_in > 0 ? p->n_state_in : p->n_initial;

  Frame fr;
  stt = prepare_frame(h, st, emb, pixel_stride, channel_stride, mask, height, width, dim,
                      p->precision == FMS_PREC_BF16_REFINE, fr);
  if (stt != FMS_OK) return stt;
  set_tiling(fr, p);
  sx.n_fg = fr.n;
  HIP_TRY(fms::launch_fill_i32(st, labels, P, -1));
  if (fr.n == 0) {
    HIP_TRY(h->wait(st));
    *n_modes = 0;
    sx.n_state_out = int32_t(std::min<int64_t>(n_seeds, std::numeric_limits<int32_t>::max()));
    if (stats) *stats = sx;
    return FMS_OK;
  }
  const int n = fr.n;
  const float thr = float(1.0 - p->bandwidth);
  const float tol = float(tol_of(p));
  const double r = double(n) / double(P);
  int* meta = h->meta.as<int>();

  // Seed order, coverage and use flags.
  HIP_TRY(h->order.ensure(size_t(n) * sizeof(int)));
  HIP_TRY(h->rank.ensure(size_t(n) * sizeof(int)));
  const size_t elig_bytes = ((size_t(n) + 15) / 16) * 16 + 16;
  HIP_TRY(h->elig.ensure(elig_bytes));
  uint64_t keys[4];
  round_keys(p->seed, keys);
  HIP_TRY(fms::launch_seed_order(st, n, half_bits(n), keys, h->order.as<int>(), h->rank.as<int>(),
                                 h->elig.as<uint8_t>(), int(elig_bytes), meta));

  int64_t n_used = 0;
  int k_modes = 0;
  bool have_nmin = false;
  double nmin = 0.0;
  for (int round = 0; round < p->max_rounds; ++round) {
    const int64_t want64 = std::min<int64_t>(n_seeds - n_used, n);
    if (want64 <= 0) break;
    const int want = int(want64);
    stt = ensure_round(h, fr, want, p->precision == FMS_PREC_BF16_REFINE);
    if (stt != FMS_OK) return stt;
    const bool bf16 = p->precision == FMS_PREC_BF16_REFINE;
    // Room for every seed of the round to become a mode.
    stt = grow_modes(h, st, fr, k_modes, want);
    if (stt != FMS_OK) return stt;
    HIP_TRY(fms::launch_select(st, h->order.as<int>(), h->elig.as<uint8_t>(), n, want, meta, h->seed_pos.as<int>(),
                               h->seed_fg.as<int>()));
    RoundOut ro;
    const bool on_device = want <= fms::kRankMax;
    stt = run_iterations(h, st, fr, want, p, thr, tol, ro, !on_device, h->seed_fg.as<int>());
    if (stt != FMS_OK) return stt;
    if (h->hmeta[META_BAD] != 0) return FMS_ERR_BAD_INPUT;
    const int m = h->hmeta[META_NSEL];
    if (m == 0) break;
    n_used += m;
    sx.rounds += 1;
    sx.seeds_used += m;

    // Prune (Alg. 2): window counts at the converged endpoints, ranking by
    // count (descending) then seed position, greedy suppression against the
    // modes kept so far and the candidates accepted before.
    int accepted = 0;
    unsigned long long round_updates = 0;
    int round_ncand = 0;
    if (on_device) {
      Xfer x;
      stt = ensure_xfer(h, want, k_modes, x);
      if (stt != FMS_OK) return stt;
      HIP_TRY(fms::launch_collect(st, h->state.as<uint8_t>(), h->cand.as<int>(), meta));
      // Ranking counts in the precision of the iteration (the BF16 form
      // recounts its refined modes in FP32 at the end of the frame).
      HIP_TRY(fms::launch_count(st, bf16, fr.dp, pick_tiling(fr, bf16, want), fr.geom.n_blocks, fr.n,
                                bf16 ? h->x16.p : h->x32.p,
                                h->y.as<float>(), h->cand.as<int>(), m, thr, h->pcount.as<int>(), x.counts, meta,
                                fms::META_NCAND));
      HIP_TRY(fms::launch_rank(st, h->cand.as<int>(), x.counts, meta, h->sorted.as<int>(), h->scount.as<int>()));
      HIP_TRY(fms::launch_simbits(st, fr.dp, h->y.as<float>(), h->sorted.as<int>(), want, h->sorted.as<int>(), nullptr,
                                  want, thr, x.bits_c, meta, fms::META_NCAND, fms::META_NCAND));
      if (k_modes > 0)
        HIP_TRY(fms::launch_simbits(st, fr.dp, h->y.as<float>(), h->sorted.as<int>(), want, nullptr,
                                    h->modes.as<float>(), k_modes, thr, x.bits_m, meta, fms::META_NCAND, -1));
      HIP_TRY(fms::launch_greedy(st, x.bits_c, x.words_c, x.bits_m, x.words_m, k_modes, h->y.as<float>(),
                                 h->sorted.as<int>(), h->scount.as<int>(), meta, fms::META_NCAND, fms::META_NACC,
                                 fr.dp, h->modes.as<float>(), h->mode_counts.as<int>()));
    } else {
      const int nc = int(ro.conv.size());
      if (nc > 0) {
        Xfer x;
        XferHost xh;
        stt = prune_inputs(h, st, fr, h->y.as<float>(), h->cand.as<int>(), nc, k_modes, thr, true, x, xh);
        if (stt != FMS_OK) return stt;
        std::vector<int> ord(nc);
        for (int a = 0; a < nc; ++a) ord[a] = a;
        std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return xh.counts[a] > xh.counts[b]; });
        std::vector<int> acc = greedy_accept(ord, xh, x, k_modes > 0);
        accepted = int(acc.size());
        if (accepted > 0) {
          HIP_TRY(h->acc.ensure(size_t(accepted) * sizeof(int)));
          int* hacc = reinterpret_cast<int*>(h->hstage);  // staging is free again after the sync above
          for (int q = 0; q < accepted; ++q) hacc[q] = acc[q];
          HIP_TRY(hipMemcpyAsync(h->acc.p, hacc, size_t(accepted) * sizeof(int), hipMemcpyHostToDevice, st));
          HIP_TRY(fms::launch_append_modes(st, fr.dp, h->y.as<float>(), h->cand.as<int>(), x.counts,
                                           h->acc.as<int>(), accepted, h->modes.as<float>(), h->mode_counts.as<int>(),
                                           k_modes));
          HIP_TRY(h->wait(st));
        }
      }
    }
    const bool acc_on_device = on_device;
    // Coverage by the new modes, and the pool left to seed; then one read of
    // the round's counters.
    HIP_TRY(fms::launch_assign(st, fr.dp, h->x32.as<float>(), n, h->modes.as<float>(), k_modes,
                               k_modes + (acc_on_device ? want : accepted), acc_on_device ? fms::META_NACC : -1, thr,
                               0, h->elig.as<uint8_t>(), h->rank.as<int>(), meta, nullptr, nullptr));
    HIP_TRY(hipMemcpyAsync(h->hmeta, meta, META_COUNT * sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(h->hmeta + META_COUNT, h->meta64.p, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                           st));
    HIP_TRY(h->wait(st));
    if (acc_on_device) accepted = h->hmeta[fms::META_NACC];
    if (on_device) {
      std::memcpy(&round_updates, h->hmeta + META_COUNT, sizeof(round_updates));
      round_ncand = h->hmeta[fms::META_NCAND];
      ro.updates = int64_t(round_updates);
      if (p->timing) ro.step_updates[bf16 ? 1 : 0] += ro.updates;
      sx.n_discarded += m - round_ncand;
    } else {
      sx.n_discarded += m - int(ro.conv.size());
    }
    sx.iterations_total += ro.steps;
    sx.refine_steps += ro.refine_steps;
    sx.seed_pixel_updates += ro.updates;
    sx.refine_unconverged += ro.refine_bad;
    sx.refine_updates += ro.refine_updates;
    add_timing(sx, ro);
    k_modes += accepted;
    const bool left = h->hmeta[META_LEFT] > 0;
    // Controller (Sec. 3.2.4).
    bool go_on = false;
    have_nmin = eq19_n_min(p->p_target, k_modes, r, &nmin);
    if (left) {
      if (!have_nmin || double(n_seeds) < p->big_l * nmin) {
        n_seeds *= 2;
        go_on = true;
      }
    }
    if (!go_on) break;
  }

  if (p->precision == FMS_PREC_BF16_REFINE && k_modes > 0 && p->refine_iters > 0) {
    // BF16 form: the frame's modes are refined in FP32 (refine_iters steps,
    // then FP32 iteration under the early stop; modes still moving at the
    // stop are dropped), recounted, and a mode that now falls inside the
    // window of an earlier kept mode is dropped (acceptance order decides).
    stt = ensure_round(h, fr, k_modes, true);
    if (stt != FMS_OK) return stt;
    RoundOut ro;
    float* mrows = h->modes.as<float>();
    HIP_TRY(fms::launch_iota(st, h->ident.as<int>(), k_modes));
    std::vector<uint8_t> settled;
    stt = run_refine(h, st, fr, mrows, h->ident.as<int>(), k_modes, p->refine_iters, p->max_iter, thr, tol, p->gamma,
                     true, p->timing != 0, ro, &settled);
    if (stt != FMS_OK) return stt;
    HIP_TRY(fms::launch_iota(st, h->ident.as<int>(), k_modes));
    Xfer x;
    XferHost xh;
    stt = prune_inputs(h, st, fr, mrows, h->ident.as<int>(), k_modes, 0, thr, true, x, xh);
    if (stt != FMS_OK) return stt;
    std::vector<int> ord;
    for (int a = 0; a < k_modes; ++a)
      if (settled[size_t(a)]) ord.push_back(a);
    std::vector<int> keep = greedy_accept(ord, xh, x, false);
    // Rewrite the rows through the (now free) centre buffer, keeping only the
    // survivors, with their recounted windows.
    HIP_TRY(fms::launch_copy_rows(st, mrows, fr.dp, h->y.as<float>(), fr.dp, k_modes, fr.dp));
    HIP_TRY(h->acc.ensure(size_t(k_modes) * sizeof(int)));
    int* hk = reinterpret_cast<int*>(h->hstage);
    for (size_t q = 0; q < keep.size(); ++q) hk[q] = keep[q];
    if (!keep.empty())
      HIP_TRY(hipMemcpyAsync(h->acc.p, hk, keep.size() * sizeof(int), hipMemcpyHostToDevice, st));
    HIP_TRY(fms::launch_append_modes(st, fr.dp, h->y.as<float>(), h->ident.as<int>(), x.counts, h->acc.as<int>(),
                                     int(keep.size()), mrows, h->mode_counts.as<int>(), 0));
    HIP_TRY(h->wait(st));
    sx.refine_merged += int(ord.size()) - int(keep.size());
    sx.refine_steps += ro.refine_steps;
    sx.refine_unconverged += ro.refine_bad;
    sx.refine_updates += ro.refine_updates;
    add_timing(sx, ro);
    k_modes = int(keep.size());
  }

  // Labels (Alg. 2): most similar mode, lowest index on ties; count pixels
  // farther than h from every mode.
  HIP_TRY(hipMemsetAsync(meta + META_LEFT, 0, sizeof(int), st));
  HIP_TRY(fms::launch_assign(st, fr.dp, h->x32.as<float>(), n, h->modes.as<float>(), 0, k_modes, -1, thr, 1, nullptr,
                             nullptr, meta, h->fg_idx.as<int>(), labels));
  HIP_TRY(hipMemcpyAsync(h->hmeta + META_LEFT, meta + META_LEFT, sizeof(int), hipMemcpyDeviceToHost, st));
  if (k_modes > k_max) {
    HIP_TRY(h->wait(st));
    *n_modes = k_modes;
    return FMS_ERR_CAPACITY;
  }
  HIP_TRY(fms::launch_copy_rows(st, h->modes.as<float>(), fr.dp, modes_out, dim, k_modes, dim));
  if (mode_counts_out && k_modes > 0)
    HIP_TRY(hipMemcpyAsync(mode_counts_out, h->mode_counts.p, size_t(k_modes) * sizeof(int), hipMemcpyDeviceToDevice,
                           st));
  HIP_TRY(h->wait(st));
  *n_modes = k_modes;
  sx.n_uncovered = h->hmeta[META_LEFT];
  sx.n_min = have_nmin ? nmin : std::numeric_limits<double>::quiet_NaN();
  int64_t next = n_seeds;
  if (have_nmin && double(n_seeds) > p->big_h * nmin) next = n_seeds - int64_t(std::ceil(nmin));
  sx.n_state_out = int32_t(std::min<int64_t>(next, std::numeric_limits<int32_t>::max()));
  if (stats) *stats = sx;
  return FMS_OK;
}

fms_status fms_shift_seeds(fms_handle h, void* stream, const float* emb, int64_t pixel_stride, int64_t channel_stride,
                           const uint8_t* mask, int32_t height, int32_t width, int32_t dim, const int32_t* seed_fg,
                           int32_t n_seeds, const fms_params* p, float* endpoints, int32_t* iters, uint8_t* converged,
                           int32_t* counts, fms_stats* stats) {
  fms_status stt = check_frame_args(h, emb, pixel_stride, channel_stride, height, width, dim);
  if (stt != FMS_OK) return stt;
  stt = check_params(p);
  if (stt != FMS_OK) return stt;
  if (n_seeds < 0 || (n_seeds > 0 && (!seed_fg || !endpoints || !iters || !converged))) return FMS_ERR_INVALID_ARG;
  DeviceGuard guard(h->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  fms_stats sx;
  std::memset(&sx, 0, sizeof(sx));
  sx.n_min = std::numeric_limits<double>::quiet_NaN();
  Frame fr;
  stt = prepare_frame(h, st, emb, pixel_stride, channel_stride, mask, height, width, dim,
                      p->precision == FMS_PREC_BF16_REFINE, fr);
  if (stt != FMS_OK) return stt;
  set_tiling(fr, p);
  sx.n_fg = fr.n;
  if (n_seeds == 0) {
    if (stats) *stats = sx;
    return FMS_OK;
  }
  if (fr.n == 0) return FMS_ERR_INVALID_ARG;
  const int m = n_seeds;
  stt = ensure_round(h, fr, m, p->precision == FMS_PREC_BF16_REFINE);
  if (stt != FMS_OK) return stt;
  int* meta = h->meta.as<int>();
  HIP_TRY(hipMemsetAsync(meta + META_BADSEED, 0, sizeof(int), st));
  HIP_TRY(fms::launch_init_seeds(st, seed_fg, m, fr.n, h->x32.as<float>(), fr.dp, h->y.as<float>(), meta));
  HIP_TRY(hipMemcpyAsync(h->hmeta, meta, META_COUNT * sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(h->wait(st));
  if (h->hmeta[META_BAD] != 0) return FMS_ERR_BAD_INPUT;
  if (h->hmeta[META_BADSEED] != 0) return FMS_ERR_INVALID_ARG;
  const float thr = float(1.0 - p->bandwidth);
  const float tol = float(tol_of(p));
  RoundOut ro;
  h->hmeta[META_NSEL] = m;
  HIP_TRY(hipMemcpyAsync(meta + META_NSEL, h->hmeta + META_NSEL, sizeof(int), hipMemcpyHostToDevice, st));
  stt = run_iterations(h, st, fr, m, p, thr, tol, ro, true);
  if (stt != FMS_OK) return stt;
  if (p->precision == FMS_PREC_BF16_REFINE && !ro.conv.empty()) {
    stt = run_refine(h, st, fr, h->y.as<float>(), h->cand.as<int>(), int(ro.conv.size()), p->refine_iters,
                     p->refine_iters, thr, tol, p->gamma, false, p->timing != 0, ro, nullptr);
    if (stt != FMS_OK) return stt;
  }
  // Window counts of every slot (the output keeps them for converged seeds).
  HIP_TRY(fms::launch_iota(st, h->ident.as<int>(), m));
  HIP_TRY(fms::launch_count(st, false, fr.dp, pick_tiling(fr, false, m), fr.geom.n_blocks, fr.n, h->x32.p,
                            h->y.as<float>(),
                            h->ident.as<int>(), m, thr, h->pcount.as<int>(), h->counts.as<int>(), nullptr, -1));
  HIP_TRY(fms::launch_lockstep_out(st, m, fr.dp, dim, h->y.as<float>(), h->state.as<uint8_t>(), h->iters.as<int>(),
                                   h->counts.as<int>(), endpoints, iters, converged, counts));
  HIP_TRY(h->wait(st));
  sx.iterations_total = ro.steps;
  sx.refine_steps = ro.refine_steps;
  sx.seed_pixel_updates = ro.updates;
  sx.refine_unconverged = ro.refine_bad;
  sx.refine_updates = ro.refine_updates;
  add_timing(sx, ro);
  sx.seeds_used = m;
  sx.n_discarded = m - int(ro.conv.size());
  if (stats) *stats = sx;
  return FMS_OK;
}

}  // extern "C"
