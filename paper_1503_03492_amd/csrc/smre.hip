// smre.hip -- host side of the SMRE projection library (C ABI in include/smre.h).
//
// Full Dykstra (Sec. 2.3, Algorithm 2): plan the region grid and the
// increment stream, then enqueue sweeps of four region-phase launches (one
// per region colour).  Every check_every sweeps a snapshot kernel, the sweep,
// and a delta kernel measure max |x - x_prev| in FP64; a one-thread kernel
// raises a device flag once it falls below tol, and every later kernel exits
// at once, so the host can enqueue ahead and read the flag a few sweeps late
// without changing the result.
//
// Incomplete Dykstra (Sec. 3.2, ICD handler and kernel listings): one launch
// per phase i = 0..num_phases-1, one wave per block of side 2^K.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <optional>
#include <string>
#include <vector>

#include "icd.hpp"
#include "checks.hpp"
#include "kernels.hpp"
#include "mc.hpp"
#include "canon.hpp"
#include "icd_nested.hpp"
#include "admm.hpp"
#include "serve_core.hpp"
#include "smre.h"

using namespace smre;

namespace {

#define HIP_OK(expr)                                      \
  do {                                                    \
    hipError_t e_ = (expr);                               \
    if (e_ != hipSuccess) {                               \
      if (getenv("SMRE_LOG"))                             \
        fprintf(stderr, "smre: %s -> %s\n", #expr, hipGetErrorString(e_)); \
      return SMRE_EDEVICE;                                \
    }                                                     \
  } while (0)

constexpr int kTimingPairs = 256;

}  // namespace

struct smre_ctx {
  int device = 0;
  void* ws = nullptr;  // cached workspace
  size_t ws_bytes = 0;
  Ctrl* ctrl = nullptr;       // device control block
  Ctrl* ctrl_host = nullptr;  // pinned mirror ring
  int* counter = nullptr;     // device int (ICD inner sweeps)
  unsigned icd_epoch = 0;     // number of the last ICD call (its non-finite flag value)
  int timing = 0;
  hipEvent_t ev[2 * kTimingPairs] = {};
  int ev_used = 0;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  std::vector<hipEvent_t> lag_ev;
  int* counters_host = nullptr;      // pinned ring of batch counters
  hipStream_t capture = nullptr;     // private stream for graph capture
  std::map<std::string, int> tuned;  // autotuned region side per batch key
  int cus = 0;
  unsigned long long* icd_cnt = nullptr;  // ICD work counters (kIcdSlots lines)
  unsigned long long* mc_tmax = nullptr;  // Monte-Carlo per-(field, side) maxima
  double* mc_q = nullptr;                 // Monte-Carlo statistic per field
  void* admm_ws = nullptr;                // ADMM working images
  size_t admm_bytes = 0;
  double* admm_slots = nullptr;           // ADMM norm partials (2 x kAdmmSlots lines)
};

namespace {

constexpr int kLag = 4;  // host reads the converged flag this many checks late

int set_device(smre_ctx* c) {
  HIP_OK(hipSetDevice(c->device));
  return SMRE_OK;
}

// ---------------------------------------------------------------- timing
struct TimingAcc {
  double ms = 0.0;
  int64_t launches = 0;
  int64_t seen = 0;         // launches offered for timing (every k-th is timed)
  std::deque<int> pending;  // event pair indices in flight
};

int timing_flush(smre_ctx* c, TimingAcc& acc, bool all) {
  while (!acc.pending.empty() && (all || (int)acc.pending.size() >= kTimingPairs)) {
    const int k = acc.pending.front();
    acc.pending.pop_front();
    HIP_OK(hipEventSynchronize(c->ev[2 * k + 1]));
    float ms = 0.f;
    HIP_OK(hipEventElapsedTime(&ms, c->ev[2 * k], c->ev[2 * k + 1]));
    acc.ms += ms;
    acc.launches += 1;
  }
  return SMRE_OK;
}

int timing_begin(smre_ctx* c, TimingAcc& acc, hipStream_t s, int* slot) {
  *slot = -1;
  if (!c->timing) return SMRE_OK;
  if (c->timing > 1 && acc.seen++ % c->timing != 0) return SMRE_OK;  // not sampled
  if ((int)acc.pending.size() >= kTimingPairs) {
    int rc = timing_flush(c, acc, false);
    if (rc) return rc;
  }
  const int k = c->ev_used;
  c->ev_used = (c->ev_used + 1) % kTimingPairs;
  HIP_OK(hipEventRecord(c->ev[2 * k], s));
  *slot = k;
  return SMRE_OK;
}

int timing_end(smre_ctx* c, TimingAcc& acc, hipStream_t s, int slot) {
  if (slot < 0) return SMRE_OK;
  HIP_OK(hipEventRecord(c->ev[2 * slot + 1], s));
  acc.pending.push_back(slot);
  return SMRE_OK;
}

// ---------------------------------------------------------------- planning
constexpr int kSigWords = 8;
struct Plan {
  int R = 16;
  int SI = 17;  // largest side of the sweep kernel instance (its LDS footprint)
  int nsides = 0;
  int sides[kMaxSides];
  double r2[kMaxSides];
  int smax = 0;
  int nry = 0, nrx = 0;
  int64_t nq = 0;  // increment elements
  int64_t nwin = 0;
  size_t qbytes = 0;
  size_t off_roff = 0, off_prev = 0, off_isum = 0, off_sig = 0, total = 0;
  std::vector<RegionStream> roff;  // page layout of each region's increments
  // device metadata blob: the region streams, then (16-byte aligned) the round
  // tables; meta_bytes covers both whether or not the blob is built
  std::vector<unsigned char> meta;
  size_t meta_rtab = 0, meta_bytes = 0;
};

// Sweep kernel instances: region side R with largest side R + 1, and R = 16
// with largest side 9 (a smaller LDS footprint, so more workgroups per CU,
// for images whose sides are all at most 9).  The instance changes where a
// region's pixels sit in LDS, not the arithmetic.
int instance_smax(int R, int smax) { return (R == 16 && smax <= 9) ? 9 : R + 1; }

// Footprint pitch of the instance (R, SI).
int footprint_pitch(int R, int SI) {
  switch (R) {
    case 8: return PhaseShape<float, float, 8, 9>::P;
    case 16: return SI == 9 ? PhaseShape<float, float, 16, 9>::P : PhaseShape<float, float, 16, 17>::P;
    case 32: return PhaseShape<float, float, 32, 33>::P;
    default: return 0;
  }
}

// Round tables of one image (layout in kernels.hpp): for every side and
// border class, the rounds of the region visiting order -- tiling offsets
// (a', b') raster, then blocks of BR x BC windows of that offset -- with each
// round's pixel offset in the footprint, its window counts and the end of its
// increment bytes.  Border classes: regions in the last row / column of
// regions (class 2) and the one before (class 1) may hold fewer anchors.
void build_round_tables(const Plan& pl, int64_t H, int64_t W, size_t es, RoundEntry* out) {
  const int R = pl.R, P = footprint_pitch(R, pl.SI), TL = round_table_len(R);
  for (int k = 0; k < pl.nsides; ++k) {
    const int S = pl.sides[k];
    const Pattern pt = pattern(R, S);
    for (int crow = 0; crow < 3; ++crow)
      for (int ccol = 0; ccol < 3; ++ccol) {
        auto extent = [&](int cls, int64_t n, int nreg) -> int {
          const int64_t o = cls == 0 ? 0 : (int64_t)(nreg - (cls == 1 ? 2 : 1)) * R;
          if (o < 0) return 0;
          return (int)std::max<int64_t>(0, std::min<int64_t>(R, n - S + 1 - o));
        };
        const int rhi = extent(crow, H, pl.nry), chi = extent(ccol, W, pl.nrx);
        RoundEntry* t = out + ((size_t)k * 9 + crow * 3 + ccol) * TL;
        uint32_t cnt = 0, rb = 0;
        for (int ap = 0; ap < std::min(S, rhi); ++ap) {
          const int nr = (rhi - ap + S - 1) / S;
          for (int bp = 0; bp < std::min(S, chi); ++bp) {
            const int nc = (chi - bp + S - 1) / S;
            for (int rby = 0; rby < nr; rby += pt.br) {
              const int nbr = std::min(pt.br, nr - rby);
              for (int rbx = 0; rbx < nc; rbx += pt.bc) {
                const int nbc = std::min(pt.bc, nc - rbx);
                const uint32_t xo = (uint32_t)((ap + S * rby) * P + (bp + S * rbx));
                rb += (uint32_t)(nbr * nbc * S * S * (int)es);
                const bool one = pt.br == 1 && pt.bc == 1;  // counts implied
                t[2 + cnt] =
                    RoundEntry{one ? xo : (xo | ((uint32_t)nbc << 16) | ((uint32_t)nbr << 20)), rb};
                ++cnt;
              }
            }
          }
        }
        t[0] = RoundEntry{cnt, 0};
        t[1] = RoundEntry{0, 0};
      }
  }
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int choose_region(int smax, int requested) {
  if (requested) return requested;
  if (smax <= 17) return 16;
  return 32;
}

int plan_project(smre_dtype dt, int64_t H, int64_t W, const smre_params* p, Plan* pl,
                 bool need_offsets, int si_force = 0) {
  if (!p || !p->sides || !p->radius2) return SMRE_EINVAL;
  if (dt != SMRE_F32 && dt != SMRE_F64) return SMRE_EINVAL;
  if (H < 1 || W < 1 || H > (1 << 20) || W > (1 << 20)) return SMRE_EINVAL;
  if (p->n_sides < 1 || p->n_sides > kMaxSides) return SMRE_EINVAL;
  if (p->max_sweeps < 1 || p->check_every < 1) return SMRE_EINVAL;
  if (p->inc != SMRE_INC_SAME && p->inc != SMRE_INC_BF16) return SMRE_EINVAL;
  if (p->inc == SMRE_INC_BF16 && dt != SMRE_F32) return SMRE_EINVAL;
  if (p->warm != 0 && p->warm != 1) return SMRE_EINVAL;
  if (p->order < SMRE_ORDER_REGION || p->order > SMRE_ORDER_ASC) return SMRE_EINVAL;
  if (!std::isfinite(p->tol) || !std::isfinite(p->guard_rel) || p->guard_rel < 0)
    return SMRE_EINVAL;
  std::vector<std::pair<int, double>> sd;
  for (int k = 0; k < p->n_sides; ++k) {
    const int s = p->sides[k];
    const double r = p->radius2[k];
    if (s < 1 || s > 32 || s > H || s > W) return SMRE_EINVAL;
    if (!std::isfinite(r)) return SMRE_ENONFINITE;
    if (!(r > 0)) return SMRE_EINVAL;
    sd.push_back({s, r});
  }
  std::sort(sd.begin(), sd.end(), [](auto& a, auto& b) { return a.first > b.first; });
  for (size_t k = 1; k < sd.size(); ++k)
    if (sd[k].first == sd[k - 1].first) return SMRE_EINVAL;
  pl->nsides = (int)sd.size();
  for (int k = 0; k < pl->nsides; ++k) {
    pl->sides[k] = sd[k].first;
    pl->r2[k] = sd[k].second;
  }
  pl->smax = pl->sides[0];
  pl->R = choose_region(pl->smax, p->region);
  if (pl->R != 8 && pl->R != 16 && pl->R != 32) return SMRE_EINVAL;
  if (pl->R < pl->smax - 1) return SMRE_EINVAL;
  // kernel instance: the caller's (a batch or server shares one), else the
  // smallest that holds the sides
  pl->SI = si_force ? si_force : instance_smax(pl->R, pl->smax);
  if (pl->SI < pl->smax || (pl->SI != pl->R + 1 && !(pl->R == 16 && pl->SI == 9)))
    return SMRE_EINVAL;
  pl->nry = (int)((H + pl->R - 1) / pl->R);
  pl->nrx = (int)((W + pl->R - 1) / pl->R);
  const size_t es = (p->inc == SMRE_INC_BF16) ? 2 : (dt == SMRE_F64 ? 8 : 4);
  const size_t xs = dt == SMRE_F64 ? 8 : 4;
  // increments per region: each side s contributes s^2 per anchor in the
  // region.  A region's increments occupy whole 1 KiB pages (so the kernel
  // writes pages back without touching another region's); the pages of the
  // regions of one colour are interleaved -- page p of the colour's b-th region
  // (in launch order) at segment_base + p * (regions of the colour) + b -- so
  // the workgroups of a launch stream one contiguous window of HBM.
  const int nreg = pl->nry * pl->nrx;
  std::vector<int32_t> npg((size_t)nreg, 0);
  int64_t nq = 0, nwin = 0, maxpg[4] = {0, 0, 0, 0}, nb[4] = {0, 0, 0, 0};
  for (int ry = 0; ry < pl->nry; ++ry)
    for (int rx = 0; rx < pl->nrx; ++rx) {
      int64_t cnt = 0;
      for (int k = 0; k < pl->nsides; ++k) {
        const int64_t s = pl->sides[k];
        const int64_t ar = std::max<int64_t>(0, std::min<int64_t>((int64_t)ry * pl->R + pl->R, H - s + 1) - (int64_t)ry * pl->R);
        const int64_t ac = std::max<int64_t>(0, std::min<int64_t>((int64_t)rx * pl->R + pl->R, W - s + 1) - (int64_t)rx * pl->R);
        cnt += s * s * ar * ac;
        nwin += ar * ac;
      }
      nq += cnt;
      const int col = (ry & 1) * 2 + (rx & 1);
      npg[(size_t)ry * pl->nrx + rx] = (int32_t)((cnt * (int64_t)es + kPage - 1) / kPage);
      maxpg[col] = std::max<int64_t>(maxpg[col], npg[(size_t)ry * pl->nrx + rx]);
      nb[col]++;
    }
  int64_t seg[4], pages = 0;
  for (int col = 0; col < 4; ++col) {
    seg[col] = pages;
    pages += maxpg[col] * nb[col];
  }
  if (pages >= (int64_t)1 << 31) return SMRE_ETOOBIG;
  if (need_offsets) {
    pl->roff.assign((size_t)nreg, RegionStream{0, 0, 0, 0});
    for (int ry = 0; ry < pl->nry; ++ry)
      for (int rx = 0; rx < pl->nrx; ++rx) {
        const int cy = ry & 1, cx = rx & 1, col = cy * 2 + cx;
        const int ncx = (pl->nrx - cx + 1) / 2;
        const int64_t b = (int64_t)(ry >> 1) * ncx + (rx >> 1);
        RegionStream& r = pl->roff[(size_t)ry * pl->nrx + rx];
        r.first = (int32_t)(seg[col] + b);
        r.npages = npg[(size_t)ry * pl->nrx + rx];
        r.stride = (int32_t)nb[col];
      }
  }
  pl->nq = nq;
  pl->nwin = nwin;
  pl->qbytes = (size_t)(pages + 1) * kPage;
  pl->meta_rtab = align_up((size_t)nreg * sizeof(RegionStream), 256);
  pl->meta_bytes =
      pl->meta_rtab + (size_t)pl->nsides * 9 * round_table_len(pl->R) * sizeof(RoundEntry);
  if (need_offsets) {
    pl->meta.assign(pl->meta_bytes, 0);
    std::memcpy(pl->meta.data(), pl->roff.data(), (size_t)nreg * sizeof(RegionStream));
    build_round_tables(*pl, H, W, es, (RoundEntry*)(pl->meta.data() + pl->meta_rtab));
  }
  pl->off_roff = pl->qbytes;
  pl->off_prev = align_up(pl->off_roff + pl->meta_bytes, 256);
  pl->off_isum = align_up(pl->off_prev + (size_t)H * W * xs, 256);
  pl->off_sig = align_up(pl->off_isum + (size_t)H * W * xs, 256);
  pl->total = align_up(pl->off_sig + kSigWords * sizeof(uint64_t), 256);
  return SMRE_OK;
}

// What a workspace's increments belong to: written at the end of a solve,
// cleared at the start of a cold one; a warm start requires a match.
void problem_signature(smre_dtype dt, int64_t H, int64_t W, const smre_params* p,
                       const Plan& pl, uint64_t* sig) {
  uint64_t h = 1469598103934665603ull;  // FNV-1a over the sorted sides and bounds
  auto mix = [&](const void* b, size_t n) {
    for (size_t i = 0; i < n; ++i) h = (h ^ ((const unsigned char*)b)[i]) * 1099511628211ull;
  };
  mix(pl.sides, sizeof(int) * pl.nsides);
  mix(pl.r2, sizeof(double) * pl.nsides);
  sig[0] = 0x534d524557524d31ull;
  sig[1] = (uint64_t)dt | ((uint64_t)p->inc << 8) | ((uint64_t)pl.R << 16);
  sig[2] = (uint64_t)H;
  sig[3] = (uint64_t)W;
  sig[4] = h;
  sig[5] = (uint64_t)pl.nq;
  sig[6] = (uint64_t)pl.qbytes;
  sig[7] = 0;
}

int ensure_ctrl(smre_ctx* c) {
  if (!c->ctrl) {
    HIP_OK(hipMalloc(&c->ctrl, sizeof(Ctrl)));
    hipLaunchKernelGGL(ctrl_init_kernel, dim3(1), dim3(1), 0, 0, c->ctrl);  // defined contents
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(0));
    HIP_OK(hipHostMalloc(&c->ctrl_host, sizeof(Ctrl) * (kLag + 2), hipHostMallocDefault));
    HIP_OK(hipMalloc(&c->counter, 64));
    c->lag_ev.resize(kLag + 2);
    for (auto& e : c->lag_ev) HIP_OK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    for (int k = 0; k < 2 * kTimingPairs; ++k) HIP_OK(hipEventCreate(&c->ev[k]));
    HIP_OK(hipEventCreate(&c->t0));
    HIP_OK(hipEventCreate(&c->t1));
    HIP_OK(hipHostMalloc(&c->counters_host, sizeof(int) * 2 * (kLag + 2), hipHostMallocDefault));
    HIP_OK(hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking));
    hipDeviceProp_t prop;
    HIP_OK(hipGetDeviceProperties(&prop, c->device));
    c->cus = prop.multiProcessorCount;
  }
  return SMRE_OK;
}

int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(8192, (n + 255) / 256)); }
int grid_rows(int64_t H) { return (int)std::max<int64_t>(1, std::min<int64_t>(4096, H)); }

// One colour of one image: grid = regions of that colour.
struct PhaseLaunch {
  int cy, cx, ncx, blocks;
  const int* done;
  int* abort;  // raised by a region job whose producer/consumer wait gave up
  unsigned char* q;
};

template <typename TX, typename TQ, int R, int SMAX, bool KAHAN>
void launch_phase(const ImageDesc& a, const PhaseLaunch& l, hipStream_t s) {
  hipLaunchKernelGGL((region_phase<TX, TQ, R, SMAX, KAHAN>), dim3(l.blocks), dim3(128), 0, s, a,
                     l.cy, l.cx, l.ncx, l.done, l.abort, l.q);
}

template <typename TX, typename TQ, bool KAHAN>
int launch_phase_r(int R, int SI, const ImageDesc& a, const PhaseLaunch& l, hipStream_t s) {
  switch (R) {
    case 8: launch_phase<TX, TQ, 8, 9, KAHAN>(a, l, s); break;
    case 16:
      if (SI == 9) launch_phase<TX, TQ, 16, 9, KAHAN>(a, l, s);
      else launch_phase<TX, TQ, 16, 17, KAHAN>(a, l, s);
      break;
    case 32: launch_phase<TX, TQ, 32, 33, KAHAN>(a, l, s); break;
    default: return SMRE_EINVAL;
  }
  HIP_OK(hipGetLastError());
  return SMRE_OK;
}

int launch_phase_any(smre_dtype dt, int inc, int kahan, int R, int SI, const ImageDesc& a,
                     const PhaseLaunch& l, hipStream_t s) {
  if (dt == SMRE_F64) return launch_phase_r<double, double, false>(R, SI, a, l, s);
  if (inc == SMRE_INC_BF16)
    return kahan ? launch_phase_r<float, bf16_t, true>(R, SI, a, l, s)
                 : launch_phase_r<float, bf16_t, false>(R, SI, a, l, s);
  return kahan ? launch_phase_r<float, float, true>(R, SI, a, l, s)
               : launch_phase_r<float, float, false>(R, SI, a, l, s);
}

// Feasibility of frames stacked fstride elements apart over the sides (each
// at most kViolMaxSide; sides longer than the image have no window and are
// skipped), folded into ctrl->viol_key as enqueued work on s: sides up to
// kFeasMaxSide in one pass per launch of up to 65535 frames, longer ones one
// launch each.  The caller resets viol_key and reads it back.
//
// cslots (may be null): an ICD call's work-counter slots (kIcdSlots of
// kIcdSlotWords words), totalled into csum in the same pass, or by
// icd_counter_sum when no side is short enough for the one-pass kernel.
template <typename TX>
int enqueue_feasibility(const void* x, int64_t H, int64_t W, int64_t ld, int64_t fstride,
                        int64_t frames, int n, const int* sides, const double* r2, Ctrl* ctrl,
                        hipStream_t s, const unsigned long long* cslots = nullptr,
                        unsigned long long* csum = nullptr) {
  static_assert(kIcdSlots == 256 && kIcdCountWords == 4, "feasibility_kernel sums 256 x 4");
  FeasSides fs;
  std::memset(&fs, 0, sizeof fs);
  int smin = 0;
  std::vector<int> longer;
  for (int k = 0; k < n; ++k) {
    const int sk = sides[k];
    if (sk < 1 || sk > kViolMaxSide) return SMRE_EINVAL;
    if (sk > H || sk > W) continue;
    if (sk > kFeasMaxSide) {
      longer.push_back(k);
      continue;
    }
    // a side listed twice keeps its smaller bound (the larger violation)
    fs.r2[sk] = fs.r2[sk] > 0.0 ? std::min(fs.r2[sk], r2[k]) : r2[k];
    fs.smax = std::max(fs.smax, sk);
    smin = smin ? std::min(smin, sk) : sk;
  }
  for (int64_t f0 = 0; f0 < frames; f0 += 65535) {
    const unsigned nz = (unsigned)std::min<int64_t>(65535, frames - f0);
    const TX* xf = (const TX*)x + f0 * fstride;
    if (fs.smax > 0) {
      const int tr = feas_tile_rows(fs.smax <= 16 ? 16 : 32);
      const dim3 grid((unsigned)((W - smin + 64) / 64), (unsigned)((H - smin + tr) / tr), nz);
      const unsigned long long* cs = f0 == 0 ? cslots : nullptr;
      if (fs.smax <= 8)
        hipLaunchKernelGGL((feasibility_kernel<TX, 8>), grid, dim3(256), 0, s, xf, fstride, ld,
                           (int)H, (int)W, fs, ctrl, cs, kIcdSlotWords, csum);
      else if (fs.smax <= 16)
        hipLaunchKernelGGL((feasibility_kernel<TX, 16>), grid, dim3(256), 0, s, xf, fstride, ld,
                           (int)H, (int)W, fs, ctrl, cs, kIcdSlotWords, csum);
      else
        hipLaunchKernelGGL((feasibility_kernel<TX, 32>), grid, dim3(256), 0, s, xf, fstride, ld,
                           (int)H, (int)W, fs, ctrl, cs, kIcdSlotWords, csum);
    } else if (cslots && f0 == 0) {
      hipLaunchKernelGGL(icd_counter_sum, dim3(1), dim3(kIcdSlots), 0, s, cslots, csum);
    }
    for (int k : longer) {
      const dim3 grid((unsigned)((W - sides[k] + kViolTileW) / kViolTileW),
                      (unsigned)((H - sides[k] + kViolTileH) / kViolTileH), nz);
      if (sides[k] <= 64)
        hipLaunchKernelGGL((violation_kernel<TX, 64>), grid, dim3(256), 0, s, xf, fstride, ld,
                           (int)H, (int)W, sides[k], r2[k], ctrl);
      else
        hipLaunchKernelGGL((violation_kernel<TX, kViolMaxSide>), grid, dim3(256), 0, s, xf,
                           fstride, ld, (int)H, (int)W, sides[k], r2[k], ctrl);
    }
  }
  HIP_OK(hipGetLastError());
  return SMRE_OK;
}

template <typename TX>
int run_violation(smre_ctx* c, const void* x, int64_t H, int64_t W, int64_t ld, int n,
                  const int* sides, const double* r2, hipStream_t s, double* out,
                  int64_t frames = 1) {
  int rc = enqueue_feasibility<TX>(x, H, W, ld, H * ld, frames, n, sides, r2, c->ctrl, s);
  if (rc) return rc;
  HIP_OK(hipMemcpyAsync(c->ctrl_host, c->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  *out = dkey_inv(c->ctrl_host->viol_key);
  return SMRE_OK;
}

// Non-finite test of the input, enqueued: raises ctrl->nonfinite.
template <typename TX>
void enqueue_nonfinite(smre_ctx* c, const void* x, int64_t H, int64_t W, int64_t ld,
                       hipStream_t s) {
  // every caller gets a cleared flag, whatever the control block held before
  hipLaunchKernelGGL(nonfinite_reset_kernel, dim3(1), dim3(1), 0, s, c->ctrl);
  hipLaunchKernelGGL((nonfinite_kernel<TX>), dim3(grid_rows(H)), dim3(256), 0, s,
                     (const TX*)x, ld, (int)H, (int)W, c->ctrl);
}

template <typename TX>
int check_nonfinite(smre_ctx* c, const void* x, int64_t H, int64_t W, int64_t ld, hipStream_t s,
                    bool* bad) {
  enqueue_nonfinite<TX>(c, x, H, W, ld, s);
  HIP_OK(hipGetLastError());
  HIP_OK(hipMemcpyAsync(c->ctrl_host, c->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  *bad = c->ctrl_host->nonfinite != 0;
  return SMRE_OK;
}

template <typename TX>
int project_impl(smre_ctx* c, smre_dtype dt, void* x, int64_t H, int64_t W, int64_t ld,
                 const smre_params* p, const Plan& pl, unsigned char* ws, hipStream_t s,
                 smre_report* rep) {
  const size_t es = (p->inc == SMRE_INC_BF16) ? 2 : sizeof(TX);
  HIP_OK(hipEventRecord(c->t0, s));
  hipLaunchKernelGGL(ctrl_reset_kernel, dim3(1), dim3(1), 0, s, c->ctrl);
  bool bad = false;
  int rc = check_nonfinite<TX>(c, x, H, W, ld, s, &bad);
  if (rc) return rc;
  if (bad) return SMRE_ENONFINITE;

  uint64_t sig[kSigWords];
  problem_signature(dt, H, W, p, pl, sig);
  TX* isum = (TX*)(ws + pl.off_isum);
  uint64_t* dsig = (uint64_t*)(ws + pl.off_sig);
  if (p->warm) {
    // the increments (and sum_S I_S) of the previous solve of this problem
    uint64_t have[kSigWords];
    HIP_OK(hipMemcpyAsync(have, dsig, sizeof have, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (std::memcmp(have, sig, sizeof sig) != 0) return SMRE_EINVAL;
    hipLaunchKernelGGL((warm_begin_kernel<TX>), dim3(grid_rows(H)), dim3(256), 0, s, (TX*)x, ld,
                       (int)H, (int)W, isum);
  } else {
    // increments start at zero (a fill kernel, not a memset: graph-safe)
    const int64_t nwords = (int64_t)(pl.qbytes / 4);
    hipLaunchKernelGGL((fill_kernel<uint32_t>), dim3(grid_for(nwords)), dim3(256), 0, s,
                       (uint32_t*)ws, nwords, 0u);
    hipLaunchKernelGGL((keep_input_kernel<TX>), dim3(grid_rows(H)), dim3(256), 0, s,
                       (const TX*)x, ld, (int)H, (int)W, isum);
  }
  // until this solve ends, the workspace holds no reusable increments
  hipLaunchKernelGGL((fill_kernel<uint64_t>), dim3(1), dim3(256), 0, s, dsig, (int64_t)kSigWords,
                     (uint64_t)0);
  HIP_OK(hipGetLastError());
  HIP_OK(hipMemcpyAsync(ws + pl.off_roff, pl.meta.data(), pl.meta.size(), hipMemcpyHostToDevice,
                        s));

  ImageDesc a{};
  a.x = x;
  a.rs = (const RegionStream*)(ws + pl.off_roff);
  a.rtab = (const RoundEntry*)(ws + pl.off_roff + pl.meta_rtab);
  a.ld = ld;
  a.q_byte = 0;
  a.H = (int)H;
  a.W = (int)W;
  a.nrx = pl.nrx;
  a.nry = pl.nry;
  a.fr = pl.R + pl.smax - 1;
  a.nsides = pl.nsides;
  a.guard = (float)p->guard_rel;
  for (int k = 0; k < pl.nsides; ++k) {
    a.sides[k] = pl.sides[k];
    a.r2f[k] = (float)pl.r2[k];
    a.rf[k] = (float)std::sqrt(pl.r2[k]);
    a.r2d[k] = pl.r2[k];
  }
  TX* prev = (TX*)(ws + pl.off_prev);
  const bool checking = p->tol > 0;
  TimingAcc tacc;
  std::deque<std::pair<int, int>> inflight;  // (lag slot, sweep)
  int lag_slot = 0;
  bool host_done = false;
  int sweep = 0;
  for (sweep = 1; sweep <= p->max_sweeps && !host_done; ++sweep) {
    const bool check = checking && (sweep % p->check_every == 0 || sweep == p->max_sweeps);
    if (check)
      hipLaunchKernelGGL((snapshot_kernel<TX>), dim3(grid_rows(H)), dim3(256), 0, s,
                         (const TX*)x, ld, (int)H, (int)W, prev, c->ctrl);
    for (int color = 0; color < 4; ++color) {
      PhaseLaunch l;
      l.cy = color >> 1;
      l.cx = color & 1;
      const int ny = (pl.nry - l.cy + 1) / 2, nx = (pl.nrx - l.cx + 1) / 2;
      l.ncx = nx;
      l.blocks = ny * nx;
      l.done = &c->ctrl->done;
      l.abort = &c->ctrl->abort;
      l.q = ws;
      if (ny <= 0 || nx <= 0) continue;
      int slot;
      rc = timing_begin(c, tacc, s, &slot);
      if (rc) return rc;
      rc = launch_phase_any(dt, p->inc, p->kahan, pl.R, pl.SI, a, l, s);
      if (rc) return rc;
      rc = timing_end(c, tacc, s, slot);
      if (rc) return rc;
    }
    if (check) {
      hipLaunchKernelGGL((delta_kernel<TX>), dim3(grid_rows(H)), dim3(256), 0, s,
                         (const TX*)x, ld, (int)H, (int)W, (const TX*)prev, c->ctrl);
      hipLaunchKernelGGL(decide_kernel, dim3(1), dim3(1), 0, s, c->ctrl, p->tol, sweep);
      HIP_OK(hipGetLastError());
      HIP_OK(hipMemcpyAsync(c->ctrl_host + 1 + lag_slot, c->ctrl, sizeof(Ctrl),
                            hipMemcpyDeviceToHost, s));
      HIP_OK(hipEventRecord(c->lag_ev[lag_slot], s));
      inflight.push_back({lag_slot, sweep});
      lag_slot = (lag_slot + 1) % (kLag + 1);
      if ((int)inflight.size() > kLag) {
        auto f = inflight.front();
        inflight.pop_front();
        HIP_OK(hipEventSynchronize(c->lag_ev[f.first]));
        if (c->ctrl_host[1 + f.first].done) host_done = true;
      }
    }
  }
  // sum_S I_S = x0 - z for a later warm start
  hipLaunchKernelGGL((increment_sum_kernel<TX>), dim3(grid_rows(H)), dim3(256), 0, s,
                     (const TX*)x, ld, (int)H, (int)W, isum);
  HIP_OK(hipGetLastError());
  HIP_OK(hipStreamSynchronize(s));
  rc = timing_flush(c, tacc, true);
  if (rc) return rc;
  HIP_OK(hipMemcpy(c->ctrl_host, c->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
  const Ctrl fin = *c->ctrl_host;
  const int sweeps_run = fin.done ? fin.done_sweep : p->max_sweeps;
  if (!fin.abort)  // the increments belong to this problem now
    HIP_OK(hipMemcpy(dsig, sig, sizeof sig, hipMemcpyHostToDevice));
  double viol = 0.0;
  rc = run_violation<TX>(c, x, H, W, ld, pl.nsides, pl.sides, pl.r2, s, &viol);
  if (rc) return rc;
  HIP_OK(hipEventRecord(c->t1, s));
  HIP_OK(hipEventSynchronize(c->t1));
  // a wait that gave up is a protocol failure: the result is not trustworthy
  if (fin.abort) return SMRE_EDEVICE;
  float ms = 0.f;
  HIP_OK(hipEventElapsedTime(&ms, c->t0, c->t1));
  if (rep) {
    rep->sweeps = sweeps_run;
    rep->converged = fin.done;
    rep->region = pl.R;
    rep->inner_sweeps = 0;
    rep->last_delta = checking ? fin.last_delta : NAN;
    rep->max_violation = viol;
    rep->elapsed_ms = ms;
    rep->kernel_ms = tacc.ms;
    rep->kernel_launches = tacc.launches;
    rep->bytes_moved = (double)sweeps_run * (2.0 * es * (double)pl.nq + 2.0 * sizeof(TX) * (double)H * W);
    rep->window_projections = (double)sweeps_run * (double)pl.nwin;
    rep->pixel_updates = (double)sweeps_run * (double)pl.nq;
  }
  if (checking && !fin.done) return SMRE_NOT_CONVERGED;
  return SMRE_OK;
}


// ---------------------------------------------------------------- canonical orders
// Full Dykstra with the sides descending (or ascending) and each side's
// tilings (a, b) in raster order, one launch per tiling (canon.hpp).
struct CanonTiling {
  int s, a, b, nr, nc, k;  // side, offset, window rows / columns, side index
  size_t off;              // first byte of the tiling's increment plane
};
struct CanonPlan {
  std::vector<CanonTiling> t;
  Plan base;  // sorted sides, bounds, counts (the region fields are unused)
  size_t qbytes = 0, off_prev = 0, off_isum = 0, off_sig = 0, total = 0;
};

int plan_canon(smre_dtype dt, int64_t H, int64_t W, const smre_params* p, CanonPlan* cp) {
  // the region planner validates the sides, bounds and options (the region
  // side plays no part in these orders)
  smre_params q = *p;
  q.region = 0;
  int rc = plan_project(dt, H, W, &q, &cp->base, false);
  if (rc) return rc;
  const Plan& pl = cp->base;
  const size_t es = (p->inc == SMRE_INC_BF16) ? 2 : (dt == SMRE_F64 ? 8 : 4);
  const size_t xs = dt == SMRE_F64 ? 8 : 4;
  cp->t.clear();
  size_t off = 0;
  for (int kk = 0; kk < pl.nsides; ++kk) {
    const int k = p->order == SMRE_ORDER_ASC ? pl.nsides - 1 - kk : kk;  // sorted descending
    const int sd = pl.sides[k];
    for (int a = 0; a < sd; ++a)
      for (int b = 0; b < sd; ++b) {
        const int nr = (int)((H - a) / sd), nc = (int)((W - b) / sd);
        if (nr <= 0 || nc <= 0) continue;
        cp->t.push_back(CanonTiling{sd, a, b, nr, nc, k, off});
        off = align_up(off + (size_t)nr * nc * sd * sd * es, 256);
      }
  }
  cp->qbytes = off;
  cp->off_prev = align_up(off, 256);
  cp->off_isum = align_up(cp->off_prev + (size_t)H * W * xs, 256);
  cp->off_sig = align_up(cp->off_isum + (size_t)H * W * xs, 256);
  cp->total = align_up(cp->off_sig + kSigWords * sizeof(uint64_t), 256);
  return SMRE_OK;
}

template <typename TX, typename TQ, int SMAX, bool KAHAN>
void launch_tiling(const TilingArgs& g, hipStream_t s) {
  const dim3 grid((unsigned)((g.nc + g.wpb - 1) / g.wpb), (unsigned)g.nr);
  hipLaunchKernelGGL((tiling_phase<TX, TQ, SMAX, KAHAN>), grid, dim3(256), 0, s, g);
}

template <typename TX>
int launch_tiling_any(int inc, int kahan, const TilingArgs& g, hipStream_t s) {
  const bool big = g.s > 16;
  if constexpr (sizeof(TX) == 8) {
    big ? launch_tiling<double, double, 32, false>(g, s) : launch_tiling<double, double, 16, false>(g, s);
  } else if (inc == SMRE_INC_BF16) {
    if (kahan) big ? launch_tiling<float, bf16_t, 32, true>(g, s) : launch_tiling<float, bf16_t, 16, true>(g, s);
    else big ? launch_tiling<float, bf16_t, 32, false>(g, s) : launch_tiling<float, bf16_t, 16, false>(g, s);
  } else {
    if (kahan) big ? launch_tiling<float, float, 32, true>(g, s) : launch_tiling<float, float, 16, true>(g, s);
    else big ? launch_tiling<float, float, 32, false>(g, s) : launch_tiling<float, float, 16, false>(g, s);
  }
  HIP_OK(hipGetLastError());
  return SMRE_OK;
}

template <typename TX>
int canon_impl(smre_ctx* c, smre_dtype dt, void* x, int64_t H, int64_t W, int64_t ld,
               const smre_params* p, const CanonPlan& cp, unsigned char* ws, hipStream_t s,
               smre_report* rep) {
  const Plan& pl = cp.base;
  const size_t es = (p->inc == SMRE_INC_BF16) ? 2 : sizeof(TX);
  HIP_OK(hipEventRecord(c->t0, s));
  hipLaunchKernelGGL(ctrl_reset_kernel, dim3(1), dim3(1), 0, s, c->ctrl);
  bool bad = false;
  int rc = check_nonfinite<TX>(c, x, H, W, ld, s, &bad);
  if (rc) return rc;
  if (bad) return SMRE_ENONFINITE;
  uint64_t sig[kSigWords];
  problem_signature(dt, H, W, p, pl, sig);
  sig[1] |= (uint64_t)p->order << 32;
  sig[6] = (uint64_t)cp.qbytes;
  TX* isum = (TX*)(ws + cp.off_isum);
  uint64_t* dsig = (uint64_t*)(ws + cp.off_sig);
  if (p->warm) {
    uint64_t have[kSigWords];
    HIP_OK(hipMemcpyAsync(have, dsig, sizeof have, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (std::memcmp(have, sig, sizeof sig) != 0) return SMRE_EINVAL;
    hipLaunchKernelGGL((warm_begin_kernel<TX>), dim3(grid_rows(H)), dim3(256), 0, s, (TX*)x, ld,
                       (int)H, (int)W, isum);
  } else {
    const int64_t nwords = (int64_t)(cp.qbytes / 4);
    hipLaunchKernelGGL((fill_kernel<uint32_t>), dim3(grid_for(nwords)), dim3(256), 0, s,
                       (uint32_t*)ws, nwords, 0u);
    hipLaunchKernelGGL((keep_input_kernel<TX>), dim3(grid_rows(H)), dim3(256), 0, s,
                       (const TX*)x, ld, (int)H, (int)W, isum);
  }
  hipLaunchKernelGGL((fill_kernel<uint64_t>), dim3(1), dim3(256), 0, s, dsig, (int64_t)kSigWords,
                     (uint64_t)0);
  HIP_OK(hipGetLastError());

  TX* prev = (TX*)(ws + cp.off_prev);
  const bool checking = p->tol > 0;
  std::deque<std::pair<int, int>> inflight;  // (lag slot, sweep)
  int lag_slot = 0, sweep = 0;
  bool host_done = false;
  int64_t launches = 0;
  for (sweep = 1; sweep <= p->max_sweeps && !host_done; ++sweep) {
    const bool check = checking && (sweep % p->check_every == 0 || sweep == p->max_sweeps);
    if (check)
      hipLaunchKernelGGL((snapshot_kernel<TX>), dim3(grid_rows(H)), dim3(256), 0, s,
                         (const TX*)x, ld, (int)H, (int)W, prev, c->ctrl);
    for (const CanonTiling& t : cp.t) {
      TilingArgs g{};
      g.x = x;
      g.q = ws + t.off;
      g.done = &c->ctrl->done;
      g.ld = ld;
      g.s = t.s;
      g.a = t.a;
      g.b = t.b;
      g.nr = t.nr;
      g.nc = t.nc;
      g.wpb = 256 / t.s;
      g.guard = (float)p->guard_rel;
      g.r2f = (float)pl.r2[t.k];
      g.rf = (float)std::sqrt(pl.r2[t.k]);
      g.r2d = pl.r2[t.k];
      if ((rc = launch_tiling_any<TX>(p->inc, p->kahan, g, s))) return rc;
      ++launches;
    }
    if (check) {
      hipLaunchKernelGGL((delta_kernel<TX>), dim3(grid_rows(H)), dim3(256), 0, s,
                         (const TX*)x, ld, (int)H, (int)W, (const TX*)prev, c->ctrl);
      hipLaunchKernelGGL(decide_kernel, dim3(1), dim3(1), 0, s, c->ctrl, p->tol, sweep);
      HIP_OK(hipGetLastError());
      HIP_OK(hipMemcpyAsync(c->ctrl_host + 1 + lag_slot, c->ctrl, sizeof(Ctrl),
                            hipMemcpyDeviceToHost, s));
      HIP_OK(hipEventRecord(c->lag_ev[lag_slot], s));
      inflight.push_back({lag_slot, sweep});
      lag_slot = (lag_slot + 1) % (kLag + 1);
      if ((int)inflight.size() > kLag) {
        auto f = inflight.front();
        inflight.pop_front();
        HIP_OK(hipEventSynchronize(c->lag_ev[f.first]));
        if (c->ctrl_host[1 + f.first].done) host_done = true;
      }
    }
  }
  hipLaunchKernelGGL((increment_sum_kernel<TX>), dim3(grid_rows(H)), dim3(256), 0, s,
                     (const TX*)x, ld, (int)H, (int)W, isum);
  HIP_OK(hipGetLastError());
  HIP_OK(hipStreamSynchronize(s));
  HIP_OK(hipMemcpy(c->ctrl_host, c->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
  const Ctrl fin = *c->ctrl_host;
  const int sweeps_run = fin.done ? fin.done_sweep : p->max_sweeps;
  HIP_OK(hipMemcpy(dsig, sig, sizeof sig, hipMemcpyHostToDevice));
  double viol = 0.0;
  rc = run_violation<TX>(c, x, H, W, ld, pl.nsides, pl.sides, pl.r2, s, &viol);
  if (rc) return rc;
  HIP_OK(hipEventRecord(c->t1, s));
  HIP_OK(hipEventSynchronize(c->t1));
  float ms = 0.f;
  HIP_OK(hipEventElapsedTime(&ms, c->t0, c->t1));
  if (rep) {
    rep->sweeps = sweeps_run;
    rep->converged = fin.done;
    rep->region = 0;
    rep->inner_sweeps = 0;
    rep->last_delta = checking ? fin.last_delta : NAN;
    rep->max_violation = viol;
    rep->elapsed_ms = ms;
    rep->kernel_ms = 0.0;
    rep->kernel_launches = launches;
    rep->bytes_moved = (double)sweeps_run * (2.0 * es * (double)pl.nq + 2.0 * sizeof(TX) * (double)H * W);
    rep->window_projections = (double)sweeps_run * (double)pl.nwin;
    rep->pixel_updates = (double)sweeps_run * (double)pl.nq;
  }
  if (checking && !fin.done) return SMRE_NOT_CONVERGED;
  return SMRE_OK;
}

template <typename T, bool MEANABS>
void launch_icd(int K, dim3 grid, const IcdArgs& a, hipStream_t s) {
  switch (K) {
    case 0: hipLaunchKernelGGL((icd_phase<T, 0, MEANABS>), grid, dim3(64), 0, s, a); break;
    case 1: hipLaunchKernelGGL((icd_phase<T, 1, MEANABS>), grid, dim3(64), 0, s, a); break;
    case 2: hipLaunchKernelGGL((icd_phase<T, 2, MEANABS>), grid, dim3(64), 0, s, a); break;
    case 3: hipLaunchKernelGGL((icd_phase<T, 3, MEANABS>), grid, dim3(64), 0, s, a); break;
    case 4: hipLaunchKernelGGL((icd_phase<T, 4, MEANABS>), grid, dim3(64), 0, s, a); break;
    default: hipLaunchKernelGGL((icd_phase<T, 5, MEANABS>), grid, dim3(64), 0, s, a); break;
  }
}

template <bool GEN, typename T>
int mc_run(smre_ctx* c, const T* fields, int64_t ld, int64_t H, int64_t W, uint64_t seed,
           int64_t f0, int64_t nf, const McSides& sd, double* q_out, double* tmax_out,
           hipStream_t s, TimingAcc& acc);
template <bool GEN, typename T>
int mc_run_buf(smre_ctx* c, const T* fields, int64_t ld, int64_t H, int64_t W, uint64_t seed,
               int64_t f0, int64_t nf, const McSides& sd, double* q_out, double* tmax_out,
               hipStream_t s, TimingAcc* acc, unsigned long long* tmax, double* q);
int mc_sides(int32_t n, const int32_t* sides, int64_t H, int64_t W, McSides* sd);

// Device scratch of one ICD call: the work counters (kIcdSlots lines).  Their
// sums and the feasibility report go through the context's control block.
struct IcdScratch {
  unsigned long long* cnt;   // kIcdSlots * kIcdSlotWords words
};
constexpr int64_t kIcdCntWords = (int64_t)kIcdSlots * kIcdSlotWords;
// words of the allocation-free scratch: the counters
constexpr int64_t kIcdScratchWords = kIcdCntWords;

}  // namespace

// Device scratch of smre_dykstra_incomplete_noalloc (32,768 bytes, held by every
// GPU the library runs on until the process ends).  In host code `scratch`
// names a host-side stand-in: kernels get its device address, looked up per
// device with hipGetSymbolAddress when a context is created.
static __device__ __align__(256) unsigned long long scratch[kIcdScratchWords];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned long long* g_scratch_ptr[kMaxDevices] = {};

// With `device` current: record the device address of `scratch` on it.
int scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return SMRE_EINVAL;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return SMRE_OK;
  void* p = nullptr;
  HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) return SMRE_EDEVICE;
  g_scratch_ptr[device] = (unsigned long long*)p;
  return SMRE_OK;
}

unsigned long long* scratch_of(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

// Phase p: lattice shift (sy[p], sx[p]), levels K down to lo[p].  fixed:
// caller-supplied device scratch (one frame; no allocation on any path, no
// per-kernel timing); null: the context's buffers, allocated on first use.
template <typename T>
int icd_impl(smre_ctx* c, void* x, int64_t H, int64_t W, int64_t ld, int64_t frames, int K,
             const double* r2, double tol, int mode, int max_inner, int nph, const int32_t* sy,
             const int32_t* sx, const int32_t* lo, hipStream_t s, smre_report* rep,
             bool checks = true, const IcdScratch* fixed = nullptr) {
  // checks: the non-finite test of the input and the feasibility report (an
  // inner call of the ADMM loop, whose inputs are its own, skips both)
  if (fixed && frames != 1) return SMRE_EINVAL;
  HIP_OK(hipEventRecord(c->t0, s));
  int rc = SMRE_OK;
  unsigned long long* cnt;
  if (fixed) {
    cnt = fixed->cnt;
  } else {
    if (!c->icd_cnt) HIP_OK(hipMalloc(&c->icd_cnt, sizeof(unsigned long long) * kIcdCntWords));
    cnt = c->icd_cnt;
  }
  // one launch clears the counters, resets the control block and runs the
  // non-finite test, which is not waited for: the phase kernels read its flag
  // and leave x alone when it holds this call's number, and the one wait at
  // the end of the call reads it with the counters and the feasibility
  // report.  Frames are stacked H * ld elements apart: one tall image of
  // frames * H rows.
  const unsigned epoch = ++c->icd_epoch;
  const int begin_grid = checks ? grid_rows(frames * H) : grid_for(kIcdCntWords);
  hipLaunchKernelGGL((icd_begin_kernel<T>), dim3(begin_grid), dim3(256), 0, s, c->ctrl,
                     checks ? 1 : 0, cnt, kIcdCntWords, checks ? (const T*)x : (const T*)nullptr,
                     ld, (int)(frames * H), (int)W, epoch);
  IcdArgs a{};
  a.ld = ld;
  a.fstride = H * ld;
  a.H = (int)H;
  a.W = (int)W;
  a.mode = mode;
  a.max_inner = max_inner;
  a.tol = tol;
  for (int k = 0; k <= K; ++k) {
    a.r2[k] = r2[k];
    a.sr2[k] = std::sqrt((float)r2[k]);
  }
  a.counters = cnt;
  a.skip = checks ? &c->ctrl->nf_epoch : nullptr;
  a.epoch = epoch;
  const int B = 1 << K;
  std::optional<TimingAcc> tacc;  // (its queue allocates: not on the fixed path)
  if (!fixed) tacc.emplace();
  for (int ph = 0; ph < nph; ++ph) {
    a.oy = sy[ph];
    a.ox = sx[ph];
    a.lmin = lo[ph];
    const int start_y = sy[ph] > 0 ? sy[ph] - B : 0, start_x = sx[ph] > 0 ? sx[ph] - B : 0;
    const int nby = (int)((H - start_y + B - 1) / B), nbx = (int)((W - start_x + B - 1) / B);
    int slot = -1;
    if (tacc && (rc = timing_begin(c, *tacc, s, &slot))) return rc;
    // frames per launch: at most 65535 and fewer than 2^31 blocks in all
    const int64_t fchunk = std::max<int64_t>(
        1, std::min<int64_t>(65535, ((int64_t)1 << 31) / ((int64_t)nbx * nby) - 1));
    a.nx_d = (uint32_t)nbx;
    a.nxy_d = (uint32_t)nbx * (uint32_t)nby;
    udiv_magic(a.nx_d, &a.nx_m, &a.nx_s);
    udiv_magic(a.nxy_d, &a.nxy_m, &a.nxy_s);
    for (int64_t f0 = 0; f0 < frames; f0 += fchunk) {
      const int64_t nf = std::min<int64_t>(fchunk, frames - f0);
      a.nblocks = (uint32_t)(nf * nbx * nby);
      // runs of blocks per wave once there are enough blocks to keep every
      // SIMD busy with several waves (wave launches are then the cost to
      // amortise); one block per wave below that
      const int64_t simds = (int64_t)std::max(1, c->cus) * 4;
      a.run = a.nblocks >= (uint32_t)(simds * 8 * 16) ? 16u
              : a.nblocks >= (uint32_t)(simds * 8 * 4) ? 4u : 1u;
      const dim3 grid((a.nblocks + a.run - 1) / a.run);
      a.x = (T*)x + f0 * H * ld;
      if (mode == SMRE_TOL_MEANABS)
        launch_icd<T, true>(K, grid, a, s);
      else
        launch_icd<T, false>(K, grid, a, s);
      HIP_OK(hipGetLastError());
    }
    if (tacc && (rc = timing_end(c, *tacc, s, slot))) return rc;
  }
  // The work counters (inner sweeps, square projections, (square, pixel)
  // updates, blocks that stopped at max_inner without meeting the tolerance)
  // are totalled in the feasibility pass when there is one.  Reported: the
  // violation over the FULL family of the levels' sides (every position, every
  // frame), i.e. how far ICD is from feasibility for the exact method.
  if (checks && rep) {  // the feasibility pass only feeds the report
    int32_t fam[6];
    double fam_r2[6];
    int nfam = 0;
    for (int k = 0; k <= K; ++k) {
      fam[nfam] = 1 << k;
      fam_r2[nfam++] = r2[k];
    }
    rc = enqueue_feasibility<T>(x, H, W, ld, H * ld, frames, nfam, fam, fam_r2, c->ctrl, s, cnt,
                                c->ctrl->icd_sum);
    if (rc) return rc;
  } else {
    hipLaunchKernelGGL(icd_counter_sum, dim3(1), dim3(kIcdSlots), 0, s, cnt, c->ctrl->icd_sum);
    HIP_OK(hipGetLastError());
  }
  HIP_OK(hipMemcpyAsync(c->ctrl_host, c->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
  HIP_OK(hipEventRecord(c->t1, s));
  HIP_OK(hipEventSynchronize(c->t1));
  if (tacc && (rc = timing_flush(c, *tacc, true))) return rc;
  const Ctrl& fin = *c->ctrl_host;
  if (checks && fin.nf_epoch == epoch) return SMRE_ENONFINITE;  // x was left as it came
  const unsigned long long* sums = fin.icd_sum;
  const double viol = (checks && rep) ? dkey_inv(fin.viol_key) : NAN;
  float ms = 0.f;
  HIP_OK(hipEventElapsedTime(&ms, c->t0, c->t1));
  if (rep) {
    rep->sweeps = nph;
    rep->converged = sums[3] == 0;
    rep->region = B;
    rep->inner_sweeps = (int32_t)std::min<unsigned long long>(sums[0], INT32_MAX);
    rep->last_delta = NAN;
    rep->max_violation = viol;
    rep->elapsed_ms = ms;
    rep->kernel_ms = tacc ? tacc->ms : 0.0;
    rep->kernel_launches = tacc ? tacc->launches : 0;
    rep->bytes_moved = 2.0 * sizeof(T) * (double)H * W * nph * (double)frames;
    rep->window_projections = (double)sums[1];
    rep->pixel_updates = (double)sums[2];
  }
  return sums[3] == 0 ? SMRE_OK : SMRE_NOT_CONVERGED;
}

// ---------------------------------------------------------------- nested ICD
// Lane layout of a divisor chain (icd_nested.hpp): the lane level m is one
// whose squares hold at most 16 pixels while the block fits the lanes the
// kernel instance allows.  Of those, the one with the fewest lanes that still
// fills a wave (fewer reduction steps per inner sweep), else the one with the
// most lanes (small blocks: as many busy lanes as the block has).  The choice
// depends on the chain only, so a frame gives the same bits alone or in a
// movie.
int nested_lanes_max(int P) { return P == 16 ? 256 : P == 9 ? 512 : 1024; }

int nested_tables(int nlev, const int32_t* side, NestedArgs* a) {
  const int B = side[nlev - 1];
  int m = -1, m_most = -1;
  for (int j = nlev - 1; j >= 0; --j) {
    const int P = side[j] * side[j];
    if (P > 16 || B * B / P > nested_lanes_max(P)) continue;
    m_most = j;                           // ends at the most lanes
    if (m < 0 && B * B / P >= 64) m = j;  // first (fewest lanes) filling a wave
  }
  if (m < 0) m = m_most;
  if (m < 0) return SMRE_EINVAL;
  const int P = side[m] * side[m];
  a->B = B;
  a->nlev = nlev;
  a->m = m;
  a->nt = B * B / P;
  for (int j = 0; j < kNestLevels; ++j) {
    a->side[j] = j < nlev ? side[j] : 0;
    a->rad[j] = (j >= 1 && j < nlev) ? side[j] / side[j - 1] : 1;
    a->grp[j] = (j > m && j < nlev) ? (side[j] / side[m]) * (side[j] / side[m]) : 1;
    a->rstart[j] = a->rend[j] = 0;
    if (j <= m) {
      const int A = side[j] * side[j];
      for (int e = 0; e < P; ++e) {
        if (e % A == 0) a->rstart[j] |= 1u << e;
        if (e % A == A - 1) a->rend[j] |= 1u << e;
      }
    }
  }
  // element e of a lane: its digits, lowest first -- the pixel inside its
  // level-0 square (raster), then the sub-square at each level up to m
  for (int e = 0; e < 16; ++e) {
    int r = 0, c = 0;
    if (e < P) {
      int u = e;
      const int a0 = side[0] * side[0];
      const int d0 = u % a0;
      u /= a0;
      r = d0 / side[0];
      c = d0 % side[0];
      for (int j = 1; j <= m; ++j) {
        const int rd = side[j] / side[j - 1], rr = rd * rd;
        const int d = u % rr;
        u /= rr;
        r += (d / rd) * side[j - 1];
        c += (d % rd) * side[j - 1];
      }
    }
    a->pr[e] = (uint8_t)r;
    a->pc[e] = (uint8_t)c;
    for (int j = 0; j < kNestLevels; ++j) {
      const int L = (j <= m) ? side[j] : 1;
      a->sqr[j][e] = (uint8_t)((r / L) * L);
      a->sqc[j][e] = (uint8_t)((c / L) * L);
    }
  }
  return SMRE_OK;
}

template <typename T, bool MEANABS>
void launch_nested(int P, dim3 grid, int threads, const NestedArgs& a, hipStream_t s) {
  switch (P) {
    case 16: hipLaunchKernelGGL((icd_nested_phase<T, 16, MEANABS>), grid, dim3(threads), 0, s, a); break;
    case 9: hipLaunchKernelGGL((icd_nested_phase<T, 9, MEANABS>), grid, dim3(threads), 0, s, a); break;
    case 4: hipLaunchKernelGGL((icd_nested_phase<T, 4, MEANABS>), grid, dim3(threads), 0, s, a); break;
    default: hipLaunchKernelGGL((icd_nested_phase<T, 1, MEANABS>), grid, dim3(threads), 0, s, a); break;
  }
}

int nested_validate(smre_ctx* c, smre_dtype dt, const void* x, int64_t H, int64_t W, int64_t ld,
                    int64_t frames, int32_t nlev, const int32_t* side, const double* r2,
                    int32_t n_phases, const int32_t* shift_y, const int32_t* shift_x,
                    const int32_t* min_level, double tol, int32_t mode, int32_t max_inner) {
  if (!c || !x || !side || !r2 || !shift_y || !shift_x || !min_level) return SMRE_EINVAL;
  if (frames < 1 || frames * H > INT32_MAX) return SMRE_EINVAL;
  if (dt != SMRE_F32 && dt != SMRE_F64) return SMRE_EINVAL;
  if (H < 1 || W < 1 || ld < W || H > (1 << 20) || W > (1 << 20)) return SMRE_EINVAL;
  if (nlev < 1 || nlev > kNestLevels || max_inner < 1 || n_phases < 1 || n_phases > 64)
    return SMRE_EINVAL;
  for (int j = 0; j < nlev; ++j) {
    if (side[j] < 1 || side[j] > 96) return SMRE_EINVAL;
    if (j > 0 && (side[j] <= side[j - 1] || side[j] % side[j - 1] != 0)) return SMRE_EINVAL;
    if (!std::isfinite(r2[j])) return SMRE_ENONFINITE;
    if (!(r2[j] > 0)) return SMRE_EINVAL;
  }
  const int B = side[nlev - 1];
  {
    const int64_t nbx = W / B + 2, nby = H / B + 2;
    if (nbx * nby >= ((int64_t)1 << 31)) return SMRE_EINVAL;
  }
  for (int p = 0; p < n_phases; ++p)
    if (shift_y[p] < 0 || shift_y[p] >= B || shift_x[p] < 0 || shift_x[p] >= B ||
        min_level[p] < 0 || min_level[p] >= nlev)
      return SMRE_EINVAL;
  if (mode != SMRE_TOL_MAXABS && mode != SMRE_TOL_MEANABS) return SMRE_EINVAL;
  if (!std::isfinite(tol)) return SMRE_EINVAL;
  NestedArgs a{};
  return nested_tables(nlev, side, &a);
}

template <typename T>
int nested_impl(smre_ctx* c, void* x, int64_t H, int64_t W, int64_t ld, int64_t frames, int nlev,
                const int32_t* side, const double* r2, double tol, int mode, int max_inner,
                int nph, const int32_t* sy, const int32_t* sx, const int32_t* lo, hipStream_t s,
                smre_report* rep) {
  HIP_OK(hipEventRecord(c->t0, s));
  int rc = SMRE_OK;
  if (!c->icd_cnt) HIP_OK(hipMalloc(&c->icd_cnt, sizeof(unsigned long long) * kIcdCntWords));
  unsigned long long* cnt = c->icd_cnt;
  // counters cleared, control block reset and the non-finite test in one
  // launch, read back with the results (as in icd_impl)
  const unsigned epoch = ++c->icd_epoch;
  hipLaunchKernelGGL((icd_begin_kernel<T>), dim3(grid_rows(frames * H)), dim3(256), 0, s, c->ctrl,
                     1, cnt, kIcdCntWords, (const T*)x, ld, (int)(frames * H), (int)W, epoch);
  NestedArgs a{};
  rc = nested_tables(nlev, side, &a);
  if (rc) return rc;
  const int P = side[a.m] * side[a.m];
  const int threads = (a.nt + 63) / 64 * 64;
  a.ld = ld;
  a.fstride = H * ld;
  a.H = (int)H;
  a.W = (int)W;
  a.mode = mode;
  a.max_inner = max_inner;
  a.tol = tol;
  for (int j = 0; j < nlev; ++j) {
    a.r2[j] = r2[j];
    a.sr2[j] = std::sqrt((float)r2[j]);
  }
  a.counters = cnt;
  a.skip = &c->ctrl->nf_epoch;
  a.epoch = epoch;
  const int B = a.B;
  TimingAcc tacc;
  for (int ph = 0; ph < nph; ++ph) {
    a.oy = sy[ph] > 0 ? sy[ph] - B : 0;
    a.ox = sx[ph] > 0 ? sx[ph] - B : 0;
    a.lo = lo[ph];
    const int nby = (int)((H - a.oy + B - 1) / B), nbx = (int)((W - a.ox + B - 1) / B);
    a.nbx = nbx;
    int slot = -1;
    if ((rc = timing_begin(c, tacc, s, &slot))) return rc;
    for (int64_t f0 = 0; f0 < frames; f0 += 65535) {
      const int64_t nf = std::min<int64_t>(65535, frames - f0);
      a.x = (T*)x + f0 * H * ld;
      const dim3 grid((unsigned)(nbx * nby), (unsigned)nf);
      if (mode == SMRE_TOL_MEANABS)
        launch_nested<T, true>(P, grid, threads, a, s);
      else
        launch_nested<T, false>(P, grid, threads, a, s);
      HIP_OK(hipGetLastError());
    }
    if ((rc = timing_end(c, tacc, s, slot))) return rc;
  }
  // reported: the violation over the full family of the levels' sides (every
  // position, every frame); the work counters totalled in the same pass
  if (rep) {
    rc = enqueue_feasibility<T>(x, H, W, ld, H * ld, frames, nlev, side, r2, c->ctrl, s, cnt,
                                c->ctrl->icd_sum);
    if (rc) return rc;
  } else {
    hipLaunchKernelGGL(icd_counter_sum, dim3(1), dim3(kIcdSlots), 0, s, cnt, c->ctrl->icd_sum);
    HIP_OK(hipGetLastError());
  }
  HIP_OK(hipMemcpyAsync(c->ctrl_host, c->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
  HIP_OK(hipEventRecord(c->t1, s));
  HIP_OK(hipEventSynchronize(c->t1));
  if ((rc = timing_flush(c, tacc, true))) return rc;
  const Ctrl& fin = *c->ctrl_host;
  if (fin.nf_epoch == epoch) return SMRE_ENONFINITE;  // x was left as it came
  const unsigned long long* sums = fin.icd_sum;
  const double viol = rep ? dkey_inv(fin.viol_key) : NAN;
  float ms = 0.f;
  HIP_OK(hipEventElapsedTime(&ms, c->t0, c->t1));
  if (rep) {
    rep->sweeps = nph;
    rep->converged = sums[3] == 0;
    rep->region = B;
    rep->inner_sweeps = (int32_t)std::min<unsigned long long>(sums[0], INT32_MAX);
    rep->last_delta = NAN;
    rep->max_violation = viol;
    rep->elapsed_ms = ms;
    rep->kernel_ms = tacc.ms;
    rep->kernel_launches = tacc.launches;
    rep->bytes_moved = 2.0 * sizeof(T) * (double)H * W * nph * (double)frames;
    rep->window_projections = (double)sums[1];
    rep->pixel_updates = (double)sums[2];
  }
  return sums[3] == 0 ? SMRE_OK : SMRE_NOT_CONVERGED;
}

// ---------------------------------------------------------------- batches
struct BatchPlan {
  int R = 16;
  int SI = 17;  // kernel instance shared by every image (instance_smax of the batch)
  int n = 0;
  std::vector<Plan> plans;
  std::vector<size_t> qoff;       // byte offset of each image's increments
  std::vector<size_t> roff_off;   // byte offset of each image's metadata blob
  std::vector<int64_t> prev_off;  // element offset of each image's snapshot
  size_t qbytes = 0, roff_elems = 0, prev_elems = 0;
  int nitems[4] = {0, 0, 0, 0};
  size_t off_roff = 0, off_desc = 0, off_ctl = 0, off_items = 0, off_cnt = 0, off_prev = 0,
         total = 0;
};

int plan_batch(smre_dtype dt, int n, const smre_batch_image* im, const smre_batch_params* bp,
               int R, BatchPlan* B, bool need_offsets) {
  B->R = R;
  B->n = n;
  int smax_all = 1;
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < im[i].n_sides && im[i].sides; ++k)
      smax_all = std::max(smax_all, (int)im[i].sides[k]);
  B->SI = instance_smax(R, smax_all);
  B->plans.assign(n, Plan());
  B->qoff.assign(n, 0);
  B->roff_off.assign(n, 0);
  B->prev_off.assign(n, 0);
  B->qbytes = B->roff_elems = B->prev_elems = 0;
  for (int c = 0; c < 4; ++c) B->nitems[c] = 0;
  const size_t xs = dt == SMRE_F64 ? 8 : 4;
  int64_t items_total = 0;
  for (int i = 0; i < n; ++i) {
    smre_params p{};
    p.n_sides = im[i].n_sides;
    p.sides = im[i].sides;
    p.radius2 = im[i].radius2;
    p.tol = im[i].tol;
    p.max_sweeps = im[i].max_sweeps;
    p.check_every = bp->check_every;
    p.region = R;
    p.inc = bp->inc;
    p.kahan = bp->kahan;
    p.guard_rel = bp->guard_rel;
    if (!im[i].x || im[i].ld < im[i].W) return SMRE_EINVAL;
    int rc = plan_project(dt, im[i].H, im[i].W, &p, &B->plans[i], need_offsets, B->SI);
    if (rc) return rc;
    B->qoff[i] = B->qbytes;
    B->qbytes += align_up(B->plans[i].qbytes, kPage);
    B->roff_off[i] = B->roff_elems;
    B->roff_elems += align_up(B->plans[i].meta_bytes, 256);
    B->prev_off[i] = (int64_t)B->prev_elems;
    B->prev_elems += (size_t)(im[i].H * im[i].W);
    const Plan& pl = B->plans[i];
    for (int ry = 0; ry < pl.nry; ++ry)
      for (int rx = 0; rx < pl.nrx; ++rx) B->nitems[(ry & 1) * 2 + (rx & 1)]++;
    items_total += (int64_t)pl.nry * pl.nrx;
  }
  B->off_roff = B->qbytes;
  B->off_desc = align_up(B->off_roff + B->roff_elems, 256);
  B->off_ctl = align_up(B->off_desc + sizeof(ImageDesc) * n, 256);
  B->off_items = align_up(B->off_ctl + sizeof(BatchCtl) * n, 256);
  B->off_cnt = align_up(B->off_items + sizeof(WorkItem) * items_total, 256);
  B->off_prev = align_up(B->off_cnt + 64, 256);
  B->total = align_up(B->off_prev + B->prev_elems * xs, 256);
  return SMRE_OK;
}

template <typename TX, typename TQ, int R, int SMAX, bool KAHAN>
int batch_grid(int cus, int want) {
  int occ = 0;
  HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &occ, (const void*)region_phase_batch<TX, TQ, R, SMAX, KAHAN>, 128, 0));
  return std::max(1, std::min(want, std::max(1, occ) * cus));
}

template <typename TX, typename TQ, bool KAHAN>
int launch_batch_phase(int R, int SI, int grid, const ImageDesc* d, BatchCtl* ctl,
                       const WorkItem* items, const int* cnt, unsigned char* q, hipStream_t s) {
  switch (R) {
    case 8:
      hipLaunchKernelGGL((region_phase_batch<TX, TQ, 8, 9, KAHAN>), dim3(grid), dim3(128), 0, s, d,
                         ctl, items, cnt, q);
      break;
    case 16:
      if (SI == 9)
        hipLaunchKernelGGL((region_phase_batch<TX, TQ, 16, 9, KAHAN>), dim3(grid), dim3(128), 0,
                           s, d, ctl, items, cnt, q);
      else
        hipLaunchKernelGGL((region_phase_batch<TX, TQ, 16, 17, KAHAN>), dim3(grid), dim3(128), 0,
                           s, d, ctl, items, cnt, q);
      break;
    case 32:
      hipLaunchKernelGGL((region_phase_batch<TX, TQ, 32, 33, KAHAN>), dim3(grid), dim3(128), 0, s,
                         d, ctl, items, cnt, q);
      break;
    default: return SMRE_EINVAL;
  }
  HIP_OK(hipGetLastError());
  return SMRE_OK;
}

template <typename TX, typename TQ, bool KAHAN>
int grid_for_batch(smre_ctx* c, int R, int SI, int want) {
  switch (R) {
    case 8: return batch_grid<TX, TQ, 8, 9, KAHAN>(c->cus, want);
    case 16:
      return SI == 9 ? batch_grid<TX, TQ, 16, 9, KAHAN>(c->cus, want)
                     : batch_grid<TX, TQ, 16, 17, KAHAN>(c->cus, want);
    default: return batch_grid<TX, TQ, 32, 33, KAHAN>(c->cus, want);
  }
}

// Everything one batched sweep needs, already on the device.
struct BatchDev {
  ImageDesc* desc;
  BatchCtl* ctl;
  WorkItem* items[4];
  int* cnt;       // cnt[0..3] items per colour, cnt[4] sweeps done, cnt[5] active images
  unsigned char* q;
  void* prev;
  int grid[4];
  int n;
  int maxh;
};

template <typename TX>
int enqueue_batch_sweep(smre_dtype dt, const smre_batch_params* bp, int R, int SI,
                        const BatchDev& D, bool check, hipStream_t s) {
  (void)dt;
  const dim3 cg(std::max(1, std::min(64, D.maxh)), D.n);
  if (check)
    hipLaunchKernelGGL((snapshot_batch<TX>), cg, dim3(256), 0, s, D.desc, D.ctl, (TX*)D.prev);
  for (int color = 0; color < 4; ++color) {
    int rc;
    if (sizeof(TX) == 8)
      rc = launch_batch_phase<double, double, false>(R, SI, D.grid[color], D.desc, D.ctl,
                                                     D.items[color], D.cnt + color, D.q, s);
    else if (bp->inc == SMRE_INC_BF16)
      rc = bp->kahan ? launch_batch_phase<float, bf16_t, true>(R, SI, D.grid[color], D.desc, D.ctl,
                                                                D.items[color], D.cnt + color, D.q, s)
                     : launch_batch_phase<float, bf16_t, false>(R, SI, D.grid[color], D.desc, D.ctl,
                                                                 D.items[color], D.cnt + color, D.q, s);
    else
      rc = bp->kahan ? launch_batch_phase<float, float, true>(R, SI, D.grid[color], D.desc, D.ctl,
                                                               D.items[color], D.cnt + color, D.q, s)
                     : launch_batch_phase<float, float, false>(R, SI, D.grid[color], D.desc, D.ctl,
                                                                D.items[color], D.cnt + color, D.q, s);
    if (rc) return rc;
  }
  if (check)
    hipLaunchKernelGGL((delta_batch<TX>), cg, dim3(256), 0, s, D.desc, D.ctl, (const TX*)D.prev);
  hipLaunchKernelGGL(decide_batch, dim3(1), dim3(256), 0, s, D.ctl, D.n, check ? 1 : 0, D.cnt + 4);
  HIP_OK(hipGetLastError());
  return SMRE_OK;
}

// Upload descriptors, control blocks and work lists for region side R; zero
// the increments.  Host staging lives in `host` until the stream is synced.
template <typename TX>
int batch_setup(smre_ctx* c, smre_dtype dt, int n, const smre_batch_image* im,
                const smre_batch_params* bp, const BatchPlan& B, unsigned char* ws,
                std::vector<unsigned char>& host, BatchDev* D, hipStream_t s) {
  (void)c;
  const size_t es = (bp->inc == SMRE_INC_BF16) ? 2 : sizeof(TX);
  (void)es;
  int64_t items_total = 0;
  for (int c2 = 0; c2 < 4; ++c2) items_total += B.nitems[c2];
  host.assign(B.off_prev - B.off_roff, 0);
  unsigned char* h = host.data();
  unsigned char* meta = h;
  ImageDesc* desc = (ImageDesc*)(h + (B.off_desc - B.off_roff));
  BatchCtl* ctl = (BatchCtl*)(h + (B.off_ctl - B.off_roff));
  WorkItem* items = (WorkItem*)(h + (B.off_items - B.off_roff));
  int* cnt = (int*)(h + (B.off_cnt - B.off_roff));
  int64_t base[4] = {0, B.nitems[0], B.nitems[0] + B.nitems[1],
                     B.nitems[0] + B.nitems[1] + B.nitems[2]};
  int64_t fill[4] = {0, 0, 0, 0};
  D->maxh = 1;
  for (int i = 0; i < n; ++i) {
    const Plan& pl = B.plans[i];
    std::memcpy(meta + B.roff_off[i], pl.meta.data(), pl.meta.size());
    ImageDesc& a = desc[i];
    a.x = im[i].x;
    a.rs = (const RegionStream*)(ws + B.off_roff + B.roff_off[i]);
    a.rtab = (const RoundEntry*)(ws + B.off_roff + B.roff_off[i] + pl.meta_rtab);
    a.ld = im[i].ld;
    a.q_byte = (int64_t)B.qoff[i];
    a.H = (int)im[i].H;
    a.W = (int)im[i].W;
    a.nrx = pl.nrx;
    a.nry = pl.nry;
    a.fr = pl.R + pl.smax - 1;
    a.nsides = pl.nsides;
    a.guard = (float)bp->guard_rel;
    for (int k = 0; k < pl.nsides; ++k) {
      a.sides[k] = pl.sides[k];
      a.r2f[k] = (float)pl.r2[k];
      a.rf[k] = (float)std::sqrt(pl.r2[k]);
      a.r2d[k] = pl.r2[k];
    }
    BatchCtl& cl = ctl[i];
    cl.done = 0;
    cl.done_sweep = 0;
    cl.converged = 0;
    cl.max_sweeps = im[i].max_sweeps;
    cl.sweeps = 0;
    cl.check_every = bp->check_every;
    cl.delta_key = 0;
    cl.last_delta = -1.0;
    cl.tol = im[i].tol;
    cl.prev_off = B.prev_off[i];
    for (int ry = 0; ry < pl.nry; ++ry)
      for (int rx = 0; rx < pl.nrx; ++rx) {
        const int col = (ry & 1) * 2 + (rx & 1);
        items[base[col] + fill[col]++] = WorkItem{i, ry * pl.nrx + rx};
      }
    D->maxh = std::max(D->maxh, (int)im[i].H);
  }
  for (int c2 = 0; c2 < 4; ++c2) cnt[c2] = B.nitems[c2];
  cnt[4] = 0;
  cnt[5] = n;
  HIP_OK(hipMemcpyAsync(ws + B.off_roff, h, host.size(), hipMemcpyHostToDevice, s));
  const int64_t nwords = (int64_t)(B.qbytes / 4);
  hipLaunchKernelGGL((fill_kernel<uint32_t>), dim3(grid_for(nwords)), dim3(256), 0, s,
                     (uint32_t*)ws, nwords, 0u);
  HIP_OK(hipGetLastError());
  D->desc = (ImageDesc*)(ws + B.off_desc);
  D->ctl = (BatchCtl*)(ws + B.off_ctl);
  for (int c2 = 0; c2 < 4; ++c2) D->items[c2] = (WorkItem*)(ws + B.off_items) + base[c2];
  D->cnt = (int*)(ws + B.off_cnt);
  D->q = ws;
  D->prev = ws + B.off_prev;
  D->n = n;
  for (int c2 = 0; c2 < 4; ++c2) {
    int g;
    if (sizeof(TX) == 8) g = grid_for_batch<double, double, false>(c, B.R, B.SI, B.nitems[c2]);
    else if (bp->inc == SMRE_INC_BF16)
      g = grid_for_batch<float, bf16_t, true>(c, B.R, B.SI, B.nitems[c2]);
    else g = grid_for_batch<float, float, true>(c, B.R, B.SI, B.nitems[c2]);
    if (bp->grid > 0) g = std::min(bp->grid, std::max(1, B.nitems[c2]));
    D->grid[c2] = std::max(1, g);
  }
  return SMRE_OK;
}

int batch_validate(smre_dtype dt, int n, const smre_batch_image* im, const smre_batch_params* bp,
                   int* smax) {
  if (n < 1 || !im || !bp) return SMRE_EINVAL;
  if (dt != SMRE_F32 && dt != SMRE_F64) return SMRE_EINVAL;
  if (bp->check_every < 1 || bp->grid < 0) return SMRE_EINVAL;
  if (bp->region != 0 && bp->region != 8 && bp->region != 16 && bp->region != 32)
    return SMRE_EINVAL;
  *smax = 0;
  for (int i = 0; i < n; ++i) {
    if (im[i].n_sides < 1 || !im[i].sides) return SMRE_EINVAL;
    for (int k = 0; k < im[i].n_sides; ++k) *smax = std::max(*smax, im[i].sides[k]);
  }
  return SMRE_OK;
}

std::vector<int> region_candidates(int smax, int requested) {
  if (requested) return {requested};
  std::vector<int> v;
  for (int R : {8, 16, 32})
    if (R >= smax - 1) v.push_back(R);
  if (v.size() > 2) v.resize(2);
  return v;
}

// Workspace of a batch: the largest layout over the tuner's candidates, then
// (when there is more than one candidate) room to save the inputs while the
// tuner runs.  *tune_off receives the start of that room.
size_t batch_bytes(smre_dtype dt, int n, const smre_batch_image* im, const smre_batch_params* bp,
                   int smax, size_t* tune_off) {
  size_t best = 0, prev = 0;
  const std::vector<int> cands = region_candidates(smax, bp->region);
  for (int R : cands) {
    BatchPlan B;
    if (plan_batch(dt, n, im, bp, R, &B, false)) return 0;
    best = std::max(best, B.total);
    prev = B.prev_elems * (dt == SMRE_F64 ? 8 : 4);
  }
  best = align_up(best, 256);
  if (tune_off) *tune_off = best;
  return cands.size() > 1 ? best + align_up(prev, 256) : best;
}

template <typename TX>
int batch_impl(smre_ctx* c, smre_dtype dt, int n, const smre_batch_image* im,
               const smre_batch_params* bp, unsigned char* ws, size_t ws_bytes, hipStream_t s,
               smre_report* reps) {
  int smax = 0;
  int rc = batch_validate(dt, n, im, bp, &smax);
  if (rc) return rc;
  // input check
  for (int i = 0; i < n; ++i) {
    hipLaunchKernelGGL(ctrl_reset_kernel, dim3(1), dim3(1), 0, s, c->ctrl);
    bool bad = false;
    rc = check_nonfinite<TX>(c, im[i].x, im[i].H, im[i].W, im[i].ld, s, &bad);
    if (rc) return rc;
    if (bad) return SMRE_ENONFINITE;
  }
  HIP_OK(hipEventRecord(c->t0, s));
  // region side: requested, cached, or tuned on a scratch run of two sweeps
  std::vector<int> cands = region_candidates(smax, bp->region);
  char keyb[160];
  snprintf(keyb, sizeof keyb, "dt%d inc%d k%d smax%d n%d", (int)dt, bp->inc, bp->kahan, smax, n);
  std::string key(keyb);
  int R = cands[0];
  std::vector<unsigned char> host;
  BatchPlan B;
  BatchDev D;
  if (cands.size() > 1 && c->tuned.count(key)) {
    R = c->tuned[key];
  } else if (cands.size() > 1) {
    // save the inputs, time two sweeps per candidate, restore
    size_t tune_off = 0;
    if (batch_bytes(dt, n, im, bp, smax, &tune_off) > ws_bytes) return SMRE_ENOMEM;
    std::vector<TX*> saved(n);
    size_t off = 0;
    for (int i = 0; i < n; ++i) {
      saved[i] = (TX*)(ws + tune_off) + off;
      off += (size_t)(im[i].H * im[i].W);
    }
    float best = 1e30f;
    for (int Rc : cands) {
      rc = plan_batch(dt, n, im, bp, Rc, &B, true);
      if (rc) return rc;
      if (B.total > ws_bytes) return SMRE_ENOMEM;
      for (int i = 0; i < n; ++i)
        HIP_OK(hipMemcpy2DAsync(saved[i], im[i].W * sizeof(TX), im[i].x, im[i].ld * sizeof(TX),
                                im[i].W * sizeof(TX), im[i].H, hipMemcpyDeviceToDevice, s));
      rc = batch_setup<TX>(c, dt, n, im, bp, B, ws, host, &D, s);
      if (rc) return rc;
      // the snapshot buffer holds the saved inputs: sweep without checks
      hipEvent_t e0 = c->ev[0], e1 = c->ev[1];
      HIP_OK(hipEventRecord(e0, s));
      for (int k = 0; k < 2; ++k) {
        rc = enqueue_batch_sweep<TX>(dt, bp, Rc, B.SI, D, false, s);
        if (rc) return rc;
      }
      HIP_OK(hipEventRecord(e1, s));
      HIP_OK(hipEventSynchronize(e1));
      float ms = 0.f;
      HIP_OK(hipEventElapsedTime(&ms, e0, e1));
      for (int i = 0; i < n; ++i)
        HIP_OK(hipMemcpy2DAsync(im[i].x, im[i].ld * sizeof(TX), saved[i], im[i].W * sizeof(TX),
                                im[i].W * sizeof(TX), im[i].H, hipMemcpyDeviceToDevice, s));
      if (ms < best) {
        best = ms;
        R = Rc;
      }
    }
    c->tuned[key] = R;
  }
  rc = plan_batch(dt, n, im, bp, R, &B, true);
  if (rc) return rc;
  if (B.total > ws_bytes) return SMRE_ENOMEM;
  rc = batch_setup<TX>(c, dt, n, im, bp, B, ws, host, &D, s);
  if (rc) return rc;

  int max_sw = 0;
  for (int i = 0; i < n; ++i) max_sw = std::max(max_sw, im[i].max_sweeps);
  // capture one plain and one checking sweep
  hipGraphExec_t gx[2] = {nullptr, nullptr};
  hipGraph_t gr[2] = {nullptr, nullptr};
  if (bp->use_graph) {
    HIP_OK(hipStreamSynchronize(s));
    for (int g = 0; g < 2; ++g) {
      HIP_OK(hipStreamBeginCapture(c->capture, hipStreamCaptureModeThreadLocal));
      int rc2 = enqueue_batch_sweep<TX>(dt, bp, R, B.SI, D, g == 1, c->capture);
      hipGraph_t graph = nullptr;
      HIP_OK(hipStreamEndCapture(c->capture, &graph));
      if (rc2) return rc2;
      gr[g] = graph;
      HIP_OK(hipGraphInstantiate(&gx[g], graph, nullptr, nullptr, 0));
    }
  }
  TimingAcc tacc;
  std::deque<std::pair<int, int>> inflight;
  int lag_slot = 0;
  bool host_done = false;
  for (int sweep = 1; sweep <= max_sw && !host_done; ++sweep) {
    const bool check = true;  // each image tests its own cadence on the device
    int slot;
    rc = timing_begin(c, tacc, s, &slot);
    if (rc) return rc;
    if (bp->use_graph) {
      HIP_OK(hipGraphLaunch(gx[check ? 1 : 0], s));
    } else {
      rc = enqueue_batch_sweep<TX>(dt, bp, R, B.SI, D, check, s);
      if (rc) return rc;
    }
    rc = timing_end(c, tacc, s, slot);
    if (rc) return rc;
    HIP_OK(hipMemcpyAsync(c->counters_host + 2 * lag_slot, D.cnt + 4, 2 * sizeof(int),
                          hipMemcpyDeviceToHost, s));
    HIP_OK(hipEventRecord(c->lag_ev[lag_slot], s));
    inflight.push_back({lag_slot, sweep});
    lag_slot = (lag_slot + 1) % (kLag + 1);
    if ((int)inflight.size() > kLag) {
      auto f = inflight.front();
      inflight.pop_front();
      HIP_OK(hipEventSynchronize(c->lag_ev[f.first]));
      if (c->counters_host[2 * f.first + 1] == 0) host_done = true;
    }
  }
  HIP_OK(hipStreamSynchronize(s));
  rc = timing_flush(c, tacc, true);
  if (rc) return rc;
  for (int g = 0; g < 2; ++g) {
    if (gx[g]) (void)hipGraphExecDestroy(gx[g]);
    if (gr[g]) (void)hipGraphDestroy(gr[g]);
  }
  std::vector<BatchCtl> ctl(n);
  HIP_OK(hipMemcpy(ctl.data(), D.ctl, sizeof(BatchCtl) * n, hipMemcpyDeviceToHost));
  for (int i = 0; i < n; ++i)
    if (ctl[i].aborted) return SMRE_EDEVICE;  // a wait gave up: results not trustworthy
  HIP_OK(hipEventRecord(c->t1, s));
  HIP_OK(hipEventSynchronize(c->t1));
  float ms = 0.f;
  HIP_OK(hipEventElapsedTime(&ms, c->t0, c->t1));
  bool all_conv = true;
  for (int i = 0; i < n; ++i) {
    const Plan& pl = B.plans[i];
    const int sw = ctl[i].done ? ctl[i].done_sweep : max_sw;
    if (im[i].tol > 0 && !ctl[i].converged) all_conv = false;
    if (reps) {
      smre_report& r = reps[i];
      double viol = 0.0;
      rc = run_violation<TX>(c, im[i].x, im[i].H, im[i].W, im[i].ld, pl.nsides, pl.sides, pl.r2,
                             s, &viol);
      if (rc) return rc;
      const size_t es = (bp->inc == SMRE_INC_BF16) ? 2 : sizeof(TX);
      r.sweeps = sw;
      r.converged = ctl[i].converged;
      r.region = R;
      r.inner_sweeps = 0;
      r.last_delta = ctl[i].last_delta;
      r.max_violation = viol;
      r.elapsed_ms = ms;
      r.kernel_ms = tacc.ms;
      r.kernel_launches = tacc.launches;
      r.bytes_moved = (double)sw * (2.0 * es * (double)pl.nq + 2.0 * sizeof(TX) * (double)(im[i].H * im[i].W));
      r.window_projections = (double)sw * (double)pl.nwin;
      r.pixel_updates = (double)sw * (double)pl.nq;
    }
  }
  return all_conv ? SMRE_OK : SMRE_NOT_CONVERGED;
}

// ---------------------------------------------------------------- serving
// HIP backend of the continuous-batching server (scheduler: serve_core.hpp).
// One device arena holds every admitted request's image, snapshot, region
// table and increments; descriptors and control blocks sit in fixed slot
// tables, so a single captured graph (snapshot, four persistent colour
// launches over the current work lists, delta, decide) serves every sweep
// whatever the mix.  Requests join between sweeps; a finished request is
// retired one sweep after its flag is set (its items are skipped meanwhile).
class Arena {
 public:
  void reset(size_t total) {
    free_.clear();
    free_[0] = total;
  }
  bool alloc(size_t n, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n, at = it->first + n;
        free_.erase(it);
        if (rest) free_[at] = rest;
        return true;
      }
    return false;
  }
  void release(size_t off, size_t n) {
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<size_t, size_t> free_;
};

class HipBackend : public smre_serve::Backend {
 public:
  explicit HipBackend(const smre_serve_config& c) : cfg_(c) {}
  ~HipBackend() override {
    (void)hipSetDevice(cfg_.device);
    if (stream_) (void)hipStreamSynchronize(stream_);
    if (gx_) (void)hipGraphExecDestroy(gx_);
    if (graph_) (void)hipGraphDestroy(graph_);
    if (arena_) (void)hipFree(arena_);
    if (tables_) (void)hipFree(tables_);
    if (hctl_) (void)hipHostFree(hctl_);
    if (hitems_) (void)hipHostFree(hitems_);
    for (auto& e : ev_)
      if (e) (void)hipEventDestroy(e);
    if (stream_) (void)hipStreamDestroy(stream_);
  }

  int init() {
    HIP_OK(hipSetDevice(cfg_.device));
    HIP_OK(hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking));
    size_t fr = 0, tot = 0;
    HIP_OK(hipMemGetInfo(&fr, &tot));
    size_t budget = cfg_.hbm_budget_bytes ? cfg_.hbm_budget_bytes : (size_t)(fr * 0.8);
    n_ = std::max(1, cfg_.max_active);
    const size_t tbl = align_up(sizeof(ImageDesc) * n_, 256) + align_up(sizeof(BatchCtl) * n_, 256) +
                       4 * align_up(sizeof(WorkItem) * kCapItems, 256) + 256 +
                       align_up(sizeof(Ctrl), 256);
    if (budget <= tbl + (1 << 20)) return SMRE_EINVAL;
    budget -= tbl;
    if (hipMalloc(&arena_, budget) != hipSuccess) {
      (void)hipGetLastError();
      return SMRE_ENOMEM;
    }
    arena_size_ = budget;
    free_.reset(budget);
    HIP_OK(hipMalloc(&tables_, tbl));
    unsigned char* t = (unsigned char*)tables_;
    desc_ = (ImageDesc*)t;
    t += align_up(sizeof(ImageDesc) * n_, 256);
    ctl_ = (BatchCtl*)t;
    t += align_up(sizeof(BatchCtl) * n_, 256);
    for (int c = 0; c < 4; ++c) {
      items_[c] = (WorkItem*)t;
      t += align_up(sizeof(WorkItem) * kCapItems, 256);
    }
    cnt_ = (int*)t;
    t += 256;
    vctrl_ = (Ctrl*)t;
    HIP_OK(hipHostMalloc(&hctl_, sizeof(BatchCtl) * n_ * 2, hipHostMallocDefault));
    HIP_OK(hipHostMalloc(&hitems_, sizeof(WorkItem) * kCapItems * 4 + 64, hipHostMallocDefault));
    for (auto& e : ev_) HIP_OK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    // every slot starts retired
    std::vector<BatchCtl> c0(n_);
    for (auto& c : c0) {
      std::memset(&c, 0, sizeof c);
      c.done = 1;
      c.check_every = 1;
    }
    HIP_OK(hipMemcpy(ctl_, c0.data(), sizeof(BatchCtl) * n_, hipMemcpyHostToDevice));
    HIP_OK(hipMemset(cnt_, 0, 64));
    slot_.assign(n_, Slot());
    int occ = 0;
    if (cfg_.inc == SMRE_INC_BF16)
      HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &occ, (const void*)region_phase_batch<float, bf16_t, 16, 17, true>, 128, 0));
    else
      HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &occ, (const void*)region_phase_batch<float, float, 16, 17, true>, 128, 0));
    hipDeviceProp_t prop;
    HIP_OK(hipGetDeviceProperties(&prop, cfg_.device));
    BatchDev D;
    D.desc = desc_;
    D.ctl = ctl_;
    for (int c = 0; c < 4; ++c) {
      D.items[c] = items_[c];
      D.grid[c] = std::max(1, occ) * prop.multiProcessorCount;
    }
    D.cnt = cnt_;
    D.q = (unsigned char*)arena_;
    D.prev = arena_;  // per-image snapshots are addressed through prev_off
    D.n = n_;
    D.maxh = 1024;
    smre_batch_params bp{};
    bp.region = 16;
    bp.inc = cfg_.inc;
    bp.kahan = cfg_.kahan;
    bp.check_every = 1;
    bp.guard_rel = cfg_.guard_rel;
    HIP_OK(hipStreamBeginCapture(stream_, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue_batch_sweep<float>(SMRE_F32, &bp, 16, 17, D, true, stream_);
    HIP_OK(hipStreamEndCapture(stream_, &graph_));
    if (rc) return rc;
    HIP_OK(hipGraphInstantiate(&gx_, graph_, nullptr, nullptr, 0));
    return SMRE_OK;
  }

  int slots() const override { return n_; }
  size_t budget() const override { return arena_size_; }

  size_t footprint(const smre_serve::Request& r) const override {
    Plan pl;
    smre_params p = params_of(r);
    if (plan_project(SMRE_F32, r.H, r.W, &p, &pl, false, 17)) return 0;
    return layout(pl, r, nullptr);
  }

  int admit(smre_serve::Request& r, int s) override {
    Slot& sl = slot_[s];
    smre_params p = params_of(r);
    sl.plan = Plan();
    int rc = plan_project(SMRE_F32, r.H, r.W, &p, &sl.plan, true, 17);
    if (rc) return rc;
    size_t off_roff, off_x, off_prev;
    size_t offs[3];
    const size_t need = layout(sl.plan, r, offs);
    off_roff = offs[0];
    off_x = offs[1];
    off_prev = offs[2];
    size_t at = 0;
    if (!free_.alloc(need, &at)) return SMRE_ENOMEM;
    sl.off = at;
    sl.size = need;
    unsigned char* base = (unsigned char*)arena_ + at;
    HIP_OK(hipSetDevice(cfg_.device));
    HIP_OK(hipMemcpyAsync(base + off_x, r.in.data(), r.in.size() * sizeof(float),
                          hipMemcpyHostToDevice, stream_));
    HIP_OK(hipMemcpyAsync(base + off_roff, sl.plan.meta.data(), sl.plan.meta.size(),
                          hipMemcpyHostToDevice, stream_));
    const int64_t nwords = (int64_t)(sl.plan.qbytes / 4);
    hipLaunchKernelGGL((fill_kernel<uint32_t>), dim3(grid_for(nwords)), dim3(256), 0, stream_,
                       (uint32_t*)base, nwords, 0u);
    HIP_OK(hipGetLastError());
    ImageDesc& a = sl.desc;
    std::memset(&a, 0, sizeof a);
    a.x = base + off_x;
    a.rs = (const RegionStream*)(base + off_roff);
    a.rtab = (const RoundEntry*)(base + off_roff + sl.plan.meta_rtab);
    a.ld = r.W;
    a.q_byte = (int64_t)at;
    a.H = r.H;
    a.W = r.W;
    a.nrx = sl.plan.nrx;
    a.nry = sl.plan.nry;
    a.fr = sl.plan.R + sl.plan.smax - 1;
    a.nsides = sl.plan.nsides;
    a.guard = (float)cfg_.guard_rel;
    for (int k = 0; k < sl.plan.nsides; ++k) {
      a.sides[k] = sl.plan.sides[k];
      a.r2f[k] = (float)sl.plan.r2[k];
      a.rf[k] = (float)std::sqrt(sl.plan.r2[k]);
      a.r2d[k] = sl.plan.r2[k];
    }
    BatchCtl& c = sl.ctl;
    std::memset(&c, 0, sizeof c);
    c.max_sweeps = r.max_sweeps;
    c.check_every = std::max(1, cfg_.check_every);
    c.tol = r.tol;
    c.last_delta = -1.0;
    c.prev_off = (int64_t)((at + off_prev) / sizeof(float));
    c.gen = ++generation_;
    HIP_OK(hipMemcpyAsync(desc_ + s, &sl.desc, sizeof(ImageDesc), hipMemcpyHostToDevice, stream_));
    HIP_OK(hipMemcpyAsync(ctl_ + s, &sl.ctl, sizeof(BatchCtl), hipMemcpyHostToDevice, stream_));
    HIP_OK(hipStreamSynchronize(stream_));  // host staging (r.in, plan, desc) released safely
    sl.active = true;
    sl.reported = false;
    sl.t_admit = smre_serve::now_s();
    dirty_ = true;
    return SMRE_OK;
  }

  int step(std::vector<int>& fin) override {
    HIP_OK(hipSetDevice(cfg_.device));
    if (dirty_) {
      int rc = upload_lists();
      if (rc) return rc;
    }
    HIP_OK(hipGraphLaunch(gx_, stream_));
    const int k = parity_;
    HIP_OK(hipMemcpyAsync(hctl_ + k * n_, ctl_, sizeof(BatchCtl) * n_, hipMemcpyDeviceToHost,
                          stream_));
    HIP_OK(hipEventRecord(ev_[k], stream_));
    parity_ ^= 1;
    // read the control blocks of the previous sweep (one sweep of lag)
    const int pk = parity_;
    if (have_prev_) {
      HIP_OK(hipEventSynchronize(ev_[pk]));
      for (int i = 0; i < n_; ++i) {
        Slot& sl = slot_[i];
        if (sl.active && !sl.reported && sl.finished_in(hctl_[pk * n_ + i])) {
          sl.last = hctl_[pk * n_ + i];
          sl.reported = true;
          fin.push_back(i);
        }
      }
    }
    have_prev_ = true;
    return SMRE_OK;
  }

  int retire(smre_serve::Request& r, int s) override {
    Slot& sl = slot_[s];
    HIP_OK(hipSetDevice(cfg_.device));
    // the sweep in flight skips this image (done flag), so x is final
    r.out.resize((size_t)r.H * r.W);
    HIP_OK(hipMemcpyAsync(r.out.data(), sl.desc.x, r.out.size() * sizeof(float),
                          hipMemcpyDeviceToHost, stream_));
    HIP_OK(hipStreamSynchronize(stream_));
    std::memset(&r.rep, 0, sizeof r.rep);
    // a wait of one of this request's region jobs gave up: its result alone
    // is not trustworthy
    if (sl.last.aborted) r.failed_alone = SMRE_EDEVICE;
    r.rep.sweeps = sl.last.done_sweep;
    r.rep.converged = sl.last.converged;
    r.rep.region = 16;
    r.rep.last_delta = sl.last.last_delta;
    double worst = 0.0;
    hipLaunchKernelGGL(ctrl_reset_kernel, dim3(1), dim3(1), 0, stream_, vctrl_);
    const int vrc = enqueue_feasibility<float>(sl.desc.x, r.H, r.W, r.W, 0, 1, sl.plan.nsides,
                                               sl.plan.sides, sl.plan.r2, vctrl_, stream_);
    if (vrc) return vrc;
    Ctrl vc;
    HIP_OK(hipMemcpyAsync(&vc, vctrl_, sizeof(Ctrl), hipMemcpyDeviceToHost, stream_));
    HIP_OK(hipStreamSynchronize(stream_));
    worst = dkey_inv(vc.viol_key);
    r.rep.max_violation = worst;
    r.rep.elapsed_ms = (smre_serve::now_s() - sl.t_admit) * 1e3;
    r.rep.bytes_moved = (double)sl.last.done_sweep *
                        (2.0 * (cfg_.inc == SMRE_INC_BF16 ? 2 : 4) * (double)sl.plan.nq +
                         8.0 * (double)r.H * r.W);
    r.rep.window_projections = (double)sl.last.done_sweep * (double)sl.plan.nwin;
    r.rep.pixel_updates = (double)sl.last.done_sweep * (double)sl.plan.nq;
    free_.release(sl.off, sl.size);
    sl.active = false;
    dirty_ = true;
    return SMRE_OK;
  }

 private:
  static constexpr int kCapItems = 1 << 18;
  struct Slot {
    bool active = false, reported = false;
    size_t off = 0, size = 0;
    Plan plan;
    ImageDesc desc;
    BatchCtl ctl;
    BatchCtl last;
    double t_admit = 0;
    // a control-block copy belongs to this occupant and says it has finished
    bool finished_in(const BatchCtl& c) const { return c.done && c.gen == ctl.gen; }
  };

  smre_params params_of(const smre_serve::Request& r) const {
    smre_params p{};
    p.n_sides = (int)r.sides.size();
    p.sides = r.sides.data();
    p.radius2 = r.r2.data();
    p.tol = r.tol;
    p.max_sweeps = r.max_sweeps;
    p.check_every = std::max(1, cfg_.check_every);
    p.region = 16;
    p.inc = cfg_.inc;
    p.kahan = cfg_.kahan;
    p.guard_rel = cfg_.guard_rel;
    return p;
  }

  // bytes of one request's block: increments (+ slack), region table, image, snapshot
  // A request's slab: increments (page-aligned, first), region offsets, x,
  // snapshot.  Sizes are whole pages so every slab starts on a page.
  size_t layout(const Plan& pl, const smre_serve::Request& r, size_t* offs) const {
    size_t o = align_up(pl.qbytes, kPage);
    if (offs) offs[0] = o;
    o = align_up(o + pl.meta_bytes, 256);
    if (offs) offs[1] = o;
    o = align_up(o + (size_t)r.H * r.W * 4, 256);
    if (offs) offs[2] = o;
    o = align_up(o + (size_t)r.H * r.W * 4, kPage);
    return o;
  }

  int upload_lists() {
    // the previous upload's staging must be consumed before it is rewritten
    HIP_OK(hipStreamSynchronize(stream_));
    int cnt[6] = {0, 0, 0, 0, 0, 0};
    WorkItem* h = hitems_;
    for (int i = 0; i < n_; ++i) {
      const Slot& sl = slot_[i];
      if (!sl.active || sl.reported) continue;
      for (int ry = 0; ry < sl.plan.nry; ++ry)
        for (int rx = 0; rx < sl.plan.nrx; ++rx) {
          const int c = (ry & 1) * 2 + (rx & 1);
          if (cnt[c] >= kCapItems) return SMRE_ENOMEM;
          h[c * kCapItems + cnt[c]++] = WorkItem{i, ry * sl.plan.nrx + rx};
        }
    }
    for (int c = 0; c < 4; ++c)
      if (cnt[c])
        HIP_OK(hipMemcpyAsync(items_[c], h + c * kCapItems, sizeof(WorkItem) * cnt[c],
                              hipMemcpyHostToDevice, stream_));
    std::memcpy(hitems_ + 4 * kCapItems, cnt, 4 * sizeof(int));
    HIP_OK(hipMemcpyAsync(cnt_, hitems_ + 4 * kCapItems, 4 * sizeof(int), hipMemcpyHostToDevice,
                          stream_));
    dirty_ = false;
    return SMRE_OK;
  }

  smre_serve_config cfg_;
  int n_ = 0;
  hipStream_t stream_ = nullptr;
  void* arena_ = nullptr;
  size_t arena_size_ = 0;
  Arena free_;
  void* tables_ = nullptr;
  ImageDesc* desc_ = nullptr;
  BatchCtl* ctl_ = nullptr;
  WorkItem* items_[4] = {};
  int* cnt_ = nullptr;
  Ctrl* vctrl_ = nullptr;  // feasibility check of a retiring request
  BatchCtl* hctl_ = nullptr;
  WorkItem* hitems_ = nullptr;
  hipEvent_t ev_[2] = {};
  int parity_ = 0;
  bool have_prev_ = false;
  bool dirty_ = false;
  int generation_ = 0;
  hipGraph_t graph_ = nullptr;
  hipGraphExec_t gx_ = nullptr;
  std::vector<Slot> slot_;
};

// ---------------------------------------------------------------- bounds
// Regularised lower incomplete gamma P(a, x): power series for x < a + 1,
// continued fraction (modified Lentz) for the complement otherwise.
double gamma_p(double a, double x) {
  if (x <= 0) return 0.0;
  const double lg = std::lgamma(a);
  if (x < a + 1.0) {
    double ap = a, sum = 1.0 / a, del = sum;
    for (int n = 0; n < 100000; ++n) {
      ap += 1.0;
      del *= x / ap;
      sum += del;
      if (std::fabs(del) < std::fabs(sum) * 1e-17) break;
    }
    return sum * std::exp(-x + a * std::log(x) - lg);
  }
  const double tiny = 1e-300;
  double b = x + 1.0 - a, cc = 1.0 / tiny, d = 1.0 / b, h = d;
  for (int i = 1; i < 100000; ++i) {
    const double an = -i * (i - a);
    b += 2.0;
    d = an * d + b;
    if (std::fabs(d) < tiny) d = tiny;
    cc = b + an / cc;
    if (std::fabs(cc) < tiny) cc = tiny;
    d = 1.0 / d;
    const double del = d * cc;
    h *= del;
    if (std::fabs(del - 1.0) < 1e-17) break;
  }
  return 1.0 - std::exp(-x + a * std::log(x) - lg) * h;
}

double chi2_quantile(int k, double p) {
  // Newton on P(k/2, x/2) = p from the Wilson-Hilferty start, bracketed.
  const double a = 0.5 * k;
  double lo = 0.0, hi = std::max(1.0, 4.0 * k + 100.0);
  while (gamma_p(a, 0.5 * hi) < p) hi *= 2;
  for (int i = 0; i < 80; ++i) {
    const double mid = 0.5 * (lo + hi);
    if (gamma_p(a, 0.5 * mid) < p) lo = mid; else hi = mid;
  }
  double x = 0.5 * (lo + hi);
  for (int i = 0; i < 20; ++i) {
    const double f = gamma_p(a, 0.5 * x) - p;
    const double pdf = std::exp((a - 1.0) * std::log(x) - 0.5 * x - a * std::log(2.0) - std::lgamma(a));
    if (!(pdf > 0)) break;
    const double xn = x - f / pdf;
    if (!(xn > 0) || std::fabs(xn - x) < 1e-16 * x) break;
    x = xn;
  }
  return x;
}

// ---------------------------------------------------------------- Monte-Carlo weights
constexpr int kMcChunk = 4096;  // fields per tile launch

int mc_sides(int32_t n, const int32_t* sides, int64_t H, int64_t W, McSides* sd) {
  if (!sides || n < 1 || n > kMcMaxSide) return SMRE_EINVAL;
  std::memset(sd, 0, sizeof(*sd));
  for (int s = 0; s <= kMcMaxSide; ++s) sd->slot[s] = -1;
  for (int k = 0; k < n; ++k) {
    const int s = sides[k];
    if (s < 1 || s > kMcMaxSide || s > H || s > W || sd->slot[s] >= 0) return SMRE_EINVAL;
    sd->slot[s] = k;
    sd->side[k] = s;
    sd->smax = std::max(sd->smax, s);
  }
  sd->n = n;
  return SMRE_OK;
}

int mc_check_shape(int64_t H, int64_t W, int64_t n_fields) {
  if (H < 1 || W < 1 || H > (1 << 20) || W > (1 << 20) || n_fields < 1) return SMRE_EINVAL;
  return SMRE_OK;
}

int mc_buffers(smre_ctx* c) {
  if (!c->mc_tmax) {
    HIP_OK(hipMalloc(&c->mc_tmax, sizeof(unsigned long long) * kMcChunk * kMcMaxSide));
    HIP_OK(hipMalloc(&c->mc_q, sizeof(double) * kMcChunk));
  }
  return SMRE_OK;
}

template <bool GEN, typename T, int SMAX>
void mc_tiles(const T* fields, int64_t fstride, int64_t ld, int H, int W, uint64_t seed,
              int64_t f0, int nf, const McSides& sd, unsigned long long* tmax, hipStream_t s) {
  constexpr int TR = mc_tile_rows(SMAX);
  const dim3 grid((unsigned)((W + kMcTileW - 1) / kMcTileW), (unsigned)((H + TR - 1) / TR),
                  (unsigned)nf);
  hipLaunchKernelGGL((mc_window_max<GEN, T, SMAX>), grid, dim3(256), 0, s, fields, fstride, ld, H,
                     W, seed, f0, sd, tmax);
}

// Q (and optionally the per-side maxima) of fields f0 .. f0 + nf - 1, drawn
// (GEN) or read from `fields`; results to host arrays.  Device buffers: tmax
// (min(nf, kMcChunk) * sd.n words) and q (min(nf, kMcChunk) doubles); acc may
// be null (no per-kernel timing).
template <bool GEN, typename T>
int mc_run_buf(smre_ctx* c, const T* fields, int64_t ld, int64_t H, int64_t W, uint64_t seed,
               int64_t f0, int64_t nf, const McSides& sd, double* q_out, double* tmax_out,
               hipStream_t s, TimingAcc* acc, unsigned long long* tmax, double* q) {
  int rc = SMRE_OK;
  const int64_t fstride = H * ld;
  for (int64_t done = 0; done < nf; done += kMcChunk) {
    const int m = (int)std::min<int64_t>(kMcChunk, nf - done);
    hipLaunchKernelGGL((fill_kernel<unsigned long long>), dim3(grid_for((int64_t)m * sd.n)),
                       dim3(256), 0, s, tmax, (int64_t)m * sd.n, 0ull);
    int slot = -1;
    if (acc && (rc = timing_begin(c, *acc, s, &slot))) return rc;
    const T* fp = GEN ? fields : fields + done * fstride;
    if (sd.smax <= 8)
      mc_tiles<GEN, T, 8>(fp, fstride, ld, (int)H, (int)W, seed, f0 + done, m, sd, tmax, s);
    else if (sd.smax <= 16)
      mc_tiles<GEN, T, 16>(fp, fstride, ld, (int)H, (int)W, seed, f0 + done, m, sd, tmax, s);
    else
      mc_tiles<GEN, T, 32>(fp, fstride, ld, (int)H, (int)W, seed, f0 + done, m, sd, tmax, s);
    HIP_OK(hipGetLastError());
    if (acc && (rc = timing_end(c, *acc, s, slot))) return rc;
    hipLaunchKernelGGL(mc_q_kernel, dim3((m + 255) / 256), dim3(256), 0, s, tmax, m, sd, q);
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(q_out + done, q, sizeof(double) * m, hipMemcpyDeviceToHost, s));
    if (tmax_out)
      HIP_OK(hipMemcpyAsync(tmax_out + done * sd.n, tmax, sizeof(double) * (size_t)m * sd.n,
                            hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));  // the buffers are reused by the next chunk
  }
  return acc ? timing_flush(c, *acc, true) : SMRE_OK;
}

template <bool GEN, typename T>
int mc_run(smre_ctx* c, const T* fields, int64_t ld, int64_t H, int64_t W, uint64_t seed,
           int64_t f0, int64_t nf, const McSides& sd, double* q_out, double* tmax_out,
           hipStream_t s, TimingAcc& acc) {
  int rc = mc_buffers(c);
  if (rc) return rc;
  return mc_run_buf<GEN, T>(c, fields, ld, H, W, seed, f0, nf, sd, q_out, tmax_out, s, &acc,
                            c->mc_tmax, c->mc_q);
}

void mc_report(smre_report* rep, const TimingAcc& acc, float ms, int64_t H, int64_t W,
               int64_t nf, const McSides& sd, double bytes) {
  if (!rep) return;
  std::memset(rep, 0, sizeof(*rep));
  double windows = 0.0;
  for (int k = 0; k < sd.n; ++k)
    windows += (double)(H - sd.side[k] + 1) * (double)(W - sd.side[k] + 1);
  rep->sweeps = 0;
  rep->converged = 1;
  rep->last_delta = NAN;
  rep->max_violation = NAN;
  rep->elapsed_ms = ms;
  rep->kernel_ms = acc.ms;
  rep->kernel_launches = acc.launches;
  rep->bytes_moved = bytes;
  rep->window_projections = windows * (double)nf;
}

int mc_statistic_gen(smre_ctx* c, int64_t H, int64_t W, const McSides& sd, uint64_t seed,
                     int64_t f0, int64_t nf, double* q_out, double* tmax_out, hipStream_t s,
                     smre_report* rep) {
  HIP_OK(hipEventRecord(c->t0, s));
  TimingAcc acc;
  int rc = mc_run<true, double>(c, nullptr, W, H, W, seed, f0, nf, sd, q_out, tmax_out, s, acc);
  if (rc) return rc;
  HIP_OK(hipEventRecord(c->t1, s));
  HIP_OK(hipEventSynchronize(c->t1));
  float ms = 0.f;
  HIP_OK(hipEventElapsedTime(&ms, c->t0, c->t1));
  mc_report(rep, acc, ms, H, W, nf, sd, 0.0);
  return SMRE_OK;
}

// ---------------------------------------------------------------- ADMM
int psf_weights(double sigma, PsfWeights* pw) {
  std::memset(pw, 0, sizeof(*pw));
  if (!(sigma >= 0) || !std::isfinite(sigma)) return SMRE_EINVAL;
  if (sigma == 0) {
    pw->R = 0;
    pw->w[0] = 1.0;
    return SMRE_OK;
  }
  const int R = (int)(4.0 * sigma + 0.5);
  if (R > kAdmmMaxRadius) return SMRE_EINVAL;
  double sum = 0.0;
  for (int k = -R; k <= R; ++k) sum += std::exp(-0.5 * (double)k * k / (sigma * sigma));
  for (int k = 0; k <= R; ++k) pw->w[k] = std::exp(-0.5 * (double)k * k / (sigma * sigma)) / sum;
  pw->R = R;
  return SMRE_OK;
}

template <typename T>
int blur(const T* in, T* tmp, T* out, int H, int W, const PsfWeights& pw, hipStream_t s) {
  hipLaunchKernelGGL((blur_rows<T>), dim3((W + 255) / 256, H), dim3(256), 0, s, in, tmp, H, W,
                     (int64_t)W, pw);
  hipLaunchKernelGGL((blur_cols<T>), dim3((W + 63) / 64, (H + kBlurColRows - 1) / kBlurColRows),
                     dim3(256), 0, s, tmp,
                     out, H, W, (int64_t)W, pw);
  HIP_OK(hipGetLastError());
  return SMRE_OK;
}

template <typename T>
int admm_impl(smre_ctx* c, smre_dtype dt, const T* I_user, T* x_user, int64_t H, int64_t W,
              int64_t ld, const smre_admm_params* p, T* eps_user, hipStream_t s,
              smre_admm_report* rep) {
  const double t_start = smre_serve::now_s();
  PsfWeights pw;
  int rc = psf_weights(p->sigma, &pw);
  if (rc) return rc;
  const int64_t n = H * W;
  const size_t img = align_up((size_t)n * sizeof(T), 256);
  const size_t need = 10 * img;
  if (c->admm_bytes < need) {
    if (c->admm_ws) HIP_OK(hipFree(c->admm_ws));
    c->admm_ws = nullptr;
    c->admm_bytes = 0;
    if (hipMalloc(&c->admm_ws, need) != hipSuccess) return SMRE_ENOMEM;
    c->admm_bytes = need;
  }
  if (!c->admm_slots)
    HIP_OK(hipMalloc(&c->admm_slots, sizeof(double) * 2 * kAdmmSlots * kAdmmSlotWords));
  unsigned char* base = (unsigned char*)c->admm_ws;
  T* I = (T*)(base + 0 * img);
  T* x = (T*)(base + 1 * img);
  T* z = (T*)(base + 2 * img);
  T* eps = (T*)(base + 3 * img);
  T* Y1 = (T*)(base + 4 * img);
  T* Y2 = (T*)(base + 5 * img);
  T* Ax = (T*)(base + 6 * img);
  T* t = (T*)(base + 7 * img);
  T* At = (T*)(base + 8 * img);
  T* tmp = (T*)(base + 9 * img);
  HIP_OK(hipMemcpy2DAsync(I, W * sizeof(T), I_user, ld * sizeof(T), W * sizeof(T), H,
                          hipMemcpyDeviceToDevice, s));
  // x = z = eps = Y1 = Y2 = 0, hence A x = 0
  hipLaunchKernelGGL((fill_kernel<T>), dim3(grid_for(6 * (int64_t)(img / sizeof(T)))), dim3(256),
                     0, s, x, (int64_t)(6 * (img / sizeof(T))), T(0));
  bool bad = false;
  rc = check_nonfinite<T>(c, I, H, W, W, s, &bad);
  if (rc) return rc;
  if (bad) return SMRE_ENONFINITE;
  AdmmCoef cf;
  cf.rho1 = p->rho1;
  cf.rho2 = p->rho2;
  cf.lam = p->lam;
  cf.alpha1 = p->alpha1;
  cf.alpha2 = p->alpha2;
  cf.inv2g = 1.0 / (2.0 * (p->gamma > 0 ? p->gamma : 0.5 * (p->rho1 + p->rho2)));
  double* slots_dx = c->admm_slots;
  double* slots_res = c->admm_slots + kAdmmSlots * kAdmmSlotWords;
  const int64_t nslot = 2 * kAdmmSlots * kAdmmSlotWords;
  std::vector<double> host((size_t)nslot);
  int32_t sy[6], sx[6], lo[6];
  for (int i = 0; i <= p->K && i < 6; ++i) {
    sy[i] = sx[i] = (1 << i) & ((1 << p->K) - 1);
    lo[i] = i;
  }
  const dim3 eg(grid_for(n)), eb(256);
  double proj_s = 0.0, dx = 0.0, res = 0.0;
  int64_t psweeps = 0;
  int it = 0;
  bool conv = false;
  for (it = 1; it <= p->max_iter; ++it) {
    hipLaunchKernelGGL((fill_kernel<double>), dim3(grid_for(nslot)), dim3(256), 0, s,
                       c->admm_slots, nslot, 0.0);
    hipLaunchKernelGGL((admm_coupling<T>), eg, eb, 0, s, n, I, Ax, eps, Y1, t, cf);
    rc = blur<T>(t, tmp, At, (int)H, (int)W, pw, s);
    if (rc) return rc;
    hipLaunchKernelGGL((admm_x_step<T>), eg, eb, 0, s, n, x, At, z, Y2, cf, slots_dx);
    rc = blur<T>(x, tmp, Ax, (int)H, (int)W, pw, s);
    if (rc) return rc;
    hipLaunchKernelGGL((admm_eps_input<T>), eg, eb, 0, s, n, I, Ax, Y1, eps, cf);
    HIP_OK(hipGetLastError());
    const double tp = smre_serve::now_s();
    smre_report pr;
    std::memset(&pr, 0, sizeof(pr));
    if (p->method == SMRE_ADMM_ICD) {
      rc = icd_impl<T>(c, eps, H, W, W, 1, p->K, p->radius2_icd, p->icd_tol, p->icd_tolmode,
                       p->icd_max_inner, p->K + 1, sy, sx, lo, s, &pr, false);
      if (rc != SMRE_OK && rc != SMRE_NOT_CONVERGED) return rc;  // a capped block is fine here
      psweeps += pr.inner_sweeps;
    } else {
      // every eps-step after the first may start from the previous one's
      // increments (the input moves little between iterations)
      smre_params fp = *p->full;
      fp.warm = (p->warm && it > 1) ? 1 : 0;
      rc = smre_dykstra_project(c, dt, eps, H, W, W, &fp, nullptr, 0, s, &pr);
      if (rc != SMRE_OK && rc != SMRE_NOT_CONVERGED) return rc;
      psweeps += pr.sweeps;
    }
    proj_s += smre_serve::now_s() - tp;
    hipLaunchKernelGGL((admm_finish<T>), eg, eb, 0, s, n, I, x, Ax, eps, z, Y1, Y2, cf,
                       slots_res);
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(host.data(), c->admm_slots, sizeof(double) * nslot,
                          hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    double sdx = 0.0, sres = 0.0;
    for (int k = 0; k < kAdmmSlots; ++k) {
      sdx += host[(size_t)k * kAdmmSlotWords];
      sres += host[(size_t)(kAdmmSlots + k) * kAdmmSlotWords];
    }
    dx = std::sqrt(sdx);
    res = std::sqrt(sres);
    if (dx <= p->delta && res <= p->delta) {
      conv = true;
      break;
    }
  }
  if (it > p->max_iter) it = p->max_iter;
  HIP_OK(hipMemcpy2DAsync(x_user, ld * sizeof(T), x, W * sizeof(T), W * sizeof(T), H,
                          hipMemcpyDeviceToDevice, s));
  if (eps_user)
    HIP_OK(hipMemcpy2DAsync(eps_user, ld * sizeof(T), eps, W * sizeof(T), W * sizeof(T), H,
                            hipMemcpyDeviceToDevice, s));
  HIP_OK(hipStreamSynchronize(s));
  if (rep) {
    rep->iterations = it;
    rep->converged = conv ? 1 : 0;
    rep->last_dx = dx;
    rep->last_residual = res;
    rep->elapsed_ms = (smre_serve::now_s() - t_start) * 1e3;
    rep->projection_ms = proj_s * 1e3;
    rep->projection_sweeps = psweeps;
  }
  return SMRE_OK;
}

}  // namespace

namespace {
int icd_validate(smre_ctx* c, smre_dtype dt, const void* x, int64_t H, int64_t W, int64_t ld,
                 int64_t frames, int32_t K, const double* r2, int32_t n_phases,
                 const int32_t* shift_y, const int32_t* shift_x, const int32_t* min_level,
                 double tol, int32_t mode, int32_t max_inner) {
  if (!c || !x || !r2 || !shift_y || !shift_x || !min_level) return SMRE_EINVAL;
  if (frames < 1 || frames * H > INT32_MAX) return SMRE_EINVAL;
  if (dt != SMRE_F32 && dt != SMRE_F64) return SMRE_EINVAL;
  if (H < 1 || W < 1 || ld < W || H > (1 << 20) || W > (1 << 20)) return SMRE_EINVAL;
  if (K < 0 || K > 5 || max_inner < 1 || n_phases < 1 || n_phases > 64) return SMRE_EINVAL;
  {
    // blocks of one frame: within the grid limits and below 2^31 per launch
    const int64_t nbx = W / (1 << K) + 2, nby = H / (1 << K) + 2;
    if (nby > 65535 || nbx * nby >= ((int64_t)1 << 31)) return SMRE_EINVAL;
  }
  for (int p = 0; p < n_phases; ++p)
    if (shift_y[p] < 0 || shift_y[p] >= (1 << K) || shift_x[p] < 0 || shift_x[p] >= (1 << K) ||
        min_level[p] < 0 || min_level[p] > K)
      return SMRE_EINVAL;
  if (mode != SMRE_TOL_MAXABS && mode != SMRE_TOL_MEANABS) return SMRE_EINVAL;
  if (!std::isfinite(tol)) return SMRE_EINVAL;
  for (int k = 0; k <= K; ++k) {
    if (!std::isfinite(r2[k])) return SMRE_ENONFINITE;
    if (!(r2[k] > 0)) return SMRE_EINVAL;
  }
  return SMRE_OK;
}
}  // namespace

extern "C" {

const char* smre_status_string(int st) {
  switch (st) {
    case SMRE_OK: return "ok";
    case SMRE_NOT_CONVERGED: return "not converged (result written)";
    case SMRE_PENDING: return "pending";
    case SMRE_EINVAL: return "invalid argument";
    case SMRE_ENONFINITE: return "non-finite input";
    case SMRE_ENOMEM: return "out of device memory / workspace too small";
    case SMRE_ETOOBIG: return "request exceeds the memory budget";
    case SMRE_EBUSY: return "queue full";
    case SMRE_EDEVICE: return "HIP runtime error";
    case SMRE_ECANCELLED: return "cancelled";
    case SMRE_EUNKNOWN_TICKET: return "unknown ticket";
    default: return "unknown status";
  }
}

int smre_ctx_create(int device, smre_ctx** out) {
  if (!out) return SMRE_EINVAL;
  int n = 0;
  HIP_OK(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return SMRE_EINVAL;
  smre_ctx* c = new smre_ctx();
  c->device = device;
  int rc = set_device(c);
  if (!rc) rc = ensure_ctrl(c);
  if (!rc) rc = scratch_init(device);
  if (rc) {
    smre_ctx_destroy(c);
    return rc;
  }
  *out = c;
  return SMRE_OK;
}

void smre_ctx_destroy(smre_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->ws) (void)hipFree(c->ws);
  if (c->ctrl) (void)hipFree(c->ctrl);
  if (c->counter) (void)hipFree(c->counter);
  if (c->ctrl_host) (void)hipHostFree(c->ctrl_host);
  for (auto& e : c->lag_ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : c->ev)
    if (e) (void)hipEventDestroy(e);
  if (c->t0) (void)hipEventDestroy(c->t0);
  if (c->t1) (void)hipEventDestroy(c->t1);
  if (c->counters_host) (void)hipHostFree(c->counters_host);
  if (c->capture) (void)hipStreamDestroy(c->capture);
  if (c->icd_cnt) (void)hipFree(c->icd_cnt);
  if (c->admm_ws) (void)hipFree(c->admm_ws);
  if (c->admm_slots) (void)hipFree(c->admm_slots);
  if (c->mc_tmax) (void)hipFree(c->mc_tmax);
  if (c->mc_q) (void)hipFree(c->mc_q);
  delete c;
}

int smre_ctx_set_timing(smre_ctx* c, int every) {
  if (!c || every < 0) return SMRE_EINVAL;
  c->timing = every;
  return SMRE_OK;
}

int smre_chi2_bounds(const int32_t* sides, int32_t n, double p, double* out) {
  if (!sides || !out || n < 1 || !(p > 0) || !(p < 1)) return SMRE_EINVAL;
  for (int k = 0; k < n; ++k) {
    if (sides[k] < 1 || sides[k] > 4096) return SMRE_EINVAL;
    out[k] = chi2_quantile(sides[k] * sides[k], p);
  }
  return SMRE_OK;
}

int smre_paper_bounds(const int32_t* sides, int32_t n, double q, double* out) {
  if (!sides || !out || n < 1 || !std::isfinite(q)) return SMRE_EINVAL;
  for (int k = 0; k < n; ++k) {
    if (sides[k] < 1) return SMRE_EINVAL;
    const double np = (double)sides[k] * sides[k];
    const double mu = std::pow(np - 0.5, 0.25);
    const double sg = std::sqrt(1.0 / (8.0 * std::sqrt(np)));
    const double b = q * sg + mu;
    if (!(b > 0)) return SMRE_EINVAL;
    out[k] = b * b * b * b;
  }
  return SMRE_OK;
}

int smre_workspace_size(smre_dtype dt, int64_t H, int64_t W, const smre_params* p,
                        size_t* bytes) {
  if (!bytes) return SMRE_EINVAL;
  if (p && p->order != SMRE_ORDER_REGION) {
    CanonPlan cp;
    int rc = plan_canon(dt, H, W, p, &cp);
    if (rc) return rc;
    *bytes = cp.total;
    return SMRE_OK;
  }
  Plan pl;
  int rc = plan_project(dt, H, W, p, &pl, false);
  if (rc) return rc;
  *bytes = pl.total;
  return SMRE_OK;
}

int smre_dykstra_project(smre_ctx* c, smre_dtype dt, void* x, int64_t H, int64_t W, int64_t ld,
                         const smre_params* p, void* workspace, size_t ws_bytes, void* stream,
                         smre_report* rep) {
  if (!c || !x) return SMRE_EINVAL;
  if (ld < W) return SMRE_EINVAL;
  Plan pl;
  CanonPlan cp;
  const bool canon = p && p->order != SMRE_ORDER_REGION;
  int rc = canon ? plan_canon(dt, H, W, p, &cp) : plan_project(dt, H, W, p, &pl, true);
  if (rc) return rc;
  const size_t total = canon ? cp.total : pl.total;
  rc = set_device(c);
  if (rc) return rc;
  unsigned char* ws = (unsigned char*)workspace;
  if (ws) {
    if (ws_bytes < total) return SMRE_ENOMEM;
  } else {
    if (c->ws_bytes < total) {
      if (c->ws) HIP_OK(hipFree(c->ws));
      c->ws = nullptr;
      c->ws_bytes = 0;
      if (hipMalloc(&c->ws, total) != hipSuccess) {
        (void)hipGetLastError();
        return SMRE_ENOMEM;
      }
      c->ws_bytes = total;
    }
    ws = (unsigned char*)c->ws;
  }
  hipStream_t s = (hipStream_t)stream;
  if (canon) {
    if (dt == SMRE_F64) return canon_impl<double>(c, dt, x, H, W, ld, p, cp, ws, s, rep);
    return canon_impl<float>(c, dt, x, H, W, ld, p, cp, ws, s, rep);
  }
  if (dt == SMRE_F64) return project_impl<double>(c, dt, x, H, W, ld, p, pl, ws, s, rep);
  return project_impl<float>(c, dt, x, H, W, ld, p, pl, ws, s, rep);
}

int smre_dykstra_incomplete(smre_ctx* c, smre_dtype dt, void* x, int64_t H, int64_t W,
                            int64_t ld, int32_t K, const double* r2, double tol, int32_t mode,
                            int32_t max_inner, int32_t nph, void* stream, smre_report* rep) {
  return smre_dykstra_incomplete_frames(c, dt, x, H, W, ld, 1, K, r2, tol, mode, max_inner, nph,
                                        stream, rep);
}

int smre_dykstra_incomplete_frames(smre_ctx* c, smre_dtype dt, void* x, int64_t H, int64_t W,
                                   int64_t ld, int64_t frames, int32_t K, const double* r2,
                                   double tol, int32_t mode, int32_t max_inner, int32_t nph,
                                   void* stream, smre_report* rep) {
  if (K < 0 || K > 6 || nph < 1 || nph > K + 1) return SMRE_EINVAL;
  int32_t sy[7], sx[7], lo[7];
  for (int i = 0; i < nph; ++i) {
    sy[i] = sx[i] = (1 << i) & ((1 << K) - 1);
    lo[i] = i;
  }
  return smre_dykstra_incomplete_family(c, dt, x, H, W, ld, frames, K, r2, nph, sy, sx, lo, tol,
                                        mode, max_inner, stream, rep);
}

int smre_dykstra_incomplete_family(smre_ctx* c, smre_dtype dt, void* x, int64_t H, int64_t W,
                                   int64_t ld, int64_t frames, int32_t K, const double* r2,
                                   int32_t n_phases, const int32_t* shift_y,
                                   const int32_t* shift_x, const int32_t* min_level, double tol,
                                   int32_t mode, int32_t max_inner, void* stream,
                                   smre_report* rep) {
  if (K == 6) {
    // 64 x 64 blocks exceed one wave's registers: the nested-hierarchy kernel
    // with the chain 1, 2, ..., 64 runs them
    if (!r2) return SMRE_EINVAL;
    const int32_t chain[7] = {1, 2, 4, 8, 16, 32, 64};
    return smre_dykstra_incomplete_nested(c, dt, x, H, W, ld, frames, 7, chain, r2, n_phases,
                                          shift_y, shift_x, min_level, tol, mode, max_inner,
                                          stream, rep);
  }
  int rc = icd_validate(c, dt, x, H, W, ld, frames, K, r2, n_phases, shift_y, shift_x, min_level,
                        tol, mode, max_inner);
  if (rc) return rc;
  rc = set_device(c);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (dt == SMRE_F64)
    return icd_impl<double>(c, x, H, W, ld, frames, K, r2, tol, mode, max_inner, n_phases,
                            shift_y, shift_x, min_level, s, rep);
  return icd_impl<float>(c, x, H, W, ld, frames, K, r2, tol, mode, max_inner, n_phases, shift_y,
                         shift_x, min_level, s, rep);
}

int smre_dykstra_incomplete_nested(smre_ctx* c, smre_dtype dt, void* x, int64_t H, int64_t W,
                                   int64_t ld, int64_t frames, int32_t n_levels,
                                   const int32_t* level_side, const double* r2, int32_t n_phases,
                                   const int32_t* shift_y, const int32_t* shift_x,
                                   const int32_t* min_level, double tol, int32_t mode,
                                   int32_t max_inner, void* stream, smre_report* rep) {
  int rc = nested_validate(c, dt, x, H, W, ld, frames, n_levels, level_side, r2, n_phases,
                           shift_y, shift_x, min_level, tol, mode, max_inner);
  if (rc) return rc;
  rc = set_device(c);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (dt == SMRE_F64)
    return nested_impl<double>(c, x, H, W, ld, frames, n_levels, level_side, r2, tol, mode,
                               max_inner, n_phases, shift_y, shift_x, min_level, s, rep);
  return nested_impl<float>(c, x, H, W, ld, frames, n_levels, level_side, r2, tol, mode,
                            max_inner, n_phases, shift_y, shift_x, min_level, s, rep);
}

int smre_dykstra_incomplete_noalloc(smre_ctx* c, smre_dtype dt, void* x, int64_t H, int64_t W,
                                    int64_t ld, int32_t K, const double* r2, double tol,
                                    int32_t mode, int32_t max_inner, int32_t nph, void* stream,
                                    smre_report* rep) {
  if (K < 0 || K > 5 || nph < 1 || nph > K + 1) return SMRE_EINVAL;
  int32_t sy[6], sx[6], lo[6];
  for (int i = 0; i < nph; ++i) {
    sy[i] = sx[i] = (1 << i) & ((1 << K) - 1);
    lo[i] = i;
  }
  int rc = icd_validate(c, dt, x, H, W, ld, 1, K, r2, nph, sy, sx, lo, tol, mode, max_inner);
  if (rc) return rc;
  // the scratch holds the work counters, whatever the image size
  rc = set_device(c);
  if (rc) return rc;
  unsigned long long* base = scratch_of(c->device);
  if (!base) return SMRE_EDEVICE;  // set up when the context was created
  const IcdScratch fs{base};
  hipStream_t s = (hipStream_t)stream;
  if (dt == SMRE_F64)
    return icd_impl<double>(c, x, H, W, ld, 1, K, r2, tol, mode, max_inner, nph, sy, sx, lo, s,
                            rep, true, &fs);
  return icd_impl<float>(c, x, H, W, ld, 1, K, r2, tol, mode, max_inner, nph, sy, sx, lo, s, rep,
                         true, &fs);
}

int smre_batch_workspace_size(smre_dtype dt, int32_t n, const smre_batch_image* im,
                              const smre_batch_params* bp, size_t* bytes) {
  if (!bytes) return SMRE_EINVAL;
  int smax = 0;
  int rc = batch_validate(dt, n, im, bp, &smax);
  if (rc) return rc;
  *bytes = batch_bytes(dt, n, im, bp, smax, nullptr);
  return *bytes ? SMRE_OK : SMRE_EINVAL;
}

int smre_dykstra_project_batch(smre_ctx* c, smre_dtype dt, int32_t n, const smre_batch_image* im,
                               const smre_batch_params* bp, void* workspace, size_t ws_bytes,
                               void* stream, smre_report* reps) {
  if (!c) return SMRE_EINVAL;
  size_t need = 0;
  int rc = smre_batch_workspace_size(dt, n, im, bp, &need);
  if (rc) return rc;
  rc = set_device(c);
  if (rc) return rc;
  unsigned char* ws = (unsigned char*)workspace;
  if (ws) {
    if (ws_bytes < need) return SMRE_ENOMEM;
  } else {
    if (c->ws_bytes < need) {
      if (c->ws) HIP_OK(hipFree(c->ws));
      c->ws = nullptr;
      c->ws_bytes = 0;
      if (hipMalloc(&c->ws, need) != hipSuccess) {
        (void)hipGetLastError();
        return SMRE_ENOMEM;
      }
      c->ws_bytes = need;
    }
    ws = (unsigned char*)c->ws;
    ws_bytes = c->ws_bytes;
  }
  hipStream_t s = (hipStream_t)stream;
  if (dt == SMRE_F64) return batch_impl<double>(c, dt, n, im, bp, ws, ws_bytes, s, reps);
  return batch_impl<float>(c, dt, n, im, bp, ws, ws_bytes, s, reps);
}

int smre_max_violation(smre_ctx* c, smre_dtype dt, const void* x, int64_t H, int64_t W,
                       int64_t ld, int32_t n, const int32_t* sides, const double* r2,
                       void* stream, double* out) {
  if (!c || !x || !sides || !r2 || !out || n < 1) return SMRE_EINVAL;
  if (H < 1 || W < 1 || ld < W) return SMRE_EINVAL;
  for (int k = 0; k < n; ++k) {
    if (sides[k] < 1 || sides[k] > H || sides[k] > W || sides[k] > kViolMaxSide)
      return SMRE_EINVAL;
    if (!(r2[k] > 0) || !std::isfinite(r2[k])) return SMRE_EINVAL;
  }
  int rc = set_device(c);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(ctrl_reset_kernel, dim3(1), dim3(1), 0, s, c->ctrl);
  if (dt == SMRE_F64) return run_violation<double>(c, x, H, W, ld, n, sides, r2, s, out);
  if (dt == SMRE_F32) return run_violation<float>(c, x, H, W, ld, n, sides, r2, s, out);
  return SMRE_EINVAL;
}

int smre_mc_fields(smre_ctx* c, int64_t H, int64_t W, uint64_t seed, int64_t field0,
                   int64_t n_fields, double* out, int64_t ld, void* stream) {
  if (!c || !out || field0 < 0 || ld < W) return SMRE_EINVAL;
  int rc = mc_check_shape(H, W, n_fields);
  if (rc) return rc;
  rc = set_device(c);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const int64_t groups = (H * W + 3) / 4;
  const unsigned gx = (unsigned)std::max<int64_t>(1, std::min<int64_t>(1024, (groups + 255) / 256));
  for (int64_t done = 0; done < n_fields; done += 65535) {
    const unsigned m = (unsigned)std::min<int64_t>(65535, n_fields - done);
    hipLaunchKernelGGL(mc_fields_kernel, dim3(gx, m), dim3(256), 0, s, out + done * H * ld, H * ld,
                       ld, (int)H, (int)W, seed, field0 + done);
    HIP_OK(hipGetLastError());
  }
  HIP_OK(hipStreamSynchronize(s));
  return SMRE_OK;
}

int smre_mc_statistic(smre_ctx* c, int64_t H, int64_t W, int32_t n_sides, const int32_t* sides,
                      uint64_t seed, int64_t field0, int64_t n_fields, double* q_out,
                      double* tmax_out, void* stream, smre_report* report) {
  if (!c || !q_out || field0 < 0) return SMRE_EINVAL;
  int rc = mc_check_shape(H, W, n_fields);
  if (rc) return rc;
  McSides sd;
  rc = mc_sides(n_sides, sides, H, W, &sd);
  if (rc) return rc;
  rc = set_device(c);
  if (rc) return rc;
  return mc_statistic_gen(c, H, W, sd, seed, field0, n_fields, q_out, tmax_out,
                          (hipStream_t)stream, report);
}

int smre_mc_statistic_fields(smre_ctx* c, smre_dtype dt, const void* fields, int64_t H, int64_t W,
                             int64_t ld, int64_t n_fields, int32_t n_sides, const int32_t* sides,
                             double* q_out, double* tmax_out, void* stream) {
  if (!c || !fields || !q_out || ld < W) return SMRE_EINVAL;
  int rc = mc_check_shape(H, W, n_fields);
  if (rc) return rc;
  McSides sd;
  rc = mc_sides(n_sides, sides, H, W, &sd);
  if (rc) return rc;
  rc = set_device(c);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  TimingAcc acc;
  if (dt == SMRE_F64)
    return mc_run<false, double>(c, (const double*)fields, ld, H, W, 0, 0, n_fields, sd, q_out,
                                 tmax_out, s, acc);
  if (dt == SMRE_F32)
    return mc_run<false, float>(c, (const float*)fields, ld, H, W, 0, 0, n_fields, sd, q_out,
                                tmax_out, s, acc);
  return SMRE_EINVAL;
}

int smre_mc_quantile(smre_ctx* c, int64_t H, int64_t W, int32_t n_sides, const int32_t* sides,
                     uint64_t seed, int64_t n_fields, double alpha, double* q_alpha, void* stream,
                     smre_report* report) {
  if (!c || !q_alpha || !(alpha > 0.0) || alpha > 1.0) return SMRE_EINVAL;
  int rc = mc_check_shape(H, W, n_fields);
  if (rc) return rc;
  McSides sd;
  rc = mc_sides(n_sides, sides, H, W, &sd);
  if (rc) return rc;
  rc = set_device(c);
  if (rc) return rc;
  std::vector<double> q((size_t)n_fields);
  rc = mc_statistic_gen(c, H, W, sd, seed, 0, n_fields, q.data(), nullptr, (hipStream_t)stream,
                        report);
  if (rc) return rc;
  // the ceil(alpha n)-th smallest sample
  int64_t k = (int64_t)std::ceil(alpha * (double)n_fields);
  k = std::min<int64_t>(std::max<int64_t>(k, 1), n_fields);
  std::nth_element(q.begin(), q.begin() + (k - 1), q.end());
  *q_alpha = q[(size_t)(k - 1)];
  return SMRE_OK;
}

int smre_admm(smre_ctx* c, smre_dtype dt, const void* I, void* x, int64_t H, int64_t W,
              int64_t ld, const smre_admm_params* p, void* eps_out, void* stream,
              smre_admm_report* rep) {
  if (!c || !I || !x || !p) return SMRE_EINVAL;
  if (dt != SMRE_F32 && dt != SMRE_F64) return SMRE_EINVAL;
  if (H < 1 || W < 1 || ld < W || H > 65535 || W > 65535) return SMRE_EINVAL;
  if (!(p->lam > 0) || !(p->rho1 > 0) || !(p->rho2 > 0) || !(p->alpha1 > 0) ||
      !(p->alpha2 > 0) || !std::isfinite(p->gamma) || !std::isfinite(p->delta) ||
      p->max_iter < 1)
    return SMRE_EINVAL;
  if (p->method == SMRE_ADMM_ICD) {
    if (p->K < 0 || p->K > 5 || !p->radius2_icd || p->icd_max_inner < 1) return SMRE_EINVAL;
    if (p->icd_tolmode != SMRE_TOL_MAXABS && p->icd_tolmode != SMRE_TOL_MEANABS)
      return SMRE_EINVAL;
    for (int k = 0; k <= p->K; ++k)
      if (!(p->radius2_icd[k] > 0) || !std::isfinite(p->radius2_icd[k])) return SMRE_EINVAL;
  } else if (p->method == SMRE_ADMM_FULL) {
    if (!p->full || p->full->warm != 0) return SMRE_EINVAL;
    if (p->warm != 0 && p->warm != 1) return SMRE_EINVAL;
  } else {
    return SMRE_EINVAL;
  }
  int rc = set_device(c);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (dt == SMRE_F64)
    return admm_impl<double>(c, dt, (const double*)I, (double*)x, H, W, ld, p, (double*)eps_out,
                             s, rep);
  return admm_impl<float>(c, dt, (const float*)I, (float*)x, H, W, ld, p, (float*)eps_out, s,
                          rep);
}

struct smre_server {
  std::unique_ptr<smre_serve::Server> srv;
};

int smre_serve_create(const smre_serve_config* cfg, smre_server** out) {
  if (!cfg || !out) return SMRE_EINVAL;
  if (cfg->max_active < 1 || cfg->queue_cap < 1) return SMRE_EINVAL;
  if (cfg->inc != SMRE_INC_SAME && cfg->inc != SMRE_INC_BF16) return SMRE_EINVAL;
  int n = 0;
  HIP_OK(hipGetDeviceCount(&n));
  if (cfg->device < 0 || cfg->device >= n) return SMRE_EINVAL;
  auto be = std::make_unique<HipBackend>(*cfg);
  const int rc = be->init();
  if (rc) return rc;
  smre_server* s = new smre_server();
  s->srv = std::make_unique<smre_serve::Server>(std::move(be), cfg->queue_cap);
  *out = s;
  return SMRE_OK;
}

void smre_serve_destroy(smre_server* s) { delete s; }

int smre_serve_submit(smre_server* s, const float* x, int32_t H, int32_t W, const smre_params* p,
                      uint64_t* ticket) {
  if (!s) return SMRE_EINVAL;
  return s->srv->submit(x, H, W, p, ticket);
}

int smre_serve_poll(smre_server* s, uint64_t ticket, float* out, size_t out_elems,
                    smre_report* rep, double* latency_s) {
  if (!s) return SMRE_EINVAL;
  return s->srv->poll(ticket, out, out_elems, rep, latency_s);
}

int smre_serve_stats(smre_server* s, smre_serve_counters* out) {
  if (!s || !out) return SMRE_EINVAL;
  const smre_serve::Stats st = s->srv->stats();
  out->submitted = st.submitted;
  out->completed = st.completed;
  out->rejected = st.rejected;
  out->failed = st.failed;
  out->active = st.active;
  out->queued = st.queued;
  out->sweeps = st.sweeps;
  out->bytes_in_use = (int64_t)st.bytes_in_use;
  out->peak_active = st.peak_active;
  out->joined_running = st.joined_running;
  return SMRE_OK;
}

}  // extern "C"

