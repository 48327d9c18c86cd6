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
#include <vector>

#include "icd.hpp"
#include "kernels.hpp"
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
  int timing = 0;
  hipEvent_t ev[2 * kTimingPairs] = {};
  int ev_used = 0;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  std::vector<hipEvent_t> lag_ev;
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
struct Plan {
  int R = 16;
  int nsides = 0;
  int sides[kMaxSides];
  double r2[kMaxSides];
  int smax = 0;
  int nry = 0, nrx = 0;
  int64_t nq = 0;  // increment elements
  int64_t nwin = 0;
  size_t qbytes = 0;
  size_t off_roff = 0, off_prev = 0, total = 0;
  std::vector<int64_t> roff;
};

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int choose_region(int smax, int requested) {
  if (requested) return requested;
  if (smax <= 17) return 16;
  return 32;
}

int plan_project(smre_dtype dt, int64_t H, int64_t W, const smre_params* p, Plan* pl,
                 bool need_offsets) {
  if (!p || !p->sides || !p->radius2) return SMRE_EINVAL;
  if (dt != SMRE_F32 && dt != SMRE_F64) return SMRE_EINVAL;
  if (H < 1 || W < 1 || H > (1 << 20) || W > (1 << 20)) return SMRE_EINVAL;
  if (p->n_sides < 1 || p->n_sides > kMaxSides) return SMRE_EINVAL;
  if (p->max_sweeps < 1 || p->check_every < 1) return SMRE_EINVAL;
  if (p->inc != SMRE_INC_SAME && p->inc != SMRE_INC_BF16) return SMRE_EINVAL;
  if (p->inc == SMRE_INC_BF16 && dt != SMRE_F32) return SMRE_EINVAL;
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
  pl->nry = (int)((H + pl->R - 1) / pl->R);
  pl->nrx = (int)((W + pl->R - 1) / pl->R);
  const size_t es = (p->inc == SMRE_INC_BF16) ? 2 : (dt == SMRE_F64 ? 8 : 4);
  const size_t xs = dt == SMRE_F64 ? 8 : 4;
  // increments per region: each side s contributes s^2 per anchor in the region
  int64_t nq = 0, nwin = 0;
  if (need_offsets) pl->roff.assign((size_t)pl->nry * pl->nrx + 1, 0);
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
      if (need_offsets) pl->roff[(size_t)ry * pl->nrx + rx] = nq;
      nq += cnt;
    }
  if (need_offsets) pl->roff.back() = nq;
  pl->nq = nq;
  pl->nwin = nwin;
  pl->qbytes = align_up((size_t)nq * es + kPage, 256);
  pl->off_roff = pl->qbytes;
  pl->off_prev = align_up(pl->off_roff + ((size_t)pl->nry * pl->nrx + 1) * 8, 256);
  pl->total = align_up(pl->off_prev + (size_t)H * W * xs, 256);
  return SMRE_OK;
}

int ensure_ctrl(smre_ctx* c) {
  if (!c->ctrl) {
    HIP_OK(hipMalloc(&c->ctrl, sizeof(Ctrl)));
    HIP_OK(hipHostMalloc(&c->ctrl_host, sizeof(Ctrl) * (kLag + 2), hipHostMallocDefault));
    HIP_OK(hipMalloc(&c->counter, 64));
    c->lag_ev.resize(kLag + 2);
    for (auto& e : c->lag_ev) HIP_OK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    for (int k = 0; k < 2 * kTimingPairs; ++k) HIP_OK(hipEventCreate(&c->ev[k]));
    HIP_OK(hipEventCreate(&c->t0));
    HIP_OK(hipEventCreate(&c->t1));
  }
  return SMRE_OK;
}

int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(8192, (n + 255) / 256)); }
int grid_rows(int64_t H) { return (int)std::max<int64_t>(1, std::min<int64_t>(4096, H)); }

template <typename TX, typename TQ, int R, bool KAHAN>
void launch_phase(const PhaseArgs& a, int blocks, hipStream_t s) {
  constexpr int SMAX = R + 1;
  hipLaunchKernelGGL((region_phase<TX, TQ, R, SMAX, KAHAN>), dim3(blocks), dim3(128), 0, s, a);
}

template <typename TX, typename TQ, bool KAHAN>
int launch_phase_r(int R, const PhaseArgs& a, int blocks, hipStream_t s) {
  switch (R) {
    case 8: launch_phase<TX, TQ, 8, KAHAN>(a, blocks, s); break;
    case 16: launch_phase<TX, TQ, 16, KAHAN>(a, blocks, s); break;
    case 32: launch_phase<TX, TQ, 32, KAHAN>(a, blocks, s); break;
    default: return SMRE_EINVAL;
  }
  HIP_OK(hipGetLastError());
  return SMRE_OK;
}

int launch_phase_any(smre_dtype dt, int inc, int kahan, int R, const PhaseArgs& a, int blocks,
                     hipStream_t s) {
  if (dt == SMRE_F64) return launch_phase_r<double, double, false>(R, a, blocks, s);
  if (inc == SMRE_INC_BF16)
    return kahan ? launch_phase_r<float, bf16_t, true>(R, a, blocks, s)
                 : launch_phase_r<float, bf16_t, false>(R, a, blocks, s);
  return kahan ? launch_phase_r<float, float, true>(R, a, blocks, s)
               : launch_phase_r<float, float, false>(R, a, blocks, s);
}

template <typename TX>
int run_violation(smre_ctx* c, const void* x, int64_t H, int64_t W, int64_t ld, int n,
                  const int* sides, const double* r2, hipStream_t s, double* out) {
  for (int k = 0; k < n; ++k) {
    const int64_t nw = (H - sides[k] + 1) * (W - sides[k] + 1);
    hipLaunchKernelGGL((violation_kernel<TX>), dim3(grid_for(nw)), dim3(256), 0, s,
                       (const TX*)x, ld, (int)H, (int)W, sides[k], r2[k], c->ctrl);
  }
  HIP_OK(hipGetLastError());
  HIP_OK(hipMemcpyAsync(c->ctrl_host, c->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  *out = dkey_inv(c->ctrl_host->viol_key);
  return SMRE_OK;
}

template <typename TX>
int check_nonfinite(smre_ctx* c, const void* x, int64_t H, int64_t W, int64_t ld, hipStream_t s,
                    bool* bad) {
  hipLaunchKernelGGL((nonfinite_kernel<TX>), dim3(grid_rows(H)), dim3(256), 0, s,
                     (const TX*)x, ld, (int)H, (int)W, c->ctrl);
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

  // increments start at zero (a fill kernel, not a memset: graph-safe)
  const int64_t nwords = (int64_t)(pl.qbytes / 4);
  hipLaunchKernelGGL((fill_kernel<uint32_t>), dim3(grid_for(nwords)), dim3(256), 0, s,
                     (uint32_t*)ws, nwords, 0u);
  HIP_OK(hipMemcpyAsync(ws + pl.off_roff, pl.roff.data(), pl.roff.size() * 8,
                        hipMemcpyHostToDevice, s));

  PhaseArgs a{};
  a.x = x;
  a.roff = (const int64_t*)(ws + pl.off_roff);
  a.q = ws;
  a.done = &c->ctrl->done;
  a.ld = ld;
  a.H = (int)H;
  a.W = (int)W;
  a.nrx = pl.nrx;
  a.fr = pl.R + pl.smax - 1;
  a.nsides = pl.nsides;
  a.kahan = p->kahan ? 1 : 0;
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
      a.cy = color >> 1;
      a.cx = color & 1;
      const int ny = (pl.nry - a.cy + 1) / 2, nx = (pl.nrx - a.cx + 1) / 2;
      a.ncx = nx;
      if (ny <= 0 || nx <= 0) continue;
      int slot;
      rc = timing_begin(c, tacc, s, &slot);
      if (rc) return rc;
      rc = launch_phase_any(dt, p->inc, p->kahan, pl.R, a, ny * nx, s);
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
  HIP_OK(hipStreamSynchronize(s));
  rc = timing_flush(c, tacc, true);
  if (rc) return rc;
  HIP_OK(hipMemcpy(c->ctrl_host, c->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
  const Ctrl fin = *c->ctrl_host;
  const int sweeps_run = fin.done ? fin.done_sweep : p->max_sweeps;
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
    rep->region = pl.R;
    rep->inner_sweeps = 0;
    rep->last_delta = checking ? fin.last_delta : NAN;
    rep->max_violation = viol;
    rep->elapsed_ms = ms;
    rep->kernel_ms = tacc.ms;
    rep->kernel_launches = tacc.launches;
    rep->bytes_moved = (double)sweeps_run * (2.0 * es * (double)pl.nq + 2.0 * sizeof(TX) * (double)H * W);
    rep->window_projections = (double)sweeps_run * (double)pl.nwin;
  }
  if (checking && !fin.done) return SMRE_NOT_CONVERGED;
  return SMRE_OK;
}

template <typename T>
int icd_impl(smre_ctx* c, void* x, int64_t H, int64_t W, int64_t ld, int K, const double* r2,
             double tol, int mode, int max_inner, int nph, hipStream_t s, smre_report* rep) {
  HIP_OK(hipEventRecord(c->t0, s));
  hipLaunchKernelGGL(ctrl_reset_kernel, dim3(1), dim3(1), 0, s, c->ctrl);
  bool bad = false;
  int rc = check_nonfinite<T>(c, x, H, W, ld, s, &bad);
  if (rc) return rc;
  if (bad) return SMRE_ENONFINITE;
  hipLaunchKernelGGL((fill_kernel<int>), dim3(1), dim3(64), 0, s, c->counter, (int64_t)1, 0);
  IcdArgs a{};
  a.x = x;
  a.ld = ld;
  a.H = (int)H;
  a.W = (int)W;
  a.mode = mode;
  a.max_inner = max_inner;
  a.tol = tol;
  for (int k = 0; k <= K; ++k) a.r2[k] = r2[k];
  a.inner_count = c->counter;
  const int B = 1 << K;
  TimingAcc tacc;
  for (int ph = 0; ph < nph; ++ph) {
    a.phase = ph;
    const int o = (1 << ph) & (B - 1);
    const int start = o > 0 ? o - B : 0;
    const int nby = (int)((H - start + B - 1) / B), nbx = (int)((W - start + B - 1) / B);
    int slot;
    rc = timing_begin(c, tacc, s, &slot);
    if (rc) return rc;
    switch (K) {
      case 0: hipLaunchKernelGGL((icd_phase<T, 0>), dim3(nbx, nby), dim3(64), 0, s, a); break;
      case 1: hipLaunchKernelGGL((icd_phase<T, 1>), dim3(nbx, nby), dim3(64), 0, s, a); break;
      case 2: hipLaunchKernelGGL((icd_phase<T, 2>), dim3(nbx, nby), dim3(64), 0, s, a); break;
      case 3: hipLaunchKernelGGL((icd_phase<T, 3>), dim3(nbx, nby), dim3(64), 0, s, a); break;
      case 4: hipLaunchKernelGGL((icd_phase<T, 4>), dim3(nbx, nby), dim3(64), 0, s, a); break;
      default: hipLaunchKernelGGL((icd_phase<T, 5>), dim3(nbx, nby), dim3(64), 0, s, a); break;
    }
    HIP_OK(hipGetLastError());
    rc = timing_end(c, tacc, s, slot);
    if (rc) return rc;
  }
  HIP_OK(hipStreamSynchronize(s));
  rc = timing_flush(c, tacc, true);
  if (rc) return rc;
  int inner = 0;
  HIP_OK(hipMemcpy(&inner, c->counter, sizeof(int), hipMemcpyDeviceToHost));
  std::vector<int> sides(K + 1);
  for (int k = 0; k <= K; ++k) sides[k] = 1 << k;
  double viol = 0.0;
  // feasibility over the aligned squares of every level is not the ICD family
  // (which is shifted); report the full-family violation of the levels' sides.
  rc = run_violation<T>(c, x, H, W, ld, K + 1, sides.data(), r2, s, &viol);
  if (rc) return rc;
  HIP_OK(hipEventRecord(c->t1, s));
  HIP_OK(hipEventSynchronize(c->t1));
  float ms = 0.f;
  HIP_OK(hipEventElapsedTime(&ms, c->t0, c->t1));
  if (rep) {
    rep->sweeps = nph;
    rep->converged = 1;
    rep->region = B;
    rep->inner_sweeps = inner;
    rep->last_delta = NAN;
    rep->max_violation = viol;
    rep->elapsed_ms = ms;
    rep->kernel_ms = tacc.ms;
    rep->kernel_launches = tacc.launches;
    rep->bytes_moved = 2.0 * sizeof(T) * (double)H * W * nph;
    double wp = 0.0;  // window projections: squares per block x inner sweeps is data dependent
    rep->window_projections = wp;
  }
  return SMRE_OK;
}

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
  delete c;
}

int smre_ctx_set_timing(smre_ctx* c, int on) {
  if (!c) return SMRE_EINVAL;
  c->timing = on ? 1 : 0;
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
  int rc = plan_project(dt, H, W, p, &pl, true);
  if (rc) return rc;
  rc = set_device(c);
  if (rc) return rc;
  unsigned char* ws = (unsigned char*)workspace;
  if (ws) {
    if (ws_bytes < pl.total) return SMRE_ENOMEM;
  } else {
    if (c->ws_bytes < pl.total) {
      if (c->ws) HIP_OK(hipFree(c->ws));
      c->ws = nullptr;
      c->ws_bytes = 0;
      if (hipMalloc(&c->ws, pl.total) != hipSuccess) {
        (void)hipGetLastError();
        return SMRE_ENOMEM;
      }
      c->ws_bytes = pl.total;
    }
    ws = (unsigned char*)c->ws;
  }
  hipStream_t s = (hipStream_t)stream;
  if (dt == SMRE_F64) return project_impl<double>(c, dt, x, H, W, ld, p, pl, ws, s, rep);
  return project_impl<float>(c, dt, x, H, W, ld, p, pl, ws, s, rep);
}

int smre_dykstra_incomplete(smre_ctx* c, smre_dtype dt, void* x, int64_t H, int64_t W,
                            int64_t ld, int32_t K, const double* r2, double tol, int32_t mode,
                            int32_t max_inner, int32_t nph, void* stream, smre_report* rep) {
  if (!c || !x || !r2) return SMRE_EINVAL;
  if (dt != SMRE_F32 && dt != SMRE_F64) return SMRE_EINVAL;
  if (H < 1 || W < 1 || ld < W || H > (1 << 20) || W > (1 << 20)) return SMRE_EINVAL;
  if (K < 0 || K > 5 || max_inner < 1 || nph < 1 || nph > K + 1) return SMRE_EINVAL;
  if (mode != SMRE_TOL_MAXABS && mode != SMRE_TOL_MEANABS) return SMRE_EINVAL;
  if (!std::isfinite(tol)) return SMRE_EINVAL;
  for (int k = 0; k <= K; ++k) {
    if (!std::isfinite(r2[k])) return SMRE_ENONFINITE;
    if (!(r2[k] > 0)) return SMRE_EINVAL;
  }
  int rc = set_device(c);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (dt == SMRE_F64)
    return icd_impl<double>(c, x, H, W, ld, K, r2, tol, mode, max_inner, nph, s, rep);
  return icd_impl<float>(c, x, H, W, ld, K, r2, tol, mode, max_inner, nph, s, rep);
}

int smre_max_violation(smre_ctx* c, smre_dtype dt, const void* x, int64_t H, int64_t W,
                       int64_t ld, int32_t n, const int32_t* sides, const double* r2,
                       void* stream, double* out) {
  if (!c || !x || !sides || !r2 || !out || n < 1) return SMRE_EINVAL;
  if (H < 1 || W < 1 || ld < W) return SMRE_EINVAL;
  for (int k = 0; k < n; ++k) {
    if (sides[k] < 1 || sides[k] > H || sides[k] > W) return SMRE_EINVAL;
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

}  // extern "C"
