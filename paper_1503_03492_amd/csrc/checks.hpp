// checks.hpp -- gfx950 device code for the convergence and feasibility
// checks of the projection library (Algorithm 2's stopping rule read as the
// largest pixel change between sweep ends, in FP64; the largest window
// violation of the ball constraints, in FP64) and small utility kernels.
#pragma once

#include "kernels.hpp"

namespace smre {

// ---------------------------------------------------------------- checks
// Order-preserving map of doubles to unsigned 64-bit keys (for atomic max).
__device__ __forceinline__ unsigned long long dkey(double d) {
  unsigned long long u = (unsigned long long)__double_as_longlong(d);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__host__ __device__ inline double dkey_inv(unsigned long long k) {
  unsigned long long u = (k >> 63) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k;
  double d;
  __builtin_memcpy(&d, &u, 8);
  return d;
}

// atomicMax of a key that skips the atomic when the stored key is already at
// least as large (a stale read only costs an unneeded atomic): with many
// blocks reporting into one address most of them then skip it.
__device__ __forceinline__ void key_max(unsigned long long* addr, unsigned long long k) {
  if (k > __hip_atomic_load(addr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(addr, k);
}

struct Ctrl {
  int done;            // converged flag read by every sweep kernel
  int done_sweep;      // sweep at which it converged
  int nonfinite;       // input check result
  int abort;           // a sweep kernel's producer/consumer wait gave up
  unsigned long long delta_key;  // running max |x - prev| of the checked sweep
  double last_delta;
  unsigned long long viol_key;   // running max violation
  unsigned long long icd_sum[4]; // an ICD call's summed work counters
  unsigned int nf_epoch;         // last ICD call (by its number) whose input was not finite
};

template <typename TX>
__device__ __forceinline__ double block_max(double v) {
  __shared__ double red[4];
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  v = red[0];
  for (int i = 1; i < (int)(blockDim.x >> 6); ++i) v = fmax(v, red[i]);
  return v;
}

// Image-wide passes: blocks stride over rows, threads over columns.
template <typename TX>
__global__ __launch_bounds__(256) void snapshot_kernel(const TX* x, int64_t ld, int H, int W,
                                                       TX* prev, Ctrl* ctrl) {
  if (ctrl->done) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) ctrl->delta_key = dkey(0.0);
  for (int r = blockIdx.x; r < H; r += gridDim.x)
    for (int col = threadIdx.x; col < W; col += blockDim.x)
      prev[(int64_t)r * W + col] = x[(int64_t)r * ld + col];
}

template <typename TX>
__global__ __launch_bounds__(256) void delta_kernel(const TX* x, int64_t ld, int H, int W,
                                                    const TX* prev, Ctrl* ctrl) {
  if (ctrl->done) return;
  double m = 0.0;
  for (int r = blockIdx.x; r < H; r += gridDim.x)
    for (int col = threadIdx.x; col < W; col += blockDim.x)
      m = fmax(m, fabs((double)x[(int64_t)r * ld + col] - (double)prev[(int64_t)r * W + col]));
  m = block_max<TX>(m);
  if (threadIdx.x == 0) key_max(&ctrl->delta_key, dkey(m));
}

__global__ void decide_kernel(Ctrl* ctrl, double tol, int sweep) {
  if (ctrl->done) return;
  const double d = dkey_inv(ctrl->delta_key);
  ctrl->last_delta = d;
  if (d < tol) {
    ctrl->done = 1;
    ctrl->done_sweep = sweep;
  }
}

// Clears the non-finite flag before a check (the flag is only ever raised
// by the check itself).
__global__ void nonfinite_reset_kernel(Ctrl* ctrl) { ctrl->nonfinite = 0; }

template <typename TX>
__global__ __launch_bounds__(256) void nonfinite_kernel(const TX* x, int64_t ld, int H, int W,
                                                        Ctrl* ctrl) {
  int bad = 0;
  for (int r = blockIdx.x; r < H; r += gridDim.x)
    for (int col = threadIdx.x; col < W; col += blockDim.x) {
      const double v = (double)x[(int64_t)r * ld + col];
      bad |= !(v - v == 0.0);
    }
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(&ctrl->nonfinite, 1);
}

// Feasibility: max over windows S of the requested sides of sum_S x^2 / r2_s - 1,
// in FP64, folded into ctrl->viol_key; blockIdx.z selects a frame of a movie
// (frames fstride elements apart).
//
// All sides up to SMAX in one pass.  A workgroup owns 4 RPL x 64 window anchors
// and stages the squares of their (4 RPL + SMAX - 1) x (64 + SMAX - 1) pixels
// in LDS.  Lane (c, g) owns anchor column c and rows RPL g .. RPL g + RPL - 1:
// it keeps h[k] = sum_{l < s} x^2[RPL g + k][c + l] for the rows its windows
// touch and grows it by one column as the side goes 1, 2, ...; a window's sum
// is then its s row sums added top to bottom.  Those are the row-then-column
// sums of violation_kernel in the same order, so both give the same bits.  The
// largest ratio of a side comes from its largest sum (x -> x / r2 - 1 does not
// decrease under rounding either).
constexpr int kFeasMaxSide = 32;
constexpr int feas_rows_per_lane(int smax) { return smax <= 16 ? 16 : 8; }
constexpr int feas_tile_rows(int smax) { return 4 * feas_rows_per_lane(smax); }
struct FeasSides {
  double r2[kFeasMaxSide + 1];  // r2[s] > 0: side s requested with that bound; 0: not
  int32_t smax;                 // largest requested side
};

//
// cslots (may be null): work counters to total in the same launch, slot t's
// word w at cslots[t * sstride + w] for t < 256 and w < 4; block (0, 0, 0)
// adds them up after its tile and writes csum[0..3] (integers: any order).
template <typename TX, int SMAX>
__global__ __launch_bounds__(256) void feasibility_kernel(const TX* __restrict__ x,
                                                          int64_t fstride, int64_t ld, int H,
                                                          int W, FeasSides fs, Ctrl* ctrl,
                                                          const unsigned long long* cslots,
                                                          int sstride, unsigned long long* csum) {
  constexpr int RPL = feas_rows_per_lane(SMAX);
  constexpr int ER = 4 * RPL + SMAX - 1, EC = 64 + SMAX - 1;
  constexpr int ROWS = RPL + SMAX - 1;  // rows one lane's windows touch
  __shared__ double sq[ER][EC];
  x += (int64_t)blockIdx.z * fstride;
  const int a0 = blockIdx.y * (4 * RPL), b0 = blockIdx.x * 64;
  // every load of the lane issued before the first is used (a fixed trip
  // count, unrolled), so their latencies overlap
  constexpr int NLD = (ER * EC + 255) / 256;
  TX v[NLD];
#pragma unroll
  for (int u = 0; u < NLD; ++u) {
    const int i = threadIdx.x + 256 * u;
    const int r = i / EC, cc = i - (i / EC) * EC;
    v[u] = TX(0);
    if (i < ER * EC && a0 + r < H && b0 + cc < W) v[u] = x[(int64_t)(a0 + r) * ld + b0 + cc];
  }
#pragma unroll
  for (int u = 0; u < NLD; ++u) {
    const int i = threadIdx.x + 256 * u;
    if (i < ER * EC) {
      const double d = (double)v[u];
      sq[i / EC][i - (i / EC) * EC] = d * d;
    }
  }
  __syncthreads();
  const int c = threadIdx.x & 63, r0 = (threadIdx.x >> 6) * RPL;
  double h[ROWS];
#pragma unroll
  for (int k = 0; k < ROWS; ++k) h[k] = 0.0;
  double worst = -1.0;
#pragma unroll
  for (int s = 1; s <= SMAX; ++s) {
    // s is a compile-time constant here, so every h[] index is static
    if (s <= fs.smax) {
#pragma unroll
      for (int k = 0; k < ROWS; ++k) h[k] += sq[r0 + k][c + s - 1];
      const int nrow = min(RPL, H - s + 1 - a0 - r0);  // anchor rows inside the image
      if (fs.r2[s] > 0.0 && b0 + c <= W - s && nrow > 0) {
        double m = 0.0;
#pragma unroll
        for (int j = 0; j < RPL; ++j) {
          if (j < nrow) {
            double n = 0.0;
#pragma unroll
            for (int k = 0; k < s; ++k) n += h[j + k];
            m = fmax(m, n);
          }
        }
        worst = fmax(worst, m / fs.r2[s] - 1.0);
      }
    }
  }
  worst = block_max<TX>(worst);
  if (threadIdx.x == 0) key_max(&ctrl->viol_key, dkey(worst));
  if (cslots && blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0) {
    __shared__ unsigned long long wsum[4][4];
    unsigned long long v[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      v[w] = cslots[(size_t)threadIdx.x * sstride + w];
      for (int o = 32; o > 0; o >>= 1) v[w] += __shfl_xor(v[w], o);
    }
    if ((threadIdx.x & 63) == 0)
#pragma unroll
      for (int w = 0; w < 4; ++w) wsum[threadIdx.x >> 6][w] = v[w];
    __syncthreads();
    if (threadIdx.x < 4)
      csum[threadIdx.x] = wsum[0][threadIdx.x] + wsum[1][threadIdx.x] + wsum[2][threadIdx.x] +
                          wsum[3][threadIdx.x];
  }
}

// Sides above kFeasMaxSide, one launch per side: a block takes 16 x 32 window
// anchors, stages the squares of the (16 + s - 1) x (32 + s - 1) pixels in LDS,
// sums each row over s columns, then those row sums over s rows (O(s) adds
// per window instead of s^2 loads).  MAXS: the longest side of the instance
// (its LDS size: two blocks per CU fit with MAXS = 64).
constexpr int kViolTileH = 16, kViolTileW = 32, kViolMaxSide = 96;
template <typename TX, int MAXS>
__global__ __launch_bounds__(256) void violation_kernel(const TX* x, int64_t fstride, int64_t ld,
                                                        int H, int W, int s, double r2,
                                                        Ctrl* ctrl) {
  x += (int64_t)blockIdx.z * fstride;
  constexpr int RT = kViolTileH + MAXS - 1, CT = kViolTileW + MAXS - 1;
  __shared__ double sq[RT][CT];
  __shared__ double hs[RT][kViolTileW];
  const int a0 = blockIdx.y * kViolTileH, b0 = blockIdx.x * kViolTileW;
  const int rows = kViolTileH + s - 1, cols = kViolTileW + s - 1;
  // a wave per row, lanes along it (no index division); four rows' loads
  // issued before the first is used
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
  for (int r0 = wv; r0 < rows; r0 += 16) {
    TX v[4][(CT + 63) / 64];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int k = 0; k < (CT + 63) / 64; ++k) {
        const int r = r0 + 4 * u, cc = ln + 64 * k;
        const int gr = a0 + r, gc = b0 + cc;
        v[u][k] = (r < rows && cc < cols && gr < H && gc < W) ? x[(int64_t)gr * ld + gc] : TX(0);
      }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int k = 0; k < (CT + 63) / 64; ++k) {
        const int r = r0 + 4 * u, cc = ln + 64 * k;
        if (r < rows && cc < cols) {
          const double d = (double)v[u][k];
          sq[r][cc] = d * d;
        }
      }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < rows * kViolTileW; i += blockDim.x) {
    const int r = i / kViolTileW, cc = i - (i / kViolTileW) * kViolTileW;
    double h = 0.0;
    for (int j = 0; j < s; ++j) h += sq[r][cc + j];
    hs[r][cc] = h;
  }
  __syncthreads();
  double m = -1.0;
  for (int i = threadIdx.x; i < kViolTileH * kViolTileW; i += blockDim.x) {
    const int r = i / kViolTileW, cc = i - (i / kViolTileW) * kViolTileW;
    if (a0 + r > H - s || b0 + cc > W - s) continue;  // window not fully inside
    double n = 0.0;
    for (int j = 0; j < s; ++j) n += hs[r + j][cc];
    m = fmax(m, n / r2 - 1.0);
  }
  m = block_max<TX>(m);
  if (threadIdx.x == 0) key_max(&ctrl->viol_key, dkey(m));
}

template <typename T>
__global__ __launch_bounds__(256) void fill_kernel(T* p, int64_t n, T v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Warm start (Dykstra's invariant x + sum_S I_S = x0): isum holds the
// previous solve's sum_S I_S = x0_prev - z_prev; the new input x0 in x is
// kept in isum and the iterate starts at x0 - sum_S I_S.
template <typename TX>
__global__ __launch_bounds__(256) void warm_begin_kernel(TX* x, int64_t ld, int H, int W,
                                                         TX* isum) {
  for (int r = blockIdx.x; r < H; r += gridDim.x)
    for (int col = threadIdx.x; col < W; col += blockDim.x) {
      const TX v = x[(int64_t)r * ld + col];
      TX& s = isum[(int64_t)r * W + col];
      x[(int64_t)r * ld + col] = v - s;
      s = v;
    }
}

// Cold start: keep the input x0 in isum.
template <typename TX>
__global__ __launch_bounds__(256) void keep_input_kernel(const TX* x, int64_t ld, int H, int W,
                                                         TX* isum) {
  for (int r = blockIdx.x; r < H; r += gridDim.x)
    for (int col = threadIdx.x; col < W; col += blockDim.x)
      isum[(int64_t)r * W + col] = x[(int64_t)r * ld + col];
}

// End of a solve: isum = x0 - z = sum_S I_S, the start of the next warm solve.
template <typename TX>
__global__ __launch_bounds__(256) void increment_sum_kernel(const TX* x, int64_t ld, int H,
                                                            int W, TX* isum) {
  for (int r = blockIdx.x; r < H; r += gridDim.x)
    for (int col = threadIdx.x; col < W; col += blockDim.x)
      isum[(int64_t)r * W + col] -= x[(int64_t)r * ld + col];
}

__device__ __forceinline__ void ctrl_reset(Ctrl* c) {
  c->done = 0;
  c->done_sweep = 0;
  c->nonfinite = 0;
  c->abort = 0;
  c->delta_key = dkey(0.0);
  c->last_delta = -1.0;
  c->viol_key = dkey(-1.0);
}

__global__ void ctrl_reset_kernel(Ctrl* c) { ctrl_reset(c); }

// A new control block: reset, and no ICD call has seen a non-finite input.
__global__ void ctrl_init_kernel(Ctrl* c) {
  ctrl_reset(c);
  c->nf_epoch = 0;
}

// Start of an ICD call in one launch: the work counters cleared; when `reset`,
// the control block reset; when x is given, its rows scanned for NaN or Inf,
// which raises nf_epoch to the call's number `epoch`.  The flag needs no
// clearing (a call's phase kernels compare it with their own number, and the
// numbers grow), so the scan shares the launch with the reset.
template <typename TX>
__global__ __launch_bounds__(256) void icd_begin_kernel(Ctrl* c, int reset,
                                                        unsigned long long* cnt, int64_t n,
                                                        const TX* __restrict__ x, int64_t ld,
                                                        int rows, int W, unsigned epoch) {
  if (reset && blockIdx.x == 0 && threadIdx.x == 0) ctrl_reset(c);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    cnt[i] = 0;
  if (!x) return;
  int bad = 0;
  for (int r = blockIdx.x; r < rows; r += gridDim.x)
    for (int col = threadIdx.x; col < W; col += blockDim.x) {
      const double v = (double)x[(int64_t)r * ld + col];
      bad |= !(v - v == 0.0);
    }
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicMax(&c->nf_epoch, epoch);
}

// ---------------------------------------------------------------- batch control
template <typename TX>
__global__ __launch_bounds__(256) void snapshot_batch(const ImageDesc* __restrict__ imgs,
                                                      BatchCtl* ctl, TX* prev) {
  const int im = blockIdx.y;
  if (ctl[im].done || (ctl[im].sweeps + 1) % ctl[im].check_every != 0) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) ctl[im].delta_key = dkey(0.0);
  const ImageDesc& a = imgs[im];
  const TX* x = (const TX*)a.x;
  TX* pv = prev + ctl[im].prev_off;
  for (int r = blockIdx.x; r < a.H; r += gridDim.x)
    for (int col = threadIdx.x; col < a.W; col += blockDim.x)
      pv[(int64_t)r * a.W + col] = x[(int64_t)r * a.ld + col];
}

template <typename TX>
__global__ __launch_bounds__(256) void delta_batch(const ImageDesc* __restrict__ imgs,
                                                   BatchCtl* ctl, const TX* prev) {
  const int im = blockIdx.y;
  if (ctl[im].done || (ctl[im].sweeps + 1) % ctl[im].check_every != 0) return;
  const ImageDesc& a = imgs[im];
  const TX* x = (const TX*)a.x;
  const TX* pv = prev + ctl[im].prev_off;
  double m = 0.0;
  for (int r = blockIdx.x; r < a.H; r += gridDim.x)
    for (int col = threadIdx.x; col < a.W; col += blockDim.x)
      m = fmax(m, fabs((double)x[(int64_t)r * a.ld + col] - (double)pv[(int64_t)r * a.W + col]));
  m = block_max<TX>(m);
  if (threadIdx.x == 0) key_max(&ctl[im].delta_key, dkey(m));
}

// One block: close the sweep for every image (check and/or sweep cap) and
// count the images still running.  counters[0] = sweeps done, [1] = active.
__global__ __launch_bounds__(256) void decide_batch(BatchCtl* ctl, int n, int check,
                                                    int* counters) {
  __shared__ int active;
  const int sweep = counters[0] + 1;
  if (threadIdx.x == 0) active = 0;
  __syncthreads();
  for (int im = threadIdx.x; im < n; im += blockDim.x) {
    BatchCtl& c = ctl[im];
    if (c.done) continue;
    const int sw = ++c.sweeps;
    bool stop = false;
    if (check && sw % c.check_every == 0) {
      const double d = dkey_inv(c.delta_key);
      c.last_delta = d;
      if (d < c.tol) {
        c.converged = 1;
        stop = true;
      }
    }
    if (sw >= c.max_sweeps || c.aborted) stop = true;
    if (stop) {
      c.done = 1;
      c.done_sweep = sw;
    } else {
      atomicAdd(&active, 1);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    counters[0] = sweep;
    counters[1] = active;
  }
}

}  // namespace smre
