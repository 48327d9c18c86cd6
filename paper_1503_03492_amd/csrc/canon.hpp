// canon.hpp -- full Dykstra in a canonical visiting order: one launch per
// tiling.
//
// Dykstra's cyclic order over overlapping sets is the caller's choice (the
// limit does not depend on it, Sec. 2.3); the canonical orders visit the sides
// descending (or ascending), and for each side s its s^2 tilings (a, b) in
// raster order -- tiling (s, a, b) being the disjoint windows
// [a + s i, a + s i + s) x [b + s j, b + s j + s) inside the image.  The
// windows of one tiling commute, so one launch projects them all (Eq.
// (dykstra:if) inside Dykstra's update).
//
// Layout: the increments of tiling t form a compact plane of the nr s x nc s
// pixels its windows cover (nr = (H - a) / s window rows, nc = (W - b) / s
// window columns), row-major, starting at element q_off[t].
//
// A workgroup of 256 lanes takes one row of windows of the tiling and
// WPB = 256 / s consecutive windows of it: lane l owns column l of that band
// (l < WPB s), keeps its s values y = x + I in registers, and sums their
// squares; the window sums add s column sums in LDS; the scale comes back
// through LDS; each lane writes x' = t y and I' = y - x' for its column.
// FP32: compensated column sums, and windows within the guard band of their
// bound are re-summed in FP64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace smre {

struct TilingArgs {
  void* x;          // image (TX), row stride ld
  void* q;          // this tiling's increment plane (TQ), nr s x nc s, row-major
  const int* done;  // converged flag: every launch exits at once once it is set
  int64_t ld;
  int32_t s, a, b;  // side and tiling offset
  int32_t nr, nc;   // window rows and columns of the tiling
  int32_t wpb;      // windows per workgroup along a row: 256 / s
  float guard;      // FP32: relative band of the FP64 recheck
  float r2f, rf;    // bound and its square root, FP32
  double r2d;
};

template <typename TQ> struct GQ;
template <> struct GQ<float> {
  static __device__ __forceinline__ float get(const float* p) { return *p; }
  static __device__ __forceinline__ void put(float* p, float v) { *p = v; }
};
template <> struct GQ<double> {
  static __device__ __forceinline__ double get(const double* p) { return *p; }
  static __device__ __forceinline__ void put(double* p, double v) { *p = v; }
};
template <> struct GQ<bf16_t> {
  static __device__ __forceinline__ float get(const bf16_t* p) { return bf2f(*p); }
  static __device__ __forceinline__ void put(bf16_t* p, float v) { *p = f2bf(v); }
};

template <typename TX, typename TQ, int SMAX, bool KAHAN>
__global__ __launch_bounds__(256) void tiling_phase(TilingArgs g) {
  __shared__ double colsum[256];
  __shared__ TX scale[256];
  __shared__ int nearw[256];
  __shared__ int any_near;
  if (*g.done) return;
  const int s = g.s;
  const int lane = threadIdx.x;
  const int wrow = blockIdx.y;                 // window row of the tiling
  const int w0 = blockIdx.x * g.wpb;           // first window column of the block
  const int nw = min(g.wpb, g.nc - w0);        // windows of this block
  const bool on = lane < nw * s;
  const int pc = w0 * s + lane;                // plane column
  const int row0 = wrow * s;                   // plane row of the band
  TX* x = (TX*)g.x + (int64_t)(g.a + row0) * g.ld + g.b + pc;
  TQ* q = (TQ*)g.q + (int64_t)row0 * (g.nc * s) + pc;
  const int64_t qld = (int64_t)g.nc * s;

  TX y[SMAX];
  TX acc = 0, comp = 0;
#pragma unroll
  for (int r = 0; r < SMAX; ++r) {
    y[r] = TX(0);
    if (r < s && on) {
      const TX yv = x[(int64_t)r * g.ld] + (TX)GQ<TQ>::get(q + r * qld);
      y[r] = yv;
      if constexpr (sizeof(TX) == 4 && KAHAN) {
        const TX t2 = __builtin_fmaf(yv, yv, -comp);
        const TX s2 = acc + t2;
        comp = (s2 - acc) - t2;
        acc = s2;
      } else if constexpr (sizeof(TX) == 4) {
        acc = __builtin_fmaf(yv, yv, acc);
      } else {
        acc = __builtin_fma(yv, yv, acc);
      }
    }
  }
  if (lane == 0) any_near = 0;
  colsum[lane] = on ? (double)(acc - comp) : 0.0;
  __syncthreads();
  // one lane per window: the window sum over its s columns, the scale
  if (lane < nw) {
    if constexpr (sizeof(TX) == 4) {
      float n = 0.f;
      for (int c = 0; c < s; ++c) n += (float)colsum[lane * s + c];
      const bool near = fabsf(n - g.r2f) <= g.guard * g.r2f;
      nearw[lane] = near;
      if (near) any_near = 1;
      scale[lane] = n > g.r2f ? g.rf * __builtin_amdgcn_rsqf(n) : 1.0f;
    } else {
      double n = 0.0;
      for (int c = 0; c < s; ++c) n += colsum[lane * s + c];
      scale[lane] = n > g.r2d ? __builtin_sqrt(g.r2d / n) : 1.0;
    }
  }
  __syncthreads();
  if constexpr (sizeof(TX) == 4) {
    if (any_near) {
      // windows within the guard band of their bound decide in FP64
      double pd = 0.0;
#pragma unroll
      for (int r = 0; r < SMAX; ++r)
        if (r < s && on) pd = __builtin_fma((double)y[r], (double)y[r], pd);
      colsum[lane] = pd;
      __syncthreads();
      if (lane < nw && nearw[lane]) {
        double nd = 0.0;
        for (int c = 0; c < s; ++c) nd += colsum[lane * s + c];
        scale[lane] = nd > g.r2d ? (float)__builtin_sqrt(g.r2d / nd) : 1.0f;
      }
      __syncthreads();
    }
  }
  if (!on) return;
  const TX t = scale[lane / s];
#pragma unroll
  for (int r = 0; r < SMAX; ++r) {
    if (r < s) {
      const TX xn = t * y[r];
      x[(int64_t)r * g.ld] = xn;
      GQ<TQ>::put(q + r * qld, y[r] - xn);
    }
  }
}

}  // namespace smre
