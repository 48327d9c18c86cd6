// mc.hpp -- gfx950 kernels of the Monte-Carlo weight estimate (Sec. 2.1).
//
// The paper balances the window bounds through q_alpha, the alpha-quantile of
//   Q = max over windows S of ((t_S)^(1/4) - mu_s) / sigma_s,   t_S = sum_S e^2,
// over fields e of i.i.d. N(0,1) values.  For a fixed side the transform is
// increasing in t_S, so Q only needs the largest t_S of each side:
// mc_window_max finds it per (field, side), mc_q_kernel transforms and
// maximises over sides.
//
// Fields.  Pixel p = i W + j of field f is normal number (p mod 4) of one
// Philox4x64-10 block (Salmon et al., "Parallel random numbers: as easy as
// 1, 2, 3", SC 2011) with counter {p / 4, f, 0, 0} and key {seed, 0}; words
// (w0, w1) and (w2, w3) give two normals each by Box-Muller with
// u = ((w >> 11) + 1/2) 2^-53.  Any pixel of any field can be drawn on its
// own, so a tile draws its own pixels (and its halo) and no field ever goes
// through HBM.
//
// Tile kernel.  A workgroup of 256 lanes owns 4 RPL x 64 window anchors of one
// field (RPL = 16 rows per lane for sides up to 16, 8 up to 32).  The squares
// of the tile plus a halo of SMAX - 1 pixels sit in LDS.  Lane (c, g) owns
// anchor column c and rows RPL g .. RPL g + RPL - 1; it keeps the row sums
// h_s[r] = sum_{l < s} e^2[r][c + l] of the RPL + SMAX - 1 rows its windows
// touch in registers and grows them by one LDS read per row as the
// side goes 1, 2, ..., so each side costs one read per row plus a sliding
// sum down the column (add the entering row, subtract the leaving one).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smre {

constexpr int kMcTileW = 64;     // anchor columns per tile (one per lane of a wave)
constexpr int kMcMaxSide = 32;
// anchor rows per lane and per tile (four waves) for a largest side SMAX
constexpr int mc_rows_per_lane(int smax) { return smax <= 16 ? 16 : 8; }
constexpr int mc_tile_rows(int smax) { return 4 * mc_rows_per_lane(smax); }

// slot[s] = output column of side s (-1: side not requested); side[k] = side
// of output column k; smax = largest requested side.
struct McSides {
  int32_t slot[kMcMaxSide + 1];
  int32_t side[kMcMaxSide];
  int32_t n;
  int32_t smax;
};

__device__ __forceinline__ void philox4x64_10(uint64_t& c0, uint64_t& c1, uint64_t& c2,
                                              uint64_t& c3, uint64_t k0, uint64_t k1) {
  constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull, kM1 = 0xCA5A826395121157ull;
  constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull, kW1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    if (round) {
      k0 += kW0;
      k1 += kW1;
    }
    const uint64_t lo0 = kM0 * c0, hi0 = __umul64hi(kM0, c0);
    const uint64_t lo1 = kM1 * c2, hi1 = __umul64hi(kM1, c2);
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
}

__device__ __forceinline__ double mc_unit(uint64_t w) {
  return ((double)(w >> 11) + 0.5) * 0x1p-53;
}

// The four normals of group g (pixels 4g .. 4g+3) of field f; pairs that no
// requested lane needs are skipped (need: bit l for pixel 4g + l).
__device__ __forceinline__ void mc_group(uint64_t seed, int64_t f, int64_t g, unsigned need,
                                         double z[4]) {
  uint64_t c0 = (uint64_t)g, c1 = (uint64_t)f, c2 = 0, c3 = 0;
  philox4x64_10(c0, c1, c2, c3, seed, 0);
  constexpr double kLn2 = 0.6931471805599453;  // ln u = ln 2 * log2 u
  // the angle 2 pi u as sincospi(2 u): 2 u is exact, so the reduction is
  // exact and cheap (within an ulp or so of sin/cos of the rounded 2 pi u)
  if (need & 3u) {
    const double r = sqrt(-2.0 * kLn2 * log2(mc_unit(c0)));
    double sn, cs;
    sincospi(2.0 * mc_unit(c1), &sn, &cs);
    z[0] = r * cs;
    z[1] = r * sn;
  }
  if (need & 12u) {
    const double r = sqrt(-2.0 * kLn2 * log2(mc_unit(c2)));
    double sn, cs;
    sincospi(2.0 * mc_unit(c3), &sn, &cs);
    z[2] = r * cs;
    z[3] = r * sn;
  }
}

// Fields f0 .. f0 + gridDim.y - 1 written to out (row stride ld, field stride
// fstride); one lane per group of four pixels.
__global__ __launch_bounds__(256) void mc_fields_kernel(double* __restrict__ out, int64_t fstride,
                                                        int64_t ld, int H, int W, uint64_t seed,
                                                        int64_t f0) {
  const int64_t f = f0 + blockIdx.y;
  const int64_t npix = (int64_t)H * W, ngroups = (npix + 3) / 4;
  double* o = out + (int64_t)blockIdx.y * fstride;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < ngroups;
       g += (int64_t)gridDim.x * blockDim.x) {
    double z[4];
    mc_group(seed, f, g, 15u, z);
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      const int64_t p = 4 * g + l;
      if (p < npix) o[(p / W) * ld + p % W] = z[l];
    }
  }
}

__device__ __forceinline__ double mc_wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Largest window sum of squares per (field, requested side) over one tile of
// mc_tile_rows(SMAX) x 64 anchors; blockIdx = (tile column, tile row, field).  GEN: draw the
// field; else read it from `fields` (field stride fstride, row stride ld).
// tmax[(f - f0) * n + k] holds the bits of a non-negative double (their
// unsigned order is the numeric order) and must start at 0.
template <bool GEN, typename T, int SMAX>
__global__ __launch_bounds__(256) void mc_window_max(const T* __restrict__ fields, int64_t fstride,
                                                     int64_t ld, int H, int W, uint64_t seed,
                                                     int64_t f0, McSides sd,
                                                     unsigned long long* __restrict__ tmax) {
  constexpr int RPL = mc_rows_per_lane(SMAX);
  constexpr int EXTR = 4 * RPL + SMAX - 1;     // tile + halo rows
  constexpr int EXT = kMcTileW + SMAX - 1;     // tile + halo columns
  constexpr int ROWS = RPL + SMAX - 1;         // rows one lane's windows touch
  __shared__ double sq[EXTR][EXT];
  __shared__ double red[SMAX][4];
  const int a0 = blockIdx.y * (4 * RPL), b0 = blockIdx.x * kMcTileW;
  const int64_t f = f0 + blockIdx.z;

  // squares of the tile and its halo; zero outside the image
  if (GEN) {
    constexpr int GPR = EXT / 4 + 2;  // groups of four pixels that can meet a tile row
    for (int i = threadIdx.x; i < EXTR * GPR; i += 256) {
      const int r = i / GPR, k = i - (i / GPR) * GPR;
      const int gr = a0 + r;
      if (gr >= H) continue;
      const int64_t p0 = (int64_t)gr * W + b0;             // tile row's first pixel
      const int64_t pend = (int64_t)gr * W + min(W, b0 + EXT);
      const int64_t g = (p0 >> 2) + k;
      unsigned need = 0;
#pragma unroll
      for (int l = 0; l < 4; ++l) {
        const int64_t p = 4 * g + l;
        if (p >= p0 && p < pend) need |= 1u << l;
      }
      if (!need) continue;
      double z[4];
      mc_group(seed, f, g, need, z);
#pragma unroll
      for (int l = 0; l < 4; ++l)
        if (need & (1u << l)) sq[r][(int)(4 * g + l - p0)] = z[l] * z[l];
    }
    for (int i = threadIdx.x; i < EXTR * EXT; i += 256) {
      const int r = i / EXT, cc = i - (i / EXT) * EXT;
      if (a0 + r >= H || b0 + cc >= W) sq[r][cc] = 0.0;
    }
  } else {
    const T* src = fields + (int64_t)blockIdx.z * fstride;
    for (int i = threadIdx.x; i < EXTR * EXT; i += 256) {
      const int r = i / EXT, cc = i - (i / EXT) * EXT;
      double v = 0.0;
      if (a0 + r < H && b0 + cc < W) v = (double)src[(int64_t)(a0 + r) * ld + b0 + cc];
      sq[r][cc] = v * v;
    }
  }
  __syncthreads();

  const int c = threadIdx.x & 63, wv = threadIdx.x >> 6, r0 = wv * RPL;
  double h[ROWS];
#pragma unroll
  for (int k = 0; k < ROWS; ++k) h[k] = 0.0;
  // anchors of this lane inside the image for side s: rows r0 + j with
  // a0 + r0 + j <= H - s, column with b0 + c <= W - s
#pragma unroll
  for (int s = 1; s <= SMAX; ++s) {
    // s is a compile-time constant here, so every h[] index is static
    if (s <= sd.smax) {
#pragma unroll
      for (int k = 0; k < ROWS; ++k) h[k] += sq[r0 + k][c + s - 1];
      if (sd.slot[s] >= 0) {
        const int nrow = min(RPL, H - s + 1 - a0 - r0);
        double m = -1.0;
        if (b0 + c <= W - s && nrow > 0) {
          double n = 0.0;
#pragma unroll
          for (int k = 0; k < s; ++k) n += h[k];
#pragma unroll
          for (int j = 0; j < RPL; ++j) {
            if (j < nrow) m = fmax(m, n);
            if (j + 1 < RPL) n = (n + h[j + s]) - h[j];
          }
        }
        m = mc_wave_max(m);
        if (c == 0) red[s - 1][wv] = m;
      }
    }
  }
  __syncthreads();
  const int s = threadIdx.x + 1;
  if (s <= SMAX && s <= sd.smax && sd.slot[s] >= 0) {
    const double m = fmax(fmax(red[s - 1][0], red[s - 1][1]), fmax(red[s - 1][2], red[s - 1][3]));
    if (m >= 0.0)
      atomicMax(&tmax[(int64_t)blockIdx.z * sd.n + sd.slot[s]],
                (unsigned long long)__double_as_longlong(m));
  }
}

// Q per field: max over requested sides of ((tmax)^(1/4) - mu_s) / sigma_s,
// mu_s = (s^2 - 1/2)^(1/4), sigma_s = (8 s)^(-1/2).
__global__ __launch_bounds__(256) void mc_q_kernel(const unsigned long long* __restrict__ tmax,
                                                   int nf, McSides sd, double* __restrict__ q) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  double Q = -INFINITY;
  for (int k = 0; k < sd.n; ++k) {
    const double npix = (double)sd.side[k] * (double)sd.side[k];
    const double mu = pow(npix - 0.5, 0.25);
    const double sigma = sqrt(1.0 / (8.0 * sqrt(npix)));
    const double t = __longlong_as_double((long long)tmax[(int64_t)f * sd.n + k]);
    Q = fmax(Q, (pow(t, 0.25) - mu) / sigma);
  }
  q[f] = Q;
}

}  // namespace smre
