// admm.hpp -- gfx950 kernels of the ADMM outer loop (Sec. 2.2, Algorithm 1).
//
// The SMRE minimises G(eps) + R(z) subject to I = A x + eps and z = x (split
// form).  Per iteration, with A the Gaussian PSF (symmetric, so A^T = A):
//   t     = rho1 (I - A x - eps) + Y1               (admm_coupling)
//   x    <- x - (-A t + rho2 (x - z) + Y2) / (2 gamma)   (admm_x_step; the
//            linearised x-update with stabilisation gamma)
//   eps   = I - A x + Y1 / rho1, then eps <- P_G(eps)    (admm_eps_input + the
//            projection kernels)
//   z     = (rho2 x + Y2) / (lam + rho2)             (R = lam/2 ||z||^2)
//   Y1   += alpha1 (I - A x - eps),  Y2 += alpha2 (x - z)   (admm_finish)
// The blur is two LDS-tiled passes (rows, then columns) with zero boundary.
// ||x_new - x||^2 and ||I - A x - eps||^2 are summed in FP64: per block, then
// one atomic add into one of kAdmmSlots slots on separate 128-byte lines.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smre {

constexpr int kAdmmMaxRadius = 32;        // PSF radius <= 32 px (sigma <= 7.9)
constexpr int kAdmmSlots = 256, kAdmmSlotWords = 16;

struct PsfWeights {
  double w[kAdmmMaxRadius + 1];  // w[|k|], k = -R..R, sum 1
  int32_t R;
};

// Row pass: out[i][j] = sum_k w[|k|] in[i][j + k], zero outside the row.  One
// block per 256 outputs of one row; the row segment plus halo sits in LDS.
template <typename T>
__global__ __launch_bounds__(256) void blur_rows(const T* __restrict__ in, T* __restrict__ out,
                                                 int H, int W, int64_t ld, PsfWeights pw) {
  __shared__ T seg[256 + 2 * kAdmmMaxRadius];
  const int i = blockIdx.y, j0 = blockIdx.x * 256, R = pw.R;
  for (int t = threadIdx.x; t < 256 + 2 * R; t += 256) {
    const int j = j0 - R + t;
    seg[t] = (j >= 0 && j < W) ? in[(int64_t)i * ld + j] : T(0);
  }
  __syncthreads();
  const int j = j0 + threadIdx.x;
  if (j >= W) return;
  T acc = (T)pw.w[0] * seg[threadIdx.x + R];
  for (int k = 1; k <= R; ++k)
    acc += (T)pw.w[k] * (seg[threadIdx.x + R - k] + seg[threadIdx.x + R + k]);
  out[(int64_t)i * ld + j] = acc;
}

// Column pass: out[i][j] = sum_k w[|k|] in[i + k][j], zero outside the
// column.  A block owns 64 columns x kBlurColRows rows of outputs (short
// tiles, so a 512^2 image still gives 256 workgroups); the kBlurColRows + 2R
// input rows of those columns sit in LDS (loads and stores coalesced along
// rows).
constexpr int kBlurColRows = 16;
template <typename T>
__global__ __launch_bounds__(256) void blur_cols(const T* __restrict__ in, T* __restrict__ out,
                                                 int H, int W, int64_t ld, PsfWeights pw) {
  constexpr int TC = 64, TR = kBlurColRows;
  __shared__ T tile[TR + 2 * kAdmmMaxRadius][TC];
  const int R = pw.R, i0 = blockIdx.y * TR, j0 = blockIdx.x * TC;
  const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
  for (int r = g; r < TR + 2 * R; r += 4) {
    const int i = i0 - R + r, j = j0 + c;
    tile[r][c] = (i >= 0 && i < H && j < W) ? in[(int64_t)i * ld + j] : T(0);
  }
  __syncthreads();
  const int j = j0 + c;
  if (j >= W) return;
  for (int r = g; r < TR; r += 4) {
    const int i = i0 + r;
    if (i >= H) break;
    T acc = (T)pw.w[0] * tile[r + R][c];
    for (int k = 1; k <= R; ++k) acc += (T)pw.w[k] * (tile[r + R - k][c] + tile[r + R + k][c]);
    out[(int64_t)i * ld + j] = acc;
  }
}

// FP64 block sum of v, then one atomic add into slot (block mod kAdmmSlots).
__device__ __forceinline__ void admm_accumulate(double v, double* slots) {
  __shared__ double part[4];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double s = (part[0] + part[1]) + (part[2] + part[3]);
    atomicAdd(slots + (blockIdx.x % kAdmmSlots) * kAdmmSlotWords, s);
  }
}

struct AdmmCoef {
  double rho1, rho2, lam, alpha1, alpha2, inv2g;
};

// t = rho1 (I - Ax - eps) + Y1
template <typename T>
__global__ __launch_bounds__(256) void admm_coupling(int64_t n, const T* __restrict__ I,
                                                     const T* __restrict__ Ax,
                                                     const T* __restrict__ eps,
                                                     const T* __restrict__ Y1, T* __restrict__ t,
                                                     AdmmCoef c) {
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += (int64_t)gridDim.x * 256)
    t[p] = (T)c.rho1 * (I[p] - Ax[p] - eps[p]) + Y1[p];
}

// x <- x - (-At + rho2 (x - z) + Y2) / (2 gamma); slots += ||dx||^2
template <typename T>
__global__ __launch_bounds__(256) void admm_x_step(int64_t n, T* __restrict__ x,
                                                   const T* __restrict__ At,
                                                   const T* __restrict__ z,
                                                   const T* __restrict__ Y2, AdmmCoef c,
                                                   double* slots) {
  double acc = 0.0;
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n;
       p += (int64_t)gridDim.x * 256) {
    const T g = -At[p] + (T)c.rho2 * (x[p] - z[p]) + Y2[p];
    const T xn = x[p] - g * (T)c.inv2g;
    const double d = (double)xn - (double)x[p];
    acc += d * d;
    x[p] = xn;
  }
  admm_accumulate(acc, slots);
}

// eps = I - Ax + Y1 / rho1 (the point the projection maps onto tau_G)
template <typename T>
__global__ __launch_bounds__(256) void admm_eps_input(int64_t n, const T* __restrict__ I,
                                                      const T* __restrict__ Ax,
                                                      const T* __restrict__ Y1,
                                                      T* __restrict__ eps, AdmmCoef c) {
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += (int64_t)gridDim.x * 256)
    eps[p] = I[p] - Ax[p] + Y1[p] / (T)c.rho1;
}

// z = (rho2 x + Y2) / (lam + rho2); res = I - Ax - eps; Y1 += alpha1 res;
// Y2 += alpha2 (x - z); slots += ||res||^2
template <typename T>
__global__ __launch_bounds__(256) void admm_finish(int64_t n, const T* __restrict__ I,
                                                   const T* __restrict__ x,
                                                   const T* __restrict__ Ax,
                                                   const T* __restrict__ eps, T* __restrict__ z,
                                                   T* __restrict__ Y1, T* __restrict__ Y2,
                                                   AdmmCoef c, double* slots) {
  double acc = 0.0;
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n;
       p += (int64_t)gridDim.x * 256) {
    const T zn = ((T)c.rho2 * x[p] + Y2[p]) / (T)(c.lam + c.rho2);
    const T res = I[p] - Ax[p] - eps[p];
    Y1[p] += (T)c.alpha1 * res;
    Y2[p] += (T)c.alpha2 * (x[p] - zn);
    z[p] = zn;
    acc += (double)res * (double)res;
  }
  admm_accumulate(acc, slots);
}

}  // namespace smre
