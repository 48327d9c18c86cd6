// icd.hpp -- incomplete Dykstra (ICD) phase kernel for gfx950.
//
// Sec. 3.2 restricts the family to squares of side 2^k (k <= K) on lattices
// shifted diagonally by 2^i and projects phase by phase: phase i works on
// blocks of side 2^K on the lattice offset by o_i = 2^i mod 2^K; a block runs
// Dykstra over its squares of side 2^K, 2^(K-1), ..., 2^i with increments
// zeroed at the phase start, until the block converges.  A phase here takes
// its shift on each axis and its lowest level as arguments, so families
// other than the paper's (shifts along one axis only, say) run unchanged.  Blocks of a phase
// are disjoint, so one wave per block runs them all in parallel.
//
// A movie of frames (same size, stacked at a fixed stride) runs in the same
// launches: blockIdx.z selects the frame, so every phase covers all frames.
//
// Layout inside a wave: the block's 4^K pixels in Morton (Z) order, NPL =
// max(1, 4^K / 64) consecutive Morton indices per lane.  A square of side 2^k
// is then an aligned run of 4^k Morton indices: inside one lane when
// 4^k <= NPL, else an aligned group of 4^k / NPL lanes, reduced with DPP and
// permlane swaps.  Pixels, increments and sums stay in registers; HBM sees
// one read and one write of x per phase.
#pragma once

#include "kernels.hpp"

namespace smre {

// Even bits 0, 2, ..., 10 of a 12-bit Morton index, packed (compaction by
// masks and shifts).
__device__ __forceinline__ int morton_x(int m) {
  unsigned x = (unsigned)m & 0x555u;
  x = (x | (x >> 1)) & 0x333u;
  x = (x | (x >> 2)) & 0x0F0Fu;
  x = (x | (x >> 4)) & 0x00FFu;
  return (int)x;
}
__device__ __forceinline__ int morton_y(int m) { return morton_x(m >> 1); }

// t = sqrt(r2 / n) if n > r2 else 1, in the precision of the image.  FP64:
// the correctly rounded quotient and root.  FP32: sqrt(r2) (computed per
// level on the host, sr2) times the hardware reciprocal square root of n,
// clamped to 1 so a window just outside the ball is never scaled up by
// rounding; one instruction instead of an IEEE divide and square root,
// within a few ulp.
template <typename T> __device__ __forceinline__ T ball_scale(T n, T r2, T sr2) {
  if constexpr (sizeof(T) == 8) return n > r2 ? __builtin_sqrt(r2 / n) : T(1);
  else return n > r2 ? __builtin_fminf(sr2 * __builtin_amdgcn_rsqf(n), 1.0f) : 1.0f;
}

template <typename T> __device__ __forceinline__ T wave_max(T v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

struct IcdArgs {
  void* x;            // frame 0; frame f at x + f * fstride elements
  int64_t fstride;
  int64_t ld;
  int32_t H, W;
  int32_t oy, ox;     // lattice shift of this phase, 0 <= shift < 2^K
  int32_t lmin;       // lowest level projected in this phase
  int32_t mode;       // 0: max |dx| < tol, 1: sum |dx| <= tol * block pixels
  int32_t max_inner;
  int32_t pad;
  double tol;
  double r2[6];
  float sr2[6];       // sqrtf((float)r2[k]) for the FP32 scale
  // Work counters (device): kIcdSlots slots of kIcdSlotWords words, one
  // 128-byte line each; a block adds its inner sweeps, square projections
  // and (square, pixel) updates to words 0, 1, 2 of slot (block id mod
  // kIcdSlots), so no line takes more than a share of the blocks' atomics.
  unsigned long long* counters;
};
constexpr int kIcdSlots = 256, kIcdSlotWords = 16;
// Words per slot that the kernel adds to: inner sweeps, square projections,
// (square, pixel) updates, blocks stopped by max_inner.
constexpr int kIcdCountWords = 4;

// One block of kIcdSlots threads: out[w] = sum over the slots of word w.
__global__ __launch_bounds__(kIcdSlots) void icd_counter_sum(const unsigned long long* cnt,
                                                             unsigned long long* out) {
  __shared__ unsigned long long red[kIcdCountWords][kIcdSlots];
  const int t = threadIdx.x;
#pragma unroll
  for (int w = 0; w < kIcdCountWords; ++w) red[w][t] = cnt[(size_t)t * kIcdSlotWords + w];
  __syncthreads();
  for (int h = kIcdSlots / 2; h > 0; h >>= 1) {
    if (t < h)
#pragma unroll
      for (int w = 0; w < kIcdCountWords; ++w) red[w][t] += red[w][t + h];
    __syncthreads();
  }
  if (t < kIcdCountWords) out[t] = red[t][0];
}

// MEANABS: stop when the block's sum of |dx| over an inner sweep is at most
// tol times its pixel count (accumulated per lane in T, summed over the wave
// in FP64); else when max |dx| < tol.
// Workgroups are dealt round-robin to the 8 XCDs (each with its own L2) in
// dispatch order.  A block of 2^K FP32 pixels per row uses part of each
// 128-byte line it touches and its horizontal neighbour uses the rest, so the
// dispatch id is mapped to the block such that each XCD gets runs of 16
// consecutive blocks (row-major over (x, y, frame)), the runs dealt to the
// XCDs in turn: neighbours inside a run share an L2 instead of fetching the
// same lines twice, and every XCD still samples the whole grid (frames of a
// movie differ in how many inner sweeps their blocks need).  A bijection on
// the grid (ids past the last whole group of 128 map to themselves); 32-bit
// arithmetic, the host keeps a launch below 2^31 blocks.
__device__ __forceinline__ void icd_block_of(unsigned& bx, unsigned& by, unsigned& bz) {
  const unsigned nx = gridDim.x, nxy = gridDim.x * gridDim.y;
  const unsigned total = nxy * gridDim.z;
  const unsigned pid = blockIdx.z * nxy + blockIdx.y * nx + blockIdx.x;
  unsigned lid = pid;
  if (pid < (total & ~127u)) {
    const unsigned xcd = pid & 7u, slot = pid >> 3;
    lid = (((slot >> 4) << 3) + xcd) * 16u + (slot & 15u);
  }
  bz = lid / nxy;
  const unsigned r = lid - bz * nxy;
  by = r / nx;
  bx = r - by * nx;
}

template <typename T, int K, bool MEANABS>
__global__ __launch_bounds__(64) void icd_phase(IcdArgs a) {
  constexpr int B = 1 << K;
  constexpr int NPX = B * B;
  constexpr int NPL = NPX >= 64 ? NPX / 64 : 1;
  const int lane = threadIdx.x;
  const int i = a.lmin;
  unsigned tx, ty, tz;
  icd_block_of(tx, ty, tz);
  const int by = (a.oy > 0 ? a.oy - B : 0) + (int)ty * B;
  const int bx = (a.ox > 0 ? a.ox - B : 0) + (int)tx * B;
  T* xg = (T*)a.x + (int64_t)tz * a.fstride;

  T x[NPL];
  bool inimg[NPL];
  int gy[NPL], gx[NPL];
  int npix = 0;
#pragma unroll
  for (int e = 0; e < NPL; ++e) {
    const int m = lane * NPL + e;
    gy[e] = by + morton_y(m);
    gx[e] = bx + morton_x(m);
    inimg[e] = m < NPX && gy[e] >= 0 && gx[e] >= 0 && gy[e] < a.H && gx[e] < a.W;
    x[e] = inimg[e] ? xg[(int64_t)gy[e] * a.ld + gx[e]] : T(0);
    npix += inimg[e];
  }
  // pixels of the block inside the image (for the mean-abs rule)
  float npf = (float)npix;
  npf = group_sum<64>(npf);

  // active[k][e]: the level-k square holding pixel e lies inside the image
  // (one test per lane when the square holds all of the lane's pixels).
  bool active[K + 1][NPL];
#pragma unroll
  for (int k = 0; k <= K; ++k)
#pragma unroll
    for (int e = 0; e < NPL; ++e) {
      if ((1 << (2 * k)) >= NPL && e > 0) {
        active[k][e] = active[k][0];
        continue;
      }
      const int L = 1 << k;
      const int sy = gy[e] - ((gy[e] - by) & (L - 1));
      const int sx = gx[e] - ((gx[e] - bx) & (L - 1));
      active[k][e] = (lane * NPL + e) < NPX && sy >= 0 && sx >= 0 && sy + L <= a.H &&
                     sx + L <= a.W;
    }

  // squares this block projects per inner sweep: one leader pixel per square
  int leaders = 0;
#pragma unroll
  for (int k = 0; k <= K; ++k)
#pragma unroll
    for (int e = 0; e < NPL; ++e)
      leaders += (k >= i && active[k][e] && ((lane * NPL + e) & ((1 << (2 * k)) - 1)) == 0);
  float nsq = (float)leaders;
  nsq = group_sum<64>(nsq);
  // (square, pixel) pairs updated per inner sweep
  int upix = 0;
#pragma unroll
  for (int k = 0; k <= K; ++k)
#pragma unroll
    for (int e = 0; e < NPL; ++e) upix += (k >= i && active[k][e]);
  float nunit = (float)upix;
  nunit = group_sum<64>(nunit);

  T q[K + 1][NPL];
#pragma unroll
  for (int k = 0; k <= K; ++k)
#pragma unroll
    for (int e = 0; e < NPL; ++e) q[k][e] = T(0);

  int it = 0;
  bool met = false;  // the stopping rule held (else the block hit max_inner)
  while (true) {
    T dsum = T(0), dmax = T(0);
#pragma unroll
    for (int k = K; k >= 0; --k) {
      if (k < i) break;
      const T r2 = (T)a.r2[k];
      const T sr2 = (T)a.sr2[k];
      T y[NPL];
#pragma unroll
      for (int e = 0; e < NPL; ++e) y[e] = x[e] - q[k][e];
      T t[NPL];
      const int sq = 1 << (2 * k);  // pixels per square
      if (sq <= NPL) {
        // squares inside one lane: consecutive runs of sq Morton indices
#pragma unroll
        for (int e0 = 0; e0 < NPL; e0 += 1) {
          if (e0 % sq) continue;
          T n = T(0);
#pragma unroll
          for (int e = 0; e < NPL; ++e)
            if (e >= e0 && e < e0 + sq) n += y[e] * y[e];
          const T tt = ball_scale(n, r2, sr2);
#pragma unroll
          for (int e = 0; e < NPL; ++e)
            if (e >= e0 && e < e0 + sq) t[e] = tt;
        }
      } else {
        T part = T(0);
#pragma unroll
        for (int e = 0; e < NPL; ++e) part += y[e] * y[e];
        T n;
        switch (sq / NPL) {
          case 2: n = group_sum<2>(part); break;
          case 4: n = group_sum<4>(part); break;
          case 8: n = group_sum<8>(part); break;
          case 16: n = group_sum<16>(part); break;
          case 32: n = group_sum<32>(part); break;
          default: n = group_sum<64>(part); break;
        }
        const T tt = ball_scale(n, r2, sr2);
#pragma unroll
        for (int e = 0; e < NPL; ++e) t[e] = tt;
      }
#pragma unroll
      for (int e = 0; e < NPL; ++e) {
        if (active[k][e]) {
          const T xn = t[e] * y[e];
          q[k][e] = xn - y[e];
          const T d = fabs(x[e] - xn);
          if (MEANABS) dsum += d;
          else dmax = fmax(dmax, d);
          x[e] = xn;
        }
      }
    }
    ++it;
    bool stop;
    if (MEANABS) {
      const double s = group_sum<64>((double)dsum);
      stop = s <= a.tol * (double)npf;
    } else {
      stop = (double)wave_max(dmax) < a.tol;
    }
    met = stop;
    if (stop || it >= a.max_inner) break;
  }
#pragma unroll
  for (int e = 0; e < NPL; ++e)
    if (inimg[e]) xg[(int64_t)gy[e] * a.ld + gx[e]] = x[e];
  if (lane == 0) {
    const unsigned blk = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    unsigned long long* c = a.counters + (blk % kIcdSlots) * kIcdSlotWords;
    atomicAdd(c + 0, (unsigned long long)it);
    atomicAdd(c + 1, (unsigned long long)it * (unsigned long long)(nsq + 0.5f));
    atomicAdd(c + 2, (unsigned long long)it * (unsigned long long)(nunit + 0.5f));
    if (!met) atomicAdd(c + 3, 1ull);  // stopped by the cap
  }
}

}  // namespace smre
