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

#include <type_traits>

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

// v clamped to [-c, c] (c > 0, v finite)
template <typename T> __device__ __forceinline__ T clamp_t(T v, T c) {
  if constexpr (sizeof(T) == 8) return fmin(fmax(v, -c), c);
  else return __builtin_amdgcn_fmed3f(v, -c, c);
}

template <typename T> __device__ __forceinline__ T fma_t(T a, T b, T c) {
  if constexpr (sizeof(T) == 8) return __builtin_fma(a, b, c);
  else return __builtin_fmaf(a, b, c);
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
  uint32_t epoch;     // this call's number (see skip)
  double tol;
  double r2[6];
  float sr2[6];       // sqrtf((float)r2[k]) for the FP32 scale
  // Work counters (device): kIcdSlots slots of kIcdSlotWords words, one
  // 128-byte line each; a block adds its inner sweeps, square projections
  // and (square, pixel) updates to words 0, 1, 2 of slot (block id mod
  // kIcdSlots), so no line takes more than a share of the blocks' atomics.
  unsigned long long* counters;
  // null, or the number of the last call whose input check found a NaN or
  // Inf: when it is this call's (epoch), every block leaves the image as it is
  const unsigned* skip;
  // q = n / d for the launch's gridDim.x and gridDim.x * gridDim.y by a
  // multiply-high and shifts (udiv_magic), so the uniform block-index split
  // costs no VALU division sequence
  uint32_t nx_m, nx_s, nx_d, nxy_m, nxy_s, nxy_d;
  uint32_t nblocks;   // blocks of this launch: nx * ny * frames (< 2^31)
  uint32_t run;       // consecutive blocks per wave (1: one block per wave)
};
constexpr int kIcdSlots = 256, kIcdSlotWords = 16;

// Division by an invariant integer d >= 1 (Granlund & Montgomery, "Division
// by invariant integers using multiplication", PLDI 1994): with
// l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1 and t = mulhi(n, m),
// n / d = (t + ((n - t) >> 1)) >> (l - 1) for every 32-bit n (d = 1: n).
__host__ __device__ inline void udiv_magic(uint32_t d, uint32_t* m, uint32_t* sh) {
  if (d <= 1) {
    *m = 0;
    *sh = 0;
    return;
  }
  uint32_t l = 0;
  while (((uint64_t)1 << l) < d) ++l;
  *m = (uint32_t)((((uint64_t)1 << 32) * (((uint64_t)1 << l) - d)) / d + 1);
  *sh = l - 1;
}
__host__ __device__ inline uint32_t udiv_apply(uint32_t n, uint32_t d, uint32_t m, uint32_t sh) {
  if (d == 1) return n;
  const uint32_t t = (uint32_t)(((uint64_t)n * m) >> 32);
  return (t + ((n - t) >> 1)) >> sh;
}
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
// tol times its pixel count (accumulated per lane and summed over the wave in
// T, compared in FP64); else when max |dx| < tol.
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
__device__ __forceinline__ unsigned icd_remap(unsigned pid, unsigned total) {
  if (pid >= (total & ~127u)) return pid;
  const unsigned xcd = pid & 7u, slot = pid >> 3;
  return (((slot >> 4) << 3) + xcd) * 16u + (slot & 15u);
}
__device__ __forceinline__ void icd_block_of(const IcdArgs& a, unsigned lid, unsigned& bx,
                                             unsigned& by, unsigned& bz) {
  bz = udiv_apply(lid, a.nxy_d, a.nxy_m, a.nxy_s);
  const unsigned r = lid - bz * a.nxy_d;
  by = udiv_apply(r, a.nx_d, a.nx_m, a.nx_s);
  bx = r - by * a.nx_d;
}

// Per-wave totals of the work counters (uniform values).
struct IcdCount {
  unsigned long long inner = 0, squares = 0, units = 0, capped = 0;
};

// One block (tx, ty) of frame tz: load, inner sweeps until the block's rule
// holds or max_inner, store.
template <typename T, int K, bool MEANABS>
__device__ __forceinline__ void icd_block(const IcdArgs& a, unsigned tx, unsigned ty, unsigned tz,
                                          IcdCount& cnt) {
  constexpr int B = 1 << K;
  constexpr int NPX = B * B;
  constexpr int NPL = NPX >= 64 ? NPX / 64 : 1;
  constexpr int J = NPL == 1 ? 0 : NPL == 4 ? 1 : 2;  // NPL = 4^J
  const int lane = threadIdx.x;
  const int i = a.lmin;
  const int by = (a.oy > 0 ? a.oy - B : 0) + (int)ty * B;
  const int bx = (a.ox > 0 ? a.ox - B : 0) + (int)tx * B;
  T* xg = (T*)a.x + (int64_t)tz * a.fstride;
  // A block lying wholly inside the image projects every square of every
  // level: it runs without per-pixel masks and with its counts known.
  const bool interior = by >= 0 && bx >= 0 && by + B <= a.H && bx + B <= a.W;

  // pixel e of the lane has Morton index lane NPL + e: the lane gives the
  // high bits (a 2^J x 2^J tile), e the position inside it
  const bool lane_on = NPX >= 64 || lane < NPX;
  const int ly = by + (morton_y(lane) << J), lx = bx + (morton_x(lane) << J);
  int gy[NPL], gx[NPL];
#pragma unroll
  for (int e = 0; e < NPL; ++e) {
    gy[e] = ly + morton_y(e);
    gx[e] = lx + morton_x(e);
  }
  T x[NPL];
  bool inimg[NPL];
  // active[k][e]: the level-k square holding pixel e lies inside the image
  // (one test per lane when the square holds all of the lane's pixels)
  bool active[K + 1][NPL];
  float npf, nsq, nunit;  // block pixels in the image; squares and (square,
                          // pixel) pairs per inner sweep
  if (interior) {
#pragma unroll
    for (int e = 0; e < NPL; ++e) {
      inimg[e] = lane_on;
      x[e] = lane_on ? xg[(int64_t)gy[e] * a.ld + gx[e]] : T(0);
    }
    npf = (float)NPX;
    int ns = 0;
    for (int k = i; k <= K; ++k) ns += 1 << (2 * (K - k));
    nsq = (float)ns;
    nunit = (float)((K - i + 1) * NPX);
  } else {
    int npix = 0;
#pragma unroll
    for (int e = 0; e < NPL; ++e) {
      inimg[e] = lane_on && gy[e] >= 0 && gx[e] >= 0 && gy[e] < a.H && gx[e] < a.W;
      x[e] = inimg[e] ? xg[(int64_t)gy[e] * a.ld + gx[e]] : T(0);
      npix += inimg[e];
    }
    npf = group_sum<64>((float)npix);
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
        active[k][e] = lane_on && sy >= 0 && sx >= 0 && sy + L <= a.H && sx + L <= a.W;
      }
    // one leader pixel per square
    int leaders = 0, upix = 0;
#pragma unroll
    for (int k = 0; k <= K; ++k)
#pragma unroll
      for (int e = 0; e < NPL; ++e) {
        leaders += (k >= i && active[k][e] && ((lane * NPL + e) & ((1 << (2 * k)) - 1)) == 0);
        upix += (k >= i && active[k][e]);
      }
    nsq = group_sum<64>((float)leaders);
    nunit = group_sum<64>((float)upix);
  }

  T q[K + 1][NPL];
#pragma unroll
  for (int k = 0; k <= K; ++k)
#pragma unroll
    for (int e = 0; e < NPL; ++e) q[k][e] = T(0);

  // (Lanes past the block's pixels, K <= 2, hold zeros that stay zero.)
  // side-1 squares: the projection onto {v : v^2 <= r2} is the clamp to
  // [-sqrt(r2), sqrt(r2)] (Eq. (dykstra:if) with one pixel)
  const T c0 = (sizeof(T) == 8) ? (T)__builtin_sqrt(a.r2[0]) : (T)a.sr2[0];

  int it = 0;
  bool met = false;  // the stopping rule held (else the block hit max_inner)
  // The top level K (K >= 1) spans lanes: its inputs y = x - q[K] and their
  // group sum n are computed at the end of the previous sweep, before the
  // stopping test, so that test's wave reduction and this one run side by
  // side (same values; on stopping they are dropped).
  constexpr int GK = (1 << (2 * K)) / NPL;  // lanes per top-level square
  T yt[NPL];
  T nt = T(0);
  auto top_inputs = [&]() {
    if constexpr (K >= 1) {
#pragma unroll
      for (int e = 0; e < NPL; ++e) yt[e] = x[e] - q[K][e];
      T part = T(0);
#pragma unroll
      for (int e = 0; e < NPL; ++e) part = fma_t(yt[e], yt[e], part);
      nt = group_sum<GK>(part);
    }
  };
  top_inputs();
  auto sweeps = [&](auto interior_tag) {
    constexpr bool IN = decltype(interior_tag)::value;
    while (true) {
      T dsum = T(0), dmax = T(0);
#pragma unroll
      for (int k = K; k >= 0; --k) {
        if (k < i) break;
        const T r2 = (T)a.r2[k];
        const T sr2 = (T)a.sr2[k];
        T y[NPL], xn[NPL];
        const int sq = 1 << (2 * k);  // pixels per square
        if (k == K && K >= 1) {
          const T tt = ball_scale(nt, r2, sr2);
#pragma unroll
          for (int e = 0; e < NPL; ++e) {
            y[e] = yt[e];
            xn[e] = tt * y[e];
          }
        } else {
#pragma unroll
          for (int e = 0; e < NPL; ++e) y[e] = x[e] - q[k][e];
          if (k == 0) {
#pragma unroll
            for (int e = 0; e < NPL; ++e) xn[e] = clamp_t(y[e], c0);
          } else if (sq <= NPL) {
            // squares inside one lane: consecutive runs of sq Morton indices
#pragma unroll
            for (int e0 = 0; e0 < NPL; e0 += sq) {
              T n = T(0);
#pragma unroll
              for (int e = e0; e < e0 + sq; ++e) n = fma_t(y[e], y[e], n);
              const T tt = ball_scale(n, r2, sr2);
#pragma unroll
              for (int e = e0; e < e0 + sq; ++e) xn[e] = tt * y[e];
            }
          } else {
            T part = T(0);
#pragma unroll
            for (int e = 0; e < NPL; ++e) part = fma_t(y[e], y[e], part);
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
            for (int e = 0; e < NPL; ++e) xn[e] = tt * y[e];
          }
        }
#pragma unroll
        for (int e = 0; e < NPL; ++e) {
          if (IN || active[k][e]) {
            q[k][e] = xn[e] - y[e];
            const T d = fabs(x[e] - xn[e]);
            if (MEANABS) dsum += d;
            else dmax = fmax(dmax, d);
            x[e] = xn[e];
          }
        }
      }
      ++it;
      top_inputs();  // the next sweep's, beside the stopping test's reduction
      bool stop;
      if (MEANABS) {
        // FP32 images: the lane sums of |dx| are FP32 already, so the wave
        // sum is FP32 too; FP64 images sum in FP64
        const double s = (double)group_sum<64>(dsum);
        stop = s <= a.tol * (double)npf;
      } else {
        stop = (double)wave_max(dmax) < a.tol;
      }
      met = stop;
      if (stop || it >= a.max_inner) break;
    }
  };
  if (interior) sweeps(std::true_type{});
  else sweeps(std::false_type{});
#pragma unroll
  for (int e = 0; e < NPL; ++e)
    if (inimg[e]) xg[(int64_t)gy[e] * a.ld + gx[e]] = x[e];
  cnt.inner += (unsigned long long)it;
  cnt.squares += (unsigned long long)it * (unsigned long long)(nsq + 0.5f);
  cnt.units += (unsigned long long)it * (unsigned long long)(nunit + 0.5f);
  cnt.capped += met ? 0ull : 1ull;  // stopped by the cap
}

// One wave per run of `run` consecutive blocks (row-major over (x, y,
// frame)).  Workgroups reach the 8 XCDs in turn, so a run's neighbouring
// blocks share one L2.  With one block per wave (small launches, where every
// wave counts), the dispatch id is remapped so each XCD still gets runs of 16
// neighbours (icd_remap).  A wave adds its counts to one counter slot.
template <typename T, int K, bool MEANABS>
__global__ __launch_bounds__(64) void icd_phase(IcdArgs a) {
  if (a.skip && *a.skip == a.epoch) return;
  IcdCount cnt;
  const unsigned w = blockIdx.x;
  if (a.run == 1) {
    unsigned tx, ty, tz;
    icd_block_of(a, icd_remap(w, a.nblocks), tx, ty, tz);
    icd_block<T, K, MEANABS>(a, tx, ty, tz, cnt);
  } else {
    const unsigned b0 = w * a.run;
    const unsigned b1 = min(a.nblocks, b0 + a.run);
    for (unsigned b = b0; b < b1; ++b) {
      unsigned tx, ty, tz;
      icd_block_of(a, b, tx, ty, tz);
      icd_block<T, K, MEANABS>(a, tx, ty, tz, cnt);
    }
  }
  if (threadIdx.x == 0) {
    unsigned long long* c = a.counters + (w % kIcdSlots) * kIcdSlotWords;
    atomicAdd(c + 0, cnt.inner);
    atomicAdd(c + 1, cnt.squares);
    atomicAdd(c + 2, cnt.units);
    if (cnt.capped) atomicAdd(c + 3, cnt.capped);
  }
}

}  // namespace smre
