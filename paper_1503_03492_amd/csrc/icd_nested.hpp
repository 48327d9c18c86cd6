// icd_nested.hpp -- incomplete Dykstra over a nested hierarchy of squares of
// any sides, for gfx950.
//
// Sec. 3.2 builds its subsets from squares of side 2^k; the hierarchy here is
// any divisor chain side[0] | side[1] | ... | side[n-1] = B (e.g. 1, 3, 6, 12,
// 24, 48, or 1, 2, ..., 64 for blocks larger than one wave holds).  A phase
// takes blocks of side B on a shifted lattice; a block runs Dykstra over its
// squares of the levels n-1 down to lo (those inside the image), increments
// zeroed at the phase start, until its stopping rule holds.  Blocks are
// disjoint, so one workgroup per block runs them all at once.
//
// Layout: the block's B^2 pixels in nested order -- the sub-squares of every
// square visited in raster order, recursively, and the pixels of a level-0
// square in raster order -- so every square of every level is a contiguous run
// of indices.  Lane t holds the P = side[m]^2 consecutive indices of the t-th
// level-m square (P <= 16): a square of a level j <= m is a run of side[j]^2
// elements inside one lane (summed by a segmented scan over the lane's
// registers); a square of a level j > m is an aligned group of
// (side[j] / side[m])^2 lanes (summed by xor butterflies when the group is a
// power of two inside a wave, else by a tree in LDS).  Pixels and increments
// stay in registers; HBM sees one read and one write of x per phase.
#pragma once

#include "icd.hpp"

namespace smre {

constexpr int kNestLevels = 7;  // a divisor chain up to side 96 has at most 7 levels

struct NestedArgs {
  void* x;                 // frame 0; frame f at x + f * fstride elements
  int64_t fstride;
  int64_t ld;
  int32_t H, W;
  int32_t oy, ox;          // lattice origin: shift - B, or 0 for shift 0
  int32_t nbx;             // blocks per lattice row
  int32_t B, nlev, lo, m;  // block side, levels, lowest level of the phase, lane level
  int32_t nt;              // lanes holding pixels: B^2 / P
  int32_t mode, max_inner;
  double tol;
  int32_t side[kNestLevels];
  int32_t grp[kNestLevels];      // lanes per square (levels above m; 1 at or below)
  int32_t rad[kNestLevels];      // side[j] / side[j - 1] (j >= 1)
  uint32_t rstart[kNestLevels];  // levels j <= m: bit e set where a square's run starts
  uint32_t rend[kNestLevels];    // ... and where it ends
  uint8_t pr[16], pc[16];        // element e: offset inside the lane's level-m square
  uint8_t sqr[kNestLevels][16];  // levels j <= m: corner of element e's square, in the
  uint8_t sqc[kNestLevels][16];  //   lane's square
  double r2[kNestLevels];
  float sr2[kNestLevels];        // sqrtf((float)r2[j]) for the FP32 scale
  unsigned long long* counters;  // kIcdSlots slots of kIcdSlotWords words (as icd_phase)
  const unsigned* skip;          // null, or the non-finite input call number (as icd_phase)
  uint32_t epoch, pad;           // this call's number
};

// Sum of v over the aligned group of G lanes containing this one; every lane
// of a group gets the same bits.  gi = lane index inside its group.  Uniform
// in G across the workgroup (the LDS paths have barriers).
//
// G a power of two: DPP and permlane steps inside the wave (lane a with lane
// a ^ 1, then a ^ 2, ...), and for G > 64 the wave totals of the group added
// as a pairwise tree after one barrier: the pairs the binary tree over lanes
// forms, so the same bits.  The wave totals go to wsum[par] and par flips, so
// the next call writes the other half (every lane has passed this call's
// barrier before it reads the other half again, at the next call's).
// Otherwise a binary tree over the lanes in LDS, a barrier per step.
template <typename T, int MAXW>  // MAXW: the most waves a workgroup has
__device__ __forceinline__ T nested_group_sum(T v, int G, int gi, int t, int nt, T* part,
                                              T (*wsum)[16], int& par) {
  if ((G & (G - 1)) == 0) {
    switch (G) {
      case 1: return v;
      case 2: return group_sum<2>(v);
      case 4: return group_sum<4>(v);
      case 8: return group_sum<8>(v);
      case 16: return group_sum<16>(v);
      case 32: return group_sum<32>(v);
      default: break;
    }
    v = group_sum<64>(v);
    if (G == 64) return v;
    const int gw = G >> 6, w0 = (t - gi) >> 6;  // waves of the group, its first
    if ((t & 63) == 0) wsum[par][t >> 6] = v;
    __syncthreads();
    T w[MAXW];
#pragma unroll
    for (int i = 0; i < MAXW; ++i) w[i] = i < gw ? wsum[par][w0 + i] : T(0);
#pragma unroll
    for (int s = 1; s < MAXW; s <<= 1)
#pragma unroll
      for (int i = 0; i + s < MAXW; i += 2 * s)
        if (i + s < gw) w[i] = w[i] + w[i + s];
    par ^= 1;
    return w[0];
  }
  part[t] = v;
  __syncthreads();
  for (int s = 1; s < G; s <<= 1) {
    if (t < nt && (gi & (2 * s - 1)) == 0 && gi + s < G) part[t] += part[t + s];
    __syncthreads();
  }
  const T r = part[t - gi];
  __syncthreads();  // before part is written again
  return r;
}

template <typename T, int P, bool MEANABS>
__global__ __launch_bounds__(P == 16 ? 256 : P == 9 ? 512 : 1024)
void icd_nested_phase(NestedArgs a) {
  if (a.skip && *a.skip == a.epoch) return;
  __shared__ T part[1024];
  __shared__ T wred[2][16];
  __shared__ unsigned long long wcnt[16][2];
  __shared__ T wsum[2][16];  // wave totals of the power-of-two group sums
  int wpar = 0;
  const int t = threadIdx.x;
  const int nwaves = (blockDim.x + 63) >> 6;
  const int wave = t >> 6, lane = t & 63;
  T* x = (T*)a.x + (int64_t)blockIdx.y * a.fstride;
  const int bry = (int)blockIdx.x / a.nbx, brx = (int)blockIdx.x - bry * a.nbx;
  const int by0 = a.oy + bry * a.B, bx0 = a.ox + brx * a.B;
  const bool has = t < a.nt;

  // corner of this lane's level-m square inside the block: the digits of t,
  // lowest first, pick a sub-square at each level above m
  int lr = 0, lc = 0;
  {
    int u = t;
    for (int j = a.m + 1; j < a.nlev; ++j) {
      const int r = a.rad[j], rr = r * r;
      const int d = u % rr;
      u /= rr;
      lr += (d / r) * a.side[j - 1];
      lc += (d % r) * a.side[j - 1];
    }
  }
  const int r0 = max(by0, 0), r1 = min(by0 + a.B, a.H);
  const int c0 = max(bx0, 0), c1 = min(bx0 + a.B, a.W);
  const bool interior = by0 >= 0 && bx0 >= 0 && by0 + a.B <= a.H && bx0 + a.B <= a.W;
  const T npix = (T)((r1 - r0) * (c1 - c0));

  T xv[P];
  uint32_t inb = 0;
#pragma unroll
  for (int e = 0; e < P; ++e) {
    const int row = by0 + lr + a.pr[e], col = bx0 + lc + a.pc[e];
    const bool ok = has && row >= 0 && col >= 0 && row < a.H && col < a.W;
    xv[e] = ok ? x[(int64_t)row * a.ld + col] : T(0);
    inb |= (uint32_t)ok << e;
  }
  // squares inside the image, per level: bit e = element e's square is
  uint32_t vm[kNestLevels];
  int gidx[kNestLevels];
  unsigned long long nsq = 0, npx = 0;  // square projections and pixel updates per inner sweep
#pragma unroll
  for (int j = 0; j < kNestLevels; ++j) {
    vm[j] = 0;
    gidx[j] = 0;
    if (j >= a.nlev || j < a.lo || !has) continue;
    const int L = a.side[j];
    if (j <= a.m) {
      uint32_t v = 0;
#pragma unroll
      for (int e = 0; e < P; ++e) {
        const int sr = by0 + lr + a.sqr[j][e], sc = bx0 + lc + a.sqc[j][e];
        const bool ok = interior || (sr >= 0 && sc >= 0 && sr + L <= a.H && sc + L <= a.W);
        v |= (uint32_t)ok << e;
      }
      vm[j] = v;
      nsq += __builtin_popcount(v & a.rstart[j]);
    } else {
      const int sr = by0 + (lr / L) * L, sc = bx0 + (lc / L) * L;
      const bool ok = interior || (sr >= 0 && sc >= 0 && sr + L <= a.H && sc + L <= a.W);
      vm[j] = ok ? ((1u << P) - 1u) : 0u;
      gidx[j] = t % a.grp[j];
      nsq += (ok && gidx[j] == 0) ? 1 : 0;
    }
    npx += __builtin_popcount(vm[j]);
  }

  T q[kNestLevels][P];
#pragma unroll
  for (int j = 0; j < kNestLevels; ++j)
#pragma unroll
    for (int e = 0; e < P; ++e) q[j][e] = T(0);

  int it = 0;
  bool met = false;
  while (it < a.max_inner) {
    T dacc = T(0);
#pragma unroll
    for (int j = kNestLevels - 1; j >= 0; --j) {
      if (j >= a.nlev || j < a.lo) continue;  // uniform
      const T r2 = (T)a.r2[j];
      const T sr2 = (T)a.sr2[j];
      T y[P], n[P];
#pragma unroll
      for (int e = 0; e < P; ++e) y[e] = xv[e] + q[j][e];
      if (j <= a.m) {
        // runs of side[j]^2 elements: a forward scan that restarts at each
        // run start, then each run's total carried back over the run
        const uint32_t st = a.rstart[j], en = a.rend[j];
        T s[P];
        T acc = T(0);
#pragma unroll
        for (int e = 0; e < P; ++e) {
          acc = ((st >> e) & 1u) ? y[e] * y[e] : fma_t(y[e], y[e], acc);
          s[e] = acc;
        }
        T tot = s[P - 1];
#pragma unroll
        for (int e = P - 1; e >= 0; --e) {
          if ((en >> e) & 1u) tot = s[e];
          n[e] = tot;
        }
      } else {
        T ps = T(0);
#pragma unroll
        for (int e = 0; e < P; ++e) ps = fma_t(y[e], y[e], ps);
        const T sum = nested_group_sum<T, (P == 16 ? 256 : P == 9 ? 512 : 1024) / 64>(
            ps, a.grp[j], gidx[j], t, a.nt, part, wsum, wpar);
#pragma unroll
        for (int e = 0; e < P; ++e) n[e] = sum;
      }
#pragma unroll
      for (int e = 0; e < P; ++e) {
        const T sc = ((vm[j] >> e) & 1u) ? ball_scale<T>(n[e], r2, sr2) : T(1);
        const T xn = sc * y[e];
        const T d = xv[e] > xn ? xv[e] - xn : xn - xv[e];
        if constexpr (MEANABS) dacc += d;
        else dacc = dacc > d ? dacc : d;
        q[j][e] = y[e] - xn;
        xv[e] = xn;
      }
    }
    ++it;
    // the block's stopping rule, the same decision in every lane: wave
    // butterflies, then the wave results in wave order
    T v = dacc;
    if constexpr (MEANABS) {
      v = group_sum<64>(v);
    } else {
      for (int o = 32; o > 0; o >>= 1) {
        const T w = __shfl_xor(v, o);
        v = v > w ? v : w;
      }
    }
    if (lane == 0) wred[it & 1][wave] = v;
    __syncthreads();
    T tot = wred[it & 1][0];
    for (int w = 1; w < nwaves; ++w) {
      const T u = wred[it & 1][w];
      if constexpr (MEANABS) tot += u;
      else tot = tot > u ? tot : u;
    }
    // the sum in the image precision, the comparison in FP64 (as icd_phase)
    if (MEANABS ? ((double)tot <= a.tol * (double)npix) : ((double)tot < a.tol)) {
      met = true;
      break;
    }
  }

#pragma unroll
  for (int e = 0; e < P; ++e) {
    if ((inb >> e) & 1u) {
      const int row = by0 + lr + a.pr[e], col = bx0 + lc + a.pc[e];
      x[(int64_t)row * a.ld + col] = xv[e];
    }
  }

  // counters: inner sweeps, square projections, (square, pixel) updates,
  // blocks stopped by max_inner
  unsigned long long c1v = nsq * (unsigned long long)it, c2v = npx * (unsigned long long)it;
  for (int o = 32; o > 0; o >>= 1) {
    c1v += __shfl_xor(c1v, o);
    c2v += __shfl_xor(c2v, o);
  }
  if (lane == 0) {
    wcnt[wave][0] = c1v;
    wcnt[wave][1] = c2v;
  }
  __syncthreads();
  if (t == 0) {
    unsigned long long s1 = 0, s2 = 0;
    for (int w = 0; w < nwaves; ++w) {
      s1 += wcnt[w][0];
      s2 += wcnt[w][1];
    }
    unsigned long long* slot =
        a.counters + (size_t)((blockIdx.x + blockIdx.y * gridDim.x) % kIcdSlots) * kIcdSlotWords;
    atomicAdd(slot + 0, (unsigned long long)it);
    atomicAdd(slot + 1, s1);
    atomicAdd(slot + 2, s2);
    if (!met) atomicAdd(slot + 3, 1ull);
  }
}

}  // namespace smre
