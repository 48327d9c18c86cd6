// kernels.hpp -- gfx950 device code of the SMRE projection library.
//
// Full Dykstra (Sec. 2.3, Algorithm 2, projection Eq. (dykstra:if)) runs as
// "region phases": the anchor plane (top-left pixels of windows) is cut into
// R x R regions, coloured 2 (p mod 2) + (q mod 2).  One launch processes all
// regions of one colour; with R >= smax - 1 their pixel footprints
// (R + smax - 1)^2 are disjoint, so the launch needs no ordering between
// workgroups.  Inside a region the workgroup visits every window anchored in
// it, side by side (descending), tiling offset by tiling offset; windows of one
// tiling are disjoint (Sec. 2.3), so a step projects all of them at once.
//
// Workgroup = 2 waves:
//   wave 0 (consumer) keeps the region's x footprint in LDS for the whole
//     phase and runs the steps: y = x + I, n = sum y^2 per window (lanes of a
//     window reduce with DPP / permlane swaps), t = sqrt(r2/n) if n > r2,
//     x' = t y, I' = y - x'.  I' is stored straight to HBM.
//   wave 1 (producer) streams the region's increments -- one contiguous
//     range of the increment buffer per region and sweep -- through a ring of
//     1 KiB pages in LDS, several loads in flight, gated by the consumer's
//     progress.  The two waves synchronise through two LDS counters only.
//
// Increment layout: for each region (raster order), its steps in visiting
// order; inside a step, rounds of up to 64/G windows; inside a round, slots
// (u, v) in order; inside a slot, the active lanes' elements contiguously.
// Every load and store of a slot is therefore one dense run of elements.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smre {

constexpr int kPage = 1024;            // bytes per prefetch page (64 lanes x 16 B)
constexpr int kSlots = 32;             // pages in the LDS ring
constexpr int kRing = kPage * kSlots;  // ring bytes
constexpr int kMaxSides = 32;
constexpr int kPrefetch = 8;           // producer loads in flight

typedef uint16_t bf16_t;  // increment storage in bfloat16 (round to nearest even)
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

template <typename TQ, typename TC> struct QStore;
template <> struct QStore<float, float> {
  static __device__ __forceinline__ float get(const unsigned char* p) { return *(const float*)p; }
  static __device__ __forceinline__ void put(float* q, float v) { *q = v; }
};
template <> struct QStore<double, double> {
  static __device__ __forceinline__ double get(const unsigned char* p) { return *(const double*)p; }
  static __device__ __forceinline__ void put(double* q, double v) { *q = v; }
};
template <> struct QStore<bf16_t, float> {
  static __device__ __forceinline__ float get(const unsigned char* p) {
    return bf2f(*(const bf16_t*)p);
  }
  static __device__ __forceinline__ void put(bf16_t* q, float v) { *q = f2bf(v); }
};

// ---------------------------------------------------------------- lane patterns
// A window of side S is served by G = GR x GC lanes: lane (jr, jc) holds the
// pixels (jr + u GR, jc + v GC), u < U, v < V.  Chosen per (R, S) by a cost
// model of rounds x (round overhead + elements per lane + reduction steps).
struct Pattern {
  int gr, gc;
};
__host__ __device__ constexpr Pattern pattern(int R, int S) {
  if (R == 8) {
    constexpr Pattern t[10] = {{1, 1}, {1, 1}, {2, 2}, {1, 4}, {4, 4}, {2, 8},
                               {2, 8}, {4, 8}, {8, 8}, {4, 16}};
    return t[S];
  }
  if (R == 16) {
    constexpr Pattern t[18] = {{1, 1}, {1, 1}, {1, 1},  {1, 2},  {1, 4},  {2, 2},
                               {2, 2}, {1, 8}, {2, 8},  {1, 16}, {4, 4},  {4, 4},
                               {2, 16}, {2, 16}, {2, 16}, {4, 16}, {4, 16}, {2, 32}};
    return t[S];
  }
  constexpr Pattern t[34] = {{1, 1},  {1, 1},  {1, 1},  {1, 1},  {1, 1},  {1, 1},  {1, 2},
                             {1, 2},  {1, 4},  {2, 2},  {2, 2},  {1, 4},  {2, 4},  {1, 16},
                             {1, 16}, {1, 16}, {1, 16}, {4, 4},  {4, 4},  {4, 4},  {4, 8},
                             {4, 8},  {4, 8},  {4, 8},  {4, 8},  {2, 32}, {2, 32}, {2, 32},
                             {2, 32}, {2, 32}, {2, 32}, {2, 32}, {2, 32}, {2, 32}};
  return t[S];
}

// ---------------------------------------------------------------- reductions
// All-reduce (sum) over aligned groups of G lanes; every lane of a group gets
// the same bits.  Steps inside a row of 16 use DPP, across rows the gfx950
// permlane swaps; all VALU, no LDS.
__device__ __forceinline__ float dpp_f(float v, int ctrl) {
  switch (ctrl) {
    case 0xB1: return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
    case 0x4E: return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));
    case 0x141: return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, false));
    default: return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xF, 0xF, false));
  }
}

template <int G> __device__ __forceinline__ float group_sum(float v) {
  if constexpr (G >= 2) v += dpp_f(v, 0xB1);   // quad_perm 1,0,3,2
  if constexpr (G >= 4) v += dpp_f(v, 0x4E);   // quad_perm 2,3,0,1
  if constexpr (G >= 8) v += dpp_f(v, 0x141);  // row_half_mirror
  if constexpr (G >= 16) v += dpp_f(v, 0x140); // row_mirror
  if constexpr (G >= 32) {
    auto p = __builtin_amdgcn_permlane16_swap(__float_as_int(v), __float_as_int(v), false, false);
    v = __int_as_float(p[0]) + __int_as_float(p[1]);
  }
  if constexpr (G >= 64) {
    auto p = __builtin_amdgcn_permlane32_swap(__float_as_int(v), __float_as_int(v), false, false);
    v = __int_as_float(p[0]) + __int_as_float(p[1]);
  }
  return v;
}

__device__ __forceinline__ double dpp_d(double v, int ctrl) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  switch (ctrl) {
    case 0xB1:
      lo = __builtin_amdgcn_update_dpp(0, lo, 0xB1, 0xF, 0xF, false);
      hi = __builtin_amdgcn_update_dpp(0, hi, 0xB1, 0xF, 0xF, false);
      break;
    case 0x4E:
      lo = __builtin_amdgcn_update_dpp(0, lo, 0x4E, 0xF, 0xF, false);
      hi = __builtin_amdgcn_update_dpp(0, hi, 0x4E, 0xF, 0xF, false);
      break;
    case 0x141:
      lo = __builtin_amdgcn_update_dpp(0, lo, 0x141, 0xF, 0xF, false);
      hi = __builtin_amdgcn_update_dpp(0, hi, 0x141, 0xF, 0xF, false);
      break;
    default:
      lo = __builtin_amdgcn_update_dpp(0, lo, 0x140, 0xF, 0xF, false);
      hi = __builtin_amdgcn_update_dpp(0, hi, 0x140, 0xF, 0xF, false);
      break;
  }
  return __hiloint2double(hi, lo);
}

template <int G> __device__ __forceinline__ double group_sum(double v) {
  if constexpr (G >= 2) v += dpp_d(v, 0xB1);
  if constexpr (G >= 4) v += dpp_d(v, 0x4E);
  if constexpr (G >= 8) v += dpp_d(v, 0x141);
  if constexpr (G >= 16) v += dpp_d(v, 0x140);
  if constexpr (G >= 32) {
    int lo = __double2loint(v), hi = __double2hiint(v);
    auto pl = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    auto ph = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    v = __hiloint2double(ph[0], pl[0]) + __hiloint2double(ph[1], pl[1]);
  }
  if constexpr (G >= 64) {
    int lo = __double2loint(v), hi = __double2hiint(v);
    auto pl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    auto ph = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    v = __hiloint2double(ph[0], pl[0]) + __hiloint2double(ph[1], pl[1]);
  }
  return v;
}

// ---------------------------------------------------------------- LDS counters
__device__ __forceinline__ int lds_load(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_store(int* p, int v) {
  // The ring data written before this store reaches LDS first: one wave's LDS
  // instructions execute in order, and the asm barrier keeps the compiler
  // from moving them across.
  __asm__ volatile("" ::: "memory");
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// ---------------------------------------------------------------- phase kernel
struct PhaseArgs {
  void* x;              // image (TX), row stride ld
  const int64_t* roff;  // increment offset (elements) of each region, raster, +1 sentinel
  void* q;              // increment stream (TQ)
  const int* done;      // device flag: converged, skip remaining work
  int64_t ld;
  int32_t H, W;
  int32_t nrx;          // regions per row
  int32_t cy, cx;       // colour of this launch
  int32_t ncx;          // regions of this colour per row
  int32_t fr;           // footprint side R + smax - 1
  int32_t nsides;
  int32_t kahan;
  float guard;          // FP32 recheck band (relative)
  int32_t sides[kMaxSides];  // descending
  float r2f[kMaxSides];
  double r2d[kMaxSides];
};

template <typename TX, typename TQ, int R, int SMAX> struct PhaseShape {
  static constexpr int FR = R + SMAX - 1;
  static constexpr int P = (FR % 2 == 0) ? FR + 1 : FR;  // odd pitch: fewer bank conflicts
};

struct Consumer {
  unsigned char* ring;
  int* ready;     // pages (relative to p_lo) present in the ring
  int* consumed;  // first page (relative) still needed
  int64_t p_lo;
  int64_t qpos;   // next increment element of this region
  int r0, c0;     // anchor origin of the region (= footprint origin)
  int lane;
};

template <typename TX, typename TQ, int R, int SMAX, int S>
__device__ __forceinline__ void run_side(const PhaseArgs& a, Consumer& c, TX* xs, int k) {
  constexpr Pattern pt = pattern(R, S);
  constexpr int GR = pt.gr, GC = pt.gc, G = GR * GC, WR = 64 / G;
  constexpr int U = (S + GR - 1) / GR, V = (S + GC - 1) / GC;
  constexpr int P = PhaseShape<TX, TQ, R, SMAX>::P;
  constexpr int ES = (int)sizeof(TQ);
  using QS = QStore<TQ, TX>;

  const int wl = c.lane / G, jj = c.lane % G, jr = jj / GC, jc = jj % GC;
  const int rhi = min(c.r0 + R, a.H - S + 1), chi = min(c.c0 + R, a.W - S + 1);
  const TX r2 = (sizeof(TX) == 8) ? (TX)a.r2d[k] : (TX)a.r2f[k];
  const double r2d = a.r2d[k];
  TQ* qg = (TQ*)a.q;

  // Per-lane rank of its element inside a slot, for the (up to) four shapes
  // of slot: full / partial row block x full / partial column block.
  int rank[2][2];
#pragma unroll
  for (int ur = 0; ur < 2; ++ur)
#pragma unroll
    for (int vc = 0; vc < 2; ++vc) {
      const int jrn = ur ? (S - (U - 1) * GR) : GR;
      const int jcn = vc ? (S - (V - 1) * GC) : GC;
      rank[ur][vc] = wl * jrn * jcn + jr * jcn + jc;
    }

  for (int oa = 0; oa < S; ++oa) {
    const int i0 = c.r0 + ((oa - c.r0 % S) % S + S) % S;
    const int nr = i0 < rhi ? (rhi - i0 + S - 1) / S : 0;
    if (nr == 0) continue;
    for (int ob = 0; ob < S; ++ob) {
      const int j0 = c.c0 + ((ob - c.c0 % S) % S + S) % S;
      const int nc = j0 < chi ? (chi - j0 + S - 1) / S : 0;
      const int nw = nr * nc;
      for (int rb = 0; rb < nw; rb += WR) {
        const int nwr = min(WR, nw - rb);
        const bool valid = wl < nwr;
        const int w = rb + wl;
        const int wy = w / nc, wx = w - (w / nc) * nc;
        const int xb = (i0 - c.r0 + wy * S + jr) * P + (j0 - c.c0 + wx * S + jc);
        const int64_t chunk = c.qpos;
        c.qpos += (int64_t)nwr * S * S;
        // wait until every page holding [chunk, qpos) is in the ring
        const int need = (int)((c.qpos * ES + kPage - 1) / kPage - c.p_lo);
        while (lds_load(c.ready) < need) __builtin_amdgcn_s_sleep(1);
        __asm__ volatile("" ::: "memory");
        const uint32_t cb = (uint32_t)((uint64_t)chunk * ES);
        TQ* qr = qg + chunk;

        TX y[U][V];
        TX acc = 0, comp = 0;
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int v = 0; v < V; ++v) {
            const int jrn = (u == U - 1) ? (S - (U - 1) * GR) : GR;
            const int jcn = (v == V - 1) ? (S - (V - 1) * GC) : GC;
            const int cuv = u * GR * S + jrn * v * GC;
            const bool in = valid && (jr < jrn) && (jc < jcn);
            TX yv = 0;
            if (in) {
              const int rk = rank[u == U - 1 ? 1 : 0][v == V - 1 ? 1 : 0];
              const uint32_t off = (cb + (uint32_t)((nwr * cuv + rk) * ES)) & (kRing - 1);
              const TX qv = QS::get(c.ring + off);
              yv = xs[xb + u * GR * P + v * GC] + qv;
            }
            y[u][v] = yv;
            if constexpr (sizeof(TX) == 4) {
              if (a.kahan) {
                const TX t2 = __builtin_fmaf(yv, yv, -comp);
                const TX s2 = acc + t2;
                comp = (s2 - acc) - t2;
                acc = s2;
              } else {
                acc = __builtin_fmaf(yv, yv, acc);
              }
            } else {
              acc = __builtin_fma(yv, yv, acc);
            }
          }
        if constexpr (sizeof(TX) == 4) acc -= comp;
        TX n = group_sum<G>(acc);
        TX t = 1;
        if constexpr (sizeof(TX) == 4) {
          // FP64 recheck of windows whose sum lies within the guard band.
          const bool near = a.guard > 0.f && fabsf(n - r2) <= a.guard * r2;
          if (__builtin_amdgcn_read_exec() & __ballot(near)) {
            double pd = 0.0;
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
              for (int v = 0; v < V; ++v) pd = __builtin_fma((double)y[u][v], (double)y[u][v], pd);
            const double nd = group_sum<G>(pd);
            if (near) {
              t = nd > r2d ? (float)__builtin_sqrt(r2d / nd) : 1.0f;
            } else if (n > r2) {
              t = __builtin_sqrtf(r2 / n);
            }
          } else if (n > r2) {
            t = __builtin_sqrtf(r2 / n);
          }
        } else {
          if (n > r2) t = __builtin_sqrt(r2 / n);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int v = 0; v < V; ++v) {
            const int jrn = (u == U - 1) ? (S - (U - 1) * GR) : GR;
            const int jcn = (v == V - 1) ? (S - (V - 1) * GC) : GC;
            const int cuv = u * GR * S + jrn * v * GC;
            const bool in = valid && (jr < jrn) && (jc < jcn);
            if (in) {
              const int rk = rank[u == U - 1 ? 1 : 0][v == V - 1 ? 1 : 0];
              const TX xn = t * y[u][v];
              xs[xb + u * GR * P + v * GC] = xn;
              QS::put(qr + (nwr * cuv + rk), y[u][v] - xn);
            }
          }
        __asm__ volatile("" ::: "memory");
        lds_store(c.consumed, (int)((c.qpos * ES) / kPage - c.p_lo));
      }
    }
  }
}

template <typename TX, typename TQ, int R, int SMAX>
__device__ __forceinline__ void dispatch_side(const PhaseArgs& a, Consumer& c, TX* xs, int k) {
  switch (a.sides[k]) {
#define SMRE_SIDE_CASE(n) \
  case n:                 \
    if constexpr (n <= SMAX) run_side<TX, TQ, R, SMAX, n>(a, c, xs, k); \
    break;
    SMRE_SIDE_CASE(1) SMRE_SIDE_CASE(2) SMRE_SIDE_CASE(3) SMRE_SIDE_CASE(4) SMRE_SIDE_CASE(5)
    SMRE_SIDE_CASE(6) SMRE_SIDE_CASE(7) SMRE_SIDE_CASE(8) SMRE_SIDE_CASE(9) SMRE_SIDE_CASE(10)
    SMRE_SIDE_CASE(11) SMRE_SIDE_CASE(12) SMRE_SIDE_CASE(13) SMRE_SIDE_CASE(14)
    SMRE_SIDE_CASE(15) SMRE_SIDE_CASE(16) SMRE_SIDE_CASE(17) SMRE_SIDE_CASE(18)
    SMRE_SIDE_CASE(19) SMRE_SIDE_CASE(20) SMRE_SIDE_CASE(21) SMRE_SIDE_CASE(22)
    SMRE_SIDE_CASE(23) SMRE_SIDE_CASE(24) SMRE_SIDE_CASE(25) SMRE_SIDE_CASE(26)
    SMRE_SIDE_CASE(27) SMRE_SIDE_CASE(28) SMRE_SIDE_CASE(29) SMRE_SIDE_CASE(30)
    SMRE_SIDE_CASE(31) SMRE_SIDE_CASE(32)
#undef SMRE_SIDE_CASE
    default: break;
  }
}

// Producer wave: copy pages [p_lo, p_hi) of the increment stream into the
// ring, kPrefetch loads in flight, never more than kSlots pages ahead of the
// consumer.
__device__ __forceinline__ void produce(const u32x4* src, int64_t p_lo, int64_t p_hi, u32x4* ring,
                                        int* ready, const int* consumed, int lane) {
  const int npg = (int)(p_hi - p_lo);
  if (npg <= 0) return;
  u32x4 buf[kPrefetch];
#pragma unroll
  for (int k = 0; k < kPrefetch; ++k) {
    const int64_t pg = p_lo + min(k, npg - 1);
    buf[k] = __builtin_nontemporal_load(src + pg * 64 + lane);
  }
  for (int base = 0; base < npg; base += kPrefetch) {
#pragma unroll
    for (int k = 0; k < kPrefetch; ++k) {
      const int pg = base + k;
      if (pg < npg) {
        while (pg >= lds_load(consumed) + kSlots) __builtin_amdgcn_s_sleep(1);
        __asm__ volatile("" ::: "memory");
        ring[(int)((p_lo + pg) % kSlots) * 64 + lane] = buf[k];
        lds_store(ready, pg + 1);
        const int64_t nx = p_lo + min(pg + kPrefetch, npg - 1);
        buf[k] = __builtin_nontemporal_load(src + nx * 64 + lane);
      }
    }
  }
}

template <typename TX, typename TQ, int R, int SMAX>
__global__ __launch_bounds__(128) void region_phase(PhaseArgs a) {
  using SH = PhaseShape<TX, TQ, R, SMAX>;
  __shared__ __attribute__((aligned(16))) unsigned char ring[kRing];
  __shared__ TX xs[SH::FR * SH::P];
  __shared__ int ctr[2];
  if (*a.done) return;

  const int b = blockIdx.x;
  const int ry = a.cy + 2 * (b / a.ncx), rx = a.cx + 2 * (b % a.ncx);
  const int region = ry * a.nrx + rx;
  const int64_t e_lo = a.roff[region], e_hi = a.roff[region + 1];
  const int64_t p_lo = (e_lo * (int64_t)sizeof(TQ)) / kPage;
  const int64_t p_hi = (e_hi * (int64_t)sizeof(TQ) + kPage - 1) / kPage;
  const int lane = threadIdx.x & 63;
  if (threadIdx.x == 0) {
    ctr[0] = 0;
    ctr[1] = 0;
  }
  __syncthreads();

  if (threadIdx.x >= 64) {
    produce((const u32x4*)a.q, p_lo, p_hi, (u32x4*)ring, &ctr[0], &ctr[1], lane);
    return;
  }

  const int r0 = ry * R, c0 = rx * R;
  const int fh = min(a.fr, a.H - r0), fw = min(a.fr, a.W - c0);
  TX* xg = (TX*)a.x;
  for (int idx = lane; idx < fh * fw; idx += 64) {
    const int i = idx / fw, j = idx - (idx / fw) * fw;
    xs[i * SH::P + j] = xg[(int64_t)(r0 + i) * a.ld + c0 + j];
  }
  __asm__ volatile("" ::: "memory");

  Consumer c{ring, &ctr[0], &ctr[1], p_lo, e_lo, r0, c0, lane};
  for (int k = 0; k < a.nsides; ++k) dispatch_side<TX, TQ, R, SMAX>(a, c, xs, k);

  __asm__ volatile("" ::: "memory");
  for (int idx = lane; idx < fh * fw; idx += 64) {
    const int i = idx / fw, j = idx - (idx / fw) * fw;
    xg[(int64_t)(r0 + i) * a.ld + c0 + j] = xs[i * SH::P + j];
  }
}

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

struct Ctrl {
  int done;            // converged flag read by every sweep kernel
  int done_sweep;      // sweep at which it converged
  int nonfinite;       // input check result
  int pad;
  unsigned long long delta_key;  // running max |x - prev| of the checked sweep
  double last_delta;
  unsigned long long viol_key;   // running max violation
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

template <typename TX>
__global__ __launch_bounds__(256) void snapshot_kernel(const TX* x, int64_t ld, int H, int W,
                                                       TX* prev, Ctrl* ctrl) {
  if (ctrl->done) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) ctrl->delta_key = dkey(0.0);
  const int64_t n = (int64_t)H * W;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / W, col = i - r * W;
    prev[i] = x[r * ld + col];
  }
}

template <typename TX>
__global__ __launch_bounds__(256) void delta_kernel(const TX* x, int64_t ld, int H, int W,
                                                    const TX* prev, Ctrl* ctrl) {
  if (ctrl->done) return;
  const int64_t n = (int64_t)H * W;
  double m = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / W, col = i - r * W;
    m = fmax(m, fabs((double)x[r * ld + col] - (double)prev[i]));
  }
  m = block_max<TX>(m);
  if (threadIdx.x == 0) atomicMax(&ctrl->delta_key, dkey(m));
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

template <typename TX>
__global__ __launch_bounds__(256) void nonfinite_kernel(const TX* x, int64_t ld, int H, int W,
                                                        Ctrl* ctrl) {
  const int64_t n = (int64_t)H * W;
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / W, col = i - r * W;
    const double v = (double)x[r * ld + col];
    bad |= !(v - v == 0.0);
  }
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(&ctrl->nonfinite, 1);
}

// Feasibility: max over windows of side s of sum x^2 / r2 - 1, in FP64.
template <typename TX>
__global__ __launch_bounds__(256) void violation_kernel(const TX* x, int64_t ld, int H, int W,
                                                        int s, double r2, Ctrl* ctrl) {
  const int64_t nw = (int64_t)(H - s + 1) * (W - s + 1);
  double m = -1.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nw;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = i / (W - s + 1), b = i - a * (W - s + 1);
    double n = 0.0;
    for (int r = 0; r < s; ++r) {
      const TX* row = x + (a + r) * ld + b;
      for (int cc = 0; cc < s; ++cc) {
        const double v = (double)row[cc];
        n = __builtin_fma(v, v, n);
      }
    }
    m = fmax(m, n / r2 - 1.0);
  }
  m = block_max<TX>(m);
  if (threadIdx.x == 0) atomicMax(&ctrl->viol_key, dkey(m));
}

template <typename T>
__global__ __launch_bounds__(256) void fill_kernel(T* p, int64_t n, T v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void ctrl_reset_kernel(Ctrl* c) {
  c->done = 0;
  c->done_sweep = 0;
  c->nonfinite = 0;
  c->delta_key = dkey(0.0);
  c->last_delta = -1.0;
  c->viol_key = dkey(-1.0);
}

}  // namespace smre
