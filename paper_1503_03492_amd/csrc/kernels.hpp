// kernels.hpp -- gfx950 device code of the SMRE projection library.
//
// Full Dykstra (Sec. 2.3, Algorithm 2, projection Eq. (dykstra:if)) runs as
// "region phases": the anchor plane (top-left pixels of windows) is cut into
// R x R regions, coloured 2 (p mod 2) + (q mod 2).  One launch processes all
// regions of one colour; with R >= smax - 1 their pixel footprints
// (R + smax - 1)^2 are disjoint, so the launch needs no ordering between
// workgroups.  Inside a region the workgroup visits every window anchored in
// it: side by side (descending), then tiling offset (a', b') relative to the
// region origin in raster order; the windows of one offset are disjoint
// (Sec. 2.3), so a step projects all of them at once.
//
// Workgroup = 2 waves:
//   wave 0 (consumer) keeps the region's x footprint in LDS for the whole
//     phase and runs the steps: y = x + I, n = sum y^2 per window (lanes of a
//     window reduce with DPP / permlane swaps), t = sqrt(r2/n) if n > r2,
//     x' = t y, I' = y - x'.  I' is written back into the ring in place.
//   wave 1 (producer) streams the region's increments -- a sequence of whole
//     1 KiB pages per region and sweep, interleaved in HBM with the pages of
//     the other regions of its colour -- through a ring of pages in LDS,
//     several loads in flight, and
//     writes every page the consumer has finished back to HBM with 16-byte
//     stores before its slot is reused.  The first pages of the ring are
//     mirrored after its end so a round's chunk is always a linear LDS range
//     to read; a round that runs into the mirror copies its updated bytes back
//     to the primary pages.  The two waves synchronise through LDS counters;
//     every wait is bounded and sets an abort flag when the bound is hit, so
//     the workgroup always drains.
//
// With one consumer wave per SIMD the step is latency- and issue-bound, so it
// is written for short dependency chains and few instructions: no vector
// memory operations in the consumer, scalar-only progress checks, a lane
// serves a fixed window slot per side (its LDS pixel and ring addresses are
// one base plus compile-time immediates), masked lanes write to a dummy LDS
// area instead of branching, and the FP64 guard-band recheck branches after
// the writes it may redo.
//
// Increment layout: each region's increments form one stream of whole 1 KiB
// pages -- its steps in visiting order; per step, rounds of up to BR x BC
// windows; per round, the valid windows in row-major order, S^2 elements each,
// ordered by slot (u, v) then lane.  The pages of the regions of one colour
// are interleaved in HBM (RegionStream).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smre {

constexpr int kPage = 1024;            // bytes per prefetch page (64 lanes x 16 B)
constexpr int kSlots = 16;             // pages in the LDS ring (power of two)
constexpr int kMaxSides = 32;
constexpr int kPrefetch = 8;           // producer loads in flight

typedef uint16_t bf16_t;  // increment storage in bfloat16 (round to nearest even)
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf16_t f2bf(float f) {
  return __builtin_bit_cast(bf16_t, (__bf16)f);  // one v_cvt_pk_bf16_f32 (round to nearest even)
}
__device__ __forceinline__ float bf2f(bf16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

constexpr int kSpinLimit = 1 << 20;   // sleeps before a wait gives up (~30 ms)

// Increment element I/O in the LDS ring (BF16 storage rounds to nearest even).
template <typename TQ, typename TC> struct QStore;
template <> struct QStore<float, float> {
  static __device__ __forceinline__ float get(const unsigned char* p) { return *(const float*)p; }
  static __device__ __forceinline__ void put(unsigned char* p, float v) { *(float*)p = v; }
};
template <> struct QStore<double, double> {
  static __device__ __forceinline__ double get(const unsigned char* p) { return *(const double*)p; }
  static __device__ __forceinline__ void put(unsigned char* p, double v) { *(double*)p = v; }
};
template <> struct QStore<bf16_t, float> {
  static __device__ __forceinline__ float get(const unsigned char* p) {
    return bf2f(*(const bf16_t*)p);
  }
  static __device__ __forceinline__ void put(unsigned char* p, float v) { *(bf16_t*)p = f2bf(v); }
};

// ---------------------------------------------------------------- lane patterns
// For side S in a region of side R, a window is served by G = GR x GC lanes
// (lane (jr, jc) holds pixels (jr + u GR, jc + v GC), u < U, v < V) and a
// round covers a block of BR x BC window slots (G BR BC = 64).  Picked per
// (R, S) by counting issued instructions per step: rounds x (per-round
// overhead + elements per lane + reduction steps).
struct Pattern {
  int gr, gc, br, bc;
};
__host__ __device__ constexpr Pattern pattern(int R, int S) {
  if (R == 8) {
    constexpr Pattern t[10] = {{1, 1, 8, 8}, {1, 1, 8, 8}, {2, 2, 4, 4}, {2, 2, 4, 4},
                               {4, 4, 2, 2}, {4, 4, 2, 2}, {4, 4, 2, 2}, {4, 4, 2, 2},
                               {8, 8, 1, 1}, {8, 8, 1, 1}};
    return t[S];
  }
  if (R == 16) {
    constexpr Pattern t[18] = {{1, 1, 8, 8}, {1, 1, 8, 8}, {1, 1, 8, 8}, {1, 1, 8, 8},
                               {2, 2, 4, 4}, {2, 2, 4, 4}, {2, 2, 4, 4}, {4, 4, 2, 2},
                               {4, 4, 2, 2}, {4, 4, 2, 2}, {4, 4, 2, 2}, {4, 4, 2, 2},
                               {4, 4, 2, 2}, {8, 8, 1, 1}, {8, 8, 1, 1}, {8, 8, 1, 1},
                               {8, 8, 1, 1}, {8, 8, 1, 1}};
    return t[S];
  }
  if (S <= 5) return {1, 1, 8, 8};
  if (S <= 8) return {2, 2, 4, 4};
  if (S <= 16) return {4, 4, 2, 2};
  return {8, 8, 1, 1};
}

template <int R, int S> struct SideShape {
  static constexpr Pattern pt = pattern(R, S);
  static constexpr int GR = pt.gr, GC = pt.gc, BR = pt.br, BC = pt.bc;
  static constexpr int G = GR * GC, WB = BR * BC;
  static constexpr int U = (S + GR - 1) / GR, V = (S + GC - 1) / GC;
  static constexpr int JRL = S - (U - 1) * GR, JCL = S - (V - 1) * GC;  // last slot extents
  static constexpr int NRM = (R + S - 1) / S;   // most windows per region row
  static constexpr int RB = (NRM + BR - 1) / BR, CB = (NRM + BC - 1) / BC;
  // furthest pixel row / column (region-relative) any lane reads
  static constexpr int MAXROW = (S - 1) + S * (RB * BR - 1) + U * GR - 1;
  static constexpr int MAXCOL = (S - 1) + S * (CB * BC - 1) + V * GC - 1;
  // furthest element (from the round start) a lane reads in the ring
  static constexpr int MAXELEM = WB * S * S + G;
  static_assert(G * WB == 64, "a round uses the whole wave");
  // element offset of slot (u, v) inside a window
  static constexpr int slot(int u, int v) {
    return u * GR * S + (u == U - 1 ? JRL : GR) * v * GC;
  }
};

template <typename TX, typename TQ, int R, int SMAX> struct PhaseShape {
  static constexpr int FR = R + SMAX - 1;
  static constexpr int mrow() {
    int m = FR;
    for (int s = 1; s <= SMAX; ++s) {
      const Pattern p = pattern(R, s);
      const int U = (s + p.gr - 1) / p.gr, nrm = (R + s - 1) / s, rb = (nrm + p.br - 1) / p.br;
      const int r = (s - 1) + s * (rb * p.br - 1) + U * p.gr;
      if (r > m) m = r;
    }
    return m;
  }
  static constexpr int mcol() {
    int m = FR;
    for (int s = 1; s <= SMAX; ++s) {
      const Pattern p = pattern(R, s);
      const int V = (s + p.gc - 1) / p.gc, nrm = (R + s - 1) / s, cb = (nrm + p.bc - 1) / p.bc;
      const int c = (s - 1) + s * (cb * p.bc - 1) + V * p.gc;
      if (c > m) m = c;
    }
    return m;
  }
  static constexpr int XROWS = mrow();
  static constexpr int P = (mcol() % 2 == 0) ? mcol() + 1 : mcol();  // odd pitch
  // scratch written by lanes without a window: largest immediate + 1
  static constexpr int dummy() {
    int m = 0;
    for (int s = 1; s <= SMAX; ++s) {
      const Pattern p = pattern(R, s);
      const int U = (s + p.gr - 1) / p.gr, V = (s + p.gc - 1) / p.gc;
      const int d = (U - 1) * p.gr * P + (V - 1) * p.gc + 1;
      if (d > m) m = d;
    }
    return m;
  }
  static constexpr int XDUMMY = XROWS * P;
  // masked lanes write to XDUMMY + lane + immediate: distinct addresses, so
  // the writes of a round's masked lanes do not serialise on one bank
  static constexpr int XSIZE = XROWS * P + dummy() + 64;
  // mirrored ring pages: enough for the largest round read
  static constexpr int mirror() {
    int m = 0;
    for (int s = 1; s <= SMAX; ++s) {
      const Pattern p = pattern(R, s);
      const int e = p.br * p.bc * s * s + p.gr * p.gc;
      if (e > m) m = e;
    }
    return (m * (int)sizeof(TQ) + kPage - 1) / kPage + 1;
  }
  static constexpr int MIRROR = mirror();
  // dummy area for the increment writes of masked lanes: largest slot
  // immediate + one element
  static constexpr int qdummy() {
    int m = 0;
    for (int s = 1; s <= SMAX; ++s) {
      const Pattern p = pattern(R, s);
      const int U = (s + p.gr - 1) / p.gr, V = (s + p.gc - 1) / p.gc;
      const int jrl = s - (U - 1) * p.gr;
      const int d = ((U - 1) * p.gr * s + jrl * (V - 1) * p.gc + 1) * (int)sizeof(TQ);
      if (d > m) m = d;
    }
    return (m + 15) / 16 * 16;
  }
  static constexpr int QD = (kSlots + MIRROR) * kPage;  // ring byte offset of the dummy area
  static constexpr int RING = QD + qdummy() + 64 * (int)sizeof(TQ);  // + one element per lane
  static_assert(MIRROR + 2 <= kSlots, "ring too small for a round");
};

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
// Where a region's increment pages lie: page p at first + p * stride (pages
// of the image's stream).  The regions of one colour interleave their pages
// (stride = regions of the colour), so the workgroups of a launch stream one
// contiguous window of HBM at a time.
struct RegionStream {
  int32_t first;
  int32_t npages;
  int32_t stride;
  int32_t pad;
};

// One round of a side's visiting order in a region (see the round tables
// below): x = pixel offset of the round's first window in the footprint (bits
// 0..15) | windows of the round along a row of windows (bits 16..19) | along
// a column (bits 20..23), the counts left zero for sides whose rounds hold
// one window; y = end of the round's increment bytes, counted from the side's
// first byte.
struct RoundEntry {
  uint32_t x, y;
};

// Round tables: for each side k and border class (row class * 3 + column
// class; class 0 = interior region, 1 = next-to-last, 2 = last region row or
// column), R * R + 2 entries: entry 0 = {number of rounds, 0}, entry 1 unused,
// entries 2.. the rounds in visiting order.  Built on the host from the same
// enumeration the oracle's region order uses.
__host__ __device__ constexpr int round_table_len(int R) { return R * R + 2; }

// Everything a region job needs about its image.  Passed by value for a
// single image; an array in device memory for a batch.
struct ImageDesc {
  void* x;                 // image (TX), row stride ld
  const RegionStream* rs;  // page layout of each region's increments
  const RoundEntry* rtab;  // round tables, [side][class][round_table_len(R)]
  int64_t ld;
  int64_t q_byte;       // first byte of this image's increments in the stream
  int32_t H, W;
  int32_t nrx, nry;     // region grid
  int32_t fr;           // footprint side R + smax - 1
  int32_t nsides;
  float guard;          // FP32 recheck band (relative)
  int32_t pad;
  int32_t sides[kMaxSides];  // descending
  float r2f[kMaxSides];
  float rf[kMaxSides];       // sqrt(r2), FP32
  double r2d[kMaxSides];
};

// Per-image state of a batched solve, in device memory.
struct BatchCtl {
  int done;                      // retired (converged or capped): its work items are skipped
  int done_sweep;                // sweep at which it was retired
  int converged;                 // 1 if the tolerance was met
  int max_sweeps;
  int sweeps;                    // sweeps this image has run (images may join at different times)
  int check_every;
  int gen;                       // occupant generation (serving: tells a slot's requests apart)
  int aborted;                   // a region job of this image hit a wait bound (device error)
  unsigned long long delta_key;  // running max |x - prev| of the checked sweep
  double last_delta;
  double tol;
  int64_t prev_off;              // element offset of the image's snapshot
};

// One region of one image (a batch's work list holds these per colour).
struct WorkItem {
  int32_t img;
  int32_t region;
};

// Bounded wait until *ctr >= target; returns the last value read (SGPR).
// When the bound is hit, or the other wave has given up, the abort flag is set
// and the wait returns, so every wave of the workgroup finishes.
__device__ __forceinline__ int wait_ge(const int* ctr, int target, int* abort) {
  int seen = __builtin_amdgcn_readfirstlane(lds_load(ctr));
  for (int spin = 0; seen < target; ++spin) {
    if (spin >= kSpinLimit || lds_load(abort)) {
      lds_store(abort, 1);
      return target;
    }
    __builtin_amdgcn_s_sleep(1);
    seen = __builtin_amdgcn_readfirstlane(lds_load(ctr));
  }
  return seen;
}

struct Consumer {
  unsigned char* ring;
  int* ready;      // pages (relative to the region's first page) present in the ring
  int* consumed;   // pages (relative) whose updated increments are all in the ring
  int* abort;      // set by a wait that gave up
  uint32_t qb;     // next increment byte of the region (relative)
  int r0, c0;      // anchor origin of the region (= footprint origin)
  int lane;
  int ready_seen;  // last value read from *ready
};

template <typename TX, typename TQ, int R, int SMAX, int S, bool KAHAN>
__device__ __forceinline__ void run_side(const ImageDesc& a, Consumer& c, TX* xs, int k,
                                         const RoundEntry* tab, int nrounds) {
  using SS = SideShape<R, S>;
  using LS = PhaseShape<TX, TQ, R, SMAX>;
  constexpr int GR = SS::GR, GC = SS::GC, G = SS::G, BR = SS::BR, BC = SS::BC;
  constexpr int U = SS::U, V = SS::V, JRL = SS::JRL, JCL = SS::JCL;
  constexpr int P = LS::P;
  constexpr int ES = (int)sizeof(TQ);
  constexpr uint32_t RMASK = kSlots * kPage - 1;
  using QS = QStore<TQ, TX>;

  const int wl = c.lane / G, jj = c.lane % G;
  const int bry = wl / BC, brx = wl % BC, jr = jj / GC, jc = jj % GC;
  const bool rl = jr < JRL, cl = jc < JCL;     // lane holds a pixel in the last row / col slot
  const int ef = jr * GC + jc, el = jr * JCL + jc;  // element of the lane inside a slot
  const int lane_x0 = (S * bry + jr) * P + (S * brx + jc);
  // per-lane dummy targets for the writes of masked lanes
  const int xdum = LS::XDUMMY + c.lane;
  const uint32_t qdum = (uint32_t)(LS::QD + c.lane * ES);
  if (nrounds <= 0) return;
  // per-side constants live in VGPRs (the loop would otherwise reload them)
  TX r2 = (sizeof(TX) == 8) ? (TX)a.r2d[k] : (TX)a.r2f[k];
  float rfl = a.rf[k], gr2 = a.guard * a.r2f[k];
  const double r2d = a.r2d[k];
  __asm__ volatile("" : "+v"(r2), "+v"(rfl), "+v"(gr2));

  // Rounds of this side in visiting order -- offsets (ap, bp) raster, then
  // row / column blocks of windows -- read from the region's round table in
  // LDS, one entry per round (the next entry is read a round ahead).
  const uint32_t qb0 = c.qb;
  uint32_t rb = 0;
  uint32_t ready_lim = (uint32_t)c.ready_seen * kPage - qb0;
  RoundEntry e = tab[0];
  uint32_t rb_end = __builtin_amdgcn_readfirstlane(e.y);
  const RoundEntry* tn = tab + 1;
  int i = 0;
  do {
    const RoundEntry en = *tn++;  // entry past the last one is in the buffer, unused
    const uint32_t nbytes = rb_end - rb;
    int nbr = 1, nbc = 1;
    if constexpr (BR > 1) nbr = (int)((e.x >> 20) & 0xF);
    if constexpr (BC > 1) nbc = (int)((e.x >> 16) & 0xF);
    // one-window blocks are always valid (a round holds at least one window)
    const bool valid = (BR == 1 || bry < nbr) && (BC == 1 || brx < nbc);
    const int woff = (bry * nbc + brx) * (S * S);
    // wait until every page holding this round's bytes is in the ring (the
    // bytes of the pages seen so far, relative to the side, bound the check)
    if (__builtin_expect(rb_end > ready_lim, 0)) {
      c.ready_seen = wait_ge(c.ready, (int)((qb0 + rb_end + kPage - 1) / kPage), c.abort);
      ready_lim = (uint32_t)c.ready_seen * kPage - qb0;
    }
    __asm__ volatile("" ::: "memory");
    const uint32_t roff = (qb0 + rb) & RMASK;
    // ring offsets of the lane's elements (full / last column slot); the
    // writes of masked lanes go to the dummy area
    const uint32_t qf = roff + (uint32_t)((woff + ef) * ES);
    const uint32_t ql = roff + (uint32_t)((woff + el) * ES);
    const uint32_t wff = valid ? qf : qdum;
    const uint32_t wfl = valid && cl ? ql : qdum;
    const uint32_t wlf = valid && rl ? qf : qdum;
    const uint32_t wll = valid && rl && cl ? ql : qdum;
    const int bx = lane_x0 + (int)((BR == 1 && BC == 1) ? e.x : (e.x & 0xFFFF));
    const int bxr = valid ? bx : 0;
    const int bxw = valid ? bx : xdum;
    const int bxw_r = valid && rl ? bx : xdum;
    const int bxw_c = valid && cl ? bx : xdum;
    const int bxw_rc = valid && rl && cl ? bx : xdum;

    // 1) LDS reads: pixels at immediates off one base, increments off two
    TX xv[U][V], qv[U][V];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int v = 0; v < V; ++v) {
        qv[u][v] = QS::get(c.ring + (v == V - 1 ? ql : qf) + SS::slot(u, v) * ES);
        xv[u][v] = xs[bxr + u * GR * P + v * GC];
      }
    // 2) y = x + I (pixels outside the window count as 0), sum of squares
    TX y[U][V];
    // FP32: two interleaved accumulators (even / odd elements), each with its
    // own compensation when KAHAN, so the dependent add chains are half as
    // long; the corrected partial sums are added at the end.
    TX acc[2] = {0, 0}, comp[2] = {0, 0};
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int v = 0; v < V; ++v) {
        TX yv = xv[u][v] + qv[u][v];
        const bool part_r = (u == U - 1) && (JRL < GR);
        const bool part_c = (v == V - 1) && (JCL < GC);
        if (part_r && part_c) yv = (rl && cl) ? yv : TX(0);
        else if (part_r) yv = rl ? yv : TX(0);
        else if (part_c) yv = cl ? yv : TX(0);
        y[u][v] = yv;
        const int h = (sizeof(TX) == 4) ? ((u * V + v) & 1) : 0;
        if constexpr (sizeof(TX) == 4 && KAHAN) {
          if (u * V + v < 2) {
            // an accumulator's first term: the compensated step from (0, 0)
            // gives acc = y^2 rounded and comp = 0 exactly (finite y), so
            // take those values instead of computing y^2 - y^2
            acc[h] = yv * yv;
          } else {
            const TX t2 = __builtin_fmaf(yv, yv, -comp[h]);
            const TX s2 = acc[h] + t2;
            comp[h] = (s2 - acc[h]) - t2;
            acc[h] = s2;
          }
        } else if constexpr (sizeof(TX) == 4) {
          acc[h] = __builtin_fmaf(yv, yv, acc[h]);
        } else {
          acc[0] = __builtin_fma(yv, yv, acc[0]);
        }
      }
    TX lane_sum;
    if constexpr (sizeof(TX) == 4 && KAHAN) lane_sum = (acc[0] - comp[0]) + (acc[1] - comp[1]);
    else if constexpr (sizeof(TX) == 4) lane_sum = acc[0] + acc[1];
    else lane_sum = acc[0];
    // the next round's byte end into a scalar register here, mid-round, so
    // the vector-to-scalar hand-off is long done when the loop test and the
    // next round's page check use it
    uint32_t rb_end_n = __builtin_amdgcn_readfirstlane(en.y);
    __asm__ volatile("" : "+s"(rb_end_n));
    const TX n = group_sum<G>(lane_sum);

    // 3) x' = t y into the footprint, I' = y - x' into the ring (pixels
    //    first, then increments, so neighbouring writes merge)
    auto write_step = [&](TX t) {
      TX xn[U][V];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const bool part_r = (u == U - 1) && (JRL < GR);
          const bool part_c = (v == V - 1) && (JCL < GC);
          xn[u][v] = t * y[u][v];
          if constexpr (BR == 1 && BC == 1) {
            // one window per round: a masked element is a pixel outside the
            // window that no other lane touches, so it gets its own value back
            // (one base for all elements, so the writes pair up)
            const bool keep = (part_r && part_c) ? (rl && cl) : part_r ? rl : part_c ? cl : true;
            xs[bx + u * GR * P + v * GC] = keep ? xn[u][v] : xv[u][v];
          } else {
            const int base = (part_r && part_c) ? bxw_rc : part_r ? bxw_r : part_c ? bxw_c : bxw;
            xs[base + u * GR * P + v * GC] = xn[u][v];
          }
        }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const uint32_t wq = (u == U - 1 && JRL < GR) ? ((v == V - 1) ? wll : wlf)
                                                      : ((v == V - 1) ? wfl : wff);
          QS::put(c.ring + wq + SS::slot(u, v) * ES, y[u][v] - xn[u][v]);
        }
    };
    if constexpr (sizeof(TX) == 4) {
      // FP32 scale; windows whose sum lies within the guard band of the
      // bound are redone with an FP64 sum after the writes
      const bool near = fabsf(n - r2) <= gr2;
      uint64_t nearmask = __ballot(near);
      __asm__ volatile("" : "+s"(nearmask) :: "memory");
      write_step(n > r2 ? rfl * __builtin_amdgcn_rsqf(n) : 1.0f);
      if (__builtin_expect(nearmask != 0, 0)) {
        double pd = 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int v = 0; v < V; ++v)
            pd = __builtin_fma((double)y[u][v], (double)y[u][v], pd);
        const double nd = group_sum<G>(pd);
        const float t64 = nd > r2d ? (float)__builtin_sqrt(r2d / nd) : 1.0f;
        write_step(near ? t64 : (n > r2 ? rfl * __builtin_amdgcn_rsqf(n) : 1.0f));
      }
    } else {
      write_step(n > r2 ? __builtin_sqrt(r2 / n) : TX(1));
    }
    // (the copy below reads, as 16-byte words, increments this lane and
    // others have just stored as elements: keep the compiler from hoisting it
    // above those stores, which alias analysis would allow for another type)
    __asm__ volatile("" ::: "memory");
    // a round that ran into the mirrored pages copies them back
    if (__builtin_expect(roff + nbytes > (uint32_t)(kSlots * kPage), 0)) {
      const int np = (int)((roff + nbytes - kSlots * kPage + kPage - 1) / kPage);
      u32x4* r4 = (u32x4*)c.ring;
      for (int p = 0; p < np; ++p) r4[p * 64 + c.lane] = r4[(kSlots + p) * 64 + c.lane];
    }
    __asm__ volatile("" ::: "memory");
    lds_store(c.consumed, (int)((qb0 + rb_end) / kPage));
    rb = rb_end;
    e = en;
    rb_end = rb_end_n;
  } while (++i < nrounds);
  c.qb = qb0 + rb;
}

template <typename TX, typename TQ, int R, int SMAX, bool KAHAN>
__device__ __forceinline__ void dispatch_side(const ImageDesc& a, Consumer& c, TX* xs, int k,
                                              const RoundEntry* tab, int nrounds) {
  switch (a.sides[k]) {
#define SMRE_SIDE_CASE(n) \
  case n:                 \
    if constexpr (n <= SMAX) run_side<TX, TQ, R, SMAX, n, KAHAN>(a, c, xs, k, tab, nrounds); \
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

// Producer wave: stream pages [0, npg) of the region's increments (gq points
// at its first page, page p at gq + p * stride pages) into the ring (slot = page mod kSlots; slots below MIRROR
// also after the ring end), kPrefetch loads in flight.  A slot is refilled
// only after its previous page has been written back to HBM, and a page is
// written back (one 16-byte store per lane) once the consumer has finished
// it.  Full batches of kPrefetch pages run branch-free so the loads stay in
// flight across batches.
template <int MIRROR>
__device__ __forceinline__ void produce(u32x4* gq, int npg, int64_t stride, u32x4* ring,
                                        int* ready, const int* consumed, int* abort, int lane) {
  if (npg <= 0) return;
  stride *= 64;  // in 16-byte units
  int cons_seen = 0, wb = 0;
  auto writeback = [&]() {
    if (wb >= cons_seen) cons_seen = wait_ge(consumed, wb + 1, abort);
    __asm__ volatile("" ::: "memory");
    const u32x4 v = ring[(wb & (kSlots - 1)) * 64 + lane];
    __builtin_nontemporal_store(v, gq + (int64_t)wb * stride + lane);
    ++wb;
  };
  auto put = [&](int rel, u32x4 v) {
    while (wb <= rel - kSlots) writeback();
    __asm__ volatile("" ::: "memory");
    const int slot = rel & (kSlots - 1);
    ring[slot * 64 + lane] = v;
    if (slot < MIRROR) ring[(kSlots + slot) * 64 + lane] = v;
    lds_store(ready, rel + 1);
  };
  u32x4 buf[kPrefetch];
#pragma unroll
  for (int k = 0; k < kPrefetch; ++k)
    buf[k] = __builtin_nontemporal_load(gq + (int64_t)min(k, npg - 1) * stride + lane);
  int base = 0;
  for (; base + kPrefetch <= npg; base += kPrefetch) {
#pragma unroll
    for (int k = 0; k < kPrefetch; ++k) {
      const int rel = base + k;
      put(rel, buf[k]);
      buf[k] = __builtin_nontemporal_load(gq + (int64_t)min(rel + kPrefetch, npg - 1) * stride + lane);
    }
  }
#pragma unroll
  for (int k = 0; k < kPrefetch; ++k)
    if (base + k < npg) put(base + k, buf[k]);
  while (wb < npg) writeback();
}

template <typename TX, typename TQ, int R, int SMAX> struct PhaseLds {
  using SH = PhaseShape<TX, TQ, R, SMAX>;
  unsigned char ring[SH::RING];
  TX xs[SH::XSIZE];
  RoundEntry tab[R * R + 2];  // the current side's rounds (+ one readable entry past the end)
  int ctr[3];  // pages ready, pages consumed, abort flag
};

// One region of one image: both waves of the workgroup enter; the caller
// resets the counters and synchronises the workgroup before and after.
template <typename TX, typename TQ, int R, int SMAX, bool KAHAN>
__device__ __forceinline__ void region_job(const ImageDesc& a, int region, unsigned char* q,
                                           PhaseLds<TX, TQ, R, SMAX>& L) {
  using SH = PhaseShape<TX, TQ, R, SMAX>;
  const int ry = region / a.nrx, rx = region - (region / a.nrx) * a.nrx;
  const RegionStream st = a.rs[region];
  const int npg = st.npages;
  const int lane = threadIdx.x & 63;

  if (threadIdx.x >= 64) {
    produce<SH::MIRROR>((u32x4*)(q + a.q_byte) + (int64_t)st.first * 64, npg, st.stride,
                        (u32x4*)L.ring, &L.ctr[0], &L.ctr[1], &L.ctr[2], lane);
    return;
  }

  const int r0 = ry * R, c0 = rx * R;
  const int fh = min(a.fr, a.H - r0), fw = min(a.fr, a.W - c0);
  TX* xg = (TX*)a.x;
  TX* xs = L.xs;
  for (int idx = lane; idx < fh * fw; idx += 64) {
    const int i = idx / fw, j = idx - (idx / fw) * fw;
    xs[i * SH::P + j] = xg[(int64_t)(r0 + i) * a.ld + c0 + j];
  }
  __asm__ volatile("" ::: "memory");

  Consumer c;
  c.ring = L.ring;
  c.ready = &L.ctr[0];
  c.consumed = &L.ctr[1];
  c.abort = &L.ctr[2];
  c.qb = 0;
  c.r0 = r0;
  c.c0 = c0;
  c.lane = lane;
  c.ready_seen = 0;
  // round tables: the next side's table is loaded into registers while the
  // current side runs and parked in LDS between sides
  const int cls = (ry == a.nry - 1 ? 2 : ry == a.nry - 2 ? 1 : 0) * 3 +
                  (rx == a.nrx - 1 ? 2 : rx == a.nrx - 2 ? 1 : 0);
  constexpr int TL = round_table_len(R);           // entries per table (16-byte multiple)
  constexpr int NPF = ((TL - 2) / 2 + 63) / 64;    // 16-byte rounds chunks per lane
  auto table = [&](int k) { return (const u32x4*)(a.rtab + ((size_t)k * 9 + cls) * TL); };
  u32x4 pf[NPF], hdr;
  auto prefetch = [&](int k) {
    const u32x4* g = table(k);
    hdr = g[0];
#pragma unroll
    for (int j = 0; j < NPF; ++j)
      if (j * 64 + lane < (TL - 2) / 2) pf[j] = g[1 + j * 64 + lane];
  };
  auto park = [&]() {
    u32x4* t4 = (u32x4*)L.tab;
#pragma unroll
    for (int j = 0; j < NPF; ++j)
      if (j * 64 + lane < (TL - 2) / 2) t4[j * 64 + lane] = pf[j];
  };
  prefetch(0);
  for (int k = 0; k < a.nsides; ++k) {
    const int nrounds = (int)__builtin_amdgcn_readfirstlane(hdr.x);
    park();
    if (k + 1 < a.nsides) prefetch(k + 1);
    __asm__ volatile("" ::: "memory");
    dispatch_side<TX, TQ, R, SMAX, KAHAN>(a, c, xs, k, L.tab, nrounds);
    __asm__ volatile("" ::: "memory");
  }
  lds_store(c.consumed, npg);  // the last, partial page too

  for (int idx = lane; idx < fh * fw; idx += 64) {
    const int i = idx / fw, j = idx - (idx / fw) * fw;
    xg[(int64_t)(r0 + i) * a.ld + c0 + j] = xs[i * SH::P + j];
  }
}

template <typename TX, typename TQ, int R, int SMAX>
__device__ __forceinline__ void reset_counters(PhaseLds<TX, TQ, R, SMAX>& L) {
  if (threadIdx.x == 0) {
    L.ctr[0] = 0;
    L.ctr[1] = 0;
    L.ctr[2] = 0;
  }
  __syncthreads();
}

// A wait inside the region job gave up (a protocol failure): raise the
// caller's flag -- the single-image call's control block or the image's
// batch control block -- which the host reports as a device error for that
// solve only.
template <typename TX, typename TQ, int R, int SMAX>
__device__ __forceinline__ void report_abort(PhaseLds<TX, TQ, R, SMAX>& L, int* flag) {
  __syncthreads();
  if (threadIdx.x == 0 && L.ctr[2]) atomicOr(flag, 1);
}

// One image, one colour: block b takes the b-th region of colour (cy, cx).
template <typename TX, typename TQ, int R, int SMAX, bool KAHAN>
__global__ __launch_bounds__(128) void region_phase(ImageDesc a, int cy, int cx, int ncx,
                                                    const int* done, int* abort_flag,
                                                    unsigned char* q) {
  __shared__ PhaseLds<TX, TQ, R, SMAX> L;
  if (*done) return;
  const int b = blockIdx.x;
  const int region = (cy + 2 * (b / ncx)) * a.nrx + cx + 2 * (b % ncx);
  reset_counters(L);
  region_job<TX, TQ, R, SMAX, KAHAN>(a, region, q, L);
  report_abort(L, abort_flag);
}

// A batch of images, one colour: a persistent grid walks the colour's work
// list; items of converged images are skipped.
template <typename TX, typename TQ, int R, int SMAX, bool KAHAN>
__global__ __launch_bounds__(128) void region_phase_batch(const ImageDesc* __restrict__ imgs,
                                                          BatchCtl* __restrict__ ctl,
                                                          const WorkItem* __restrict__ items,
                                                          const int* __restrict__ nitems,
                                                          unsigned char* q) {
  __shared__ PhaseLds<TX, TQ, R, SMAX> L;
  const int n = *nitems;
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const WorkItem w = items[it];
    if (ctl[w.img].done) continue;
    reset_counters(L);
    region_job<TX, TQ, R, SMAX, KAHAN>(imgs[w.img], w.region, q, L);
    report_abort(L, &ctl[w.img].aborted);
  }
}

}  // namespace smre
