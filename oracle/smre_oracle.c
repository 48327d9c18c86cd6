/*
 * smre_oracle.c -- reference oracle for the SMRE projection (TEST INFRASTRUCTURE).
 *
 * This file is the slow, plain, obviously-correct CPU implementation that the
 * HIP library is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or helper with the HIP library, and the library never calls it.
 *
 * Everything is IEEE double, sequential, built with -O2 -ffp-contract=off.
 *
 * Paper: "Parallel Statistical Multi-resolution Estimation" (arXiv 1503.03492).
 *   - feasible sets tau_s and their intersection tau_G: Sec. 2, Eqs. (tau_s), (tau_G)
 *   - single-set projection p_s: Sec. 2.3, Eq. (dykstra:if)
 *   - Dykstra's cyclic projection with per-set increments: Sec. 2.3, Algorithm 2
 *   - disjoint sets commute, overlapping order matters: Sec. 2.3 (end)
 *   - weights c_s(alpha) from the fourth-root transform: Sec. 2.1
 *   - incomplete Dykstra (ICD) set family and product of projections: Sec. 3.2
 *     and its kernel description (Listing "incomplete implementation").
 *
 * Readings of the paper used here (each also listed in the design notes):
 *   - The bound of a window is r2 = 1/c_s, so the constraint is sum_S v^2 <= r2.
 *   - The increment update follows the kernel listing of Sec. 3.2, which is
 *     standard Dykstra: with I = -q, y = x + I, x' = p_S(y), I' = y - x'.
 *     (The one-line update printed in Algorithm 2 drops the old increment.)
 *   - The window family is every s x s square lying fully inside the image.
 *   - A projection rescales iff sum y^2 > r2 (strict, Eq. dykstra:if); the
 *     scale factor is t = sqrt(r2 / n).
 *   - The sweep stopping rule is max_i |x_i - x_prev_i| < tol between the
 *     iterates at the end of consecutive sweeps.
 *   - ICD: phase i (i = 0..K) uses blocks of side 2^K on the lattice shifted
 *     diagonally by (2^i mod 2^K); inside a block, levels k = K..i (squares of
 *     side 2^k) are projected by Dykstra with increments zeroed at the start of
 *     the phase, until the block converges.
 *
 * Parity pins (what fixes this code independently of itself) live in
 * tests/test_oracle_*.py: closed forms (single ball, disjoint sets, feasible
 * input), KKT certificate, variational inequality, brute-force QCQP, symmetry,
 * nonexpansiveness, order independence, chi-square closed forms vs SciPy.
 */
#define _DEFAULT_SOURCE /* madvise */
#include <math.h>
#include <stdint.h>
#include <sys/mman.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_ORDER_DESC 0   /* sides descending, offsets raster, windows raster */
#define ORACLE_ORDER_ASC 1    /* sides ascending, otherwise as DESC              */
#define ORACLE_ORDER_REGION 2 /* region-coloured order (see oracle_dykstra)      */

#define ORACLE_TOL_MAXABS 0
#define ORACLE_TOL_MEANABS 1

/* ------------------------------------------------------------------------- */
/* Chi-square quantiles (window bounds)                                        */
/* ------------------------------------------------------------------------- */

/* CDF of the chi-square law with k degrees of freedom, from the closed forms of
 * the regularised lower incomplete gamma function at half-integer order:
 *   k even: P = 1 - exp(-h) sum_{j < k/2} h^j / j!                      (h = x/2)
 *   k odd : P = erf(sqrt h) - exp(-h) sum_{j=0}^{(k-3)/2} h^(j+1/2) / Gamma(j+3/2)
 * The finite sums are the first terms of series that add up to 1 (even k) and
 * erf(sqrt h) (odd k), so below the mode P is taken as the sum of the remaining
 * terms instead, which avoids cancellation in the lower tail.  Each term is
 * evaluated in log space so large k does not underflow. */
static double chi2_term(int k, double h, double lh, int j) {
  if (k % 2 == 0) return exp(-h + j * lh - lgamma(j + 1.0));
  return exp(-h + (j + 0.5) * lh - lgamma(j + 1.5));
}

double oracle_chi2_cdf(int k, double x) {
  if (x <= 0.0) return 0.0;
  double h = 0.5 * x;
  double lh = log(h);
  int j0 = (k % 2 == 0) ? k / 2 : (k - 1) / 2; /* first term not in the finite sum */
  if (h < j0) {
    double p = 0.0;
    for (int j = j0; j < j0 + 100000; ++j) {
      double t = chi2_term(k, h, lh, j);
      p += t;
      if (t < 1e-18 * p) break;
    }
    return p;
  }
  double tail = 0.0;
  for (int j = 0; j < j0; ++j) tail += chi2_term(k, h, lh, j);
  return (k % 2 == 0) ? 1.0 - tail : erf(sqrt(h)) - tail;
}

/* chi-square density, used for the Newton polish of the quantile. */
static double chi2_pdf(int k, double x) {
  if (x <= 0.0) return 0.0;
  return exp((0.5 * k - 1.0) * log(x) - 0.5 * x - 0.5 * k * log(2.0) - lgamma(0.5 * k));
}

/* Quantile: bisection on [0, hi] to a narrow bracket, then Newton steps kept
 * inside the bracket. */
double oracle_chi2_quantile(int k, double p) {
  if (k <= 0 || !(p > 0.0) || !(p < 1.0)) return NAN;
  double lo = 0.0, hi = k + 20.0 * sqrt(2.0 * k) + 50.0;
  while (oracle_chi2_cdf(k, hi) < p) hi *= 2.0;
  for (int it = 0; it < 200 && (hi - lo) > 1e-9 * hi; ++it) {
    double mid = 0.5 * (lo + hi);
    if (oracle_chi2_cdf(k, mid) < p) lo = mid; else hi = mid;
  }
  double x = 0.5 * (lo + hi);
  for (int it = 0; it < 50; ++it) {
    double f = oracle_chi2_cdf(k, x) - p;
    double d = chi2_pdf(k, x);
    if (d <= 0.0) break;
    double xn = x - f / d;
    if (xn <= lo || xn >= hi) break;
    if (fabs(xn - x) <= 1e-15 * x) { x = xn; break; }
    x = xn;
  }
  return x;
}

/* Bound of a window with n pixels from the paper's weights (Sec. 2.1):
 * mu = (n - 1/2)^(1/4), sigma^2 = 1/(8 sqrt n), c = (q sigma + mu)^(-4),
 * and the bound on the sum of squares is 1/c = (q sigma + mu)^4. */
double oracle_paper_bound(int64_t npix, double q_alpha) {
  double n = (double)npix;
  double mu = pow(n - 0.5, 0.25);
  double sigma = sqrt(1.0 / (8.0 * sqrt(n)));
  return pow(q_alpha * sigma + mu, 4.0);
}

/* ------------------------------------------------------------------------- */
/* Full Dykstra                                                               */
/* ------------------------------------------------------------------------- */

typedef struct {
  int32_t n;          /* number of sides                      */
  int32_t side[64];   /* sides sorted descending              */
  double r2[64];      /* bound per sorted side                */
  int64_t tbase[64];  /* first tiling index of each side      */
  int64_t ntilings;   /* T = sum of side^2                    */
} side_table;

static int make_side_table(const int32_t* sides, const double* r2, int32_t nsides, int64_t H,
                           int64_t W, side_table* st) {
  if (nsides < 1 || nsides > 64) return -1;
  st->n = nsides;
  for (int k = 0; k < nsides; ++k) {
    if (sides[k] < 1 || sides[k] > H || sides[k] > W) return -1;
    if (!(r2[k] > 0.0) || !isfinite(r2[k])) return -1;
    st->side[k] = sides[k];
    st->r2[k] = r2[k];
  }
  /* insertion sort, descending; reject duplicates */
  for (int a = 1; a < nsides; ++a)
    for (int b = a; b > 0 && st->side[b] > st->side[b - 1]; --b) {
      int32_t ts = st->side[b]; st->side[b] = st->side[b - 1]; st->side[b - 1] = ts;
      double tr = st->r2[b]; st->r2[b] = st->r2[b - 1]; st->r2[b - 1] = tr;
    }
  for (int a = 1; a < nsides; ++a)
    if (st->side[a] == st->side[a - 1]) return -1;
  int64_t t = 0;
  for (int k = 0; k < nsides; ++k) { st->tbase[k] = t; t += (int64_t)st->side[k] * st->side[k]; }
  st->ntilings = t;
  return 0;
}

/* Projection of one window, Eq. (dykstra:if), inside Dykstra's update:
 *   y = x + I on the window, n = sum y^2 (row-major order),
 *   x <- t y with t = sqrt(r2/n) if n > r2 else 1,  I <- y - x. */
/* ORACLE_MUTANT (tests only) plants one plausible mistake so the test suite can
 * show that its pins catch it; the shipped oracle is built without it. */
#ifndef ORACLE_MUTANT
#define ORACLE_MUTANT 0
#endif
static void project_window(double* x, double* inc, int64_t W, int64_t i0, int64_t j0, int32_t s,
                           double r2, double* ybuf) {
  double n = 0.0;
  int64_t k = 0;
  for (int64_t i = i0; i < i0 + s; ++i)
    for (int64_t j = j0; j < j0 + s; ++j, ++k) {
#if ORACLE_MUTANT == 2
      double y = x[i * W + j] - inc[i * W + j]; /* wrong sign of the increment */
#else
      double y = x[i * W + j] + inc[i * W + j];
#endif
      ybuf[k] = y;
#if ORACLE_MUTANT == 3
      if (i < i0 + s - 1) n += y * y; /* dropped last row of the window sum */
#else
      n += y * y;
#endif
    }
  double t = 1.0;
#if ORACLE_MUTANT == 4
  if (n > r2) t = r2 / n; /* missing square root */
#else
  if (n > r2) t = sqrt(r2 / n);
#endif
  k = 0;
  for (int64_t i = i0; i < i0 + s; ++i)
    for (int64_t j = j0; j < j0 + s; ++j, ++k) {
      double xn = t * ybuf[k];
#if ORACLE_MUTANT == 1
      inc[i * W + j] = x[i * W + j] - xn; /* update printed in Algorithm 2: old increment dropped */
#else
      inc[i * W + j] = ybuf[k] - xn;
#endif
      x[i * W + j] = xn;
    }
}

/* All windows of tiling (s, a, b) whose anchor (top-left pixel) lies in the
 * anchor rectangle [ilo, ihi) x [jlo, jhi). */
static void project_tiling_part(double* x, double* inc, int64_t H, int64_t W, int32_t s, int32_t a,
                                int32_t b, double r2, int64_t ilo, int64_t ihi, int64_t jlo,
                                int64_t jhi, double* ybuf) {
  if (ihi > H - s + 1) ihi = H - s + 1;
  if (jhi > W - s + 1) jhi = W - s + 1;
  int64_t i = ilo + (((a - ilo) % s) + s) % s;
  int64_t j0 = jlo + (((b - jlo) % s) + s) % s;
  for (; i < ihi; i += s)
    for (int64_t j = j0; j < jhi; j += s) project_window(x, inc, W, i, j, s, r2, ybuf);
}

/* Worker threads for the sweeps (1: plain sequential loops).  Windows of one
 * tiling are disjoint, and so are the footprints of the regions of one colour
 * in the region order, so the work split between threads touches disjoint
 * pixels and increments: every thread count gives bitwise the same iterates. */
static int g_threads = 1;

int oracle_set_threads(int n) {
#ifdef _OPENMP
  g_threads = n < 1 ? 1 : n;
#else
  (void)n;
  g_threads = 1;
#endif
  return g_threads;
}

/*
 * One Dykstra sweep visits every window of the family once (Algorithm 2).
 * Windows of one tiling (s, a, b) -- the squares [a+s p, a+s p+s) x [b+s q, ...)
 * inside the image -- are disjoint, so their order is immaterial (Sec. 2.3).
 *
 * ORDER_DESC / ORDER_ASC: for each side (descending / ascending), for each
 * offset (a, b) in raster order, the whole tiling.
 *
 * ORDER_REGION(R): the anchor plane is cut into R x R regions; region (p, q)
 * gets colour 2 (p mod 2) + (q mod 2).  For colour 0, 1, 2, 3 in turn, for
 * every region of that colour, for each side descending, for each offset
 * (a', b') in raster order counted from the region origin (p R, q R), the
 * windows anchored at (p R + a' + s i, q R + b' + s j) inside the region --
 * the part of tiling ((p R + a') mod s, (q R + b') mod s) in the region.  With
 * R >= smax - 1 two regions of one colour touch disjoint pixels, so the order
 * of regions within a colour is immaterial as well.
 */
static void sweep_region(double* x, double* incs, int64_t H, int64_t W, const side_table* st,
                         int64_t R, int64_t p, int64_t q, double* ybuf) {
  int64_t HW = H * W;
  for (int k = 0; k < st->n; ++k) {
    int32_t s = st->side[k];
    for (int32_t ap = 0; ap < s; ++ap)
      for (int32_t bp = 0; bp < s; ++bp) {
        /* offsets (ap, bp) count from the region origin */
        int32_t a = (int32_t)((p * R + ap) % s), b = (int32_t)((q * R + bp) % s);
        double* inc = incs + (st->tbase[k] + (int64_t)a * s + b) * HW;
        project_tiling_part(x, inc, H, W, s, a, b, st->r2[k], p * R, p * R + R, q * R,
                            q * R + R, ybuf);
      }
  }
}

static void sweep(double* x, double* incs, int64_t H, int64_t W, const side_table* st, int order,
                  int32_t region, double* ybuf) {
  int64_t HW = H * W;
  const int nt = g_threads;
  const size_t ybytes = (size_t)st->side[0] * st->side[0] * sizeof(double);
  if (order == ORACLE_ORDER_DESC || order == ORACLE_ORDER_ASC) {
    for (int kk = 0; kk < st->n; ++kk) {
      int k = (order == ORACLE_ORDER_DESC) ? kk : st->n - 1 - kk;
      int32_t s = st->side[k];
      for (int32_t a = 0; a < s; ++a)
        for (int32_t b = 0; b < s; ++b) {
          double* inc = incs + (st->tbase[k] + (int64_t)a * s + b) * HW;
          if (nt == 1) {
            project_tiling_part(x, inc, H, W, s, a, b, st->r2[k], 0, H, 0, W, ybuf);
            continue;
          }
          /* one band of window rows per iteration: disjoint windows */
          int64_t nrows = (H - a) / s;
#pragma omp parallel num_threads(nt)
          {
            double* yb = (double*)malloc(ybytes);
#pragma omp for schedule(static)
            for (int64_t r = 0; r < nrows; ++r)
              project_tiling_part(x, inc, H, W, s, a, b, st->r2[k], a + r * s, a + r * s + 1, 0,
                                  W, yb);
            free(yb);
          }
        }
    }
    return;
  }
  int64_t R = region;
  int64_t nry = (H + R - 1) / R, nrx = (W + R - 1) / R;
  for (int color = 0; color < 4; ++color) {
    if (nt == 1) {
      for (int64_t p = color >> 1; p < nry; p += 2)
        for (int64_t q = color & 1; q < nrx; q += 2)
          sweep_region(x, incs, H, W, st, R, p, q, ybuf);
      continue;
    }
    /* the regions of one colour have disjoint footprints */
    int64_t npy = (nry - (color >> 1) + 1) / 2, npx = (nrx - (color & 1) + 1) / 2;
#pragma omp parallel num_threads(nt)
    {
      double* yb = (double*)malloc(ybytes);
#pragma omp for schedule(dynamic, 4)
      for (int64_t r = 0; r < npy * npx; ++r)
        sweep_region(x, incs, H, W, st, R, (color >> 1) + 2 * (r / npx),
                     (color & 1) + 2 * (r % npx), yb);
      free(yb);
    }
  }
}

/* Sum over every window S of the family of its increment I_S at each pixel
 * (canonical tiling layout; entries of a tiling plane outside its windows are
 * ignored). */
static void increment_sum(const double* incs, int64_t H, int64_t W, const side_table* st,
                          double* acc) {
  int64_t HW = H * W;
  memset(acc, 0, (size_t)HW * sizeof(double));
  for (int k = 0; k < st->n; ++k) {
    int32_t s = st->side[k];
    for (int32_t a = 0; a < s; ++a)
      for (int32_t b = 0; b < s; ++b) {
        const double* inc = incs + (st->tbase[k] + (int64_t)a * s + b) * HW;
        for (int64_t i0 = a; i0 + s <= H; i0 += s)
          for (int64_t j0 = b; j0 + s <= W; j0 += s)
            for (int64_t i = i0; i < i0 + s; ++i)
              for (int64_t j = j0; j < j0 + s; ++j) acc[i * W + j] += inc[i * W + j];
      }
  }
}

/* Large buffers (the increments: T H W doubles) on 2 MiB boundaries with
 * transparent huge pages requested: a region touches a few rows of every
 * tiling plane, which with 4 KiB pages costs a TLB miss per row. */
static double* alloc_big(size_t n) {
  void* p = NULL;
  size_t bytes = n * sizeof(double);
  if (posix_memalign(&p, (size_t)2 << 20, bytes ? bytes : 1) != 0) return NULL;
#ifdef MADV_HUGEPAGE
  madvise(p, bytes, MADV_HUGEPAGE);
#endif
  return (double*)p;
}

static int dykstra_run(const double* x0, int64_t H, int64_t W, const int32_t* sides,
                       int32_t nsides, const double* r2, int32_t order, int32_t region,
                       double tol, int32_t max_sweeps, double* z, double* incs, int warm,
                       int32_t* sweeps_out, double* delta_out) {
  side_table st;
  if (H < 1 || W < 1 || max_sweeps < 1) return -1;
  if (make_side_table(sides, r2, nsides, H, W, &st) != 0) return -1;
  if (order == ORACLE_ORDER_REGION && (region < 1 || region < st.side[0] - 1)) return -1;
  if (order < 0 || order > 2) return -1;
  if (warm && !incs) return -1;
  int64_t HW = H * W;
  int own = 0;
  if (!incs) {
    incs = alloc_big((size_t)(st.ntilings * HW));
    if (!incs) return -1;
    own = 1;
  }
  double* prev = (double*)malloc((size_t)HW * sizeof(double));
  double* ybuf = (double*)malloc((size_t)st.side[0] * st.side[0] * sizeof(double));
  if (!prev || !ybuf) { free(prev); free(ybuf); if (own) free(incs); return -1; }
  if (warm) {
    /* Dykstra's invariant x + sum_S I_S = x0 fixes the start from given
     * increments: x = x0 - sum_S I_S. */
    increment_sum(incs, H, W, &st, prev);
#if ORACLE_MUTANT == 10
    for (int64_t i = 0; i < HW; ++i) z[i] = x0[i]; /* start ignores the given increments */
#else
    for (int64_t i = 0; i < HW; ++i) z[i] = x0[i] - prev[i];
#endif
  } else {
    memset(incs, 0, (size_t)(st.ntilings * HW) * sizeof(double));
    if (z != x0) memcpy(z, x0, (size_t)HW * sizeof(double));
  }
  int32_t sw = 0;
  double delta = INFINITY;
  while (sw < max_sweeps) {
    memcpy(prev, z, (size_t)HW * sizeof(double));
    sweep(z, incs, H, W, &st, order, region, ybuf);
    ++sw;
    delta = 0.0;
    for (int64_t i = 0; i < HW; ++i) {
      double d = fabs(z[i] - prev[i]);
      if (d > delta) delta = d;
    }
    if (tol > 0.0 && delta < tol) break;
  }
  if (sweeps_out) *sweeps_out = sw;
  if (delta_out) *delta_out = delta;
  free(prev);
  free(ybuf);
  if (own) free(incs);
  return 0;
}

/*
 * Dykstra projection of x0 onto the intersection of the window balls.
 *   x0, z      : H x W row-major (z may alias a copy of x0; x0 is not written)
 *   sides, r2  : nsides window sides and their bounds (sum of squares <= r2)
 *   order      : ORACLE_ORDER_*; region: R for ORACLE_ORDER_REGION
 *   tol        : stop after the first sweep with max|x - x_prev| < tol
 *                (tol <= 0: run exactly max_sweeps sweeps)
 *   incs       : optional T x H x W increments I (canonical tiling index:
 *                sides descending, then a, then b); zero-initialised here.
 * Returns 0, or -1 on invalid arguments / allocation failure.
 */
int oracle_dykstra(const double* x0, int64_t H, int64_t W, const int32_t* sides, int32_t nsides,
                   const double* r2, int32_t order, int32_t region, double tol,
                   int32_t max_sweeps, double* z, double* incs, int32_t* sweeps_out,
                   double* delta_out) {
  return dykstra_run(x0, H, W, sides, nsides, r2, order, region, tol, max_sweeps, z, incs, 0,
                     sweeps_out, delta_out);
}

/*
 * Dykstra started from given increments (a warm start, e.g. from the
 * projection of a nearby input, as when Algorithm 1 projects a slowly changing
 * point every iteration).  Dykstra is block-coordinate minimisation of the
 * dual function of the projection, so it reaches the same limit from any
 * increments; the iterate starts at x = x0 - sum_S I_S so that the invariant
 * x + sum_S I_S = x0 holds from the first window on.  incs (T x H x W,
 * canonical layout, required) holds the start on entry and the final
 * increments on return; other arguments as oracle_dykstra.
 */
int oracle_dykstra_warm(const double* x0, int64_t H, int64_t W, const int32_t* sides,
                        int32_t nsides, const double* r2, int32_t order, int32_t region,
                        double tol, int32_t max_sweeps, double* z, double* incs,
                        int32_t* sweeps_out, double* delta_out) {
  return dykstra_run(x0, H, W, sides, nsides, r2, order, region, tol, max_sweeps, z, incs, 1,
                     sweeps_out, delta_out);
}

/* Number of windows of the family (each side: (H-s+1)(W-s+1)). */
int64_t oracle_window_count(int64_t H, int64_t W, const int32_t* sides, int32_t nsides) {
  int64_t n = 0;
  for (int k = 0; k < nsides; ++k) n += (H - sides[k] + 1) * (W - sides[k] + 1);
  return n;
}

/* ------------------------------------------------------------------------- */
/* Checks: feasibility and the KKT certificate                                 */
/* ------------------------------------------------------------------------- */

/* max over all windows S of (sum_S z^2) / r2_S - 1; <= 0 means feasible. */
double oracle_max_violation(const double* z, int64_t H, int64_t W, const int32_t* sides,
                            int32_t nsides, const double* r2) {
  double worst = -INFINITY;
  for (int k = 0; k < nsides; ++k) {
    int32_t s = sides[k];
    for (int64_t i0 = 0; i0 + s <= H; ++i0)
      for (int64_t j0 = 0; j0 + s <= W; ++j0) {
        double n = 0.0;
        for (int64_t i = i0; i < i0 + s; ++i)
          for (int64_t j = j0; j < j0 + s; ++j) n += z[i * W + j] * z[i * W + j];
        double v = n / r2[k] - 1.0;
        if (v > worst) worst = v;
      }
  }
  return worst;
}

/*
 * KKT certificate of z = P(x0) from Dykstra's increments I (canonical layout).
 * At the projection onto an intersection of balls B_S = {sum_S v^2 <= r2_S}:
 *   x0 - z = sum_S I_S,  I_S = mu_S z_S with mu_S >= 0, mu_S = 0 unless
 *   sum_S z^2 = r2_S.  Reported (out[0..5]):
 *   0: max feasibility violation (as oracle_max_violation)
 *   1: max_i |x0_i - z_i - sum_S I_S,i|
 *   2: max_S ||I_S - mu_S z_S||_inf with mu_S = <I_S, z_S>/||z_S||^2
 *   3: min_S mu_S
 *   4: max ||I_S||_inf over windows with sum_S z^2 < (1 - slack) r2_S
 *   5: max_S mu_S
 */
int oracle_kkt(const double* x0, const double* z, const double* incs, int64_t H, int64_t W,
               const int32_t* sides, int32_t nsides, const double* r2, double slack,
               double* out) {
  side_table st;
  if (make_side_table(sides, r2, nsides, H, W, &st) != 0) return -1;
  int64_t HW = H * W;
  double* acc = (double*)calloc((size_t)HW, sizeof(double));
  if (!acc) return -1;
  double feas = -INFINITY, res = 0.0, mumin = INFINITY, mumax = 0.0, inact = 0.0;
  for (int k = 0; k < st.n; ++k) {
    int32_t s = st.side[k];
    for (int32_t a = 0; a < s; ++a)
      for (int32_t b = 0; b < s; ++b) {
        const double* inc = incs + (st.tbase[k] + (int64_t)a * s + b) * HW;
        for (int64_t i0 = a; i0 + s <= H; i0 += s)
          for (int64_t j0 = b; j0 + s <= W; j0 += s) {
            double zz = 0.0, iz = 0.0, imax = 0.0;
            for (int64_t i = i0; i < i0 + s; ++i)
              for (int64_t j = j0; j < j0 + s; ++j) {
                double zv = z[i * W + j], iv = inc[i * W + j];
                zz += zv * zv;
                iz += iv * zv;
                acc[i * W + j] += iv;
                if (fabs(iv) > imax) imax = fabs(iv);
              }
            double v = zz / st.r2[k] - 1.0;
            if (v > feas) feas = v;
            double mu = zz > 0.0 ? iz / zz : 0.0;
            if (mu < mumin) mumin = mu;
            if (mu > mumax) mumax = mu;
            for (int64_t i = i0; i < i0 + s; ++i)
              for (int64_t j = j0; j < j0 + s; ++j) {
                double r = fabs(inc[i * W + j] - mu * z[i * W + j]);
                if (r > res) res = r;
              }
            if (zz < (1.0 - slack) * st.r2[k] && imax > inact) inact = imax;
          }
      }
  }
  double inv = 0.0;
  for (int64_t i = 0; i < HW; ++i) {
    double d = fabs(x0[i] - z[i] - acc[i]);
    if (d > inv) inv = d;
  }
  free(acc);
  out[0] = feas; out[1] = inv; out[2] = res; out[3] = mumin; out[4] = inact; out[5] = mumax;
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Incomplete Dykstra (ICD), Sec. 3.2                                          */
/* ------------------------------------------------------------------------- */

/*
 * P_incomplete = P_{Omega^K} o ... o P_{Omega^0} applied to x0.
 *   K          : blocks have side 2^K; levels k = 0..K have square side 2^k
 *   r2[k]      : bound of a square of side 2^k (k = 0..K)
 *   tol, mode  : block stopping rule after an inner sweep:
 *                ORACLE_TOL_MAXABS  -> max |x - x_new| < tol
 *                ORACLE_TOL_MEANABS -> sum |x - x_new| <= tol * (pixels of block)
 *   max_inner  : cap on inner sweeps per block (at least one always runs)
 *   num_phases : phases i = 0 .. num_phases-1 (the paper's family: K+1)
 * Phase i: offset o = 2^i mod 2^K on both axes; blocks are the cells of the
 * lattice o + 2^K Z^2 clipped to the image; a block runs Dykstra over the
 * squares of side 2^k (k = K down to i) of that lattice that lie inside the
 * image, with its increments zeroed at the start of the phase.
 * inner_total (optional) receives the sum of inner sweeps over all blocks.
 */
/* A family of ICD phases: phase p uses blocks of side 2^K on the lattice
 * whose origin is shifted by (shift_y[p], shift_x[p]) (0 <= shift < 2^K;
 * blocks cut by the image edge are clipped) and projects, inside each block,
 * onto its squares of side 2^k for k = K down to min_level[p] by Dykstra with
 * increments zeroed at the phase start, until the block converges.  The
 * paper's family (Sec. 3.2) is phase i = 0..K with both shifts 2^i mod 2^K and
 * lowest level i; other shifts (e.g. along one axis only) are the variants the
 * paper leaves open. */
int oracle_icd_family(const double* x0, int64_t H, int64_t W, int32_t K, const double* r2,
                      double tol, int32_t mode, int32_t max_inner, int32_t n_phases,
                      const int32_t* shift_y, const int32_t* shift_x, const int32_t* min_level,
                      double* z, int64_t* inner_total) {
  if (H < 1 || W < 1 || K < 0 || K > 10 || max_inner < 1 || n_phases < 1) return -1;
  int64_t HW = H * W, B = (int64_t)1 << K;
  for (int k = 0; k <= K; ++k)
    if (!(r2[k] > 0.0) || !isfinite(r2[k])) return -1;
  for (int32_t ph = 0; ph < n_phases; ++ph)
    if (shift_y[ph] < 0 || shift_y[ph] >= B || shift_x[ph] < 0 || shift_x[ph] >= B ||
        min_level[ph] < 0 || min_level[ph] > K)
      return -1;
  double* q = (double*)calloc((size_t)((K + 1) * HW), sizeof(double));
  double* ybuf = (double*)malloc((size_t)(B * B) * sizeof(double));
  if (!q || !ybuf) { free(q); free(ybuf); return -1; }
  if (z != x0) memcpy(z, x0, (size_t)HW * sizeof(double));
  int64_t total = 0;
  for (int32_t ph = 0; ph < n_phases; ++ph) {
    const int lo = min_level[ph];
    int64_t start_y = shift_y[ph] > 0 ? shift_y[ph] - B : 0;
    int64_t start_x = shift_x[ph] > 0 ? shift_x[ph] - B : 0;
    for (int64_t by = start_y; by < H; by += B)
      for (int64_t bx = start_x; bx < W; bx += B) {
        int64_t ylo = by < 0 ? 0 : by, yhi = by + B < H ? by + B : H;
        int64_t xlo = bx < 0 ? 0 : bx, xhi = bx + B < W ? bx + B : W;
        int64_t npix = (yhi - ylo) * (xhi - xlo);
        for (int k = lo; k <= K; ++k)
          for (int64_t i = ylo; i < yhi; ++i)
            for (int64_t j = xlo; j < xhi; ++j) q[k * HW + i * W + j] = 0.0;
        for (int32_t it = 0; it < max_inner; ++it) {
          double dsum = 0.0, dmax = 0.0;
          for (int k = K; k >= lo; --k) {
            int64_t L = (int64_t)1 << k;
            double* qk = q + k * HW;
            for (int64_t sy = by; sy < by + B; sy += L)
              for (int64_t sx = bx; sx < bx + B; sx += L) {
                if (sy < 0 || sx < 0 || sy + L > H || sx + L > W) continue;
                double n = 0.0;
                int64_t c = 0;
                for (int64_t i = sy; i < sy + L; ++i)
                  for (int64_t j = sx; j < sx + L; ++j, ++c) {
                    double y = z[i * W + j] - qk[i * W + j];
                    ybuf[c] = y;
                    n += y * y;
                  }
                double t = 1.0;
                if (n > r2[k]) t = sqrt(r2[k] / n);
                c = 0;
                for (int64_t i = sy; i < sy + L; ++i)
                  for (int64_t j = sx; j < sx + L; ++j, ++c) {
                    double xn = t * ybuf[c];
                    qk[i * W + j] = xn - ybuf[c];
                    double d = fabs(z[i * W + j] - xn);
                    dsum += d;
                    if (d > dmax) dmax = d;
                    z[i * W + j] = xn;
                  }
              }
          }
          ++total;
          if (mode == ORACLE_TOL_MEANABS) {
            if (dsum <= tol * (double)npix) break;
          } else if (dmax < tol) {
            break;
          }
        }
      }
  }
  if (inner_total) *inner_total = total;
  free(q);
  free(ybuf);
  return 0;
}

/* ICD over a nested hierarchy of squares of any sides (Sec. 3.2 with the
 * sides 2^k replaced by a divisor chain; Sec. 5 leaves the partition open).
 *   side[j], j = 0..n_lev-1 : square side of level j, ascending, each dividing
 *                             the next; the block side is B = side[n_lev-1]
 *   r2[j]                   : bound of a square of level j
 *   phase p                 : blocks of side B on the lattice shifted by
 *                             (shift_y[p], shift_x[p]), 0 <= shift < B, clipped
 *                             by the image edge; each block runs Dykstra over
 *                             its level-j squares that lie inside the image,
 *                             levels j = n_lev-1 down to min_level[p], with
 *                             increments zeroed at the phase start
 * The stopping rule and max_inner are those of oracle_icd_family; the paper's
 * family is side[j] = 2^j, shifts 2^i mod 2^K, lowest level i. */
int oracle_icd_nested(const double* x0, int64_t H, int64_t W, int32_t n_lev, const int32_t* side,
                      const double* r2, double tol, int32_t mode, int32_t max_inner,
                      int32_t n_phases, const int32_t* shift_y, const int32_t* shift_x,
                      const int32_t* min_level, double* z, int64_t* inner_total) {
  if (H < 1 || W < 1 || n_lev < 1 || n_lev > 16 || max_inner < 1 || n_phases < 1) return -1;
  for (int j = 0; j < n_lev; ++j) {
    if (side[j] < 1 || side[j] > 4096 || !(r2[j] > 0.0) || !isfinite(r2[j])) return -1;
    if (j > 0 && (side[j] <= side[j - 1] || side[j] % side[j - 1] != 0)) return -1;
  }
  const int64_t B = side[n_lev - 1], HW = H * W;
  for (int32_t ph = 0; ph < n_phases; ++ph)
    if (shift_y[ph] < 0 || shift_y[ph] >= B || shift_x[ph] < 0 || shift_x[ph] >= B ||
        min_level[ph] < 0 || min_level[ph] >= n_lev)
      return -1;
  /* one increment plane per level (a pixel lies in one square per level) */
  double* inc = (double*)calloc((size_t)(n_lev * HW), sizeof(double));
  double* ybuf = (double*)malloc((size_t)(B * B) * sizeof(double));
  if (!inc || !ybuf) { free(inc); free(ybuf); return -1; }
  if (z != x0) memcpy(z, x0, (size_t)HW * sizeof(double));
  int64_t total = 0;
  for (int32_t ph = 0; ph < n_phases; ++ph) {
    const int lo = min_level[ph];
#if ORACLE_MUTANT == 12
    const int64_t oy = shift_y[ph] ? shift_y[ph] - B : 0, ox = shift_y[ph] ? shift_y[ph] - B : 0;
#else
    const int64_t oy = shift_y[ph] ? shift_y[ph] - B : 0, ox = shift_x[ph] ? shift_x[ph] - B : 0;
#endif
    for (int64_t by = oy; by < H; by += B)
      for (int64_t bx = ox; bx < W; bx += B) {
        const int64_t r0 = by > 0 ? by : 0, r1 = by + B < H ? by + B : H;
        const int64_t c0 = bx > 0 ? bx : 0, c1 = bx + B < W ? bx + B : W;
        const int64_t npix = (r1 - r0) * (c1 - c0);
        for (int j = lo; j < n_lev; ++j)
          for (int64_t i = r0; i < r1; ++i)
            memset(inc + j * HW + i * W + c0, 0, (size_t)(c1 - c0) * sizeof(double));
        for (int32_t it = 0; it < max_inner; ++it) {
          double dsum = 0.0, dmax = 0.0;
          for (int j = n_lev - 1 - (ORACLE_MUTANT == 11 && n_lev > 1); j >= lo; --j) {
            const int64_t L = side[j];
            double* I = inc + j * HW;
            for (int64_t sy = by; sy < by + B; sy += L)
              for (int64_t sx = bx; sx < bx + B; sx += L) {
                if (sy < 0 || sx < 0 || sy + L > H || sx + L > W) continue;
                /* Eq. (dykstra:if): y = x + I, x' = t y, I' = y - x' */
                double n = 0.0;
                int64_t c = 0;
                for (int64_t i = sy; i < sy + L; ++i)
                  for (int64_t q = sx; q < sx + L; ++q, ++c) {
#if ORACLE_MUTANT == 13
                    ybuf[c] = z[i * W + q] + I[(sy + q - sx) * W + sx + i - sy]; /* transposed */
#else
                    ybuf[c] = z[i * W + q] + I[i * W + q];
#endif
                    n += ybuf[c] * ybuf[c];
                  }
                const double t = n > r2[j] ? sqrt(r2[j] / n) : 1.0;
                c = 0;
                for (int64_t i = sy; i < sy + L; ++i)
                  for (int64_t q = sx; q < sx + L; ++q, ++c) {
                    const double xn = t * ybuf[c];
                    const double d = fabs(z[i * W + q] - xn);
                    dsum += d;
                    if (d > dmax) dmax = d;
                    I[i * W + q] = ybuf[c] - xn;
                    z[i * W + q] = xn;
                  }
              }
          }
          ++total;
          if (mode == ORACLE_TOL_MEANABS ? dsum <= tol * (double)npix : dmax < tol) break;
        }
      }
  }
  if (inner_total) *inner_total = total;
  free(inc);
  free(ybuf);
  return 0;
}

/* The paper's ICD (Sec. 3.2): phases i = 0 .. num_phases - 1, both shifts
 * 2^i mod 2^K, lowest level i. */
int oracle_icd(const double* x0, int64_t H, int64_t W, int32_t K, const double* r2, double tol,
               int32_t mode, int32_t max_inner, int32_t num_phases, double* z,
               int64_t* inner_total) {
  if (K < 0 || K > 10 || num_phases < 1 || num_phases > K + 1) return -1;
  int32_t sy[11], sx[11], lo[11];
  for (int32_t i = 0; i < num_phases; ++i) {
    sy[i] = sx[i] = (int32_t)(((int64_t)1 << i) & (((int64_t)1 << K) - 1));
    lo[i] = i;
  }
  return oracle_icd_family(x0, H, W, K, r2, tol, mode, max_inner, num_phases, sy, sx, lo, z,
                           inner_total);
}

/* ------------------------------------------------------------------------- */
/* Monte-Carlo weights (Sec. 2.1)                                              */
/* ------------------------------------------------------------------------- */

/* The paper balances the window bounds through q_alpha, the alpha-quantile of
 *   Q = max over windows S of ((t_S)^(1/4) - mu_s) / sigma_s,  t_S = sum_S e^2,
 * for a field e of i.i.d. N(0,1) values, with mu_s = (|S| - 1/2)^(1/4) and
 * sigma_s^2 = 1/(8 sqrt|S|).  The paper does not say how the fields are drawn;
 * here they come from a counter-based generator so that any field can be
 * recomputed on its own:
 *   Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 *   easy as 1, 2, 3", SC 2011): a 4 x 64-bit counter block is mixed by ten
 *   rounds; each round multiplies words 0 and 2 by fixed odd constants, takes
 *   the 128-bit products apart and recombines them with words 1 and 3 and the
 *   key; the key is advanced by two Weyl constants between rounds.
 *   Pixel p = i W + j of field f is normal number (p mod 4) of the block with
 *   counter {p / 4, f, 0, 0} and key {seed, 0}; the words (w0, w1) and (w2, w3)
 *   become two normals each by the Box-Muller transform with
 *   u = ((w >> 11) + 1/2) 2^-53. */

#define PHILOX_M0 0xD2E7470EE14C6C93ULL
#define PHILOX_M1 0xCA5A826395121157ULL
#define PHILOX_W0 0x9E3779B97F4A7C15ULL
#define PHILOX_W1 0xBB67AE8584CAA73BULL

void oracle_philox4x64_10(const uint64_t* ctr, const uint64_t* key, uint64_t* out) {
  uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0 && ORACLE_MUTANT != 6) {
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
    unsigned __int128 p0 = (unsigned __int128)PHILOX_M0 * c0;
    unsigned __int128 p1 = (unsigned __int128)PHILOX_M1 * c2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

static double unit_open(uint64_t w) { return ((double)(w >> 11) + 0.5) * 0x1p-53; }

/* Field f (H x W, row-major) of the Monte-Carlo sample. */
void oracle_mc_field(uint64_t seed, int64_t f, int64_t H, int64_t W, double* out) {
  const double two_pi = 6.283185307179586;
  for (int64_t p = 0; p < H * W; ++p) {
    uint64_t ctr[4] = {(uint64_t)(p / 4), (uint64_t)f, 0, 0}, key[2] = {seed, 0}, w[4];
    oracle_philox4x64_10(ctr, key, w);
    int lane = (int)(p % 4);
    double u0 = unit_open(w[lane < 2 ? 0 : 2]);
    double u1 = unit_open(w[lane < 2 ? 1 : 3]);
#if ORACLE_MUTANT == 9
    double r = sqrt(-log(u0));
#else
    double r = sqrt(-2.0 * log(u0));
#endif
    out[p] = (lane % 2 == 0) ? r * cos(two_pi * u1) : r * sin(two_pi * u1);
  }
}

/* Q of one field, from the definition: every window S of every listed side,
 * t_S summed directly, transformed and maximised.  tmax_out[k] (may be NULL)
 * receives max_S t_S over the windows of side sides[k] (-1 if none fits). */
double oracle_mc_statistic(const double* e, int64_t H, int64_t W, const int32_t* sides,
                           int32_t nsides, double* tmax_out) {
  double Q = -INFINITY;
  for (int k = 0; k < nsides; ++k) {
    const int32_t s = sides[k];
    const double npix = (double)s * (double)s;
#if ORACLE_MUTANT == 5
    const double mu = pow(npix, 0.25);
#else
    const double mu = pow(npix - 0.5, 0.25);
#endif
    const double sigma = sqrt(1.0 / (8.0 * sqrt(npix)));
    double tmax = -1.0;
    for (int64_t i0 = 0; i0 + s <= H; ++i0)
      for (int64_t j0 = 0; j0 + s <= W; ++j0) {
        double t = 0.0;
        for (int64_t i = i0; i < i0 + s; ++i)
          for (int64_t j = j0; j < j0 + s - (ORACLE_MUTANT == 7); ++j) t += e[i * W + j] * e[i * W + j];
        if (t > tmax) tmax = t;
        double v = (pow(t, 0.25) - mu) / sigma;
        if (v > Q) Q = v;
      }
    if (tmax_out) tmax_out[k] = tmax;
  }
  return Q;
}

static int cmp_double(const void* a, const void* b) {
  double x = *(const double*)a, y = *(const double*)b;
  return (x > y) - (x < y);
}

/* Empirical alpha-quantile of n samples: the smallest sample q with at least
 * ceil(alpha n) samples <= q, i.e. the ceil(alpha n)-th order statistic
 * (0 < alpha <= 1).  Returns NaN for invalid arguments. */
double oracle_order_quantile(const double* q, int64_t n, double alpha) {
  if (n < 1 || !(alpha > 0.0) || alpha > 1.0) return NAN;
  double* v = (double*)malloc((size_t)n * sizeof(double));
  if (!v) return NAN;
  memcpy(v, q, (size_t)n * sizeof(double));
  qsort(v, (size_t)n, sizeof(double), cmp_double);
  int64_t k = (int64_t)ceil(alpha * (double)n);
  if (k < 1) k = 1;
  if (k > n) k = n;
  double r = v[ORACLE_MUTANT == 8 && k < n ? k : k - 1];
  free(v);
  return r;
}
