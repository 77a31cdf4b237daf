/*
 * cfs_oracle.c -- plain, single-threaded FP64 reference of the chaos game of
 * a composable function system (CFS).
 *
 * TEST INFRASTRUCTURE ONLY.  This file exists so that tests, the smoke check
 * and the benchmark's CPU baseline can check the GPU library against an
 * obviously correct implementation.  The product path never links, loads or
 * calls it, and it shares no code, header, table or constant generator with
 * the GPU library.
 *
 * What is computed (Schloss, "Composable function systems as a
 * general-purpose rendering framework"):
 *   - Section 1 and Section 3 (opening paragraphs): the chaos game.  A single
 *     point starts at a random position; each step it applies one function of
 *     the system chosen at random, and after the step it is histogrammed
 *     (splatted) onto the output image.
 *   - Section 1 (description of fig. "workflow"): the colour of a splat is the
 *     index of the function that moved the point there.
 *   - Section 3 (discussion of fig. "circle", panels B and C) and the caption
 *     of fig. "workflow": the composed spatial transform acts on a COPY of the
 *     point; the original keeps iterating.  That copy is what is splatted.
 *
 * Where the paper is silent (random number generator, selection rule, binning,
 * burn-in, Gaussian kernel), this file follows the readings listed in the
 * design notes of the repository; each function below states its reading.
 *
 * Conventions: parameters arrive as FP32 values and are widened to FP64, so
 * that the only difference to a GPU path that computes in FP32 is arithmetic
 * rounding.  No FMA contraction (compile with -ffp-contract=off).  Loops are
 * written in the order of the method, with no blocking or reordering.
 *
 * Parity status of each function is recorded next to it.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL -1

/* Final-transform kinds understood by the oracle (named by the tests). */
#define ORC_FINAL_IDENTITY 0
#define ORC_FINAL_SWIRL 1
#define ORC_FINAL_TWIST_CAMERA 2
#define ORC_FINAL_STRETCH 3
#define ORC_FINAL_RING 4

#define ORC_MAX_MAPS 64

/* Map kinds. */
#define ORC_MAP_AFFINE 0
#define ORC_MAP_CIRCLE 1
#define ORC_MAX_DIM 3

/* ------------------------------------------------------------------------ */
/* Philox4x32-10.                                                           */
/* Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as easy as 1, 2, 3" */
/* (SC'11).  Each of the 10 rounds multiplies counter words 0 and 2 by two  */
/* fixed 32-bit constants to 64-bit products; the high halves are xored     */
/* with the other two counter words and the two key words, the low halves    */
/* move over, and the key advances by two Weyl constants between rounds.    */
/* Pinned by the published known-answer vectors.                           */
/* ------------------------------------------------------------------------ */
static const uint32_t PHILOX_MUL0 = 0xD2511F53u;
static const uint32_t PHILOX_MUL1 = 0xCD9E8D57u;
static const uint32_t PHILOX_WEYL0 = 0x9E3779B9u;
static const uint32_t PHILOX_WEYL1 = 0xBB67AE85u;

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                       uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += PHILOX_WEYL0;
      k1 += PHILOX_WEYL1;
    }
    uint64_t prod0 = (uint64_t)PHILOX_MUL0 * (uint64_t)x0;
    uint64_t prod1 = (uint64_t)PHILOX_MUL1 * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
    uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Batch helper for tests: out[i] = philox(ctrs[i], key). */
void orc_philox_many(uint64_t seed, const uint32_t *ctrs, uint32_t *out,
                     int64_t n) {
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  for (int64_t i = 0; i < n; ++i) orc_philox4x32_10(ctrs + 4 * i, key, out + 4 * i);
}

/* ------------------------------------------------------------------------ */
/* Function selection (Section 1 / Section 3: "a new function is chosen at  */
/* random" every step; the paper gives no rule).  Reading: inverse CDF over */
/* integer thresholds.  thresh[i] = ceil(2^32 * P_i) with P_i the FP64       */
/* left-to-right cumulative probability, thresh[n-1] = 2^32.  With no        */
/* probabilities (all equal) the thresholds are the exact integers           */
/* ceil((i+1) * 2^32 / n).  The index drawn by u is min{ i : u < thresh[i] }.*/
/* Pinned exhaustively over all 2^32 values of u by the tests.               */
/* ------------------------------------------------------------------------ */
int orc_thresholds(const double *prob, int n, uint64_t *thresh) {
  if (n < 1 || n > ORC_MAX_MAPS) return ORC_EINVAL;
  const uint64_t two32 = (uint64_t)1 << 32;
  if (prob == NULL) {
    for (int i = 0; i < n; ++i)
      thresh[i] = ((uint64_t)(i + 1) * two32 + (uint64_t)(n - 1)) / (uint64_t)n;
  } else {
    double cum = 0.0;
    for (int i = 0; i < n; ++i) {
      if (!(prob[i] >= 0.0) || !isfinite(prob[i])) return ORC_EINVAL;
      cum += prob[i];
      double scaled = ceil(ldexp(cum, 32));
      thresh[i] = scaled >= ldexp(1.0, 32) ? two32 : (uint64_t)scaled;
    }
    if (fabs(cum - 1.0) > 1e-6) return ORC_EINVAL;
  }
  thresh[n - 1] = two32;
  return ORC_OK;
}

int orc_select(uint32_t u, const uint64_t *thresh, int n) {
  for (int i = 0; i < n; ++i)
    if ((uint64_t)u < thresh[i]) return i;
  return n - 1; /* unreachable: thresh[n-1] = 2^32 > u */
}

/* Exhaustive check helper: counts[i] = #{u in [0, 2^32) : select(u) = i},
 * evaluated with a plain per-u search (slow by design). */
void orc_select_histogram(const uint64_t *thresh, int n, uint64_t *counts) {
  for (int i = 0; i < n; ++i) counts[i] = 0;
  uint32_t u = 0;
  do {
    counts[orc_select(u, thresh, n)]++;
    ++u;
  } while (u != 0);
}

/* ------------------------------------------------------------------------ */
/* System, run and image descriptions (oracle's own types).                 */
/* ------------------------------------------------------------------------ */
typedef struct {
  int32_t dim;           /* 2 or 3 */
  int32_t n_maps;        /* 1..64 */
  const float *A;        /* [n_maps][dim][dim] row-major */
  const float *b;        /* [n_maps][dim] */
  const double *prob;    /* [n_maps] or NULL for equal probabilities */
  int32_t final_kind;    /* ORC_FINAL_* */
  const float *final_params; /* up to 24 values, meaning per kind */
  const int32_t *kind;   /* [n_maps] ORC_MAP_* or NULL (all affine) */
  int32_t compose;       /* 0: transform a copy; 1: feed the transformed point back */
} orc_system;

typedef struct {
  uint64_t seed;
  uint32_t instance;
  uint32_t n_points;
  uint32_t point_offset; /* global id of the first point */
  uint32_t n_iters;      /* T: map applications per point in this call */
  uint32_t burn_in;      /* B: steps 1..B of the whole game are not splatted */
  uint32_t iter_offset;  /* K: steps taken before this call (0: start from the
                            initial point; else from final_p, which is then
                            read as well as written) */
} orc_run;

typedef struct {
  int32_t width, height, channels;
  float lo[2], hi[2];
} orc_window;

/* Random streams (reading; the paper only names a random-number scribble
 * and a simple PRNG scheme).  Key = (seed low word, seed high word).
 * Counter = (global point id, block, instance, tag).  Tag 1, block 0 gives the
 * initial point; tag 0, block j gives the four draws of iterations 4j+1..4j+4. */
static void point_stream(const orc_run *r, uint32_t pid, uint32_t block,
                         uint32_t tag, uint32_t out[4]) {
  uint32_t key[2] = {(uint32_t)r->seed, (uint32_t)(r->seed >> 32)};
  uint32_t ctr[4] = {pid, block, r->instance, tag};
  orc_philox4x32_10(ctr, key, out);
}

/* Map draw of global step g >= 1 of point pid: word (g-1) mod 4 of Philox
 * block (pid, (g-1)/4, instance, 0); the block is fetched at the first step
 * of a call and whenever a new block starts.  A game cut into calls at any
 * step therefore draws the same words as one call (Section 3: the chaos
 * game is one sequence of steps per point). */
static uint32_t step_draw(const orc_run *r, uint32_t pid, uint32_t g, int first,
                          uint32_t words[4]) {
  if (first || (g - 1) % 4 == 0) point_stream(r, pid, (g - 1) / 4, 0, words);
  return words[(g - 1) % 4];
}

/* Steps of this call that are not splatted: the part of the burn-in that
 * lies in it (a call inside the burn-in splats nothing). */
static uint32_t call_burn_in(const orc_run *r) {
  const uint32_t b = r->burn_in > r->iter_offset ? r->burn_in - r->iter_offset : 0u;
  return b < r->n_iters ? b : r->n_iters;
}

/* Initial point (Section 3: the chaos game "starts with a single point
 * randomly chosen").  Reading: uniform on the 2^-24 grid of [0,1)^dim, one
 * 24-bit word per coordinate; exact in FP32 and FP64. */
static void initial_point(const orc_run *r, uint32_t pid, int dim, double p[3]) {
  uint32_t w[4];
  point_stream(r, pid, 0, 1, w);
  for (int c = 0; c < dim; ++c) p[c] = ldexp((double)(w[c] >> 8), -24);
}

/* Circle map (Section 3, the circle equation; 2D).  Reading of the garbled
 * equation: with u = x^2 + y^2 (= r^2) and v = theta / (2 pi), theta the
 * polar angle in [0, 2 pi), the new point has radius sqrt(v) and angle
 * pi (u + f), where f is the map's id (0 or 1; taken from b_k[0]).  The map
 * sends (u, v) to (v, (u + f) / 2), so it keeps the uniform measure of the
 * unit disk and sends the disk onto its upper (f = 0) or lower (f = 1) half. */
static void circle_map(double f, double p[3]) {
  const double two_pi = 6.283185307179586476925286766559;
  double u = p[0] * p[0] + p[1] * p[1];
  double th = atan2(p[1], p[0]);
  if (th < 0.0) th += two_pi;
  double r2 = sqrt(th / two_pi);
  double th2 = 0.5 * two_pi * (u + f);
  p[0] = r2 * cos(th2);
  p[1] = r2 * sin(th2);
}

/* Apply map k: p <- A_k p + b_k (Section 3: each function maps P_n to P_{n+1};
 * the configured systems are affine), or the circle map for circle kinds. */
static void apply_map(const orc_system *s, int k, double p[3]) {
  int d = s->dim;
  if (s->kind && s->kind[k] == ORC_MAP_CIRCLE) {
    circle_map((double)s->b[k * d], p);
    return;
  }
  double q[3] = {0, 0, 0};
  for (int r = 0; r < d; ++r) {
    double acc = 0.0;
    for (int c = 0; c < d; ++c) acc += (double)s->A[(k * d + r) * d + c] * p[c];
    q[r] = acc + (double)s->b[k * d + r];
  }
  for (int r = 0; r < d; ++r) p[r] = q[r];
}

/* Composed transform applied to a COPY q of the point p (caption of fig.
 * "workflow"; Section 3, fig. "circle" B).  p itself is never changed here.
 *  SWIRL (2D)   params {cx, cy, kappa, tx, ty}: with d = p - c and r = |d|,
 *               q = c + t + R(kappa r) d   (a swirl r,th -> r, th + kappa r,
 *               then a translation).
 *  STRETCH (2D) params {sx, sy}: q = (sx x, y - sy cos x)  (the stretch
 *               equation of Section 3 is sx = 2, sy = 1).
 *  RING (2D)    params {r_in, r_out}: the point at radius r about the origin
 *               moves along its ray to radius
 *               R = sqrt(r_in^2 + (r_out^2 - r_in^2) r^2)  (the origin goes
 *               to (r_in, 0)).  It sends the uniform unit disk to the uniform
 *               annulus r_in <= R < r_out: the "rings" object of Section 3's
 *               multiple-objects scene (a topologically non-trivial object
 *               from the disk primitive; the paper gives no formula).
 *  TWIST_CAMERA (3D) params {kappa, cx, cy, cz, M[12], fx, fy}: twist the
 *               copy about the vertical axis through c by the angle
 *               kappa (y - cy), then map it to view space v = R w + tr with
 *               w = q - c and M = [R | tr] row-major 3x4; the projected point
 *               is (fx v_x / v_z, fy v_y / v_z), depth v_z.
 * On return q holds the 2D image-plane position; depth is set for 3D. */
static void final_transform(const orc_system *s, const double p[3], double q[2],
                            double *depth) {
  const float *fp = s->final_params;
  switch (s->final_kind) {
    case ORC_FINAL_SWIRL: {
      double cx = fp[0], cy = fp[1], kappa = fp[2], tx = fp[3], ty = fp[4];
      double dx = p[0] - cx, dy = p[1] - cy;
      double r = sqrt(dx * dx + dy * dy);
      double ang = kappa * r;
      double c = cos(ang), sn = sin(ang);
      q[0] = cx + tx + (c * dx - sn * dy);
      q[1] = cy + ty + (sn * dx + c * dy);
      break;
    }
    case ORC_FINAL_STRETCH: {
      q[0] = (double)fp[0] * p[0];
      q[1] = p[1] - (double)fp[1] * cos(p[0]);
      break;
    }
    case ORC_FINAL_RING: {
      double ri = fp[0], ro = fp[1];
      double r2 = p[0] * p[0] + p[1] * p[1];
      double R = sqrt(ri * ri + (ro * ro - ri * ri) * r2);
      if (r2 > 0.0) {
        double r = sqrt(r2);
        q[0] = R * (p[0] / r);
        q[1] = R * (p[1] / r);
      } else {
        q[0] = R;
        q[1] = 0.0;
      }
      break;
    }
    case ORC_FINAL_TWIST_CAMERA: {
      double kappa = fp[0], cx = fp[1], cy = fp[2], cz = fp[3];
      double wx = p[0] - cx, wy = p[1] - cy, wz = p[2] - cz;
      double ang = kappa * wy;
      double c = cos(ang), sn = sin(ang);
      double tx = c * wx - sn * wz;
      double tz = sn * wx + c * wz;
      double w[3] = {tx, wy, tz};
      double v[3];
      for (int r = 0; r < 3; ++r) {
        double acc = 0.0;
        for (int cc = 0; cc < 3; ++cc) acc += (double)fp[4 + r * 4 + cc] * w[cc];
        v[r] = acc + (double)fp[4 + r * 4 + 3];
      }
      double fx = fp[16], fy = fp[17];
      q[0] = fx * v[0] / v[2];
      q[1] = fy * v[1] / v[2];
      *depth = v[2];
      break;
    }
    default: /* identity: the first two coordinates */
      q[0] = p[0];
      q[1] = p[1];
      break;
  }
}

/* Binning (reading; the paper only says the point colours "the appropriate
 * pixel"): half-open window [lo, hi), pixel i = floor((q - lo) * W / (hi - lo)),
 * points outside the window or NaN are dropped, row 0 at lo_y.
 * Returns 1 and sets (ix, iy) when the point lands on the image.
 * The fractional pixel coordinates are returned in fx, fy for guard-band
 * bookkeeping by the tests. */
static int bin_point(const orc_window *w, const double q[2], int *ix, int *iy,
                     double *fx, double *fy) {
  double sx = (double)w->width / ((double)w->hi[0] - (double)w->lo[0]);
  double sy = (double)w->height / ((double)w->hi[1] - (double)w->lo[1]);
  double x = (q[0] - (double)w->lo[0]) * sx;
  double y = (q[1] - (double)w->lo[1]) * sy;
  *fx = x;
  *fy = y;
  if (!(x >= 0.0 && x < (double)w->width)) return 0;
  if (!(y >= 0.0 && y < (double)w->height)) return 0;
  *ix = (int)floor(x);
  *iy = (int)floor(y);
  return 1;
}

static int check_common(const orc_system *s, const orc_run *r, const orc_window *w,
                        uint64_t *thresh) {
  if (!s || !r || !w) return ORC_EINVAL;
  if (s->dim < 2 || s->dim > 3) return ORC_EINVAL;
  if (s->n_maps < 1 || s->n_maps > ORC_MAX_MAPS) return ORC_EINVAL;
  if (s->kind)
    for (int i = 0; i < s->n_maps; ++i) {
      if (s->kind[i] != ORC_MAP_AFFINE && s->kind[i] != ORC_MAP_CIRCLE) return ORC_EINVAL;
      if (s->kind[i] == ORC_MAP_CIRCLE && s->dim != 2) return ORC_EINVAL;
    }
  if (w->width < 1 || w->height < 1 || w->channels < 1) return ORC_EINVAL;
  if (!(w->hi[0] > w->lo[0]) || !(w->hi[1] > w->lo[1])) return ORC_EINVAL;
  return orc_thresholds(s->prob, s->n_maps, thresh);
}

/* ------------------------------------------------------------------------ */
/* Plain chaos game with an integer count histogram.                        */
/* For every point: draw p0; for t = 1..T draw u_t, select k_t, apply f_kt; */
/* when t > B transform a copy and add 1 to its pixel.  With channels == 1  */
/* every splat goes to channel 0; otherwise the channel is k_t (colour by   */
/* the function that moved the point there).  The image ACCUMULATES.        */
/* Optional outputs: final positions [N][dim], last index [N],               */
/* index sequence [N][T], fractional pixel coordinates of every splat        */
/* [N][T-B][2] (NaN when dropped), dropped-splat counter.                    */
/* ------------------------------------------------------------------------ */
int orc_chaos_count(const orc_system *s, const orc_run *r, const orc_window *w,
                    uint32_t *img, double *final_p, uint8_t *last_k,
                    uint8_t *idx, double *splat_xy, uint64_t *dropped) {
  uint64_t thresh[ORC_MAX_MAPS];
  int rc = check_common(s, r, w, thresh);
  if (rc) return rc;
  if (w->channels != 1 && w->channels != s->n_maps) return ORC_EINVAL;
  if (s->final_kind == ORC_FINAL_TWIST_CAMERA) return ORC_EINVAL;
  if (s->compose != 0 && s->compose != 1) return ORC_EINVAL;
  if (s->compose && s->dim != 2) return ORC_EINVAL;
  if (r->iter_offset && !final_p) return ORC_EINVAL;
  const int d = s->dim;
  const uint32_t T = r->n_iters, B = call_burn_in(r), K = r->iter_offset;
  const size_t plane = (size_t)w->width * (size_t)w->height;
  uint64_t n_drop = 0;
  for (uint32_t n = 0; n < r->n_points; ++n) {
    uint32_t pid = r->point_offset + n;
    double p[3] = {0, 0, 0};
    if (K)
      for (int c = 0; c < d; ++c) p[c] = final_p[(size_t)n * d + c];
    else
      initial_point(r, pid, d, p);
    uint32_t words[4] = {0, 0, 0, 0};
    int k = 0;
    for (uint32_t t = 1; t <= T; ++t) {
      uint32_t u = step_draw(r, pid, K + t, t == 1, words);
      k = orc_select(u, thresh, s->n_maps);
      if (idx) idx[(size_t)n * T + (t - 1)] = (uint8_t)k;
      apply_map(s, k, p);
      if (s->compose) {
        /* reuse (fig. "circle" C): the transformed point is the new point */
        double q0[2], d0 = 0.0;
        final_transform(s, p, q0, &d0);
        p[0] = q0[0];
        p[1] = q0[1];
      }
      if (t > B) {
        double q[2], depth = 0.0, fx, fy;
        int ix, iy;
        if (s->compose) {
          q[0] = p[0];
          q[1] = p[1];
        } else {
          final_transform(s, p, q, &depth);
        }
        int hit = bin_point(w, q, &ix, &iy, &fx, &fy);
        if (splat_xy) {
          size_t o = ((size_t)n * (T - B) + (t - B - 1)) * 2;
          splat_xy[o] = fx;
          splat_xy[o + 1] = fy;
        }
        if (hit) {
          int ch = (w->channels == 1) ? 0 : k;
          img[(size_t)ch * plane + (size_t)iy * w->width + ix] += 1u;
        } else {
          n_drop++;
        }
      }
    }
    if (final_p)
      for (int c = 0; c < d; ++c) final_p[(size_t)n * d + c] = p[c];
    if (last_k) last_k[n] = (uint8_t)k;
  }
  if (dropped) *dropped += n_drop;
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Several objects from one primitive (Section 3, "multiple objects from a   */
/* single primitive", fig. "space"): after each step of the chaos game the   */
/* point is repositioned once per object -- a transform of its own, then a   */
/* placement -- and each object's copy is splatted, while the point itself   */
/* keeps iterating.  Duplication (the "stars" of that scene): an object with */
/* n_copies > 1 sends each splat to one copy, drawn from a random stream,    */
/* and places copy c with offsets and a scale that another random stream     */
/* derives from c alone, so every point agrees on where copy c is and no     */
/* copy table is stored.  Readings (the paper gives no formulas):            */
/*   object transform: one of the 2D final kinds, then q' = P q + t;         */
/*   copy draw of iteration t: word (t-1) mod 4 of the Philox block          */
/*     (pid, (t-1)/4, instance, 2); object o of the scene takes              */
/*     c = floor(((2o + 1) u mod 2^32) n_copies / 2^32) (an odd multiplier   */
/*     is a bijection of the words, so c is uniform for every object);       */
/*   copy placement: Philox block (c, o, instance, 3); words 0, 1 and 2 give */
/*     e_i = (w_i >> 8) 2^-24, offset = lo + span e_{0,1}, scale =           */
/*     s_lo + s_span e_2; the copy is q'' = scale q' + offset.              */
/* Every object splats into its own channel of a count image that           */
/* ACCUMULATES; splat_xy (nullable) gets [n][t - B - 1][o] positions.       */
/* ------------------------------------------------------------------------ */
#define ORC_MAX_OBJECTS 8

typedef struct {
  int32_t final_kind;          /* ORC_FINAL_IDENTITY, _SWIRL, _STRETCH or _RING */
  const float *final_params;   /* up to 24 values */
  float place[6];              /* P row-major (a00 a01 a10 a11), then t */
  int32_t channel;
  uint32_t n_copies;           /* 1 = no duplication */
  float copy_lo[2], copy_span[2];
  float scale_lo, scale_span;
} orc_object;

int orc_chaos_scene(const orc_system *s, const orc_object *obj, int n_obj,
                    const orc_run *r, const orc_window *w, uint32_t *img,
                    double *splat_xy, uint64_t *dropped) {
  uint64_t thresh[ORC_MAX_MAPS];
  int rc = check_common(s, r, w, thresh);
  if (rc) return rc;
  if (s->dim != 2 || s->final_kind != ORC_FINAL_IDENTITY || s->compose) return ORC_EINVAL;
  if (r->iter_offset || r->burn_in > r->n_iters) return ORC_EINVAL;
  if (n_obj < 1 || n_obj > ORC_MAX_OBJECTS) return ORC_EINVAL;
  int any_copies = 0;
  for (int o = 0; o < n_obj; ++o) {
    int fk = obj[o].final_kind;
    if (fk != ORC_FINAL_IDENTITY && fk != ORC_FINAL_SWIRL && fk != ORC_FINAL_STRETCH &&
        fk != ORC_FINAL_RING)
      return ORC_EINVAL;
    if (obj[o].channel < 0 || obj[o].channel >= w->channels) return ORC_EINVAL;
    if (obj[o].n_copies < 1) return ORC_EINVAL;
    if (obj[o].n_copies > 1) any_copies = 1;
  }
  const uint32_t T = r->n_iters, B = r->burn_in;
  const size_t plane = (size_t)w->width * (size_t)w->height;
  const uint32_t key[2] = {(uint32_t)r->seed, (uint32_t)(r->seed >> 32)};
  uint64_t n_drop = 0;
  for (uint32_t n = 0; n < r->n_points; ++n) {
    uint32_t pid = r->point_offset + n;
    double p[3] = {0, 0, 0};
    initial_point(r, pid, 2, p);
    uint32_t words[4] = {0, 0, 0, 0}, cwords[4] = {0, 0, 0, 0};
    for (uint32_t t = 1; t <= T; ++t) {
      if ((t - 1) % 4 == 0) {
        point_stream(r, pid, (t - 1) / 4, 0, words);
        if (any_copies) point_stream(r, pid, (t - 1) / 4, 2, cwords);
      }
      int k = orc_select(words[(t - 1) % 4], thresh, s->n_maps);
      apply_map(s, k, p);
      if (t <= B) continue;
      for (int o = 0; o < n_obj; ++o) {
        const orc_object *ob = &obj[o];
        orc_system so = *s;
        so.final_kind = ob->final_kind;
        so.final_params = ob->final_params;
        double g[2], depth = 0.0, q[2];
        final_transform(&so, p, g, &depth);
        q[0] = (double)ob->place[0] * g[0] + (double)ob->place[1] * g[1] + (double)ob->place[4];
        q[1] = (double)ob->place[2] * g[0] + (double)ob->place[3] * g[1] + (double)ob->place[5];
        if (ob->n_copies > 1) {
          uint32_t v = (uint32_t)((2u * (uint32_t)o + 1u) * cwords[(t - 1) % 4]);
          uint32_t c = (uint32_t)(((uint64_t)v * ob->n_copies) >> 32);
          uint32_t ctr[4] = {c, (uint32_t)o, r->instance, 3u}, cw[4];
          orc_philox4x32_10(ctr, key, cw);
          double e0 = ldexp((double)(cw[0] >> 8), -24);
          double e1 = ldexp((double)(cw[1] >> 8), -24);
          double e2 = ldexp((double)(cw[2] >> 8), -24);
          double sc = (double)ob->scale_lo + (double)ob->scale_span * e2;
          q[0] = sc * q[0] + ((double)ob->copy_lo[0] + (double)ob->copy_span[0] * e0);
          q[1] = sc * q[1] + ((double)ob->copy_lo[1] + (double)ob->copy_span[1] * e1);
        }
        double fx, fy;
        int ix, iy;
        int hit = bin_point(w, q, &ix, &iy, &fx, &fy);
        if (splat_xy) {
          size_t at = (((size_t)n * (T - B) + (t - B - 1)) * (size_t)n_obj + (size_t)o) * 2;
          splat_xy[at] = q[0];
          splat_xy[at + 1] = q[1];
        }
        if (hit)
          img[(size_t)ob->channel * plane + (size_t)iy * w->width + ix] += 1u;
        else
          n_drop++;
      }
    }
  }
  if (dropped) *dropped += n_drop;
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* 3D chaos game with a depth buffer.  Each splat keeps, per pixel, the      */
/* minimum of key = (FP32 bit pattern of the view depth) << 32 | k (nearest */
/* point wins, ties broken by function index), and counts every splat in a  */
/* density image.  Splats behind the near plane are dropped.                */
/* depth_buf and density ACCUMULATE (min and sum).                          */
/* ------------------------------------------------------------------------ */
int orc_chaos_depth(const orc_system *s, const orc_run *r, const orc_window *w,
                    float near_plane, uint64_t *depth_buf, uint32_t *density,
                    double *final_p, uint8_t *last_k, double *splat_xyz,
                    uint64_t *dropped) {
  uint64_t thresh[ORC_MAX_MAPS];
  int rc = check_common(s, r, w, thresh);
  if (rc) return rc;
  if (s->dim != 3 || s->final_kind != ORC_FINAL_TWIST_CAMERA || s->compose) return ORC_EINVAL;
  if (r->iter_offset && !final_p) return ORC_EINVAL;
  const uint32_t T = r->n_iters, B = call_burn_in(r), K = r->iter_offset;
  uint64_t n_drop = 0;
  for (uint32_t n = 0; n < r->n_points; ++n) {
    uint32_t pid = r->point_offset + n;
    double p[3];
    if (K)
      for (int c = 0; c < 3; ++c) p[c] = final_p[(size_t)n * 3 + c];
    else
      initial_point(r, pid, 3, p);
    uint32_t words[4] = {0, 0, 0, 0};
    int k = 0;
    for (uint32_t t = 1; t <= T; ++t) {
      k = orc_select(step_draw(r, pid, K + t, t == 1, words), thresh, s->n_maps);
      apply_map(s, k, p);
      if (t > B) {
        double q[2], z = 0.0, fx, fy;
        int ix, iy;
        final_transform(s, p, q, &z);
        int hit = (z > (double)near_plane) && bin_point(w, q, &ix, &iy, &fx, &fy);
        if (splat_xyz) {
          size_t o = ((size_t)n * (T - B) + (t - B - 1)) * 3;
          splat_xyz[o] = hit ? fx : NAN;
          splat_xyz[o + 1] = hit ? fy : NAN;
          splat_xyz[o + 2] = z;
        }
        if (hit) {
          float zf = (float)z;
          uint32_t zbits;
          memcpy(&zbits, &zf, sizeof zbits);
          uint64_t key = ((uint64_t)zbits << 32) | (uint64_t)k;
          size_t pix = (size_t)iy * w->width + ix;
          if (key < depth_buf[pix]) depth_buf[pix] = key;
          density[pix] += 1u;
        } else {
          n_drop++;
        }
      }
    }
    if (final_p)
      for (int c = 0; c < 3; ++c) final_p[(size_t)n * 3 + c] = p[c];
    if (last_k) last_k[n] = (uint8_t)k;
  }
  if (dropped) *dropped += n_drop;
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Gaussian soft splat (differentiable form).                              */
/* Reading: separable shifted-truncated Gaussian                            */
/*   g(d) = exp(-d^2 / (2 s^2)) - exp(-R^2 / (2 s^2))  for |d| < R = 3 s,   */
/*   g(d) = 0 otherwise,                                                    */
/* with d = (pixel centre) - (point), both in pixel units.  The weight of   */
/* pixel (i, j) is g(i + 0.5 - x) g(j + 0.5 - y); taps off the image are    */
/* skipped.  D = sum of weights / (N (T - B)).  g is continuous, so the     */
/* density is a continuous function of the map parameters.                  */
/* Identity final transform only (the configured differentiable system).    */
/* ------------------------------------------------------------------------ */
static double gauss_g(double dd, double sigma) {
  double R = 3.0 * sigma;
  if (!(fabs(dd) < R)) return 0.0;
  return exp(-dd * dd / (2.0 * sigma * sigma)) - exp(-R * R / (2.0 * sigma * sigma));
}

static double gauss_dg(double dd, double sigma) {
  double R = 3.0 * sigma;
  if (!(fabs(dd) < R)) return 0.0;
  return -dd / (sigma * sigma) * exp(-dd * dd / (2.0 * sigma * sigma));
}

/* Pixel-coordinate scale of the window. */
static void window_scale(const orc_window *w, double *sx, double *sy) {
  *sx = (double)w->width / ((double)w->hi[0] - (double)w->lo[0]);
  *sy = (double)w->height / ((double)w->hi[1] - (double)w->lo[1]);
}

static void gauss_splat_one(const orc_window *w, double sigma, double weight,
                            const double p[3], double *density) {
  double sx, sy;
  window_scale(w, &sx, &sy);
  double x = (p[0] - (double)w->lo[0]) * sx;
  double y = (p[1] - (double)w->lo[1]) * sy;
  if (!isfinite(x) || !isfinite(y)) return;
  double R = 3.0 * sigma;
  long i0 = (long)floor(x - R) - 1, i1 = (long)floor(x + R) + 1;
  long j0 = (long)floor(y - R) - 1, j1 = (long)floor(y + R) + 1;
  for (long j = j0; j <= j1; ++j) {
    if (j < 0 || j >= w->height) continue;
    double gy = gauss_g((double)j + 0.5 - y, sigma);
    if (gy == 0.0) continue;
    for (long i = i0; i <= i1; ++i) {
      if (i < 0 || i >= w->width) continue;
      double gx = gauss_g((double)i + 0.5 - x, sigma);
      if (gx == 0.0) continue;
      density[(size_t)j * w->width + i] += weight * gx * gy;
    }
  }
}

int orc_splat_gauss(const orc_system *s, const orc_run *r, const orc_window *w,
                    double sigma, double *density, double *final_p) {
  uint64_t thresh[ORC_MAX_MAPS];
  int rc = check_common(s, r, w, thresh);
  if (rc) return rc;
  if (s->dim != 2 || s->final_kind != ORC_FINAL_IDENTITY || !(sigma > 0.0) || s->kind)
    return ORC_EINVAL;
  if (r->iter_offset || r->burn_in > r->n_iters) return ORC_EINVAL;
  const uint32_t T = r->n_iters, B = r->burn_in;
  if (T == B || r->n_points == 0) return ORC_OK;
  const double weight = 1.0 / ((double)r->n_points * (double)(T - B));
  for (uint32_t n = 0; n < r->n_points; ++n) {
    uint32_t pid = r->point_offset + n;
    double p[3] = {0, 0, 0};
    initial_point(r, pid, 2, p);
    uint32_t words[4] = {0, 0, 0, 0};
    for (uint32_t t = 1; t <= T; ++t) {
      if ((t - 1) % 4 == 0) point_stream(r, pid, (t - 1) / 4, 0, words);
      int k = orc_select(words[(t - 1) % 4], thresh, s->n_maps);
      apply_map(s, k, p);
      if (t > B) gauss_splat_one(w, sigma, weight, p, density);
    }
    if (final_p) {
      final_p[2 * (size_t)n] = p[0];
      final_p[2 * (size_t)n + 1] = p[1];
    }
  }
  return ORC_OK;
}

/* Gradient of the splatted density through the trajectory (reverse mode).
 * Given G = dL/dD [H][W], returns grad [n_maps][dim*dim + dim] laid out as
 * (A row-major, then b) per map, OVERWRITTEN.
 * With p_t = A_{k_t} p_{t-1} + b_{k_t} and s_t = dL/dp_t through the splat of
 * step t (zero for t <= B), the adjoint is
 *   lam_T = s_T,  lam_t = s_t + A_{k_{t+1}}^T lam_{t+1},
 * and each step contributes dL/dA_{k_t} += lam_t p_{t-1}^T, dL/db_{k_t} += lam_t.
 * Each point's trajectory is stored whole here (plain; the GPU recomputes
 * it from checkpoints). */
int orc_splat_gauss_backward(const orc_system *s, const orc_run *r,
                             const orc_window *w, double sigma,
                             const double *dLdD, double *grad) {
  uint64_t thresh[ORC_MAX_MAPS];
  int rc = check_common(s, r, w, thresh);
  if (rc) return rc;
  if (s->dim != 2 || s->final_kind != ORC_FINAL_IDENTITY || !(sigma > 0.0) || s->kind)
    return ORC_EINVAL;
  if (r->iter_offset || r->burn_in > r->n_iters) return ORC_EINVAL;
  const int n_par = 6;
  for (int i = 0; i < s->n_maps * n_par; ++i) grad[i] = 0.0;
  const uint32_t T = r->n_iters, B = r->burn_in;
  if (T == B || r->n_points == 0) return ORC_OK;
  const double weight = 1.0 / ((double)r->n_points * (double)(T - B));
  double sx, sy;
  window_scale(w, &sx, &sy);
  const double R = 3.0 * sigma;
  double *traj = (double *)malloc(sizeof(double) * 2 * (T + 1));
  int *ks = (int *)malloc(sizeof(int) * (T + 1));
  if (!traj || !ks) {
    free(traj);
    free(ks);
    return ORC_EINVAL;
  }
  for (uint32_t n = 0; n < r->n_points; ++n) {
    uint32_t pid = r->point_offset + n;
    double p[3] = {0, 0, 0};
    initial_point(r, pid, 2, p);
    traj[0] = p[0];
    traj[1] = p[1];
    uint32_t words[4] = {0, 0, 0, 0};
    ks[0] = -1;
    for (uint32_t t = 1; t <= T; ++t) {
      if ((t - 1) % 4 == 0) point_stream(r, pid, (t - 1) / 4, 0, words);
      int k = orc_select(words[(t - 1) % 4], thresh, s->n_maps);
      apply_map(s, k, p);
      ks[t] = k;
      traj[2 * t] = p[0];
      traj[2 * t + 1] = p[1];
    }
    double lam[2] = {0.0, 0.0};
    for (uint32_t t = T; t >= 1; --t) {
      /* carry: A_{k_{t+1}}^T lam_{t+1} */
      double carry[2] = {0.0, 0.0};
      if (t < T) {
        const float *An = s->A + (size_t)ks[t + 1] * 4;
        carry[0] = (double)An[0] * lam[0] + (double)An[2] * lam[1];
        carry[1] = (double)An[1] * lam[0] + (double)An[3] * lam[1];
      }
      /* direct term s_t */
      double st[2] = {0.0, 0.0};
      if (t > B) {
        double x = (traj[2 * t] - (double)w->lo[0]) * sx;
        double y = (traj[2 * t + 1] - (double)w->lo[1]) * sy;
        if (isfinite(x) && isfinite(y)) {
          long i0 = (long)floor(x - R) - 1, i1 = (long)floor(x + R) + 1;
          long j0 = (long)floor(y - R) - 1, j1 = (long)floor(y + R) + 1;
          for (long j = j0; j <= j1; ++j) {
            if (j < 0 || j >= w->height) continue;
            double dy = (double)j + 0.5 - y;
            double gy = gauss_g(dy, sigma), dgy = gauss_dg(dy, sigma);
            for (long i = i0; i <= i1; ++i) {
              if (i < 0 || i >= w->width) continue;
              double dx = (double)i + 0.5 - x;
              double gx = gauss_g(dx, sigma), dgx = gauss_dg(dx, sigma);
              double G = dLdD[(size_t)j * w->width + i] * weight;
              /* d(dx)/dp_x = -sx, d(dy)/dp_y = -sy */
              st[0] += G * dgx * gy * (-sx);
              st[1] += G * gx * dgy * (-sy);
            }
          }
        }
      }
      lam[0] = st[0] + carry[0];
      lam[1] = st[1] + carry[1];
      int k = ks[t];
      double *g = grad + (size_t)k * n_par;
      double px = traj[2 * (t - 1)], py = traj[2 * (t - 1) + 1];
      g[0] += lam[0] * px;
      g[1] += lam[0] * py;
      g[2] += lam[1] * px;
      g[3] += lam[1] * py;
      g[4] += lam[0];
      g[5] += lam[1];
    }
  }
  free(traj);
  free(ks);
  return ORC_OK;
}

int orc_version(void) { return 1; }
