/*
 * graphgen.c -- seeded synthetic graph generators (raw edge pairs).
 *
 * This module holds no triangle / support / truss arithmetic.  It only draws
 * edge lists, so both the GPU library and the CPU oracle can be fed the same
 * input.  Every random number comes from a counter-based stream: the value
 * used for (sample i, level l) depends only on (seed, i, l), so output is
 * identical for any thread count.
 *
 * Generators
 *   - Kronecker / R-MAT (the Graph500-style power-law family the paper names
 *     among its synthetic data sets, Sec. II), with an optional seeded
 *     bijective relabelling of vertex ids.
 *   - Erdos-Renyi G(n, M): M independent uniform pairs.
 *   - Random geometric graph on the unit torus.
 *
 * Output pairs are raw: duplicates, both directions and self-loops may appear;
 * normalisation is the consumer's job.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014). */
static inline uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* Stream bases: one per purpose so streams never overlap. */
static inline uint64_t stream_base(uint64_t seed, uint64_t tag) {
  return mix64(mix64(seed) ^ (tag * 0xD1B54A32D192ED03ULL));
}

uint64_t gg_mix64(uint64_t z) { return mix64(z); }

/* Bijection on [0, 2^scale): rounds of odd-multiply-add and xorshift, all
 * modulo 2^scale, each invertible. */
static inline uint32_t perm_apply(uint32_t x, int scale, const uint64_t *k1,
                                  const uint64_t *k2) {
  if (scale == 0) return 0;
  uint64_t mask = (scale >= 64) ? ~0ULL : ((1ULL << scale) - 1ULL);
  uint64_t y = x;
  int sh = (scale + 1) / 2;
  for (int r = 0; r < 4; ++r) {
    y = (y * k1[r] + k2[r]) & mask;
    y ^= y >> sh;
  }
  return (uint32_t)y;
}

static void perm_keys(uint64_t seed, int scale, uint64_t *k1, uint64_t *k2) {
  uint64_t base = stream_base(seed, 2);
  uint64_t mask = (1ULL << scale) - 1ULL;
  for (int r = 0; r < 4; ++r) {
    k1[r] = (mix64(base ^ (uint64_t)(2 * r)) | 1ULL) & mask;
    if (k1[r] == 0) k1[r] = 1; /* scale 0 guard (mask 0) */
    k2[r] = mix64(base ^ (uint64_t)(2 * r + 1)) & mask;
  }
}

uint32_t gg_permute_vertex(uint64_t seed, int scale, uint32_t x) {
  uint64_t k1[4], k2[4];
  perm_keys(seed, scale, k1, k2);
  return perm_apply(x, scale, k1, k2);
}

/*
 * R-MAT: samples = edge_factor * 2^scale pairs.  Each pair descends `scale`
 * levels; at level l the quadrant is chosen by one 32-bit draw r compared with
 * the integer thresholds floor(a*2^32), floor((a+b)*2^32), floor((a+b+c)*2^32):
 * a -> (0,0), b -> (0,1), c -> (1,0), d -> (1,1).  Level 0 decides the most
 * significant bit.  If permute != 0, both endpoints are relabelled by the
 * seeded bijection above.
 * Returns 0, or -1 on bad arguments.
 */
int gg_rmat(int scale, int64_t n_samples, double a, double b, double c,
            uint64_t seed, int permute, int32_t *src, int32_t *dst) {
  if (scale < 0 || scale > 30 || n_samples < 0) return -1;
  if (a < 0 || b < 0 || c < 0 || a + b + c > 1.0) return -1;
  const double two32 = 4294967296.0;
  const uint64_t ta = (uint64_t)floor(a * two32);
  const uint64_t tab = (uint64_t)floor((a + b) * two32);
  const uint64_t tabc = (uint64_t)floor((a + b + c) * two32);
  const uint64_t base = stream_base(seed, 1);
  uint64_t k1[4], k2[4];
  perm_keys(seed, scale, k1, k2);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n_samples; ++i) {
    uint32_t u = 0, v = 0;
    for (int l = 0; l < scale; ++l) {
      uint64_t r = mix64(base ^ (((uint64_t)i << 6) | (uint64_t)l)) >> 32;
      uint32_t bu, bv;
      if (r < ta) { bu = 0; bv = 0; }
      else if (r < tab) { bu = 0; bv = 1; }
      else if (r < tabc) { bu = 1; bv = 0; }
      else { bu = 1; bv = 1; }
      u = (u << 1) | bu;
      v = (v << 1) | bv;
    }
    if (permute) {
      u = perm_apply(u, scale, k1, k2);
      v = perm_apply(v, scale, k1, k2);
    }
    src[i] = (int32_t)u;
    dst[i] = (int32_t)v;
  }
  return 0;
}

/* Uniform draw in [0, n) by multiply-shift of the high 32 bits. */
static inline uint32_t bounded(uint64_t x, uint32_t n) {
  return (uint32_t)(((x >> 32) * (uint64_t)n) >> 32);
}

/* Erdos-Renyi G(n, M): M independent uniform ordered pairs. */
int gg_er(int32_t n, int64_t n_samples, uint64_t seed, int32_t *src,
          int32_t *dst) {
  if (n <= 0 || n_samples < 0) return -1;
  const uint64_t base = stream_base(seed, 3);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n_samples; ++i) {
    src[i] = (int32_t)bounded(mix64(base ^ (2 * (uint64_t)i)), (uint32_t)n);
    dst[i] = (int32_t)bounded(mix64(base ^ (2 * (uint64_t)i + 1)), (uint32_t)n);
  }
  return 0;
}

/* Coordinates of the RGG points: 53-bit uniforms in [0,1). */
void gg_rgg_points(int32_t n, uint64_t seed, double *x, double *y) {
  const uint64_t base = stream_base(seed, 4);
  for (int64_t i = 0; i < n; ++i) {
    x[i] = (double)(mix64(base ^ (2 * (uint64_t)i)) >> 11) * 0x1.0p-53;
    y[i] = (double)(mix64(base ^ (2 * (uint64_t)i + 1)) >> 11) * 0x1.0p-53;
  }
}

static inline double torus_d2(double x0, double y0, double x1, double y1) {
  double dx = fabs(x0 - x1), dy = fabs(y0 - y1);
  if (dx > 0.5) dx = 1.0 - dx;
  if (dy > 0.5) dy = 1.0 - dy;
  return dx * dx + dy * dy;
}

/*
 * Random geometric graph on the unit torus: pairs i < j with torus distance
 * squared < r2.  Writes at most cap pairs; returns the number of pairs found
 * (may exceed cap: call again with a larger buffer), or -1 on bad arguments.
 */
int64_t gg_rgg(int32_t n, double r2, uint64_t seed, int32_t *src, int32_t *dst,
               int64_t cap) {
  if (n <= 0 || r2 <= 0) return -1;
  double *x = (double *)malloc(sizeof(double) * (size_t)n);
  double *y = (double *)malloc(sizeof(double) * (size_t)n);
  if (!x || !y) { free(x); free(y); return -1; }
  gg_rgg_points(n, seed, x, y);
  double r = sqrt(r2);
  int g = (int)floor(1.0 / r);
  int64_t cnt = 0;
  if (g < 3) {
    for (int32_t i = 0; i < n; ++i)
      for (int32_t j = i + 1; j < n; ++j)
        if (torus_d2(x[i], y[i], x[j], y[j]) < r2) {
          if (cnt < cap) { src[cnt] = i; dst[cnt] = j; }
          ++cnt;
        }
    free(x); free(y);
    return cnt;
  }
  /* Bucket points into a g x g grid (cell side 1/g >= r). */
  int64_t ncell = (int64_t)g * g;
  int32_t *head = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ncell + 1));
  int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *cell = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!head || !order || !cell) {
    free(x); free(y); free(head); free(order); free(cell);
    return -1;
  }
  memset(head, 0, sizeof(int32_t) * (size_t)(ncell + 1));
  for (int32_t i = 0; i < n; ++i) {
    int cx = (int)(x[i] * g), cy = (int)(y[i] * g);
    if (cx >= g) cx = g - 1;
    if (cy >= g) cy = g - 1;
    cell[i] = cx * g + cy;
    head[cell[i] + 1]++;
  }
  for (int64_t c = 0; c < ncell; ++c) head[c + 1] += head[c];
  {
    int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)ncell);
    memcpy(fill, head, sizeof(int32_t) * (size_t)ncell);
    for (int32_t i = 0; i < n; ++i) order[fill[cell[i]]++] = i;
    free(fill);
  }
  for (int32_t i = 0; i < n; ++i) {
    int cx = cell[i] / g, cy = cell[i] % g;
    for (int ddx = -1; ddx <= 1; ++ddx)
      for (int ddy = -1; ddy <= 1; ++ddy) {
        int nx = (cx + ddx + g) % g, ny = (cy + ddy + g) % g;
        int64_t c = (int64_t)nx * g + ny;
        for (int32_t t = head[c]; t < head[c + 1]; ++t) {
          int32_t j = order[t];
          if (j <= i) continue;
          if (torus_d2(x[i], y[i], x[j], y[j]) < r2) {
            if (cnt < cap) { src[cnt] = i; dst[cnt] = j; }
            ++cnt;
          }
        }
      }
  }
  free(x); free(y); free(head); free(order); free(cell);
  return cnt;
}
