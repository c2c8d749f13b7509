/*
 * Seeded synthetic voxel scenes.
 *
 * This module only produces INPUTS: dense uint8 chunks (0 = empty, 1..255 =
 * material ID, x fastest, then y, then z) and camera poses.  It contains no
 * part of the SVDAG method (no downsampling, no octree, no traversal), so the
 * CPU oracle and the GPU library can both consume its output without sharing
 * any of the method's arithmetic.
 *
 * The paper evaluates on voxelised San Miguel / Sponza and a Minecraft city
 * (Section 4); those datasets are replaced by these procedural stand-ins:
 *
 *   kind 0  "noise64"     single 64^3 chunk, 3D value noise (4 octaves,
 *                         wavelength 16) above its 70th percentile (~30%
 *                         fill), material uniform in 1..15 per solid voxel.
 *   kind 1  "terrain1024" single 1024^3 chunk: heightfield from 2D fBm
 *                         (6 octaves, wavelength 512, amplitude 400, centre
 *                         512), caves carved by 3D fBm (2 octaves, wavelength
 *                         64) below h-4, 8 materials banded by height.
 *   kind 2  "map512"      16x16x1 chunks of 512^3: same terrain (centre 256)
 *                         plus seeded solid boxes ("buildings", 4..64 per
 *                         side, ~5% of the ground area), materials 9..15.
 *   kind 3  "map1024"     32x32x1 chunks of 1024^3, terrain as kind 1 plus
 *                         boxes as kind 2.
 *   kind 4  "custom"      like kind 2 with caller-chosen chunk size and grid
 *                         (small worlds for tests): terrain wavelength 64,
 *                         cave wavelength 16, box sides 2..12.
 *
 * Randomness: splitmix64 (Steele, Lea, Flood 2014) as published; lattice
 * values are splitmix64 chains over (seed, i, j, k) mapped to [0,1) with 53
 * bits.  Value noise interpolates lattice values trilinearly with the
 * smoothstep fade 3t^2 - 2t^3.  All noise arithmetic is double precision.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SG_EXPORT __attribute__((visibility("default")))

static inline uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

static inline double lattice(uint64_t seed, int64_t i, int64_t j, int64_t k) {
  uint64_t h = splitmix64(seed ^ (uint64_t)i);
  h = splitmix64(h ^ (uint64_t)j);
  h = splitmix64(h ^ (uint64_t)k);
  return (double)(h >> 11) * 0x1p-53;
}

static inline double fade(double t) { return t * t * (3.0 - 2.0 * t); }
static inline double lerp(double a, double b, double t) { return a + (b - a) * t; }

static inline int64_t floordiv(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) q--;
  return q;
}

/* 2D value noise at integer position (x, y) with integer wavelength lam. */
static double vnoise2(uint64_t seed, int64_t x, int64_t y, int64_t lam) {
  int64_t i = floordiv(x, lam), j = floordiv(y, lam);
  double fx = fade((double)(x - i * lam) / (double)lam);
  double fy = fade((double)(y - j * lam) / (double)lam);
  double a = lerp(lattice(seed, i, j, 0), lattice(seed, i + 1, j, 0), fx);
  double b = lerp(lattice(seed, i, j + 1, 0), lattice(seed, i + 1, j + 1, 0), fx);
  return lerp(a, b, fy);
}

/* Normalised fBm in [0,1): octave o has amplitude 2^-o and wavelength lam0/2^o. */
static double fbm2(uint64_t seed, int64_t x, int64_t y, int octaves, int64_t lam0) {
  double s = 0.0, w = 0.0, amp = 1.0;
  for (int o = 0; o < octaves; o++) {
    s += amp * vnoise2(seed + 0x1000ull * (uint64_t)o, x, y, lam0 >> o);
    w += amp;
    amp *= 0.5;
  }
  return s / w;
}

static inline int ilog2_i64(int64_t v) { int l = 0; while (((int64_t)1 << (l + 1)) <= v) l++; return l; }

/*
 * 3D fBm evaluated along one x-row [x0, x0+n) at fixed (y, z).  Wavelengths
 * are powers of two.  The y/z interpolation is done once per lattice x point,
 * then each voxel needs one x lerp per octave, with the fade weight taken
 * from a table over x mod wavelength.
 */
static void fbm3_row(uint64_t seed, int64_t x0, int64_t n, int64_t y, int64_t z,
                     int octaves, int64_t lam0, double* out, double* scratch) {
  double w = 0.0, amp = 1.0;
  double fx_tab[1024];
  for (int64_t t = 0; t < n; t++) out[t] = 0.0;
  for (int o = 0; o < octaves; o++) {
    const uint64_t so = seed + 0x1000ull * (uint64_t)o;
    const int64_t lam = lam0 >> o;
    const int sh = ilog2_i64(lam);
    const int64_t j = y >> sh, k = z >> sh;
    const double fy = fade((double)(y - (j << sh)) / (double)lam);
    const double fz = fade((double)(z - (k << sh)) / (double)lam);
    const int64_t i0 = x0 >> sh, i1 = ((x0 + n - 1) >> sh) + 1;
    for (int64_t i = i0; i <= i1; i++) {
      double a = lerp(lattice(so, i, j, k), lattice(so, i, j + 1, k), fy);
      double b = lerp(lattice(so, i, j, k + 1), lattice(so, i, j + 1, k + 1), fy);
      scratch[i - i0] = lerp(a, b, fz);
    }
    for (int64_t r = 0; r < lam; r++) fx_tab[r] = fade((double)r / (double)lam);
    for (int64_t t = 0; t < n; t++) {
      const int64_t x = x0 + t;
      const int64_t i = (x >> sh) - i0;
      out[t] += amp * lerp(scratch[i], scratch[i + 1], fx_tab[x & (lam - 1)]);
    }
    w += amp;
    amp *= 0.5;
  }
  for (int64_t t = 0; t < n; t++) out[t] /= w;
}

/*
 * Lattice values of a 3D fBm over one chunk, precomputed per octave, so that
 * rows of the chunk interpolate without rehashing.  Same values and the same
 * interpolation order as fbm3_row, hence identical results.
 */
typedef struct {
  int octaves;
  int64_t lam0;
  uint64_t seed;
  int64_t i0[8], j0[8], k0[8], n[8];
  double* v[8];
} sg_lattice;

static void lattice_init(sg_lattice* L, uint64_t seed, int octaves, int64_t lam0, int64_t X0, int64_t Y0,
                         int64_t Z0, int64_t S) {
  L->octaves = octaves;
  L->lam0 = lam0;
  L->seed = seed;
  for (int o = 0; o < octaves; o++) {
    const uint64_t so = seed + 0x1000ull * (uint64_t)o;
    const int sh = ilog2_i64(lam0 >> o);
    const int64_t n = ((S - 1) >> sh) + 3;
    L->i0[o] = X0 >> sh; L->j0[o] = Y0 >> sh; L->k0[o] = Z0 >> sh; L->n[o] = n;
    L->v[o] = (double*)malloc((size_t)(n * n * n) * sizeof(double));
    for (int64_t c = 0; c < n; c++)
      for (int64_t b = 0; b < n; b++)
        for (int64_t a = 0; a < n; a++)
          L->v[o][a + n * (b + n * c)] = lattice(so, L->i0[o] + a, L->j0[o] + b, L->k0[o] + c);
  }
}

static void lattice_free(sg_lattice* L) {
  for (int o = 0; o < L->octaves; o++) free(L->v[o]);
}

static void fbm3_row_tab(const sg_lattice* L, int64_t x0, int64_t nx, int64_t y, int64_t z, double* out,
                         double* scratch) {
  double w = 0.0, amp = 1.0;
  double fx_tab[1024];
  for (int64_t t = 0; t < nx; t++) out[t] = 0.0;
  for (int o = 0; o < L->octaves; o++) {
    const int64_t lam = L->lam0 >> o;
    const int sh = ilog2_i64(lam);
    const int64_t j = y >> sh, k = z >> sh, n = L->n[o];
    const double fy = fade((double)(y - (j << sh)) / (double)lam);
    const double fz = fade((double)(z - (k << sh)) / (double)lam);
    const int64_t i0 = x0 >> sh, i1 = ((x0 + nx - 1) >> sh) + 1;
    const double* V = L->v[o];
    const int64_t jb = j - L->j0[o], kb = k - L->k0[o];
    for (int64_t i = i0; i <= i1; i++) {
      const int64_t ia = i - L->i0[o];
      double a = lerp(V[ia + n * (jb + n * kb)], V[ia + n * (jb + 1 + n * kb)], fy);
      double b = lerp(V[ia + n * (jb + n * (kb + 1))], V[ia + n * (jb + 1 + n * (kb + 1))], fy);
      scratch[i - i0] = lerp(a, b, fz);
    }
    for (int64_t r = 0; r < lam; r++) fx_tab[r] = fade((double)r / (double)lam);
    for (int64_t t = 0; t < nx; t++) {
      const int64_t x = x0 + t;
      const int64_t i = (x >> sh) - i0;
      out[t] += amp * lerp(scratch[i], scratch[i + 1], fx_tab[x & (lam - 1)]);
    }
    w += amp;
    amp *= 0.5;
  }
  for (int64_t t = 0; t < nx; t++) out[t] /= w;
}

/* ------------------------------------------------------------------------ */

typedef struct {
  int32_t x0, y0, z0, x1, y1, z1; /* inclusive-exclusive box in voxels */
  uint8_t mat;
} sg_box;
_Static_assert(sizeof(sg_box) == 28, "sg_world_params documents a 28-byte box record");

typedef struct {
  int kind;
  uint64_t seed;
  uint32_t chunk_log2;
  uint32_t grid[3];
  int terrain;        /* 0 = value-noise blob, 1 = terrain */
  int64_t centre;     /* terrain centre height */
  double amp;         /* terrain amplitude */
  int64_t zmax;       /* world height in voxels */
  double cave_tau;    /* cave threshold on 3D fBm */
  int64_t terrain_lam; /* wavelength of the first terrain octave */
  int64_t cave_lam;    /* wavelength of the first cave octave */
  int box_lo, box_hi;  /* box side range, voxels */
  int nbox;
  sg_box* boxes;
} sg_world;

/* Cave threshold: the 90th percentile of the 2-octave, wavelength-64 3D fBm
 * (measured once over 2^22 seeded samples; about 10% of the underground is
 * carved). */
#define SG_CAVE_TAU 0.6803

static int64_t terrain_h(const sg_world* w, int64_t x, int64_t y) {
  double f = fbm2(w->seed ^ 0x7E44A1Cull, x, y, 6, w->terrain_lam);
  int64_t h = (int64_t)floor((double)w->centre + w->amp * (f - 0.5));
  if (h > w->zmax - 1) h = w->zmax - 1;
  if (h < 0) h = 0;
  return h;
}

static void make_boxes(sg_world* w) {
  const int64_t X = (int64_t)w->grid[0] << w->chunk_log2;
  const int64_t Y = (int64_t)w->grid[1] << w->chunk_log2;
  /* boxes cover ~5% of the ground: mean side of the uniform range squared */
  const int span = w->box_hi - w->box_lo + 1;
  const double mean = 0.5 * (double)(w->box_lo + w->box_hi);
  int n = (int)((double)X * (double)Y * 0.05 / (mean * mean));
  w->nbox = n;
  w->boxes = (sg_box*)calloc((size_t)(n > 0 ? n : 1), sizeof(sg_box));
  uint64_t s = splitmix64(w->seed ^ 0xB0C5B0C5ull);
  for (int b = 0; b < n; b++) {
    uint64_t r0 = splitmix64(s + 4ull * (uint64_t)b + 0);
    uint64_t r1 = splitmix64(s + 4ull * (uint64_t)b + 1);
    uint64_t r2 = splitmix64(s + 4ull * (uint64_t)b + 2);
    uint64_t r3 = splitmix64(s + 4ull * (uint64_t)b + 3);
    int32_t sx = w->box_lo + (int32_t)(r0 % (uint64_t)span);
    int32_t sy = w->box_lo + (int32_t)((r0 >> 20) % (uint64_t)span);
    int32_t sz = w->box_lo + (int32_t)((r0 >> 40) % (uint64_t)span);
    int32_t x0 = (int32_t)(r1 % (uint64_t)(X - sx + 1));
    int32_t y0 = (int32_t)(r2 % (uint64_t)(Y - sy + 1));
    int64_t base = w->zmax;
    for (int32_t y = y0; y < y0 + sy; y++)
      for (int32_t x = x0; x < x0 + sx; x++) {
        int64_t h = terrain_h(w, x, y);
        if (h < base) base = h;
      }
    sg_box* bx = &w->boxes[b];
    bx->x0 = x0; bx->x1 = x0 + sx;
    bx->y0 = y0; bx->y1 = y0 + sy;
    bx->z0 = (int32_t)base;
    bx->z1 = (int32_t)((base + sz) < w->zmax ? (base + sz) : w->zmax);
    bx->mat = (uint8_t)(9 + (r3 % 7));
  }
}

SG_EXPORT sg_world* sg_world_new(int kind, uint64_t seed, uint32_t chunk_log2,
                                 uint32_t gx, uint32_t gy, uint32_t gz) {
  sg_world* w = (sg_world*)calloc(1, sizeof(sg_world));
  if (!w) return NULL;
  w->kind = kind;
  w->seed = seed;
  w->cave_tau = SG_CAVE_TAU;
  w->terrain_lam = 512; w->cave_lam = 64; w->box_lo = 4; w->box_hi = 64;
  switch (kind) {
    case 0: w->chunk_log2 = 6; w->grid[0] = w->grid[1] = w->grid[2] = 1; w->terrain = 0; break;
    case 1: w->chunk_log2 = 10; w->grid[0] = w->grid[1] = w->grid[2] = 1; w->terrain = 1;
            w->centre = 512; w->amp = 400.0; break;
    case 2: w->chunk_log2 = 9; w->grid[0] = w->grid[1] = 16; w->grid[2] = 1; w->terrain = 1;
            w->centre = 256; w->amp = 400.0; break;
    case 3: w->chunk_log2 = 10; w->grid[0] = w->grid[1] = 32; w->grid[2] = 1; w->terrain = 1;
            w->centre = 512; w->amp = 400.0; break;
    case 4: w->chunk_log2 = chunk_log2; w->grid[0] = gx; w->grid[1] = gy; w->grid[2] = gz;
            w->terrain = 1;
            w->centre = (int64_t)((gz << chunk_log2) / 2);
            w->amp = 0.78 * (double)(gz << chunk_log2);
            w->terrain_lam = 64; w->cave_lam = 16; w->box_lo = 2; w->box_hi = 12; break;
    default: free(w); return NULL;
  }
  w->zmax = (int64_t)w->grid[2] << w->chunk_log2;
  if (kind >= 2) make_boxes(w); else { w->nbox = 0; w->boxes = NULL; }
  return w;
}

SG_EXPORT void sg_world_free(sg_world* w) {
  if (!w) return;
  free(w->boxes);
  free(w);
}

SG_EXPORT void sg_world_info(const sg_world* w, uint32_t* chunk_log2, uint32_t grid[3], int* nbox) {
  *chunk_log2 = w->chunk_log2;
  grid[0] = w->grid[0]; grid[1] = w->grid[1]; grid[2] = w->grid[2];
  *nbox = w->nbox;
}

/* The parameters a second implementation of the terrain generator needs:
 * ip = {terrain, centre, zmax, terrain_lam, cave_lam, nbox}, dp = {amp,
 * cave_tau}; *boxes points at the world's nbox boxes in paint order (later
 * boxes overwrite earlier ones), each 6 int32 bounds then the material byte,
 * padded to 28 bytes.  The pointer stays valid while the world lives. */
SG_EXPORT void sg_world_params(const sg_world* w, int64_t ip[6], double dp[2], const void** boxes) {
  ip[0] = w->terrain; ip[1] = w->centre; ip[2] = w->zmax;
  ip[3] = w->terrain_lam; ip[4] = w->cave_lam; ip[5] = w->nbox;
  dp[0] = w->amp; dp[1] = w->cave_tau;
  *boxes = w->boxes;
}

SG_EXPORT int64_t sg_height(const sg_world* w, int64_t x, int64_t y) {
  if (!w->terrain) return -1;
  return terrain_h(w, x, y);
}

static int cmp_double(const void* a, const void* b) {
  double x = *(const double*)a, y = *(const double*)b;
  return (x > y) - (x < y);
}

/* Noise blob chunk: 3D value noise, 4 octaves, wavelength 16, solid above the
 * 70th percentile, material 1 + (hash mod 15). */
static void gen_noise(const sg_world* w, uint8_t* out) {
  const int64_t S = (int64_t)1 << w->chunk_log2;
  const size_t n = (size_t)(S * S * S);
  double* v = (double*)malloc(n * sizeof(double));
  double* tmp = (double*)malloc(n * sizeof(double));
  double* scr = (double*)malloc((size_t)(S + 8) * sizeof(double));
  for (int64_t z = 0; z < S; z++)
    for (int64_t y = 0; y < S; y++)
      fbm3_row(w->seed, 0, S, y, z, 4, 16, v + (size_t)((z * S + y) * S), scr);
  memcpy(tmp, v, n * sizeof(double));
  /* 70th percentile: value of rank floor(0.7 n) in ascending order */
  qsort(tmp, n, sizeof(double), cmp_double);
  size_t kth = (size_t)(0.7 * (double)n);
  const double thr = tmp[kth];
  for (size_t idx = 0; idx < n; idx++) {
    if (v[idx] > thr) {
      uint64_t h = splitmix64(w->seed ^ 0x3A7E41A1ull ^ splitmix64((uint64_t)idx));
      out[idx] = (uint8_t)(1 + h % 15);
    } else {
      out[idx] = 0;
    }
  }
  free(v); free(tmp); free(scr);
}

/* Terrain (+ caves + boxes) chunk at chunk coordinates (cx, cy, cz),
 * z-slab [za, zb) of it. */
typedef struct {
  const sg_world* w;
  uint32_t cx, cy, cz;
  int64_t za, zb;
  const int64_t* hh;
  const sg_lattice* cave;
  uint8_t* out;
} sg_job;

static void* gen_terrain_slab(void* arg) {
  const sg_job* J = (const sg_job*)arg;
  const sg_world* w = J->w;
  const int64_t S = (int64_t)1 << w->chunk_log2;
  const int64_t X0 = (int64_t)J->cx * S, Y0 = (int64_t)J->cy * S, Z0 = (int64_t)J->cz * S;
  double* row = (double*)malloc((size_t)S * sizeof(double));
  double* scr = (double*)malloc((size_t)(S + 8) * sizeof(double));
  for (int64_t z = J->za; z < J->zb; z++) {
    const int64_t Z = Z0 + z;
    const uint8_t band = (uint8_t)(1 + (8 * Z) / w->zmax);
    for (int64_t y = 0; y < S; y++) {
      uint8_t* o = J->out + (size_t)((z * S + y) * S);
      const int64_t* hr = J->hh + y * S;
      int need_cave = 0, any = 0;
      for (int64_t x = 0; x < S; x++) {
        any |= (Z <= hr[x]);
        need_cave |= (Z < hr[x] - 4);
      }
      if (!any) { memset(o, 0, (size_t)S); continue; }
      if (need_cave) fbm3_row_tab(J->cave, X0, S, Y0 + y, Z, row, scr);
      for (int64_t x = 0; x < S; x++) {
        uint8_t m = 0;
        if (Z <= hr[x]) {
          m = band;
          if (Z < hr[x] - 4 && row[x] > w->cave_tau) m = 0;
        }
        o[x] = m;
      }
    }
  }
  free(row); free(scr);
  return NULL;
}

static void gen_terrain(const sg_world* w, uint32_t cx, uint32_t cy, uint32_t cz, uint8_t* out,
                        int nthreads) {
  const int64_t S = (int64_t)1 << w->chunk_log2;
  const int64_t X0 = (int64_t)cx * S, Y0 = (int64_t)cy * S, Z0 = (int64_t)cz * S;
  int64_t* hh = (int64_t*)malloc((size_t)(S * S) * sizeof(int64_t));
  for (int64_t y = 0; y < S; y++)
    for (int64_t x = 0; x < S; x++) hh[y * S + x] = terrain_h(w, X0 + x, Y0 + y);
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 64) nthreads = 64;
  if (nthreads > S) nthreads = (int)S;
  sg_lattice cave;
  lattice_init(&cave, w->seed ^ 0xCA7ECA7Eull, 2, w->cave_lam, X0, Y0, Z0, S);
  sg_job jobs[64];
  pthread_t th[64];
  for (int t = 0; t < nthreads; t++) {
    jobs[t].w = w; jobs[t].cx = cx; jobs[t].cy = cy; jobs[t].cz = cz;
    jobs[t].za = S * t / nthreads; jobs[t].zb = S * (t + 1) / nthreads;
    jobs[t].hh = hh; jobs[t].cave = &cave; jobs[t].out = out;
  }
  for (int t = 1; t < nthreads; t++) pthread_create(&th[t], NULL, gen_terrain_slab, &jobs[t]);
  gen_terrain_slab(&jobs[0]);
  for (int t = 1; t < nthreads; t++) pthread_join(th[t], NULL);
  lattice_free(&cave);
  /* boxes overwrite terrain; later boxes overwrite earlier ones */
  for (int b = 0; b < w->nbox; b++) {
    const sg_box* bx = &w->boxes[b];
    int64_t xa = bx->x0 > X0 ? bx->x0 : X0, xb = bx->x1 < X0 + S ? bx->x1 : X0 + S;
    int64_t ya = bx->y0 > Y0 ? bx->y0 : Y0, yb = bx->y1 < Y0 + S ? bx->y1 : Y0 + S;
    int64_t za = bx->z0 > Z0 ? bx->z0 : Z0, zb = bx->z1 < Z0 + S ? bx->z1 : Z0 + S;
    if (xa >= xb || ya >= yb || za >= zb) continue;
    for (int64_t z = za; z < zb; z++)
      for (int64_t y = ya; y < yb; y++)
        memset(out + (size_t)(((z - Z0) * S + (y - Y0)) * S + (xa - X0)), bx->mat, (size_t)(xb - xa));
  }
  free(hh);
}

/* Fill `out` (S^3 bytes) with chunk (cx, cy, cz), using up to `nthreads`
 * threads.  The output does not depend on the thread count.  Returns 0 on
 * success. */
SG_EXPORT int sg_gen_chunk(const sg_world* w, uint32_t cx, uint32_t cy, uint32_t cz, uint8_t* out,
                           int nthreads) {
  if (!w || !out) return -1;
  if (cx >= w->grid[0] || cy >= w->grid[1] || cz >= w->grid[2]) return -1;
  if (!w->terrain) gen_noise(w, out);
  else gen_terrain(w, cx, cy, cz, out, nthreads);
  return 0;
}

/* Seeded samples of the cave fBm, used once to fix SG_CAVE_TAU. */
SG_EXPORT void sg_cave_samples(uint64_t seed, int64_t n, double* out) {
  double scr[64];  /* one-voxel rows need at most 3 lattice points */
  for (int64_t s = 0; s < n; s++) {
    uint64_t r = splitmix64(seed + (uint64_t)s);
    int64_t x = (int64_t)(r & 0xFFFF), y = (int64_t)((r >> 16) & 0xFFFF), z = (int64_t)((r >> 32) & 0x3FF);
    fbm3_row(seed ^ 0xCA7ECA7Eull, x, 1, y, z, 2, 64, out + s, scr);
  }
}

SG_EXPORT uint64_t sg_splitmix64(uint64_t x) { return splitmix64(x); }
