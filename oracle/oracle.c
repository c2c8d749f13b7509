/*
 * CPU oracle for chunked-SVDAG primary-ray traversal.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the library.  Shares no code with
 * the GPU library.  Plain and slow on purpose; 128-bit integers everywhere a
 * product could overflow.  Build with -ffp-contract=off (camera frame).
 *
 * Paper references are to Fang, Wang, Wang, "Aokana: A GPU-Driven Voxel
 * Rendering Framework for Open World Games" (PACMCGIT 2025).
 */
#include "oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

typedef __int128 i128;

/* ========================================================================
 * Camera -> integer ray frame.
 *
 * The paper gives no camera equations.  Reading used here: pinhole camera,
 * vertical FOV, +z up, pixel centres at +0.5, row 0 at the top.  The
 * unnormalised direction of pixel (px, py) is affine in the pixel index,
 *     d = fwd + ((2(px+0.5)/W - 1) tau a) right + ((1 - 2(py+0.5)/H) tau) up'
 *       = A + px BX + py BY,
 * tau = tan(vfov/2), a = W/H.  A, BX, BY are rounded to integers at scale
 * 2^G, G the largest exponent for which all four corner directions have
 * every component below 2^31 in magnitude; the origin is rounded at 2^16.
 * ======================================================================== */
static void cross3(const double a[3], const double b[3], double r[3]) {
  r[0] = a[1] * b[2] - a[2] * b[1];
  r[1] = a[2] * b[0] - a[0] * b[2];
  r[2] = a[0] * b[1] - a[1] * b[0];
}

int or_camera_frame(const float pos[3], const float target[3], const float up[3],
                    float vfov_deg, uint32_t W, uint32_t H, or_frame* out) {
  double f[3], u0[3], fn[3], r[3], rn[3], u[3];
  if (W == 0 || H == 0) return -1;
  if (!(vfov_deg > 0.0f && vfov_deg < 180.0f)) return -1;
  for (int i = 0; i < 3; i++) {
    f[i] = (double)target[i] - (double)pos[i];
    u0[i] = (double)up[i];
  }
  double fl = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
  if (!(fl > 0.0)) return -1;
  for (int i = 0; i < 3; i++) fn[i] = f[i] / fl;
  cross3(fn, u0, r);
  double rl = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  if (!(rl > 0.0)) return -1;
  for (int i = 0; i < 3; i++) rn[i] = r[i] / rl;
  cross3(rn, fn, u);
  const double half = (double)vfov_deg * (M_PI / 360.0);
  const double tau = tan(half);
  const double a = (double)W / (double)H;
  const double sx0 = ((1.0 / (double)W - 1.0) * tau) * a;
  const double sy0 = (1.0 - 1.0 / (double)H) * tau;
  const double sbx = ((2.0 / (double)W) * tau) * a;
  const double sby = -((2.0 / (double)H) * tau);
  double A[3], BX[3], BY[3];
  for (int i = 0; i < 3; i++) {
    A[i] = (fn[i] + sx0 * rn[i]) + sy0 * u[i];
    BX[i] = sbx * rn[i];
    BY[i] = sby * u[i];
  }
  const int64_t LIM = (int64_t)1 << 31;
  int G;
  for (G = 40; G >= 0; G--) {
    int64_t qa[3], qx[3], qy[3];
    int ok = 1;
    for (int i = 0; i < 3; i++) {
      qa[i] = (int64_t)rint(ldexp(A[i], G));
      qx[i] = (int64_t)rint(ldexp(BX[i], G));
      qy[i] = (int64_t)rint(ldexp(BY[i], G));
    }
    for (int c = 0; c < 4 && ok; c++) {
      int64_t px = (c & 1) ? (int64_t)W - 1 : 0;
      int64_t py = (c & 2) ? (int64_t)H - 1 : 0;
      for (int i = 0; i < 3; i++) {
        int64_t d = qa[i] + px * qx[i] + py * qy[i];
        if (d >= LIM || d <= -LIM) ok = 0;
      }
    }
    if (ok) {
      for (int i = 0; i < 3; i++) {
        out->A[i] = qa[i];
        out->BX[i] = qx[i];
        out->BY[i] = qy[i];
      }
      break;
    }
  }
  if (G < 0) return -1;
  out->G = G;
  out->W = W;
  out->H = H;
  for (int i = 0; i < 3; i++) {
    int64_t o = (int64_t)rint(ldexp((double)pos[i], 16));
    /* guard band: |plane - O| < 2^32 for every plane of a world <= 2^15 */
    if (o <= -((int64_t)1 << 31) || o >= ((int64_t)1 << 32)) return -2;
    out->O[i] = o;
  }
  return 0;
}

/* ========================================================================
 * LOD pyramid (Section 3.4): a level-n voxel aggregates 8 level-(n-1)
 * voxels; it is solid iff at least density = 2 of them are non-empty.
 * Material: most frequent material of the solid children, ties to the
 * smallest ID.
 * ======================================================================== */
void or_downsample(const uint8_t* src, uint32_t R, uint8_t* dst) {
  const uint32_t h = R / 2;
  for (uint32_t z = 0; z < h; z++)
    for (uint32_t y = 0; y < h; y++)
      for (uint32_t x = 0; x < h; x++) {
        uint8_t m[8];
        int solid = 0;
        for (int i = 0; i < 8; i++) {
          uint32_t sx = 2 * x + (i & 1), sy = 2 * y + ((i >> 1) & 1), sz = 2 * z + ((i >> 2) & 1);
          m[i] = src[(size_t)sx + (size_t)R * ((size_t)sy + (size_t)R * sz)];
          solid += m[i] != 0;
        }
        /* mode of the solid children: count each value among the eight */
        uint8_t out = 0;
        if (solid >= 2) {
          int best = 0;
          for (int i = 0; i < 8; i++) {
            if (!m[i]) continue;
            int n = 0;
            for (int j = 0; j < 8; j++) n += m[j] == m[i];
            if (n > best || (n == best && m[i] < out)) { best = n; out = m[i]; }
          }
        }
        dst[(size_t)x + (size_t)h * ((size_t)y + (size_t)h * z)] = out;
      }
}

/* ========================================================================
 * SVO -> DAG (Sections 3.2, 2.2).
 *
 * Levels count cells: level 0 = one cell, level 2 = a 4x4x4 leaf cube stored
 * as a 64-bit bitmap, level log2(R) = the root.  Child octant of a child cube
 * at offset (dx,dy,dz) in {0,1}^3 is dx | dy<<1 | dz<<2.  Bit b of a leaf
 * bitmap is 8*octant(2x2x2 sub-block) + octant(cell in the sub-block), so
 * ascending bits are depth-first order.  Identical subtrees are merged level
 * by level.
 *
 * Serialisation (paper's node format): node = [mask][count][ptr x popcount].
 * Pointers of nodes at level >= 4 are word offsets of child nodes; pointers
 * of level-3 nodes are indices into the leaf array.  Nodes are grouped by
 * level from the root down; within a level, and for the leaf array, in order
 * of first reference when the level above is scanned in its order with
 * children in ascending octant.
 * ======================================================================== */
typedef struct {
  uint32_t mask;
  uint32_t child[8];  /* ids of the next level down (leaf ids at level 3) */
  uint64_t count;
} or_tnode;

typedef struct {
  or_tnode* v;
  uint32_t n, cap;
  uint32_t* slot;     /* open addressing: id + 1, 0 = free */
  uint32_t nslot;
} or_ltab;

typedef struct {
  uint64_t* v;
  uint32_t n, cap;
  uint32_t* slot;
  uint32_t nslot;
} or_leaftab;

static uint64_t or_mix(uint64_t h) {
  h ^= h >> 33;
  h *= 0xff51afd7ed558ccdull;
  h ^= h >> 33;
  h *= 0xc4ceb9fe1a85ec53ull;
  h ^= h >> 33;
  return h;
}

static uint64_t tnode_hash(const or_tnode* t) {
  uint64_t h = or_mix(t->mask + 0x1234567ull);
  for (int i = 0; i < 8; i++) h = or_mix(h ^ (t->child[i] + 0x9e3779b97f4a7c15ull * (uint64_t)(i + 1)));
  return h;
}

static int tnode_eq(const or_tnode* a, const or_tnode* b) {
  if (a->mask != b->mask) return 0;
  for (int i = 0; i < 8; i++)
    if (a->child[i] != b->child[i]) return 0;
  return 1;
}

static void ltab_grow(or_ltab* t) {
  uint32_t ns = t->nslot ? t->nslot * 2 : 1024;
  uint32_t* s = (uint32_t*)calloc(ns, sizeof(uint32_t));
  for (uint32_t i = 0; i < t->n; i++) {
    uint64_t h = tnode_hash(&t->v[i]) & (ns - 1);
    while (s[h]) h = (h + 1) & (ns - 1);
    s[h] = i + 1;
  }
  free(t->slot);
  t->slot = s;
  t->nslot = ns;
}

static uint32_t ltab_intern(or_ltab* t, const or_tnode* x) {
  if (2 * (t->n + 1) > t->nslot) ltab_grow(t);
  uint64_t h = tnode_hash(x) & (t->nslot - 1);
  while (t->slot[h]) {
    uint32_t id = t->slot[h] - 1;
    if (tnode_eq(&t->v[id], x)) return id;
    h = (h + 1) & (t->nslot - 1);
  }
  if (t->n == t->cap) {
    t->cap = t->cap ? 2 * t->cap : 256;
    t->v = (or_tnode*)realloc(t->v, (size_t)t->cap * sizeof(or_tnode));
  }
  t->v[t->n] = *x;
  t->slot[h] = t->n + 1;
  return t->n++;
}

static void leaftab_grow(or_leaftab* t) {
  uint32_t ns = t->nslot ? t->nslot * 2 : 1024;
  uint32_t* s = (uint32_t*)calloc(ns, sizeof(uint32_t));
  for (uint32_t i = 0; i < t->n; i++) {
    uint64_t h = or_mix(t->v[i]) & (ns - 1);
    while (s[h]) h = (h + 1) & (ns - 1);
    s[h] = i + 1;
  }
  free(t->slot);
  t->slot = s;
  t->nslot = ns;
}

static uint32_t leaftab_intern(or_leaftab* t, uint64_t bits) {
  if (2 * (t->n + 1) > t->nslot) leaftab_grow(t);
  uint64_t h = or_mix(bits) & (t->nslot - 1);
  while (t->slot[h]) {
    uint32_t id = t->slot[h] - 1;
    if (t->v[id] == bits) return id;
    h = (h + 1) & (t->nslot - 1);
  }
  if (t->n == t->cap) {
    t->cap = t->cap ? 2 * t->cap : 256;
    t->v = (uint64_t*)realloc(t->v, (size_t)t->cap * sizeof(uint64_t));
  }
  t->v[t->n] = bits;
  t->slot[h] = t->n + 1;
  return t->n++;
}

typedef struct {
  const uint8_t* g;
  uint32_t R;
  or_ltab lv[16];     /* index = level (3..root) */
  or_leaftab leaves;
} or_bctx;

static inline uint8_t gat(const or_bctx* c, uint32_t x, uint32_t y, uint32_t z) {
  return c->g[(size_t)x + (size_t)c->R * ((size_t)y + (size_t)c->R * z)];
}

/* Returns the unique id of the cube's subtree at `level`, or -1 if empty. */
static int64_t build_rec(or_bctx* c, uint32_t x0, uint32_t y0, uint32_t z0, uint32_t level) {
  if (level == 2) {
    uint64_t bits = 0;
    for (int b = 0; b < 64; b++) {
      int o1 = b >> 3, o0 = b & 7;
      uint32_t x = x0 + 2 * (o1 & 1) + (o0 & 1);
      uint32_t y = y0 + 2 * ((o1 >> 1) & 1) + ((o0 >> 1) & 1);
      uint32_t z = z0 + 2 * ((o1 >> 2) & 1) + ((o0 >> 2) & 1);
      if (gat(c, x, y, z)) bits |= 1ull << b;
    }
    if (!bits) return -1;
    return leaftab_intern(&c->leaves, bits);
  }
  const uint32_t h = 1u << (level - 1);
  or_tnode t;
  memset(&t, 0, sizeof(t));
  for (int i = 0; i < 8; i++) {
    int64_t id = build_rec(c, x0 + h * (i & 1), y0 + h * ((i >> 1) & 1), z0 + h * ((i >> 2) & 1), level - 1);
    if (id >= 0) {
      t.mask |= 1u << i;
      t.child[i] = (uint32_t)id;
      t.count += (level == 3) ? (uint64_t)__builtin_popcountll(c->leaves.v[id])
                              : c->lv[level - 1].v[id].count;
    }
  }
  if (!t.mask) return -1;
  return ltab_intern(&c->lv[level], &t);
}

/* DFS walk in the serialised DAG: appends the grid materials of the solid
 * cells in depth-first order (ascending octant, then ascending leaf bit). */
static void dfs_materials(const or_dag* d, const uint8_t* g, uint32_t off, uint32_t level,
                          uint32_t x0, uint32_t y0, uint32_t z0, uint8_t* mats, uint32_t* n) {
  const uint32_t mask = d->words[off];
  const uint32_t h = 1u << (level - 1);
  uint32_t slot = 0;
  for (int i = 0; i < 8; i++) {
    if (!((mask >> i) & 1)) continue;
    const uint32_t ptr = d->words[off + 2 + slot++];
    const uint32_t cx = x0 + h * (i & 1), cy = y0 + h * ((i >> 1) & 1), cz = z0 + h * ((i >> 2) & 1);
    if (level > 3) {
      dfs_materials(d, g, ptr, level - 1, cx, cy, cz, mats, n);
    } else {
      const uint64_t bits = d->leaves[ptr];
      for (int b = 0; b < 64; b++) {
        if (!((bits >> b) & 1)) continue;
        int o1 = b >> 3, o0 = b & 7;
        uint32_t x = cx + 2 * (o1 & 1) + (o0 & 1);
        uint32_t y = cy + 2 * ((o1 >> 1) & 1) + ((o0 >> 1) & 1);
        uint32_t z = cz + 2 * ((o1 >> 2) & 1) + ((o0 >> 2) & 1);
        mats[(*n)++] = g[(size_t)x + (size_t)d->R * ((size_t)y + (size_t)d->R * z)];
      }
    }
  }
}

static int ilog2u(uint32_t v) { int l = 0; while ((1u << (l + 1)) <= v && l < 31) l++; return l; }

or_dag* or_dag_build(const uint8_t* grid, uint32_t R) {
  if (R < 8 || (R & (R - 1)) || R > 1024) return NULL;
  or_dag* d = (or_dag*)calloc(1, sizeof(or_dag));
  d->R = R;
  d->root_level = (uint32_t)ilog2u(R);
  or_bctx c;
  memset(&c, 0, sizeof(c));
  c.g = grid;
  c.R = R;
  const uint32_t L = d->root_level;
  int64_t root = build_rec(&c, 0, 0, 0, L);
  if (root >= 0) {
    /* canonical order, level by level */
    uint32_t* order[16];
    uint32_t norder[16];
    uint8_t* seen[16];
    memset(norder, 0, sizeof(norder));
    for (uint32_t l = 3; l <= L; l++) {
      order[l] = (uint32_t*)malloc((size_t)(c.lv[l].n ? c.lv[l].n : 1) * sizeof(uint32_t));
      seen[l] = (uint8_t*)calloc(c.lv[l].n ? c.lv[l].n : 1, 1);
    }
    uint32_t* leaf_order = (uint32_t*)malloc((size_t)(c.leaves.n ? c.leaves.n : 1) * sizeof(uint32_t));
    uint32_t* leaf_index = (uint32_t*)malloc((size_t)(c.leaves.n ? c.leaves.n : 1) * sizeof(uint32_t));
    uint8_t* leaf_seen = (uint8_t*)calloc(c.leaves.n ? c.leaves.n : 1, 1);
    uint32_t nleaf = 0;
    order[L][norder[L]++] = (uint32_t)root;
    seen[L][root] = 1;
    for (uint32_t l = L; l >= 3; l--) {
      for (uint32_t k = 0; k < norder[l]; k++) {
        const or_tnode* t = &c.lv[l].v[order[l][k]];
        for (int i = 0; i < 8; i++) {
          if (!((t->mask >> i) & 1)) continue;
          uint32_t cid = t->child[i];
          if (l > 3) {
            if (!seen[l - 1][cid]) { seen[l - 1][cid] = 1; order[l - 1][norder[l - 1]++] = cid; }
          } else {
            if (!leaf_seen[cid]) { leaf_seen[cid] = 1; leaf_index[cid] = nleaf; leaf_order[nleaf++] = cid; }
          }
        }
      }
      if (l == 3) break;
    }
    /* word offsets */
    uint32_t* woff[16];
    uint64_t off = 0;
    for (uint32_t l = L; l >= 3; l--) {
      woff[l] = (uint32_t*)malloc((size_t)(c.lv[l].n ? c.lv[l].n : 1) * sizeof(uint32_t));
      for (uint32_t k = 0; k < norder[l]; k++) {
        const or_tnode* t = &c.lv[l].v[order[l][k]];
        woff[l][order[l][k]] = (uint32_t)off;
        off += 2 + (uint32_t)__builtin_popcount(t->mask);
      }
      d->level_nodes[l] = norder[l];
      if (l == 3) break;
    }
    d->level_nodes[2] = nleaf;
    d->n_words = (uint32_t)off;
    d->words = (uint32_t*)malloc((size_t)off * sizeof(uint32_t));
    for (uint32_t l = L; l >= 3; l--) {
      for (uint32_t k = 0; k < norder[l]; k++) {
        const or_tnode* t = &c.lv[l].v[order[l][k]];
        uint32_t w = woff[l][order[l][k]];
        d->words[w] = t->mask;
        d->words[w + 1] = (uint32_t)t->count;
        uint32_t slot = 0;
        for (int i = 0; i < 8; i++) {
          if (!((t->mask >> i) & 1)) continue;
          d->words[w + 2 + slot++] = (l > 3) ? woff[l - 1][t->child[i]] : leaf_index[t->child[i]];
        }
      }
      if (l == 3) break;
    }
    d->n_leaves = nleaf;
    d->leaves = (uint64_t*)malloc((size_t)(nleaf ? nleaf : 1) * sizeof(uint64_t));
    for (uint32_t k = 0; k < nleaf; k++) d->leaves[k] = c.leaves.v[leaf_order[k]];
    d->n_solid = d->words[1];
    /* DFS material array and its run blocks (Section 3.3, e_c = 0) */
    uint8_t* mats = (uint8_t*)malloc((size_t)d->n_solid + 1);
    uint32_t n = 0;
    dfs_materials(d, grid, 0, L, 0, 0, 0, mats, &n);
    uint32_t nb = 0;
    for (uint32_t i = 0; i < n; i++)
      if (i == 0 || mats[i] != mats[i - 1]) nb++;
    d->n_rle = nb;
    d->rle_start = (uint32_t*)malloc((size_t)(nb ? nb : 1) * sizeof(uint32_t));
    d->rle_mat = (uint8_t*)malloc((size_t)(nb ? nb : 1));
    nb = 0;
    for (uint32_t i = 0; i < n; i++)
      if (i == 0 || mats[i] != mats[i - 1]) { d->rle_start[nb] = i; d->rle_mat[nb] = mats[i]; nb++; }
    free(mats);
    for (uint32_t l = 3; l <= L; l++) { free(order[l]); free(seen[l]); free(woff[l]); }
    free(leaf_order); free(leaf_index); free(leaf_seen);
  }
  for (uint32_t l = 0; l < 16; l++) { free(c.lv[l].v); free(c.lv[l].slot); }
  free(c.leaves.v);
  free(c.leaves.slot);
  return d;
}

void or_dag_free(or_dag* d) {
  if (!d) return;
  free(d->words); free(d->leaves); free(d->rle_start); free(d->rle_mat);
  free(d);
}

/* Touch marks of one DAG (counting instrumentation, see or_touch_frame):
 * child pointers read on the way down, leaf bitmaps read, child pointers of
 * a solid cell's path (whose prefix counts a hit reads), run starts probed
 * and run materials read.  NULL arrays mark nothing. */
typedef struct {
  uint8_t* words;   /* [n_words]: child pointer read */
  uint8_t* pre;     /* [n_words]: prefix of this child read (hit paths) */
  uint8_t* leaves;  /* [n_leaves] */
  uint8_t* rle;     /* [n_rle]: run start probed */
  uint8_t* mat;     /* [n_rle]: run material read */
} or_marks;

static void mark(uint8_t* m, uint32_t i) {
  if (m) __atomic_store_n(&m[i], (uint8_t)1, __ATOMIC_RELAXED);
}

static int dag_lookup(const or_dag* d, uint32_t x, uint32_t y, uint32_t z, uint32_t* dfs,
                      uint32_t* empty_level, const or_marks* mk, uint32_t* siblings);

/* Point query.  The DFS index is the sum, along the root-to-leaf path, of the
 * subtree counts of the preceding siblings, plus the set bits below the
 * cell's bit in its leaf bitmap (Section 3.3). */
int or_dag_lookup(const or_dag* d, uint32_t x, uint32_t y, uint32_t z, uint32_t* dfs,
                  uint32_t* empty_level) {
  return dag_lookup(d, x, y, z, dfs, empty_level, NULL, NULL);
}

/* `siblings` (may be NULL) gets, for a solid cell, the number of preceding
 * set siblings summed over the internal levels of its path: the subtree
 * counts that the DFS index adds up (Section 3.3). */
static int dag_lookup(const or_dag* d, uint32_t x, uint32_t y, uint32_t z, uint32_t* dfs,
                      uint32_t* empty_level, const or_marks* mk, uint32_t* siblings) {
  if (d->n_words == 0) { *empty_level = d->root_level; return 0; }
  uint32_t path[16];
  uint32_t np = 0;
  uint32_t off = 0, acc = 0, nsib = 0;
  for (uint32_t l = d->root_level; l >= 3; l--) {
    const uint32_t mask = d->words[off];
    const uint32_t s = l - 1;
    const int oct = (int)(((x >> s) & 1) | (((y >> s) & 1) << 1) | (((z >> s) & 1) << 2));
    if (!((mask >> oct) & 1)) { *empty_level = l - 1; return 0; }
    uint32_t slot = 0;
    for (int i = 0; i < oct; i++) {
      if (!((mask >> i) & 1)) continue;
      const uint32_t p = d->words[off + 2 + slot];
      acc += (l > 3) ? d->words[p + 1] : (uint32_t)__builtin_popcountll(d->leaves[p]);
      slot++;
    }
    nsib += slot;
    const uint32_t ptr = d->words[off + 2 + slot];
    if (mk) {
      mark(mk->words, off + 2 + slot);
      path[np++] = off + 2 + slot;
    }
    if (l == 3) {
      const uint64_t bits = d->leaves[ptr];
      if (mk) mark(mk->leaves, ptr);
      const int o1 = (int)(((x >> 1) & 1) | (((y >> 1) & 1) << 1) | (((z >> 1) & 1) << 2));
      const int o0 = (int)((x & 1) | ((y & 1) << 1) | ((z & 1) << 2));
      if (!((bits >> (8 * o1)) & 0xFF)) { *empty_level = 1; return 0; }
      const int b = 8 * o1 + o0;
      if (!((bits >> b) & 1)) { *empty_level = 0; return 0; }
      acc += (uint32_t)__builtin_popcountll(bits & ((1ull << b) - 1));
      *dfs = acc;
      if (siblings) *siblings = nsib;
      /* a hit reads the prefix count of every child on its path, from the
       * root's child down to the leaf (one per internal level) */
      if (mk)
        for (uint32_t i = 0; i < np; i++) mark(mk->pre, path[i]);
      return 1;
    }
    off = ptr;
  }
  return 0; /* not reached: root_level >= 3 */
}

static uint8_t dag_material(const or_dag* d, uint32_t i, const or_marks* mk, uint32_t* probes);

/* Material of DFS index i: the run block with the largest start <= i. */
uint8_t or_dag_material(const or_dag* d, uint32_t i) { return dag_material(d, i, NULL, NULL); }

/* `probes` (may be NULL) gets the number of run starts the search compares. */
static uint8_t dag_material(const or_dag* d, uint32_t i, const or_marks* mk, uint32_t* probes) {
  uint32_t lo = 0, hi = d->n_rle; /* answer in [lo, hi) */
  if (probes) *probes = 0;
  while (hi - lo > 1) {
    uint32_t mid = lo + (hi - lo) / 2;
    if (probes) (*probes)++;
    if (mk) mark(mk->rle, mid);
    if (d->rle_start[mid] <= i) lo = mid; else hi = mid;
  }
  if (mk) mark(mk->mat, lo);
  return d->rle_mat[lo];
}

static void expand_rec(const or_dag* d, uint32_t off, uint32_t level, uint32_t x0, uint32_t y0,
                       uint32_t z0, uint32_t* k, uint8_t* out) {
  const uint32_t mask = d->words[off];
  const uint32_t h = 1u << (level - 1);
  uint32_t slot = 0;
  for (int i = 0; i < 8; i++) {
    if (!((mask >> i) & 1)) continue;
    const uint32_t ptr = d->words[off + 2 + slot++];
    const uint32_t cx = x0 + h * (i & 1), cy = y0 + h * ((i >> 1) & 1), cz = z0 + h * ((i >> 2) & 1);
    if (level > 3) { expand_rec(d, ptr, level - 1, cx, cy, cz, k, out); continue; }
    const uint64_t bits = d->leaves[ptr];
    for (int b = 0; b < 64; b++) {
      if (!((bits >> b) & 1)) continue;
      int o1 = b >> 3, o0 = b & 7;
      uint32_t x = cx + 2 * (o1 & 1) + (o0 & 1);
      uint32_t y = cy + 2 * ((o1 >> 1) & 1) + ((o0 >> 1) & 1);
      uint32_t z = cz + 2 * ((o1 >> 2) & 1) + ((o0 >> 2) & 1);
      out[(size_t)x + (size_t)d->R * ((size_t)y + (size_t)d->R * z)] = or_dag_material(d, (*k)++);
    }
  }
}

void or_dag_expand(const or_dag* d, uint8_t* out) {
  memset(out, 0, (size_t)d->R * d->R * d->R);
  if (d->n_words == 0) return;
  uint32_t k = 0;
  expand_rec(d, 0, d->root_level, 0, 0, 0, &k, out);
}

/* ========================================================================
 * World of chunks.
 * ======================================================================== */
struct or_world {
  uint32_t chunk_log2, grid[3], lod_count, nchunks;
  or_dag** dags;        /* [chunk * lod_count + lod] */
  uint8_t** dense;      /* optional dense LOD grids */
};

or_world* or_world_new(uint32_t chunk_log2, const uint32_t grid[3], uint32_t lod_count) {
  if (chunk_log2 < 3 || chunk_log2 > 10 || lod_count < 1 || lod_count > 4) return NULL;
  if (chunk_log2 - (lod_count - 1) < 3) return NULL;
  for (int a = 0; a < 3; a++)
    if (grid[a] < 1 || ((uint64_t)grid[a] << chunk_log2) > 32768) return NULL;
  or_world* w = (or_world*)calloc(1, sizeof(or_world));
  w->chunk_log2 = chunk_log2;
  memcpy(w->grid, grid, sizeof(w->grid));
  w->lod_count = lod_count;
  w->nchunks = grid[0] * grid[1] * grid[2];
  w->dags = (or_dag**)calloc((size_t)w->nchunks * lod_count, sizeof(or_dag*));
  w->dense = (uint8_t**)calloc((size_t)w->nchunks * lod_count, sizeof(uint8_t*));
  return w;
}

void or_world_free(or_world* w) {
  if (!w) return;
  for (uint32_t i = 0; i < w->nchunks * w->lod_count; i++) { or_dag_free(w->dags[i]); free(w->dense[i]); }
  free(w->dags);
  free(w->dense);
  free(w);
}

int or_world_set_dag(or_world* w, uint32_t chunk, uint32_t lod, or_dag* d) {
  if (chunk >= w->nchunks || lod >= w->lod_count) return -1;
  if (d && d->R != (1u << (w->chunk_log2 - lod))) return -1;
  size_t i = (size_t)chunk * w->lod_count + lod;
  or_dag_free(w->dags[i]);
  w->dags[i] = d;
  return 0;
}

int or_world_set_dense(or_world* w, uint32_t chunk, uint32_t lod, const uint8_t* g) {
  if (chunk >= w->nchunks || lod >= w->lod_count) return -1;
  size_t i = (size_t)chunk * w->lod_count + lod;
  size_t R = (size_t)1 << (w->chunk_log2 - lod);
  free(w->dense[i]);
  w->dense[i] = (uint8_t*)malloc(R * R * R);
  memcpy(w->dense[i], g, R * R * R);
  return 0;
}

/* LOD pick: LOD = number of thresholds T with |camera - chunk centre| >= T
 * (the distance term of Eq. 1 with the chunk centre), compared exactly as
 * squared fixed-point integers; "<" keeps the finer LOD. */
void or_lod_pick(const or_world* w, const int64_t O[3], const uint32_t thr[3], uint8_t* lods) {
  const int64_t S = (int64_t)1 << w->chunk_log2;
  for (uint32_t cz = 0; cz < w->grid[2]; cz++)
    for (uint32_t cy = 0; cy < w->grid[1]; cy++)
      for (uint32_t cx = 0; cx < w->grid[0]; cx++) {
        const int64_t cc[3] = {cx, cy, cz};
        i128 d2 = 0;
        for (int a = 0; a < 3; a++) {
          i128 diff = (i128)O[a] - (i128)(cc[a] * S + S / 2) * 65536;
          d2 += diff * diff;
        }
        uint32_t lod = 0;
        for (uint32_t j = 0; j + 1 < w->lod_count; j++) {
          i128 t = (i128)thr[j] * 65536;
          if (d2 >= t * t) lod++;
        }
        lods[cx + w->grid[0] * (cy + w->grid[1] * cz)] = (uint8_t)lod;
      }
}

/* ========================================================================
 * Traversal.
 *
 * p(t) = (O + t D) / 2^16 voxels, t >= 0.  The level-s cell of a point is
 * floor(p / 2^s) (half-open cells).  The ray visits the distinct values of
 * floor(p(t)) as t grows.  An "instant" is (t, phase): phase 0 = at t,
 * phase 1 = just after t.  A boundary crossing on an axis with D > 0 takes
 * effect at t (class 0); one with D < 0 takes effect just after t (class 1).
 * Crossings are applied in (t, class) order, equal keys together.
 * The hit is the first visited cell inside the world that is solid in the
 * grid of its chunk at that chunk's picked LOD.  (The paper's traversal is
 * "similar to ESVO" in floating point; this exact definition replaces it.)
 * ======================================================================== */
typedef struct { i128 N, Dd; int ph; } or_key; /* t = N / Dd, Dd > 0 */

static int key_cmp(or_key a, or_key b) {
  i128 l = a.N * b.Dd, r = b.N * a.Dd;
  if (l < r) return -1;
  if (l > r) return 1;
  return (a.ph > b.ph) - (a.ph < b.ph);
}

static i128 floordiv128(i128 a, i128 b) { /* b > 0 */
  i128 q = a / b;
  if ((a % b) != 0 && a < 0) q -= 1;
  return q;
}

/* Level-s cell coordinate of axis a at instant k. */
static int64_t cell_at(int64_t O, int64_t D, or_key k, int s) {
  const i128 v = (i128)O * k.Dd + k.N * (i128)D;  /* p(t) * 2^16 * Dd */
  const i128 den = k.Dd << (16 + s);
  i128 q = floordiv128(v, den);
  if (D < 0 && k.ph == 1 && v == q * den) q -= 1; /* on a boundary, moving down */
  return (int64_t)q;
}

/* Exit key of the level-s cell c (coordinates in units of 2^s voxels) and the
 * mask of axes that cross at that key.  Returns 0 if the ray never leaves. */
static int exit_key(const int64_t O[3], const int64_t D[3], const int64_t c[3], int s,
                    or_key* out, int* axes) {
  int have = 0;
  for (int a = 0; a < 3; a++) {
    if (D[a] == 0) continue;
    or_key k;
    if (D[a] > 0) { k.N = (((i128)c[a] + 1) << (s + 16)) - O[a]; k.Dd = D[a]; k.ph = 0; }
    else { k.N = (i128)O[a] - ((i128)c[a] << (s + 16)); k.Dd = -(i128)D[a]; k.ph = 1; }
    if (!have) { *out = k; *axes = 1 << a; have = 1; continue; }
    int cmp = key_cmp(k, *out);
    if (cmp < 0) { *out = k; *axes = 1 << a; }
    else if (cmp == 0) *axes |= 1 << a;
  }
  return have;
}

typedef struct {
  const or_world* w;
  const uint8_t* lods;
  int mode;
  /* touch instrumentation (NULL when off): marks per DAG [chunk * lod_count
   * + lod], chunks visited and DAGs entered */
  const or_marks* marks;
  uint8_t* chunk_marks;
  uint8_t* dag_marks;
} or_tctx;

/* Occupancy of world LOD-k cell c in chunk ci.  Returns 1 if solid (and the
 * material), else 0 with *skip = level (in cells) of an empty cube around it. */
static int occupied(const or_tctx* T, uint32_t ci, uint32_t k, const int64_t c[3],
                    const int64_t base[3], uint8_t* mat, uint32_t* skip, int32_t* elev,
                    uint32_t* siblings, uint32_t* probes) {
  const or_world* w = T->w;
  const size_t i = (size_t)ci * w->lod_count + k;
  const uint32_t x = (uint32_t)(c[0] - base[0]), y = (uint32_t)(c[1] - base[1]), z = (uint32_t)(c[2] - base[2]);
  *elev = -1;
  if (T->mode & 2) {
    const uint32_t R = 1u << (w->chunk_log2 - k);
    const uint8_t m = w->dense[i] ? w->dense[i][(size_t)x + (size_t)R * ((size_t)y + (size_t)R * z)] : 0;
    *skip = 0;
    if (m) { *mat = m; return 1; }
    *elev = 0;
    return 0;
  }
  const or_dag* d = w->dags[i];
  if (!d) { *skip = (T->mode & 1) ? w->chunk_log2 - k : 0; *elev = (int32_t)(w->chunk_log2 - k); return 0; }
  uint32_t dfs = 0, lev = 0;
  const or_marks* mk = T->marks ? &T->marks[i] : NULL;
  if (dag_lookup(d, x, y, z, &dfs, &lev, mk, siblings)) { *mat = dag_material(d, dfs, mk, probes); return 1; }
  *skip = (T->mode & 1) ? lev : 0;
  *elev = (int32_t)lev;
  return 0;
}

/* Counting (test instrumentation): the non-empty cubes of the chunk's DAG
 * that the ray enters, from the cubes around each looked-up cell above its
 * largest empty cube.  A straight ray never re-enters a cube, so a cube is
 * new iff it differs from the same level's cube around the previous lookup. */
static void count_cubes(or_counts* cnt, const int64_t c[3], const int64_t base[3], int32_t elev,
                        int top, int64_t prev[3], int* have_prev) {
  for (int l = elev + 1; l <= top; l++) {
    if (*have_prev && ((c[0] - base[0]) >> l) == ((prev[0] - base[0]) >> l) &&
        ((c[1] - base[1]) >> l) == ((prev[1] - base[1]) >> l) &&
        ((c[2] - base[2]) >> l) == ((prev[2] - base[2]) >> l))
      continue;
    if (l == top) cnt->chunk_entries++;
    else if (l >= 3) cnt->node_cubes++;
    else if (l == 2) cnt->leaf_cubes++;
  }
  for (int a = 0; a < 3; a++) prev[a] = c[a];
  *have_prev = 1;
}

static void trace_one(const or_tctx* T, const int64_t O[3], const int64_t D[3], or_hit* h,
                      or_counts* cnt) {
  const or_world* w = T->w;
  const int CL = (int)w->chunk_log2;
  const int64_t ext[3] = {(int64_t)w->grid[0] << CL, (int64_t)w->grid[1] << CL, (int64_t)w->grid[2] << CL};
  h->hit = 0; h->x = h->y = h->z = 0; h->lod = 0; h->face = 0; h->material = 0; h->chunk = -1;
  h->t = INFINITY; h->t_num = 0; h->t_den = 0;

  /* world entry: the latest lower bound of the per-axis slab intervals */
  or_key cur = {0, 1, 0};
  for (int a = 0; a < 3; a++) {
    or_key k;
    if (D[a] > 0) { k.N = -(i128)O[a]; k.Dd = D[a]; k.ph = 0; }
    else if (D[a] < 0) { k.N = (i128)O[a] - ((i128)ext[a] << 16); k.Dd = -(i128)D[a]; k.ph = 1; }
    else continue;
    if (key_cmp(k, cur) > 0) cur = k;
  }

  for (;;) {
    int64_t cc[3];
    for (int a = 0; a < 3; a++) cc[a] = cell_at(O[a], D[a], cur, CL);
    for (int a = 0; a < 3; a++)
      if (cc[a] < 0 || cc[a] >= (int64_t)w->grid[a]) return; /* outside the world: miss */
    const uint32_t ci = (uint32_t)(cc[0] + (int64_t)w->grid[0] * (cc[1] + (int64_t)w->grid[1] * cc[2]));
    const int k = T->lods[ci];
    const or_dag* dk = w->dags[(size_t)ci * w->lod_count + k];
    const int counting = cnt && !(T->mode & 2) && dk && dk->n_words;
    int64_t prev[3] = {0, 0, 0};
    int have_prev = 0;
    if (cnt) cnt->chunk_visits++;
    mark(T->chunk_marks, ci);
    if (dk && dk->n_words) mark(T->dag_marks, (uint32_t)((size_t)ci * w->lod_count + k));
    const int64_t base[3] = {cc[0] << (CL - k), cc[1] << (CL - k), cc[2] << (CL - k)};
    int64_t c[3];
    for (int a = 0; a < 3; a++) c[a] = cell_at(O[a], D[a], cur, k);
    for (;;) {
      uint8_t mat = 0;
      uint32_t skip = 0, siblings = 0, probes = 0;
      int32_t elev = -1;
      const int solid = occupied(T, ci, (uint32_t)k, c, base, &mat, &skip, &elev, &siblings, &probes);
      if (counting) count_cubes(cnt, c, base, elev, CL - k, prev, &have_prev);
      if (solid) {
        if (counting) {
          cnt->preceding_siblings = (int32_t)siblings;
          cnt->run_probes = (int32_t)probes;
        }
        h->hit = 1;
        h->x = (int32_t)(c[0] << k); h->y = (int32_t)(c[1] << k); h->z = (int32_t)(c[2] << k);
        h->lod = k;
        h->material = mat;
        h->chunk = (int32_t)ci;
        /* face: lowest axis whose entry plane of this cell is crossed at the hit key */
        for (int a = 0; a < 3 && !h->face; a++) {
          if (D[a] == 0) continue;
          or_key e;
          if (D[a] > 0) { e.N = ((i128)c[a] << (k + 16)) - O[a]; e.Dd = D[a]; e.ph = 0; }
          else { e.N = (i128)O[a] - (((i128)c[a] + 1) << (k + 16)); e.Dd = -(i128)D[a]; e.ph = 1; }
          if (key_cmp(e, cur) == 0) h->face = 1 + 2 * a + (D[a] < 0);
        }
        const long double nd = sqrtl((long double)D[0] * D[0] + (long double)D[1] * D[1] +
                                     (long double)D[2] * D[2]);
        h->t = (double)(((long double)cur.N / (long double)cur.Dd) * nd / 65536.0L);
        h->t_num = (double)cur.N;
        h->t_den = (double)cur.Dd;
        return;
      }
      /* step out of the empty cube of level `skip` (cells) around c */
      const int s = k + (int)skip;
      int64_t cs[3];
      for (int a = 0; a < 3; a++) cs[a] = c[a] >> skip;
      or_key nk = cur;
      int axes = 0;
      if (!exit_key(O, D, cs, s, &nk, &axes)) return; /* D == 0: never leaves */
      cur = nk;
      if (skip == 0) {
        for (int a = 0; a < 3; a++)
          if (axes & (1 << a)) c[a] += (D[a] > 0) ? 1 : -1;
      } else {
        for (int a = 0; a < 3; a++) c[a] = cell_at(O[a], D[a], cur, k);
      }
      if ((c[0] >> (CL - k)) != cc[0] || (c[1] >> (CL - k)) != cc[1] || (c[2] >> (CL - k)) != cc[2])
        break; /* left the chunk */
    }
  }
}

typedef struct {
  const or_tctx* T;
  or_counts* counts;
  const int64_t* O;
  const int32_t* D;
  const or_frame* f;
  const uint32_t* idx;
  uint32_t lo, hi;
  or_hit* out;
} or_job;

static void* trace_job(void* arg) {
  const or_job* J = (const or_job*)arg;
  for (uint32_t i = J->lo; i < J->hi; i++) {
    int64_t D[3];
    const int64_t* O;
    if (J->f) {
      const uint32_t p = J->idx ? J->idx[i] : i;
      const int64_t px = p % J->f->W, py = p / J->f->W;
      for (int a = 0; a < 3; a++) D[a] = J->f->A[a] + px * J->f->BX[a] + py * J->f->BY[a];
      O = J->f->O;
    } else {
      for (int a = 0; a < 3; a++) D[a] = J->D[3 * (size_t)i + a];
      O = J->O;
    }
    if (J->counts) memset(&J->counts[i], 0, sizeof(or_counts));
    trace_one(J->T, O, D, &J->out[i], J->counts ? &J->counts[i] : NULL);
  }
  return NULL;
}

static void run_jobs(or_job* base, uint32_t n, int nthreads) {
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  if ((uint32_t)nthreads > n) nthreads = n ? (int)n : 1;
  or_job jobs[256];
  pthread_t th[256];
  for (int t = 0; t < nthreads; t++) {
    jobs[t] = *base;
    jobs[t].lo = (uint32_t)((uint64_t)n * t / nthreads);
    jobs[t].hi = (uint32_t)((uint64_t)n * (t + 1) / nthreads);
  }
  for (int t = 1; t < nthreads; t++) pthread_create(&th[t], NULL, trace_job, &jobs[t]);
  trace_job(&jobs[0]);
  for (int t = 1; t < nthreads; t++) pthread_join(th[t], NULL);
}

void or_trace(const or_world* w, const uint8_t* lods, const int64_t O[3], const int32_t* D,
              uint32_t n, or_hit* out, int mode, int nthreads) {
  or_tctx T = {w, lods, mode, NULL, NULL, NULL};
  or_job J = {&T, NULL, O, D, NULL, NULL, 0, n, out};
  run_jobs(&J, n, nthreads);
}

void or_trace_frame(const or_world* w, const uint8_t* lods, const or_frame* f,
                    const uint32_t* idx, uint32_t n, or_hit* out, int mode, int nthreads,
                    or_counts* counts) {
  or_tctx T = {w, lods, mode, NULL, NULL, NULL};
  or_job J = {&T, counts, NULL, NULL, f, idx, 0, n, out};
  run_jobs(&J, n, nthreads);
}

/* Counting instrumentation: the bytes of the device layout that the rays
 * of a frame touch, each counted once (see oracle.h). */
void or_touch_frame(const or_world* w, const uint8_t* lods, const or_frame* f, int nthreads,
                    or_touched* out) {
  const size_t nd = (size_t)w->nchunks * w->lod_count;
  or_marks* mk = (or_marks*)calloc(nd, sizeof(or_marks));
  for (size_t i = 0; i < nd; i++) {
    const or_dag* d = w->dags[i];
    if (!d) continue;
    mk[i].words = (uint8_t*)calloc(d->n_words ? d->n_words : 1, 1);
    mk[i].pre = (uint8_t*)calloc(d->n_words ? d->n_words : 1, 1);
    mk[i].leaves = (uint8_t*)calloc(d->n_leaves ? d->n_leaves : 1, 1);
    mk[i].rle = (uint8_t*)calloc(d->n_rle ? d->n_rle : 1, 1);
    mk[i].mat = (uint8_t*)calloc(d->n_rle ? d->n_rle : 1, 1);
  }
  uint8_t* cm = (uint8_t*)calloc(w->nchunks, 1);
  uint8_t* dm = (uint8_t*)calloc(nd, 1);
  const uint32_t n = f->W * f->H;
  or_hit* hits = (or_hit*)malloc((size_t)n * sizeof(or_hit));
  or_tctx T = {w, lods, 1, mk, cm, dm};
  or_job J = {&T, NULL, NULL, NULL, f, NULL, 0, n, hits};
  run_jobs(&J, n, nthreads);
  memset(out, 0, sizeof(*out));
  out->rays = n;
  for (uint32_t h = 0; h < n; h++) out->hits += hits[h].hit != 0;
  for (size_t i = 0; i < nd; i++) {
    const or_dag* d = w->dags[i];
    if (!d) continue;
    for (uint32_t j = 0; j < d->n_words; j++) {
      out->child_words += mk[i].words[j];
      out->prefixes += mk[i].pre[j];
    }
    for (uint32_t j = 0; j < d->n_leaves; j++) out->leaves += mk[i].leaves[j];
    for (uint32_t j = 0; j < d->n_rle; j++) {
      out->run_starts += mk[i].rle[j];
      out->run_materials += mk[i].mat[j];
    }
    out->dags += dm[i];
    free(mk[i].words); free(mk[i].pre); free(mk[i].leaves); free(mk[i].rle); free(mk[i].mat);
  }
  for (uint32_t c = 0; c < w->nchunks; c++) out->chunks += cm[c];
  free(mk); free(cm); free(dm); free(hits);
}
