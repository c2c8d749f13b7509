// gfx950 kernels of libsvdag: per-view chunk stage and per-pixel SVDAG trace.
//
// Traversal (Section 3.5 ray marching, made exact).  A ray is
// p(t) = (O + t D) / 2^16 voxels with integer O, D.  A time is a rational
// Nt/Dt plus a phase (0 = at t, 1 = just after t); a boundary crossing on an
// axis with D > 0 takes effect at t, one with D < 0 just after t, so events
// are ordered by (t, class) and equal keys are stepped together.
//
// Each ray is mirrored on the axes where D < 0 (as ESVO does), so that every
// direction component is >= 0 and every cell coordinate only grows; a
// mirrored axis keeps class 1 (its cells are closed at their upper plane).
// A plane of axis a at numerator N = X - O_a (fixed point) is crossed at the
// key (N / |D_a|, class_a); it is behind the current instant iff
//     N * 2 Dt  <  T_a = 2 Nt |D_a| + 1 + phase - class_a,
// one 32x32->64-bit multiply-add per test, T_a being refreshed once per
// step.  The exit planes of the current cell are kept as numerators E_a:
// a mid-plane is E_a - half a cell, a child's exits are E_a or the mid-plane,
// a step adds one cell.  No division anywhere in the kernel.
//
// The walk is one hierarchy: chunk grid (level chunk_log2, in voxels), the
// chunk's DAG levels down to 8^3 nodes (level k+3 for LOD k), the 4^3 leaf
// bitmap (k+2), its 2^3 sub-blocks (k+1) and cells (k).  Entering a non-empty
// cell finds its child that holds the current instant with three mid-plane
// tests; an empty cell is left by one exact step at its level, and the walk
// goes on at the neighbour: a sibling in the same parent (when the cell was
// the lower of its pair on every stepped axis, read off its octant), or the
// child of the lowest common ancestor of the old and new cells (highest
// changed coordinate bit) that holds the new cell, found from the
// coordinates without plane tests.  The node words of the current path live
// in LDS.  Hits are resolved after the loop (DFS index, material run through
// the run directory, t, face).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "svdag_internal.h"

// Walk events (iter, descend, exit, sibling, pop, chunk_next, chunk_visit,
// chunk_enter, hit) for a host build that counts them; empty in the library.
#ifndef SVD_WALK_EVENT
#define SVD_WALK_EVENT(e) do {} while (0)
#endif

namespace svd {

struct DescBatch {
  DevDag d[4];
};

__global__ void set_desc_kernel(DevDag* dst, DescBatch b, uint32_t n) {
  const uint32_t i = threadIdx.x;
  if (i < n) dst[i] = b.d[i];
}

int launch_set_desc(DevDag* dst, const DevDag* src, uint32_t n, void* stream) {
  if (n > 4) return svd_fail(SVD_EINVAL, "internal: descriptor batch > 4");
  DescBatch b;
  for (uint32_t i = 0; i < n; i++) b.d[i] = src[i];
  hipLaunchKernelGGL(set_desc_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, dst, b, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return svd_fail(SVD_EDEVICE, "set_desc launch: %s", hipGetErrorString(e));
  return SVD_OK;
}

// ------------------------------------------------------------- chunk stage
// One thread per chunk.  LOD = number of thresholds reached by the camera to
// chunk-centre distance (Eq. 1 distance term), compared exactly as squared
// 128-bit integers.  Cull: the chunk's tight box at that LOD lies strictly on
// the outer side of a side plane of the view cone (exact 128-bit), so no
// pixel ray can reach a solid cell of it.
__host__ __device__ inline uint32_t stage_chunk(const StageParams& p, uint32_t ci) {
  const uint32_t cc[3] = {ci % p.grid[0], (ci / p.grid[0]) % p.grid[1], ci / (p.grid[0] * p.grid[1])};
  const int64_t S = (int64_t)1 << p.chunk_log2;
  unsigned __int128 d2 = 0;
  _Pragma("unroll") for (int a = 0; a < 3; a++) {
    const __int128 diff = (__int128)p.O[a] - (__int128)(((int64_t)cc[a] * S + S / 2) << 16);
    d2 += (unsigned __int128)(diff * diff);
  }
  uint32_t k = 0;
  _Pragma("unroll") for (uint32_t j = 0; j < 3; j++) {
    if (j + 1 >= p.lod_count) break;
    const unsigned __int128 t = (unsigned __int128)p.thr[j] << 16;
    if (d2 >= t * t) k++;
  }
  const DevDag& d = p.desc[(size_t)ci * 4 + k];
  uint32_t v = k;
  if (d.solid == 0) {
    v |= kViewEmpty;
  } else if (p.cull) {
    __int128 lo[3], hi[3];
    _Pragma("unroll") for (int a = 0; a < 3; a++) {
      const int64_t base = (int64_t)cc[a] * S;
      lo[a] = ((__int128)(base + ((int64_t)d.lo[a] << k)) << 16) - p.O[a];
      hi[a] = ((__int128)(base + ((int64_t)(d.hi[a] + 1) << k)) << 16) - p.O[a];
    }
    bool culled = false;
    _Pragma("unroll") for (int i = 0; i < 4; i++) {
      __int128 s = 0;
      _Pragma("unroll") for (int a = 0; a < 3; a++) s += (__int128)p.n[i][a] * (p.n[i][a] >= 0 ? hi[a] : lo[a]);
      if (s < 0) culled = true;
    }
    if (culled) v |= kViewCulled;
  }
  // a chunk that rays may enter at an LOD that is described but not loaded
  if (!(v & (kViewCulled | kViewEmpty)) && d.nodes == 0) v |= kViewMissing;
  return v;
}

uint32_t host_stage_chunk(const StageParams& p, uint32_t ci) { return stage_chunk(p, ci); }

__global__ void chunk_stage_kernel(StageParams p) {
  const uint32_t ci = blockIdx.x * blockDim.x + threadIdx.x;
  if (ci >= p.nchunks) return;
  p.view[ci] = stage_chunk(p, ci);
}

int launch_chunk_stage(const StageParams& p, void* stream) {
  const uint32_t threads = 64;
  const uint32_t blocks = (p.nchunks + threads - 1) / threads;
  hipLaunchKernelGGL(chunk_stage_kernel, dim3(blocks), dim3(threads), 0, (hipStream_t)stream, p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return svd_fail(SVD_EDEVICE, "chunk stage launch: %s", hipGetErrorString(e));
  return SVD_OK;
}

// ------------------------------------------------------------------- trace
constexpr int kBlock = 256;      // 4 waves; each wave traces one 64-pixel tile at a time
constexpr int kStackLevels = 8;  // node levels 3..10
constexpr uint32_t kMaxIter = 1u << 22;
constexpr uint32_t kFaultChunk = 0xFFFFFFFEu;
constexpr uint32_t kMissingChunk = 0xFFFFFFFDu;

enum : uint32_t { kRunning = 0, kHit = 1, kMiss = 2, kFault = 3, kNotLoaded = 4 };

__host__ __device__ __forceinline__ uint32_t float_bits(float f) {
  union { float f; uint32_t u; } v;
  v.f = f;
  return v.u;
}

// DAG arrays live in global memory (the world's pool); naming the address
// space lets the loads be global_load rather than flat_load.
#define SVD_GLOBAL __attribute__((address_space(1)))
typedef const SVD_GLOBAL uint32_t* gptr32;
typedef const SVD_GLOBAL uint64_t* gptr64;
typedef const SVD_GLOBAL uint8_t* gptr8;

// Ray in mirrored coordinates and its current instant.
struct Ray {
  int64_t Om[3];    // mirrored origin, voxels * 2^16
  uint32_t Oml[3];  // low 32 bits of Om: plane numerators in [0, 2^32) are exact mod 2^32
  uint32_t ad[3];   // |D_a|
  uint32_t ad2[3];  // 2 |D_a| (< 2^32)
  uint32_t mm;      // mirror mask (bit a: D_a < 0) = class bits
  uint32_t Nt, ph, D2;      // instant Nt / (D2 / 2), phase
  uint64_t T[3];    // 2 Nt |D_a| + 1 + ph - class_a

  __host__ __device__ __forceinline__ uint32_t cls(int a) const { return (mm >> a) & 1u; }
  // Is the plane of axis a with numerator N >= 0 behind the current instant?
  __host__ __device__ __forceinline__ bool past_n(int a, uint32_t N) const {
    return (uint64_t)N * D2 < T[a];
  }
  // Same for a plane given in mirrored fixed point (possibly behind the origin).
  __host__ __device__ __forceinline__ bool past(int a, int64_t X16) const {
    const int64_t N = X16 - Om[a];
    return (N < 0) | past_n(a, (uint32_t)N);
  }
  __host__ __device__ __forceinline__ void set_time(uint32_t n, uint32_t d2, uint32_t c) {
    Nt = n;
    ph = c;
    D2 = d2;
    _Pragma("unroll") for (int a = 0; a < 3; a++) T[a] = (uint64_t)n * ad2[a] + (1u + c - cls(a));
  }
};

// Bit i of m (i < 32): one bit-field extract on the GPU.
__host__ __device__ __forceinline__ uint32_t bit_at(uint32_t m, uint32_t i) {
#ifdef __HIP_DEVICE_COMPILE__
  return __builtin_amdgcn_ubfe(m, i, 1);
#else
  return (m >> i) & 1u;
#endif
}

// Leave the current cell (any level; E its exit-plane numerators): the
// earliest exit plane sets the ray's new instant.  `step` gets the axes that
// step (bit a; every axis that ties).  False when D == 0: the ray never
// leaves the cell.
__host__ __device__ __forceinline__ bool exit_cell(Ray& r, const uint32_t E[3], uint32_t& step) {
  // Key of axis a, scaled against axis b: E_a * 2|D_b| + class_a.
  uint32_t bE = E[0], bA2 = r.ad2[0], bC = r.cls(0), sm = 1u;
  _Pragma("unroll") for (int a = 1; a < 3; a++) {
    const uint64_t ka = (uint64_t)E[a] * bA2 + r.cls(a);
    const uint64_t kb = (uint64_t)bE * r.ad2[a] + bC;
    const bool lt = ka < kb, eq = ka == kb;
    bE = lt ? E[a] : bE;
    bA2 = lt ? r.ad2[a] : bA2;
    bC = lt ? r.cls(a) : bC;
    sm = lt ? (1u << a) : (eq ? sm | (1u << a) : sm);
  }
  if (bA2 == 0) return false;
  r.set_time(bE, bA2, bC);  // 2|D| of the exit axis
  step = sm;
  return true;
}

// One level down: the child of cell c (level lev, exit numerators E) that
// holds the current instant, by three mid-plane tests.  Updates c, E and lev
// to the child and returns its octant in the unmirrored node.
__host__ __device__ __forceinline__ uint32_t descend(const Ray& r, int32_t c[3], uint32_t E[3], int& lev) {
  const uint32_t half = 1u << (lev - 1 + 16);
  uint32_t bits = 0;
  _Pragma("unroll") for (int a = 0; a < 3; a++) {
    const uint32_t nm = E[a] - half;  // mid-plane numerator
    const uint32_t b = (uint32_t)(E[a] < half) | (uint32_t)r.past_n(a, nm);
    c[a] = 2 * c[a] + (int32_t)b;
    E[a] = b ? E[a] : nm;
    bits |= b << a;
  }
  lev--;
  return bits ^ r.mm;
}

// Enter the non-empty child `oct` (a cube at level lev) of the current node:
// a node or leaf word from the DAG (node words of levels >= k + 3 go on the
// path stack; a leaf's word carries its sub-block summary, and its bitmap is
// read), or a sub-block of the current leaf.  `mask` becomes the child's
// children mask.
__host__ __device__ __forceinline__ void enter_child(int lev, int k, uint32_t oct, uint32_t& mask, uint32_t& ptr,
                                                     uint32_t& lmask, uint64_t& bitmap, gptr32 nodes, gptr64 leaves,
                                                     uint32_t* stk, uint32_t ss) {
  if (lev >= k + 2) {
    const uint32_t w = nodes[ptr + __builtin_popcount(mask & ((1u << oct) - 1u))];
    mask = w >> kPtrBits;
    ptr = w & kPtrMask;
    if (lev >= k + 3) {
      stk[(lev - 3) * ss] = w;
    } else {
      lmask = mask;
      bitmap = leaves[ptr];
    }
  } else {
    mask = (uint32_t)(bitmap >> (8 * oct)) & 0xFFu;
  }
}

// The whole per-pixel path: ray setup, world entry, chunk walk, DAG
// traversal, hit resolve.  `stk` is this ray's node-word stack (levels 3..10,
// element stride `ss`).
__host__ __device__ inline uint4 trace_pixel(const TraceParams& p, uint32_t px, uint32_t py,
                                             uint32_t* stk, uint32_t ss, uint32_t start) {
  const int CL = (int)p.chunk_log2;
  int32_t D[3];
  Ray r;
  r.mm = 0;
  _Pragma("unroll") for (int a = 0; a < 3; a++) {
    D[a] = (int32_t)(p.A[a] + (int64_t)px * p.BX[a] + (int64_t)py * p.BY[a]);
    r.ad[a] = (uint32_t)(D[a] < 0 ? -(int64_t)D[a] : (int64_t)D[a]);
    r.ad2[a] = 2u * r.ad[a];
    const int64_t ext16 = (int64_t)p.grid[a] << (CL + 16);
    if (D[a] < 0) r.mm |= 1u << a;
    r.Om[a] = D[a] < 0 ? ext16 - p.O[a] : p.O[a];
    r.Oml[a] = (uint32_t)r.Om[a];
  }

  // World entry: the latest lower bound of the per-axis slabs (mirrored
  // world = [0, ext) per axis, entered through plane 0).
  uint32_t n0 = 0, d0 = 1, c0 = 0;
  _Pragma("unroll") for (int a = 0; a < 3; a++) {
    // a class-1 axis starting exactly on plane 0 still enters just after t = 0
    if (r.Om[a] > 0 || r.ad[a] == 0) continue;
    const uint32_t n = (uint32_t)(-r.Om[a]), cl = r.cls(a);
    const uint64_t l = (uint64_t)n * d0, q = (uint64_t)n0 * r.ad[a];
    if (l > q || (l == q && cl > c0)) { n0 = n; d0 = r.ad[a]; c0 = cl; }
  }
  uint32_t status = kRunning;
  // Start bound of the tile (beam pass): no cell the ray can hit lies within
  // Chebyshev distance `start` voxels of the camera, and the ray is at that
  // distance at t = start 2^16 / max|D_a|; begin there if that is later.
  if (start == kBeamNone) {
    status = kMiss;
  } else if (start) {
    const uint32_t m01 = r.ad[0] > r.ad[1] ? r.ad[0] : r.ad[1];
    const uint32_t mad = m01 > r.ad[2] ? m01 : r.ad[2];
    const uint32_t nb = start << 16;
    if ((uint64_t)nb * d0 > (uint64_t)n0 * mad) { n0 = nb; d0 = mad; c0 = 0; }
  }
  r.set_time(n0, 2u * d0, c0);

  int32_t c[3];
  uint32_t E[3];  // exit-plane numerators of cell c at level lev
  _Pragma("unroll") for (int a = 0; a < 3; a++) {
    const int64_t ext16 = (int64_t)p.grid[a] << (CL + 16);
    if (!r.past(a, 0) || r.past(a, ext16)) status = kMiss;
    // chunk coordinate at the entry instant: binary search over chunk planes
    uint32_t lo = 0, hi = p.grid[a];
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (r.past(a, (int64_t)mid << (CL + 16))) lo = mid; else hi = mid;
    }
    c[a] = (int32_t)lo;
    E[a] = ((lo + 1) << (CL + 16)) - r.Oml[a];
  }

  int lev = CL, k = 0;
  uint32_t mask = 0, lmask = 0, ptr = 0, ci = 0, iter = 0;
  uint64_t bitmap = 0;
  gptr32 nodes = nullptr;
  gptr64 leaves = nullptr;
  // Chunk walk: c and E describe the current chunk (level CL).
  while (status == kRunning) {
    if (++iter > kMaxIter) { status = kFault; break; }
#ifdef __HIP_DEVICE_COMPILE__
    // Issue priority of the wave: rays that keep crossing chunks are the long
    // ones (far, grazing rays), and their tiles are the launch's critical
    // path.  The wave raises its priority as a ray reaches its 2nd, 4th and
    // 8th chunk, so the SIMD's arbiter issues its instructions ahead of waves
    // whose rays ended nearby (scheduling only; the tile loop resets it).
    if (iter == 2) __builtin_amdgcn_s_setprio(1);
    if (iter == 4) __builtin_amdgcn_s_setprio(2);
    if (iter == 8) __builtin_amdgcn_s_setprio(3);
#endif
    SVD_WALK_EVENT(chunk_visit);
    if (c[0] >= (int32_t)p.grid[0] || c[1] >= (int32_t)p.grid[1] || c[2] >= (int32_t)p.grid[2]) {
      status = kMiss;  // left the world
      break;
    }
    uint32_t co[3];
    _Pragma("unroll") for (int a = 0; a < 3; a++) co[a] = r.cls(a) ? p.grid[a] - 1 - (uint32_t)c[a] : (uint32_t)c[a];
    ci = co[0] + p.grid[0] * (co[1] + p.grid[1] * co[2]);
    const uint32_t v = p.view[ci];
    if (!(v & (kViewCulled | kViewEmpty))) {
      if (v & kViewMissing) {
        status = kNotLoaded;
        break;
      }
      k = (int)(v & kViewLodMask);
      const DevDag* dag = &p.desc[(size_t)ci * 4 + k];
      // Every solid cell of the chunk lies in its tight box.  Cell
      // coordinates of the mirrored ray never decrease, so a ray already at
      // or past the box's upper face on some axis meets none of them: cross
      // the chunk as an empty one.  (A face behind the origin wraps to a
      // numerator near 2^32; the test may then read it as not passed, which
      // only forgoes the skip.)
      bool beyond = false;
      _Pragma("unroll") for (int a = 0; a < 3; a++) {
        const uint32_t b = r.cls(a) ? (1u << (CL - k)) - dag->lo[a] : dag->hi[a] + 1u;
        beyond |= r.past_n(a, ((((uint32_t)c[a] << (CL - k)) + b) << (k + 16)) - r.Oml[a]);
      }
      if (!beyond) {
      SVD_WALK_EVENT(chunk_enter);
      nodes = (gptr32)dag->nodes;
      leaves = (gptr64)dag->leaves;
      const uint32_t root = dag->root;
      stk[(CL - 3) * ss] = root;
      mask = root >> kPtrBits;
      ptr = 0;
      // Into the root's child that holds the current instant.  From here on
      // c (level lev) is a cell whose parent's children mask is `mask` and
      // whose octant in that parent is `oct`.
      lev = CL;
      uint32_t oct = descend(r, c, E, lev);
      // DAG walk inside the chunk, until a hit or the ray leaves the chunk.
      // An iteration enters c and descends one level if c is not empty, then
      // leaves the cell it is in if that one is empty.  Leaving a cell finds
      // the next cell without mid-plane tests: a sibling in the same parent
      // (its octant differs on the stepped axes), or the child of the lowest
      // common ancestor that holds the new cell (the ancestor's mask comes
      // from the path stack).  No iteration guard: each exit moves the cell
      // forward on some axis of the mirrored ray and each descent lowers the
      // level, so the walk inside a chunk ends whatever the DAG holds.
      for (;;) {
        SVD_WALK_EVENT(iter);
        uint32_t full = bit_at(mask, oct);
        // A non-empty cell at the LOD's level (the walk never goes below
        // level k, so lev <= k means lev == k) is the hit.  The loop leaves
        // without setting the status: the hit is the one exit with the
        // current cell non-empty, read after the loop.
        if (full && lev <= k) {
          SVD_WALK_EVENT(hit);
          break;
        }
        if (full) {
          SVD_WALK_EVENT(descend);
          enter_child(lev, k, oct, mask, ptr, lmask, bitmap, nodes, leaves, stk, ss);
          oct = descend(r, c, E, lev);
          full = (mask >> oct) & 1u;
        }
        if (!full) {
          SVD_WALK_EVENT(exit);
          uint32_t step;
          if (!exit_cell(r, E, step)) break;  // D == 0: the ray never leaves the cell
          if (((oct ^ r.mm) & step) == 0) {
            SVD_WALK_EVENT(sibling);
            // the cell was the lower of its pair on every stepped axis: the
            // new cell is its sibling, one cell on along those axes
            _Pragma("unroll") for (int a = 0; a < 3; a++) {
              const uint32_t s = (step >> a) & 1u;
              E[a] += s << (lev + 16);
              c[a] += (int32_t)s;
            }
            oct ^= step;
          } else {
            // the lowest common ancestor of the old and new cells is the
            // level above the highest changed coordinate bit; the new cell
            // lies in its child at level nl (or in the next chunk, level CL)
            uint32_t diff = 0;
            _Pragma("unroll") for (int a = 0; a < 3; a++) {
              const int32_t n = c[a] + (int32_t)((step >> a) & 1u);
              diff |= (uint32_t)(c[a] ^ n);
              c[a] = n;
            }
            const int pl = lev + (32 - __builtin_clz(diff));
            const int nl = min(pl - 1, CL);
            _Pragma("unroll") for (int a = 0; a < 3; a++) {
              c[a] >>= (nl - lev);
              E[a] = ((uint32_t)(c[a] + 1) << (nl + 16)) - r.Oml[a];
            }
            if (pl > CL) {  // into the next chunk (level CL)
              SVD_WALK_EVENT(chunk_next);
              break;
            }
            SVD_WALK_EVENT(pop);
            lev = nl;
            oct = (((uint32_t)c[0] & 1u) | (((uint32_t)c[1] & 1u) << 1) | (((uint32_t)c[2] & 1u) << 2)) ^ r.mm;
            if (pl >= k + 3) {
              const uint32_t w = stk[(pl - 3) * ss];
              mask = w >> kPtrBits;
              ptr = w & kPtrMask;
            } else if (pl == k + 2) {
              mask = lmask;
            } else {  // pl == k + 1: the sub-block of the leaf
              const uint32_t o1 = ((((uint32_t)c[0] >> 1) & 1u) | ((((uint32_t)c[1] >> 1) & 1u) << 1) |
                                   ((((uint32_t)c[2] >> 1) & 1u) << 2)) ^ r.mm;
              mask = (uint32_t)(bitmap >> (8 * o1)) & 0xFFu;
            }
          }
        }
      }
      // the loop's exits: a hit (the current cell non-empty), the next chunk,
      // or a ray that never moves (D == 0) in an empty cell: a miss
      if ((mask >> oct) & 1u) status = kHit;
      else if ((r.ad2[0] | r.ad2[1] | r.ad2[2]) == 0) status = kMiss;
      continue;
      }
    }
    // an empty or culled chunk, or one whose solid cells all lie behind the
    // ray: cross it
    uint32_t step;
    if (!exit_cell(r, E, step)) { status = kMiss; break; }
    _Pragma("unroll") for (int a = 0; a < 3; a++) {
      const uint32_t s = (step >> a) & 1u;
      E[a] += s << (CL + 16);
      c[a] += (int32_t)s;
    }
  }

  uint4 rec = make_uint4(0u, 0u, 0x7F800000u /* +inf */, 0xFFFFFFFFu);
  if (status == kFault) rec.w = kFaultChunk;
  if (status == kNotLoaded) rec.w = kMissingChunk;
  if (status == kHit) {
    // unmirrored LOD-k cell
    int32_t h[3];
    _Pragma("unroll") for (int a = 0; a < 3; a++)
      h[a] = r.cls(a) ? (int32_t)((p.grid[a] << (CL - k)) - 1) - c[a] : c[a];
    const DevDag* dag = &p.desc[(size_t)ci * 4 + k];
    // DFS index (Section 3.3): counts of earlier siblings along the path
    const gptr32 pre = (gptr32)dag->pre;
    uint32_t dfs = 0;
    for (int L = CL; L >= k + 3; L--) {
      const uint32_t w = stk[(L - 3) * ss];
      const int s = L - 1 - k;
      const uint32_t o = ((h[0] >> s) & 1) | (((h[1] >> s) & 1) << 1) | (((h[2] >> s) & 1) << 2);
      dfs += pre[(w & kPtrMask) + __builtin_popcount((w >> kPtrBits) & ((1u << o) - 1u))];
    }
    const uint32_t o1 = ((h[0] >> 1) & 1) | (((h[1] >> 1) & 1) << 1) | (((h[2] >> 1) & 1) << 2);
    const uint32_t o0 = (h[0] & 1) | ((h[1] & 1) << 1) | ((h[2] & 1) << 2);
    dfs += (uint32_t)__builtin_popcountll(bitmap & ((1ull << (8 * o1 + o0)) - 1ull));
    // material: the last run starting at or before the DFS index, searched
    // between the two run-directory entries around it
    const gptr32 rs = (gptr32)dag->rle_start;
    const uint32_t nr = dag->rle_n;
    const gptr32 dir = (gptr32)dag->rle_dir + (dfs >> run_dir_shift(nr, dag->solid));
    uint32_t lo = dir[0], hi = dir[1] + 1u;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (rs[mid] <= dfs) lo = mid; else hi = mid;
    }
    const uint32_t mat = ((gptr8)(rs + nr))[lo];
    // entry face: lowest axis whose entry plane is crossed at the hit instant
    // (the direction is recomputed here rather than kept through the walk)
    uint32_t face = 0;
    double len2 = 0.0;
    _Pragma("unroll") for (int a = 0; a < 3; a++) {
      const uint32_t ada = r.ad2[a] >> 1;
      len2 += (double)ada * (double)ada;
      if (face || !ada) continue;
      const uint32_t cl = r.cls(a);
      const int64_t X16 = (int64_t)(cl ? h[a] + 1 : h[a]) << (k + 16);
      const int64_t ne = cl ? p.O[a] - X16 : X16 - p.O[a];
      if (ne >= 0 && cl == r.ph && (uint64_t)ne * (r.D2 >> 1) == (uint64_t)r.Nt * ada) face = 1 + 2 * a + cl;
    }
    const double len = sqrt(len2);
    const float t = (float)(((double)r.Nt / (double)(r.D2 >> 1)) * len * (1.0 / 65536.0));
    rec.x = ((uint32_t)h[0] << k) | (((uint32_t)h[1] << k) << 16);
    rec.y = ((uint32_t)h[2] << k) | ((uint32_t)k << 16) | (face << 20) | (1u << 23) | (mat << 24);
    rec.z = float_bits(t);
    rec.w = ci;
  }
  return rec;
}

// Next tile (or first of `claim` tiles) of the wave from its home queue, or
// from the following queues once that one is dry; false when all are.
// Queue q hands out the band [total q / kQueues, total (q + 1) / kQueues).
__device__ __forceinline__ bool take_tiles(uint32_t* queue, uint32_t total, uint32_t claim, uint32_t home,
                                           uint32_t lane, uint32_t& qi, uint32_t& t0, uint32_t& t1) {
  for (; qi < kQueues; qi++) {
    const uint32_t q = (home + qi) % kQueues;
    const uint32_t lo = (uint32_t)((uint64_t)total * q / kQueues);
    const uint32_t hi = (uint32_t)((uint64_t)total * (q + 1) / kQueues);
    uint32_t t = 0;
    if (lane == 0) t = atomicAdd(&queue[q * kQueueStride], claim);
    t = __builtin_amdgcn_readlane(t, 0);  // wave-uniform: the tile math and view lookup stay scalar
    if (t < hi - lo) {
      t0 = lo + t;
      t1 = t0 + claim < hi ? t0 + claim : hi;
      return true;
    }
  }
  return false;
}

// Tiles of queue q in the per-view trace: the tile rows y with y % kQueues
// == q, each left to right, rows top to bottom.  Interleaving the rows
// spreads every part of the image (the costly rows around a horizon, the
// cheap sky) over all the queues, so that they run dry together and each
// ends on the image's last rows, instead of one queue's band of costly
// rows finishing alone.
__host__ __device__ __forceinline__ uint32_t row_queue_tiles(uint32_t q, uint32_t tiles_x, uint32_t tiles_y) {
  return q < tiles_y ? ((tiles_y - 1 - q) / kQueues + 1) * tiles_x : 0u;
}
__host__ __device__ __forceinline__ uint32_t row_queue_tile(uint32_t q, uint32_t j, uint32_t tiles_x) {
  return (q + kQueues * (j / tiles_x)) * tiles_x + j % tiles_x;
}

// Next tile of the wave from its home queue (row-interleaved), or from the
// following queues once that one is dry; false when all are.
__device__ __forceinline__ bool take_row_tile(uint32_t* queue, uint32_t tiles_x, uint32_t tiles_y, uint32_t home,
                                              uint32_t lane, uint32_t& qi, uint32_t& t) {
  for (; qi < kQueues; qi++) {
    const uint32_t q = (home + qi) % kQueues;
    uint32_t j = 0;
    if (lane == 0) j = atomicAdd(&queue[q * kQueueStride], 1u);
    j = __builtin_amdgcn_readlane(j, 0);  // wave-uniform: the tile math stays scalar
    if (j < row_queue_tiles(q, tiles_x, tiles_y)) {
      t = row_queue_tile(q, j, tiles_x);
      return true;
    }
  }
  return false;
}

// Held to 6 waves per SIMD (80 VGPRs at most; it fits in fewer).
// Persistent: a machine-filling grid whose waves each take 64-pixel tiles
// (tile_w x 64/tile_w) from the per-XCD, row-interleaved queues until the
// image is done, so that no wave idles while the slower waves of its
// work-group finish (ray costs vary widely per tile).  Waves that find every
// queue dry count themselves out; the last one clears the queues, so every
// launch starts from zero.
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6, 6))) void trace_kernel(TraceParams p) {
  __shared__ uint32_t stk[kStackLevels][kBlock];
  const uint32_t tid = threadIdx.x, lane = tid & 63;
  const uint32_t tw = p.tile_w, tw_log2 = __builtin_ctz(p.tile_w), th = 64u >> tw_log2;
  const uint32_t home = blockIdx.x % kQueues;
  const uint32_t tiles_y = p.total_tiles / p.tiles_x;
  uint32_t qi = 0;
  for (;;) {
    uint32_t t = 0;
    if (!take_row_tile(p.queue, p.tiles_x, tiles_y, home, lane, qi, t)) {
      if (lane == 0 && atomicAdd(&p.queue[kQueues * kQueueStride], 1u) == gridDim.x * (kBlock / 64) - 1) {
        for (uint32_t i = 0; i <= kQueues; i++) atomicExch(&p.queue[i * kQueueStride], 0u);
      }
      break;
    }
    __builtin_amdgcn_s_setprio(0);  // a new tile starts at the lowest priority
    const uint32_t x0 = (t % p.tiles_x) * tw, y0 = (t / p.tiles_x) * th;
    const uint32_t px = x0 + (lane & (tw - 1)), py = y0 + (lane >> tw_log2);
    uint4* out = reinterpret_cast<uint4*>(p.out);
    const uint32_t start = p.beam ? out[(size_t)y0 * p.W + x0].x : 0u;  // read before the tile is written
    if (px < p.W && py < p.H) out[(size_t)py * p.W + px] = trace_pixel(p, px, py, &stk[0][tid], kBlock, start);
  }
}

int trace_occupancy(uint32_t* blocks_per_cu) {
  int n = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, trace_kernel, kBlock, 0);
  if (e != hipSuccess || n < 1) return svd_fail(SVD_EDEVICE, "occupancy query failed");
  *blocks_per_cu = (uint32_t)n;
  return SVD_OK;
}

int launch_trace(const TraceParams& p, uint32_t blocks, void* stream, void* start, void* stop) {
  if (start || stop)
    hipExtLaunchKernelGGL(trace_kernel, dim3(blocks), dim3(kBlock), 0, (hipStream_t)stream, (hipEvent_t)start,
                          (hipEvent_t)stop, 0, p);
  else
    hipLaunchKernelGGL(trace_kernel, dim3(blocks), dim3(kBlock), 0, (hipStream_t)stream, p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return svd_fail(SVD_EDEVICE, "trace launch: %s", hipGetErrorString(e));
  return SVD_OK;
}

// ------------------------------------------------------------- beam pass
// ESVO's beam optimisation (Section 2.2: a coarse pass that moves the rays'
// starting points; Section 4.1 compares against it), made exact.  One lane
// per wave tile computes a lower bound d on the Chebyshev distance from the
// camera to every cell that a ray of the tile could hit: the minimum over
// the cubes that may hold such a cell (chunk tight boxes, then DAG children
// down to 2^3 sub-blocks of the picked LOD, or a whole chunk whose LOD is not
// loaded) that reach the cone of the tile's corner rays.  Every pixel ray of
// the tile lies in that cone (directions are affine in the pixel), and a
// ray point at time t < d 2^16 / max|D_a| is nearer than d in the Chebyshev
// norm, so it lies outside every such closed cube: the ray visits only empty
// cells before that time, and starting its walk there (same exact instant
// arithmetic as the world entry) changes no record.
//
// The cone test runs in FP32 with a margin that covers its rounding.  Side
// plane i has the exact i64 normal m_i = C_i x C_(i+1) (|C| < 2^31), scaled
// by a power of two so that its largest component lies in [1/2, 1), then
// rounded to FP32 (relative error <= 2^-24).  For a cube [lo, lo + s]
// (integer voxels in [0, 2^15], s <= 2^10) the largest value of n_i . (x - o)
// over it is
//   n_i . lo + s P_i - n_i . o,    P_i = sum of the positive components,
// evaluated with FMAs from the FP32 camera position o (in (-2^15, 2^16), so
// rounded by at most 2^-8 per axis).  Every partial sum stays below 2^18, so
// the four FMAs of the test err by at most 4 2^-6, the three of n_i . o by
// 9 2^-8, the normal's rounding by 3 2^-24 2^17 and the camera's by 3 2^-8:
// less than 0.14 together.  A cube is dropped
// only when that value is below -1.  Distances are integer: with of / oc the
// camera position rounded down / up to whole voxels, a cube is at least
// max(lo - oc, of - (lo + s), 0) voxels away on each axis.
struct BeamCone {
  float n[4][3];
  float pos[4];  // sum of the positive components of n_i
  float c[4];    // n_i . o
  int32_t of[3], oc[3];
  uint32_t mm;   // near-first octant order: bit a set when the tile looks down axis a
};

__host__ __device__ inline bool beam_cone(const BeamParams& p, uint32_t x0, uint32_t y0, uint32_t x1, uint32_t y1,
                                          BeamCone& q) {
  int64_t C[4][3];
  const uint32_t px[4] = {x0, x1, x1, x0}, py[4] = {y0, y0, y1, y1};
  _Pragma("unroll") for (int i = 0; i < 4; i++)
    _Pragma("unroll") for (int a = 0; a < 3; a++) C[i][a] = p.A[a] + (int64_t)px[i] * p.BX[a] + (int64_t)py[i] * p.BY[a];
  q.mm = 0;
  float o[3];
  _Pragma("unroll") for (int a = 0; a < 3; a++) {
    if (C[0][a] + C[2][a] < 0) q.mm |= 1u << a;
    o[a] = (float)((double)p.O[a] * (1.0 / 65536.0));
    q.of[a] = (int32_t)(p.O[a] >> 16);
    q.oc[a] = (int32_t)(-((-p.O[a]) >> 16));
  }
  _Pragma("unroll") for (int i = 0; i < 4; i++) {
    const int64_t* u = C[i];
    const int64_t* v = C[(i + 1) & 3];
    const int64_t m[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
    __int128 s0 = 0, s1 = 0;
    _Pragma("unroll") for (int a = 0; a < 3; a++) {
      s0 += (__int128)m[a] * C[(i + 2) & 3][a];
      s1 += (__int128)m[a] * C[(i + 3) & 3][a];
    }
    int sg;
    if (s0 >= 0 && s1 >= 0 && (s0 > 0 || s1 > 0)) sg = 1;
    else if (s0 <= 0 && s1 <= 0 && (s0 < 0 || s1 < 0)) sg = -1;
    else return false;  // degenerate cone (a one-pixel row or column)
    uint64_t big = 0;
    _Pragma("unroll") for (int a = 0; a < 3; a++) {
      const uint64_t am = m[a] < 0 ? (uint64_t)0 - (uint64_t)m[a] : (uint64_t)m[a];
      big = am > big ? am : big;
    }
    int e = 0;  // 2^e > big >= 2^(e-1): scale so the largest component is in [1/2, 1)
    while (e < 64 && (big >> e)) e++;
    q.pos[i] = 0.0f;
    q.c[i] = 0.0f;
    _Pragma("unroll") for (int a = 0; a < 3; a++) {
      q.n[i][a] = (float)sg * (float)ldexp((double)m[a], -e);
      q.pos[i] += q.n[i][a] > 0.0f ? q.n[i][a] : 0.0f;
      q.c[i] = fmaf(q.n[i][a], o[a], q.c[i]);
    }
  }
  return true;
}

// Closed cube [lo, lo + s] (voxels) entirely outside the cone?
__host__ __device__ __forceinline__ bool beam_outside(const BeamCone& q, const int32_t lo[3], int32_t s) {
  const float l0 = (float)lo[0], l1 = (float)lo[1], l2 = (float)lo[2], fs = (float)s;
  bool out = false;
  _Pragma("unroll") for (int i = 0; i < 4; i++) {
    const float v = fmaf(q.n[i][0], l0, fmaf(q.n[i][1], l1, fmaf(q.n[i][2], l2, fmaf(fs, q.pos[i], -q.c[i]))));
    out |= v < -1.0f;
  }
  return out;
}

// Chebyshev distance from the camera to the closed cube [lo, lo + s], in
// whole voxels rounded down, at most 65535.
__host__ __device__ __forceinline__ uint32_t beam_dist(const BeamCone& q, const int32_t lo[3], int32_t s) {
  int32_t d = 0;
  _Pragma("unroll") for (int a = 0; a < 3; a++) {
    const int32_t e0 = lo[a] - q.oc[a], e1 = q.of[a] - (lo[a] + s);
    d = e0 > d ? e0 : d;
    d = e1 > d ? e1 : d;
  }
  return (uint32_t)(d < 65535 ? d : 65535);
}

// Children mask with bit i standing for octant i ^ mm: the near-first order.
__host__ __device__ __forceinline__ uint32_t beam_order(uint32_t m, uint32_t mm) {
  if (mm & 1u) m = ((m & 0x55u) << 1) | ((m >> 1) & 0x55u);
  if (mm & 2u) m = ((m & 0x33u) << 2) | ((m >> 2) & 0x33u);
  if (mm & 4u) m = ((m & 0x0Fu) << 4) | ((m >> 4) & 0x0Fu);
  return m;
}

// Start bound of the tile with pixel corners (x0, y0)..(x1, y1).  Chunks are
// visited shell by shell around the camera's chunk, and inside each a
// depth-first walk of the DAG takes the near octants first; both are cut by
// the bound found so far.  One loop drives the shell walk and the DAG walk,
// so lanes of a wave at different stages of their tiles never wait on each
// other's inner loops.  `stk` holds the DAG path (two words per node level,
// element stride `ss`).
__host__ __device__ inline uint32_t beam_tile(const BeamParams& p, uint32_t x0, uint32_t y0, uint32_t x1, uint32_t y1,
                                              uint32_t* stk, uint32_t ss) {
  BeamCone q;
  if (!beam_cone(p, x0, y0, x1, y1, q)) return 0u;
  const int CL = (int)p.chunk_log2;
  const int32_t S = (int32_t)1 << CL;
  const int32_t g[3] = {(int32_t)p.grid[0], (int32_t)p.grid[1], (int32_t)p.grid[2]};
  int32_t c0[3], rmin = 0, rmax = 0;
  _Pragma("unroll") for (int a = 0; a < 3; a++) {
    c0[a] = q.of[a] >> CL;  // chunk of the camera (floor), maybe outside the grid
    const int32_t in = c0[a] < 0 ? -c0[a] : (c0[a] >= g[a] ? c0[a] - g[a] + 1 : 0);
    const int32_t out = c0[a] < 0 ? g[a] - 1 - c0[a] : (c0[a] >= g[a] ? c0[a] : (c0[a] > g[a] - 1 - c0[a] ? c0[a] : g[a] - 1 - c0[a]));
    rmin = in > rmin ? in : rmin;
    rmax = out > rmax ? out : rmax;
  }
  // Shell cursor: shell r (every axis range clipped to the grid is non-empty
  // from rmin on), row (y, z) in the clipped ranges, x across the row: every
  // cell on the shell's top and bottom faces and side rows, only the two ends
  // on the other rows.
  int32_t r = rmin;
  int32_t z = c0[2] - r < 0 ? 0 : c0[2] - r;
  int32_t y = c0[1] - r < 0 ? 0 : c0[1] - r;
  int32_t x = c0[0] - r;
  uint32_t best = kBeamNone;
  int L = 0;  // level of the DAG node being walked; 0 between chunks
  int k = 0;
  uint32_t wd = 0, rem = 0;
  int32_t org[3] = {0, 0, 0};
  gptr32 nodes = nullptr;
  for (;;) {
    if (L == 0) {
      // every chunk of shell r is at least (r - 1) chunks away on some axis
      if (r > rmax || (r >= 1 && best != kBeamNone && (uint32_t)((r - 1) * S) >= best)) break;
      const int32_t cx = x, cy = y, cz = z;
      const bool face = r == 0 || z == c0[2] - r || z == c0[2] + r || y == c0[1] - r || y == c0[1] + r;
      x += face ? 1 : 2 * r;
      if (x > c0[0] + r) {
        x = c0[0] - r;
        const int32_t yh = c0[1] + r >= g[1] ? g[1] - 1 : c0[1] + r;
        if (++y > yh) {
          y = c0[1] - r < 0 ? 0 : c0[1] - r;
          const int32_t zh = c0[2] + r >= g[2] ? g[2] - 1 : c0[2] + r;
          if (++z > zh) {
            r++;
            z = c0[2] - r < 0 ? 0 : c0[2] - r;
            y = c0[1] - r < 0 ? 0 : c0[1] - r;
            x = c0[0] - r;
          }
        }
      }
      if (cx < 0 || cx >= g[0]) continue;
      const uint32_t ci = (uint32_t)cx + p.grid[0] * ((uint32_t)cy + p.grid[1] * (uint32_t)cz);
      const uint32_t v = p.view[ci];
      if (v & (kViewCulled | kViewEmpty)) continue;
      k = (int)(v & kViewLodMask);
      org[0] = cx * S;
      org[1] = cy * S;
      org[2] = cz * S;
      if (v & kViewMissing) {  // rays must reach it to report it
        const uint32_t d = beam_dist(q, org, S);
        if (d < best && !beam_outside(q, org, S)) best = d;
        continue;
      }
      const DevDag* dag = &p.desc[(size_t)ci * 4 + k];
      nodes = (gptr32)dag->nodes;
      wd = dag->root;
      rem = beam_order(wd >> kPtrBits, q.mm);
      L = CL;
      continue;
    }
    if (rem == 0) {  // node done: back to its parent
      if (L == CL) {
        L = 0;
        continue;
      }
      L++;
      wd = stk[(2 * (L - 3)) * ss];
      rem = stk[(2 * (L - 3) + 1) * ss];
      _Pragma("unroll") for (int a = 0; a < 3; a++) org[a] &= ~((1 << L) - 1);
      continue;
    }
    const uint32_t o = (uint32_t)__builtin_ctz(rem) ^ q.mm;
    rem &= rem - 1u;
    const int32_t half = 1 << (L - 1);
    const int32_t lo[3] = {org[0] + ((o & 1) ? half : 0), org[1] + ((o & 2) ? half : 0),
                           org[2] + ((o & 4) ? half : 0)};
    const uint32_t d = beam_dist(q, lo, half);
    if (d >= best || beam_outside(q, lo, half)) continue;
    if (L - 1 == k + 1) {  // a 2^3 sub-block of a leaf: as fine as the bound goes
      best = d;
      continue;
    }
    const uint32_t cw = nodes[(wd & kPtrMask) + __builtin_popcount((wd >> kPtrBits) & ((1u << o) - 1u))];
    stk[(2 * (L - 3)) * ss] = wd;
    stk[(2 * (L - 3) + 1) * ss] = rem;
    L--;
    wd = cw;
    rem = beam_order(cw >> kPtrBits, q.mm);
    _Pragma("unroll") for (int a = 0; a < 3; a++) org[a] = lo[a];
  }
  return best;
}

constexpr int kBeamBlock = 64;

__global__ __launch_bounds__(kBeamBlock) void beam_kernel(BeamParams p) {
  __shared__ uint32_t stk[2 * kStackLevels][kBeamBlock];
  const uint32_t t = blockIdx.x * kBeamBlock + threadIdx.x;
  if (t >= p.total_tiles) return;
  const uint32_t th = 64 / p.tile_w;
  const uint32_t x0 = (t % p.tiles_x) * p.tile_w, y0 = (t / p.tiles_x) * th;
  const uint32_t x1 = min(x0 + p.tile_w, p.W) - 1, y1 = min(y0 + th, p.H) - 1;
  const uint32_t d = beam_tile(p, x0, y0, x1, y1, &stk[0][threadIdx.x], kBeamBlock);
  reinterpret_cast<uint32_t*>(p.out)[((size_t)y0 * p.W + x0) * 4] = d;
}

int launch_beam(const BeamParams& p, void* stream, void* start) {
  const uint32_t blocks = (p.total_tiles + kBeamBlock - 1) / kBeamBlock;
  if (start)
    hipExtLaunchKernelGGL(beam_kernel, dim3(blocks), dim3(kBeamBlock), 0, (hipStream_t)stream, (hipEvent_t)start,
                          nullptr, 0, p);
  else
    hipLaunchKernelGGL(beam_kernel, dim3(blocks), dim3(kBeamBlock), 0, (hipStream_t)stream, p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return svd_fail(SVD_EDEVICE, "beam launch: %s", hipGetErrorString(e));
  return SVD_OK;
}

// ----------------------------------------------------------- batched views
// Many views of uneven size in one pass: a chunk stage over (view, chunk)
// pairs, then a persistent trace whose waves take 64-pixel tiles of any
// view from one work queue, so small views fill the machine as well as large
// ones.  All per-batch values come from device memory (BatchHeader and
// BatchView), so the three launches are captured once as a graph.
// Zero the queue counters and the done counter that follows them.
__global__ void batch_reset_kernel(uint32_t* queue) {
  if (threadIdx.x <= kQueues) queue[threadIdx.x * kQueueStride] = 0;
}

int launch_queue_clear(uint32_t* queue, void* stream) {
  hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, queue);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return svd_fail(SVD_EDEVICE, "queue clear launch: %s", hipGetErrorString(e));
  return SVD_OK;
}

__global__ void batch_stage_kernel(BatchParams p) {
  const uint32_t v = blockIdx.y;
  const uint32_t ci = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= p.hdr->nviews || ci >= p.nchunks) return;
  const BatchView& bv = p.views[v];
  StageParams sp;
  _Pragma("unroll") for (int a = 0; a < 3; a++) {
    sp.O[a] = bv.O[a];
    sp.grid[a] = p.grid[a];
    sp.thr[a] = p.thr[a];
    _Pragma("unroll") for (int i = 0; i < 4; i++) sp.n[i][a] = bv.n[i][a];
  }
  sp.chunk_log2 = p.chunk_log2;
  sp.lod_count = p.lod_count;
  sp.cull = bv.cull;
  sp.nchunks = p.nchunks;
  sp.desc = p.desc;
  sp.view = nullptr;
  p.view_tables[(size_t)v * p.nchunks + ci] = stage_chunk(sp, ci);
}

// Held to 80 VGPRs (6 blocks of 4 waves per CU), which it fits without
// spilling; left alone the compiler takes 83 and only 5 blocks fit.
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6, 6))) void batch_trace_kernel(BatchParams p) {
  __shared__ uint32_t stk[kStackLevels][kBlock];
  const uint32_t tid = threadIdx.x, lane = tid & 63;
  const uint32_t total = p.hdr->total_tiles, nviews = p.hdr->nviews;
  const uint32_t claim = p.hdr->claim, tw = p.hdr->tile_w, th = 64 / tw, beam = p.hdr->beam;
  const uint32_t home = blockIdx.x % kQueues;
  uint32_t qi = 0;
  for (;;) {
    // one queue access per wave: lane 0 claims, the wave shares the index
    uint32_t t0 = 0, t1 = 0;
    if (!take_tiles(p.queue, total, claim, home, lane, qi, t0, t1)) break;
    for (uint32_t t = t0; t < t1; t++) {
      __builtin_amdgcn_s_setprio(0);  // a new tile starts at the lowest priority
      uint32_t lo = 0, hi = nviews;  // view holding global tile t
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (p.views[mid].tile_base <= t) lo = mid; else hi = mid;
      }
      const BatchView& bv = p.views[lo];
      const uint32_t lt = t - bv.tile_base;
      const uint32_t x0 = (lt % bv.tiles_x) * tw, y0 = (lt / bv.tiles_x) * th;
      const uint32_t px = x0 + lane % tw, py = y0 + lane / tw;
      uint4* out = reinterpret_cast<uint4*>(bv.out);
      const uint32_t start = beam ? out[(size_t)y0 * bv.W + x0].x : 0u;  // read before the tile is written
      if (px >= bv.W || py >= bv.H) continue;
      TraceParams tp;
      _Pragma("unroll") for (int a = 0; a < 3; a++) {
        tp.O[a] = bv.O[a];
        tp.A[a] = bv.A[a];
        tp.BX[a] = bv.BX[a];
        tp.BY[a] = bv.BY[a];
        tp.grid[a] = p.grid[a];
      }
      tp.chunk_log2 = p.chunk_log2;
      tp.view = p.view_tables + (size_t)lo * p.nchunks;
      tp.desc = p.desc;
      out[(size_t)py * bv.W + px] = trace_pixel(tp, px, py, &stk[0][tid], kBlock, start);
    }
  }
}

int batch_trace_occupancy(uint32_t* blocks_per_cu) {
  int n = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_trace_kernel, kBlock, 0);
  if (e != hipSuccess || n < 1) return svd_fail(SVD_EDEVICE, "occupancy query failed");
  *blocks_per_cu = (uint32_t)n;
  return SVD_OK;
}

// Beam pass over every tile of the batch (grid-stride: the grid is fixed when
// the graph is captured).
__global__ __launch_bounds__(kBeamBlock) void batch_beam_kernel(BatchParams p) {
  __shared__ uint32_t stk[2 * kStackLevels][kBeamBlock];
  if (!p.hdr->beam) return;
  const uint32_t total = p.hdr->total_tiles, nviews = p.hdr->nviews;
  const uint32_t tw = p.hdr->tile_w, th = 64 / tw;
  for (uint32_t t = blockIdx.x * kBeamBlock + threadIdx.x; t < total; t += gridDim.x * kBeamBlock) {
    uint32_t lo = 0, hi = nviews;  // view holding global tile t
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (p.views[mid].tile_base <= t) lo = mid; else hi = mid;
    }
    const BatchView& bv = p.views[lo];
    BeamParams bp;
    _Pragma("unroll") for (int a = 0; a < 3; a++) {
      bp.O[a] = bv.O[a];
      bp.A[a] = bv.A[a];
      bp.BX[a] = bv.BX[a];
      bp.BY[a] = bv.BY[a];
      bp.grid[a] = p.grid[a];
    }
    bp.W = bv.W;
    bp.H = bv.H;
    bp.tiles_x = bv.tiles_x;
    bp.tile_w = tw;
    bp.chunk_log2 = p.chunk_log2;
    bp.view = p.view_tables + (size_t)lo * p.nchunks;
    bp.desc = p.desc;
    const uint32_t lt = t - bv.tile_base;
    const uint32_t x0 = (lt % bv.tiles_x) * tw, y0 = (lt / bv.tiles_x) * th;
    const uint32_t x1 = min(x0 + tw, bv.W) - 1, y1 = min(y0 + th, bv.H) - 1;
    const uint32_t d = beam_tile(bp, x0, y0, x1, y1, &stk[0][threadIdx.x], kBeamBlock);
    reinterpret_cast<uint32_t*>(bv.out)[((size_t)y0 * bv.W + x0) * 4] = d;
  }
}

int launch_batch(const BatchParams& p, uint32_t trace_blocks, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, s, p.queue);
  hipLaunchKernelGGL(batch_stage_kernel, dim3((p.nchunks + 63) / 64, p.max_views), dim3(64), 0, s, p);
  // one-wave beam blocks, twice as many waves as the trace: the beam walk is
  // latency-bound, and blocks past the last tile (or of a batch without the
  // beam) exit at once
  hipLaunchKernelGGL(batch_beam_kernel, dim3(trace_blocks * 8), dim3(kBeamBlock), 0, s, p);
  hipLaunchKernelGGL(batch_trace_kernel, dim3(trace_blocks), dim3(kBlock), 0, s, p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return svd_fail(SVD_EDEVICE, "batch launch: %s", hipGetErrorString(e));
  return SVD_OK;
}

int launch_batch_direct(const BatchParams& p, uint32_t views, uint32_t trace_blocks, bool beam, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, s, p.queue);
  hipLaunchKernelGGL(batch_stage_kernel, dim3((p.nchunks + 63) / 64, views), dim3(64), 0, s, p);
  if (beam) hipLaunchKernelGGL(batch_beam_kernel, dim3(trace_blocks * 8), dim3(kBeamBlock), 0, s, p);
  hipLaunchKernelGGL(batch_trace_kernel, dim3(trace_blocks), dim3(kBlock), 0, s, p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return svd_fail(SVD_EDEVICE, "batch launch: %s", hipGetErrorString(e));
  return SVD_OK;
}

// ------------------------------------------------------ allocation-free batch
// Batch area of svd_batch_trace_frames_static (queue block, header, views,
// per-(view, chunk) tables), kStaticScratchBytes per GPU, held until the
// process ends.  In host code `scratch` names a host-side stand-in, not
// device memory: host code only ever uses the device address that
// hipGetSymbolAddress returns for the current device (static_device).
static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

int static_device(StaticDevice* out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static StaticDevice dev_state[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return svd_fail(SVD_EDEVICE, "static batch: hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return svd_fail(SVD_EDEVICE, "static batch: device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(mu);
  StaticDevice& d = dev_state[dev];
  if (!d.scratch) {
    uint8_t* ptr = nullptr;
    e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return svd_fail(SVD_EDEVICE, "static batch: hipGetSymbolAddress: %s", hipGetErrorString(e));
    int cus = 0, n = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess || cus < 1) return svd_fail(SVD_EDEVICE, "static batch: cannot query the device");
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_trace_kernel, kBlock, 0);
    if (e != hipSuccess || n < 1) return svd_fail(SVD_EDEVICE, "static batch: occupancy query failed");
    d.cus = (uint32_t)cus;
    d.per_cu = (uint32_t)n;
    d.scratch = ptr;  // set last: a set-up that failed is retried on the next call
  }
  *out = d;
  return SVD_OK;
}

// Views travel as kernel arguments, so no host staging buffer (and no copy
// from host memory) is needed; a block copies them word by word.
struct ViewPack {
  uint32_t hdr[sizeof(BatchHeader) / 4];
  uint32_t count, with_hdr, pad[2];
  uint32_t words[kPackViews * (sizeof(BatchView) / 4)];
};

__global__ __launch_bounds__(256) void set_views_kernel(uint32_t* dst, uint32_t* hdr_dst, ViewPack pk) {
  const uint32_t t = threadIdx.x, n = pk.count * (uint32_t)(sizeof(BatchView) / 4);
  for (uint32_t i = t; i < n; i += 256) dst[i] = pk.words[i];
  if (pk.with_hdr && t < sizeof(BatchHeader) / 4) hdr_dst[t] = pk.hdr[t];
}

int launch_set_views(BatchView* dst, const BatchView* src, uint32_t count, BatchHeader* hdr_dst,
                     const BatchHeader* hdr, void* stream) {
  if (count > kPackViews) return svd_fail(SVD_EINVAL, "internal: view pack > %u", kPackViews);
  ViewPack pk;
  memset(&pk, 0, sizeof(pk));
  if (hdr) memcpy(pk.hdr, hdr, sizeof(BatchHeader));
  pk.count = count;
  pk.with_hdr = hdr != nullptr;
  memcpy(pk.words, src, (size_t)count * sizeof(BatchView));
  hipLaunchKernelGGL(set_views_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream, reinterpret_cast<uint32_t*>(dst),
                     reinterpret_cast<uint32_t*>(hdr_dst), pk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return svd_fail(SVD_EDEVICE, "view pack launch: %s", hipGetErrorString(e));
  return SVD_OK;
}

}  // namespace svd
