// gfx950 kernels of libsvdag: per-view chunk stage and per-pixel SVDAG trace.
//
// Traversal (Section 3.5 ray marching, made exact).  A ray is
// p(t) = (O + t D) / 2^16 voxels with integer O, D.  A time is a rational
// Nt/Dt plus a phase (0 = at t, 1 = just after t); a boundary crossing on an
// axis with D > 0 takes effect at t, one with D < 0 just after t, so events
// are ordered by (t, class) and equal keys are stepped together.  Every
// comparison is a cross-multiplication of 32-bit values (one v_mad_u64_u32),
// with no division in the loop.
//
// The walk is one hierarchy: chunk grid (level chunk_log2, in voxels), the
// chunk's DAG levels down to 8^3 nodes (level k+3 for LOD k), the 4^3 leaf
// bitmap (k+2), its 2^3 sub-blocks (k+1) and cells (k).  At a non-empty node
// the child containing the current instant is found with three mid-plane
// tests; an empty child is left by one exact step at its level, followed by
// a pop to the lowest common ancestor of the old and new cells (highest
// differing coordinate bit).  The node words of the current path live in LDS.
#include <hip/hip_runtime.h>

#include "svdag_internal.h"

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
__global__ void chunk_stage_kernel(StageParams p) {
  const uint32_t ci = blockIdx.x * blockDim.x + threadIdx.x;
  if (ci >= p.nchunks) return;
  const uint32_t cc[3] = {ci % p.grid[0], (ci / p.grid[0]) % p.grid[1], ci / (p.grid[0] * p.grid[1])};
  const int64_t S = (int64_t)1 << p.chunk_log2;
  unsigned __int128 d2 = 0;
  for (int a = 0; a < 3; a++) {
    const __int128 diff = (__int128)p.O[a] - (__int128)(((int64_t)cc[a] * S + S / 2) << 16);
    d2 += (unsigned __int128)(diff * diff);
  }
  uint32_t k = 0;
  for (uint32_t j = 0; j + 1 < p.lod_count; j++) {
    const unsigned __int128 t = (unsigned __int128)p.thr[j] << 16;
    if (d2 >= t * t) k++;
  }
  const DevDag& d = p.desc[(size_t)ci * 4 + k];
  uint32_t v = k;
  if (d.solid == 0) {
    v |= kViewEmpty;
  } else if (p.cull) {
    __int128 lo[3], hi[3];
    for (int a = 0; a < 3; a++) {
      const int64_t base = (int64_t)cc[a] * S;
      lo[a] = ((__int128)(base + ((int64_t)d.lo[a] << k)) << 16) - p.O[a];
      hi[a] = ((__int128)(base + ((int64_t)(d.hi[a] + 1) << k)) << 16) - p.O[a];
    }
    bool culled = false;
    for (int i = 0; i < 4; i++) {
      __int128 s = 0;
      for (int a = 0; a < 3; a++) s += (__int128)p.n[i][a] * (p.n[i][a] >= 0 ? hi[a] : lo[a]);
      if (s < 0) culled = true;
    }
    if (culled) v |= kViewCulled;
  }
  p.view[ci] = v;
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
constexpr int kBlock = 256;      // 4 waves; each wave is one 8x8 pixel tile
constexpr int kStackLevels = 8;  // node levels 3..10
constexpr uint32_t kMaxIter = 1u << 22;
constexpr uint32_t kFaultChunk = 0xFFFFFFFEu;

// Is p_a >= X (fixed point) at the current instant?
__device__ __forceinline__ bool plane_ge(int64_t X, int64_t O, int dsg, uint32_t ad, uint32_t Nt,
                                         uint32_t Dt, uint32_t ph) {
  const int64_t U = X - O;
  if (dsg > 0) return U <= 0 || (uint64_t)(uint32_t)U * Dt <= (uint64_t)Nt * ad;
  if (dsg < 0) {
    if (U > 0) return false;
    const uint64_t l = (uint64_t)Nt * ad, r = (uint64_t)(uint32_t)(-U) * Dt;
    return ph ? (l < r) : (l <= r);
  }
  return U <= 0;
}

// 8-bit mask of the non-empty bytes of a leaf bitmap (= non-empty 2^3 sub-blocks).
__device__ __forceinline__ uint32_t leaf_summary(uint64_t b) {
  b |= b >> 4;
  b |= b >> 2;
  b |= b >> 1;
  b &= 0x0101010101010101ull;
  return (uint32_t)((b * 0x0102040810204080ull) >> 56);
}

__global__ __launch_bounds__(kBlock) void trace_kernel(TraceParams p) {
  __shared__ uint32_t stk[kStackLevels][kBlock];
  const uint32_t tid = threadIdx.x;
  // Work-groups are dealt to the 8 XCDs round-robin; give each XCD a
  // contiguous run of 16x16 pixel blocks so that its L2 sees neighbouring
  // rays.
  const uint32_t per_xcd = (p.nblocks + 7) / 8;
  const uint32_t blk = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (blk >= p.nblocks) return;
  const uint32_t lane = tid & 63, wv = tid >> 6;
  const uint32_t px = (blk % p.tiles_x) * 16 + (wv & 1) * 8 + (lane & 7);
  const uint32_t py = (blk / p.tiles_x) * 16 + (wv >> 1) * 8 + (lane >> 3);
  if (px >= p.W || py >= p.H) return;

  const int CL = (int)p.chunk_log2;
  int dsg[3];
  uint32_t ad[3];
  int32_t D[3];
  for (int a = 0; a < 3; a++) {
    D[a] = (int32_t)(p.A[a] + (int64_t)px * p.BX[a] + (int64_t)py * p.BY[a]);
    dsg[a] = (D[a] > 0) - (D[a] < 0);
    ad[a] = (uint32_t)(D[a] < 0 ? -(int64_t)D[a] : (int64_t)D[a]);
  }

  // World entry: the latest lower bound of the per-axis slab intervals.
  uint32_t Nt = 0, Dt = 1, ph = 0;
  for (int a = 0; a < 3; a++) {
    uint32_t n = 0, cls = 0;
    bool cand = false;
    if (dsg[a] > 0 && p.O[a] < 0) { n = (uint32_t)(-p.O[a]); cls = 0; cand = true; }
    if (dsg[a] < 0) {
      const int64_t v = p.O[a] - ((int64_t)p.grid[a] << (CL + 16));
      if (v >= 0) { n = (uint32_t)v; cls = 1; cand = true; }
    }
    if (!cand) continue;
    const uint64_t l = (uint64_t)n * Dt, r = (uint64_t)Nt * ad[a];
    if (l > r || (l == r && cls > ph)) { Nt = n; Dt = ad[a]; ph = cls; }
  }

  uint4 rec = make_uint4(0u, 0u, __float_as_uint(__builtin_inff()), 0xFFFFFFFFu);
  bool inside = true;
  for (int a = 0; a < 3; a++) {
    const int64_t ext = (int64_t)p.grid[a] << (CL + 16);
    inside = inside && plane_ge(0, p.O[a], dsg[a], ad[a], Nt, Dt, ph) &&
             !plane_ge(ext, p.O[a], dsg[a], ad[a], Nt, Dt, ph);
  }
  if (inside) {
    // cell coordinates at the entry instant: one exact division per axis
    int32_t c[3];
    for (int a = 0; a < 3; a++) {
      const uint64_t v = (uint64_t)(p.O[a] * (int64_t)Dt + (int64_t)Nt * D[a]);  // p * 2^16 * Dt >= 0
      const uint64_t den = (uint64_t)Dt << 16;
      uint64_t q = v / den;
      if (dsg[a] < 0 && ph && q * den == v) q -= 1;
      c[a] = (int32_t)(q >> CL);
    }
    int lev = CL, k = 0;
    bool at_chunk = true;
    uint32_t mask = 0, ptr = 0, ci = 0;
    uint64_t bitmap = 0;
    const uint32_t* nodes = nullptr;
    const uint64_t* leaves = nullptr;
    const DevDag* dag = nullptr;
    uint32_t iter = 0;
    for (;;) {
      if (++iter > kMaxIter) { rec.w = kFaultChunk; break; }
      bool step = false;
      if (at_chunk) {
        if (c[0] < 0 || c[1] < 0 || c[2] < 0 || c[0] >= (int32_t)p.grid[0] || c[1] >= (int32_t)p.grid[1] ||
            c[2] >= (int32_t)p.grid[2])
          break;  // left the world: miss
        ci = (uint32_t)c[0] + p.grid[0] * ((uint32_t)c[1] + p.grid[1] * (uint32_t)c[2]);
        const uint32_t v = p.view[ci];
        if (v & (kViewCulled | kViewEmpty)) {
          step = true;
        } else {
          k = (int)(v & kViewLodMask);
          dag = &p.desc[(size_t)ci * 4 + k];
          nodes = (const uint32_t*)dag->nodes;
          leaves = (const uint64_t*)dag->leaves;
          const uint32_t root = dag->root;
          stk[CL - 3][tid] = root;
          mask = root >> kPtrBits;
          ptr = 0;
          at_chunk = false;
        }
      }
      if (!step) {
        // descend: child octant of the current instant inside cell c (level lev)
        uint32_t oct = 0;
        for (int a = 0; a < 3; a++) {
          const int64_t X = (int64_t)(2 * c[a] + 1) << (lev - 1 + 16);
          const uint32_t bit = plane_ge(X, p.O[a], dsg[a], ad[a], Nt, Dt, ph) ? 1u : 0u;
          c[a] = 2 * c[a] + (int32_t)bit;
          oct |= bit << a;
        }
        lev--;
        if ((mask >> oct) & 1u) {
          if (lev == k) {
            // ---- hit: DFS index (Section 3.3), material, t, face
            const uint32_t* pre = (const uint32_t*)dag->pre;
            uint32_t dfs = 0;
            for (int L = CL; L >= k + 3; L--) {
              const uint32_t w = stk[L - 3][tid];
              const int s = L - 1 - k;
              const uint32_t o = ((c[0] >> s) & 1) | (((c[1] >> s) & 1) << 1) | (((c[2] >> s) & 1) << 2);
              dfs += pre[(w & kPtrMask) + __builtin_popcount((w >> kPtrBits) & ((1u << o) - 1u))];
            }
            const uint32_t o1 = ((c[0] >> 1) & 1) | (((c[1] >> 1) & 1) << 1) | (((c[2] >> 1) & 1) << 2);
            const uint32_t o0 = (c[0] & 1) | ((c[1] & 1) << 1) | ((c[2] & 1) << 2);
            const uint32_t b = 8 * o1 + o0;
            dfs += (uint32_t)__builtin_popcountll(bitmap & ((1ull << b) - 1ull));
            const uint32_t* rs = (const uint32_t*)dag->rle_start;
            uint32_t lo = 0, hi = dag->rle_n;
            while (hi - lo > 1) {
              const uint32_t mid = (lo + hi) >> 1;
              if (rs[mid] <= dfs) lo = mid; else hi = mid;
            }
            const uint32_t mat = ((const uint8_t*)dag->rle_mat)[lo];
            uint32_t face = 0;
            for (int a = 0; a < 3 && !face; a++) {
              if (!dsg[a]) continue;
              const int64_t X = (int64_t)(dsg[a] > 0 ? c[a] : c[a] + 1) << (k + 16);
              const int64_t ne = dsg[a] > 0 ? X - p.O[a] : p.O[a] - X;
              const uint32_t cls = dsg[a] < 0;
              if (ne >= 0 && cls == ph && (uint64_t)ne * Dt == (uint64_t)Nt * ad[a]) face = 1 + 2 * a + cls;
            }
            const double len = sqrt((double)D[0] * D[0] + (double)D[1] * D[1] + (double)D[2] * D[2]);
            const float t = (float)(((double)Nt / (double)Dt) * len * (1.0 / 65536.0));
            rec.x = ((uint32_t)c[0] << k) | (((uint32_t)c[1] << k) << 16);
            rec.y = ((uint32_t)c[2] << k) | ((uint32_t)k << 16) | (face << 20) | (1u << 23) | (mat << 24);
            rec.z = __float_as_uint(t);
            rec.w = ci;
            break;
          }
          if (lev >= k + 3) {
            const uint32_t w = nodes[ptr + __builtin_popcount(mask & ((1u << oct) - 1u))];
            stk[lev - 3][tid] = w;
            mask = w >> kPtrBits;
            ptr = w & kPtrMask;
          } else if (lev == k + 2) {
            const uint32_t w = nodes[ptr + __builtin_popcount(mask & ((1u << oct) - 1u))];
            bitmap = leaves[w & kPtrMask];
            mask = leaf_summary(bitmap);
          } else {
            mask = (uint32_t)(bitmap >> (8 * oct)) & 0xFFu;
          }
          continue;
        }
      }
      // ---- step out of the empty cell c at level lev
      uint32_t bn = 0, bd = 1, bc = 0, smask = 0;
      for (int a = 0; a < 3; a++) {
        if (!dsg[a]) continue;
        const int64_t X = (int64_t)(dsg[a] > 0 ? c[a] + 1 : c[a]) << (lev + 16);
        const uint32_t n = (uint32_t)(dsg[a] > 0 ? X - p.O[a] : p.O[a] - X);
        const uint32_t cls = dsg[a] < 0;
        if (!smask) { bn = n; bd = ad[a]; bc = cls; smask = 1u << a; continue; }
        const uint64_t l = (uint64_t)n * bd, r = (uint64_t)bn * ad[a];
        if (l < r || (l == r && cls < bc)) { bn = n; bd = ad[a]; bc = cls; smask = 1u << a; }
        else if (l == r && cls == bc) smask |= 1u << a;
      }
      if (!smask) break;  // D == 0: the ray never leaves this cell
      Nt = bn; Dt = bd; ph = bc;
      uint32_t diff = 0;
      for (int a = 0; a < 3; a++) {
        if (!((smask >> a) & 1)) continue;
        const int32_t nc = c[a] + dsg[a];
        diff |= (uint32_t)(nc ^ c[a]);
        c[a] = nc;
      }
      const int pl = lev + (32 - __builtin_clz(diff));  // lowest common ancestor level
      if (pl > CL) {
        for (int a = 0; a < 3; a++) c[a] >>= (CL - lev);
        lev = CL;
        at_chunk = true;
        continue;
      }
      for (int a = 0; a < 3; a++) c[a] >>= (pl - lev);
      lev = pl;
      if (lev >= k + 3) {
        const uint32_t w = stk[lev - 3][tid];
        mask = w >> kPtrBits;
        ptr = w & kPtrMask;
      } else if (lev == k + 2) {
        mask = leaf_summary(bitmap);
      } else {
        const uint32_t o1 = (c[0] & 1) | ((c[1] & 1) << 1) | ((c[2] & 1) << 2);
        mask = (uint32_t)(bitmap >> (8 * o1)) & 0xFFu;
      }
    }
  }
  reinterpret_cast<uint4*>(p.out)[(size_t)py * p.W + px] = rec;
}

int launch_trace(const TraceParams& p, void* stream) {
  const uint32_t blocks = (p.nblocks + 7) / 8 * 8;
  hipLaunchKernelGGL(trace_kernel, dim3(blocks), dim3(kBlock), 0, (hipStream_t)stream, p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return svd_fail(SVD_EDEVICE, "trace launch: %s", hipGetErrorString(e));
  return SVD_OK;
}

}  // namespace svd
