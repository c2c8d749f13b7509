// Test infrastructure: the library's kernel logic (chunk stage, beam pass,
// per-pixel trace from kernels.hip) run on the host over the same device
// images, so CPU-only test runs check it against the oracle; likewise the GPU
// scene generator's per-element code, checked against the host generator.  Not part of
// libsvdag; nothing here touches a GPU.
#include <cstdint>

// Walk events of trace_pixel, counted per host thread (see hk_trace_counts).
struct WalkCounts {
  uint64_t iter, descend, exit, sibling, pop, chunk_next, chunk_visit, chunk_enter, hit;
};
static thread_local WalkCounts g_walk;
#ifdef __HIP_DEVICE_COMPILE__
#define SVD_WALK_EVENT(e) do {} while (0)  // the device pass of this host-only file counts nothing
#else
#define SVD_WALK_EVENT(e) (g_walk.e++)
#endif

#include "kernels.hip"
#include "../paper_2505_02017_amd/scenes/scenegen_gpu.hip"

#include <algorithm>
#include <cstring>
#include <thread>
#include <vector>

using namespace svd;

struct HkWorld {
  svd_world_desc desc;
  uint32_t n = 0;
  std::vector<DevDag> tab;                   // descriptor table, addresses into `image`
  std::vector<std::vector<uint8_t>> image;   // per chunk: the blob's device image
};

extern "C" HkWorld* hk_world_new(const svd_world_desc* d) {
  HkWorld* w = new HkWorld();
  w->desc = *d;
  w->n = d->grid[0] * d->grid[1] * d->grid[2];
  w->tab.assign((size_t)w->n * 4, DevDag());
  memset(w->tab.data(), 0, w->tab.size() * sizeof(DevDag));
  w->image.resize(w->n);
  return w;
}

extern "C" void hk_world_free(HkWorld* w) { delete w; }

// All LODs of b as chunk ci (a copy of its device image), or only their
// descriptions (addresses zero) when `describe_only`.
extern "C" int hk_upload(HkWorld* w, uint32_t ci, const svd_blob* b, int describe_only) {
  if (ci >= w->n || b->lod_count != w->desc.lod_count) return SVD_EINVAL;
  w->image[ci] = b->image;
  const uint64_t base = (uint64_t)(uintptr_t)w->image[ci].data();
  for (uint32_t k = 0; k < 4; k++) {
    DevDag& d = w->tab[(size_t)ci * 4 + k];
    memset(&d, 0, sizeof(d));
    if (k >= b->lod_count) continue;
    const LodData& L = b->lod[k];
    if (!describe_only) {
      d.nodes = base + L.off_nodes;
      d.leaves = base + L.off_leaves;
      d.pre = base + L.off_pre;
      d.rle_start = base + L.off_rle_start;
      d.rle_dir = base + L.off_rle_dir;
    }
    d.rle_n = (uint32_t)L.rle_start.size();
    d.root = L.root_word;
    d.solid = L.n_solid;
    for (int a = 0; a < 3; a++) {
      d.lo[a] = L.lo[a];
      d.hi[a] = L.hi[a];
    }
  }
  return SVD_OK;
}

// Stage, optional beam pass (16x4 tiles, as the per-view launch) and trace
// of every pixel; records in `out` (width*height x 16 bytes), the view table
// in `view_out` (may be NULL).  With `counts` (may be NULL), the walk events
// summed over all pixels, in WalkCounts order, then per 64-pixel tile the
// largest count of inner-loop iterations of one pixel, summed over tiles, and
// the number of tiles.
static int trace_impl(HkWorld* w, const svd_ray_frame* f, uint32_t flags, svd_hit* out, uint32_t* view_out,
                      uint32_t threads, uint64_t* counts);

extern "C" int hk_trace(HkWorld* w, const svd_ray_frame* f, uint32_t flags, svd_hit* out, uint32_t* view_out,
                        uint32_t threads) {
  return trace_impl(w, f, flags, out, view_out, threads, nullptr);
}

extern "C" int hk_trace_counts(HkWorld* w, const svd_ray_frame* f, uint32_t flags, svd_hit* out, uint32_t threads,
                               uint64_t* counts) {
  return trace_impl(w, f, flags, out, nullptr, threads, counts);
}

static int trace_impl(HkWorld* w, const svd_ray_frame* f, uint32_t flags, svd_hit* out, uint32_t* view_out,
                      uint32_t threads, uint64_t* counts) {
  StageParams sp;
  memset(&sp, 0, sizeof(sp));
  memcpy(sp.O, f->O, sizeof(sp.O));
  sp.cull = !(flags & SVD_NO_CULL) && cull_planes(f, sp.n);
  memcpy(sp.grid, w->desc.grid, sizeof(sp.grid));
  sp.chunk_log2 = w->desc.chunk_log2;
  sp.lod_count = w->desc.lod_count;
  memcpy(sp.thr, w->desc.lod_threshold, sizeof(sp.thr));
  sp.nchunks = w->n;
  sp.desc = w->tab.data();
  std::vector<uint32_t> view(w->n);
  for (uint32_t ci = 0; ci < w->n; ci++) view[ci] = host_stage_chunk(sp, ci);
  if (view_out) memcpy(view_out, view.data(), w->n * 4);

  const uint32_t W = f->width, H = f->height;
  const uint32_t tw = kViewTileW, th = 64 / kViewTileW;
  const uint32_t tiles_x = (W + tw - 1) / tw, tiles_y = (H + th - 1) / th;
  std::vector<uint32_t> start((size_t)tiles_x * tiles_y, 0);
  BeamParams bp;
  memset(&bp, 0, sizeof(bp));
  memcpy(bp.O, f->O, sizeof(bp.O));
  memcpy(bp.A, f->A, sizeof(bp.A));
  memcpy(bp.BX, f->BX, sizeof(bp.BX));
  memcpy(bp.BY, f->BY, sizeof(bp.BY));
  bp.W = W;
  bp.H = H;
  memcpy(bp.grid, w->desc.grid, sizeof(bp.grid));
  bp.chunk_log2 = w->desc.chunk_log2;
  bp.view = view.data();
  bp.desc = w->tab.data();
  TraceParams tp;
  memset(&tp, 0, sizeof(tp));
  memcpy(tp.O, f->O, sizeof(tp.O));
  memcpy(tp.A, f->A, sizeof(tp.A));
  memcpy(tp.BX, f->BX, sizeof(tp.BX));
  memcpy(tp.BY, f->BY, sizeof(tp.BY));
  tp.W = W;
  tp.H = H;
  memcpy(tp.grid, w->desc.grid, sizeof(tp.grid));
  tp.chunk_log2 = w->desc.chunk_log2;
  tp.view = view.data();
  tp.desc = w->tab.data();

  const uint32_t nt = std::max(1u, std::min(threads, 64u));
  constexpr int kEvents = sizeof(WalkCounts) / sizeof(uint64_t);
  std::vector<uint64_t> part((size_t)nt * (kEvents + 2), 0);
  auto run_rows = [&](uint32_t t0) {
    g_walk = WalkCounts{};
    uint64_t* mine = &part[(size_t)t0 * (kEvents + 2)];
    for (uint32_t ty = t0; ty < tiles_y; ty += nt) {
      for (uint32_t tx = 0; tx < tiles_x; tx++) {
        uint64_t tile_max = 0;
        uint32_t s = 0;
        if (flags & SVD_BEAM) {
          uint32_t bstk[2 * 8];
          const uint32_t x0 = tx * tw, y0 = ty * th;
          s = beam_tile(bp, x0, y0, std::min(x0 + tw, W) - 1, std::min(y0 + th, H) - 1, bstk, 1);
        }
        start[(size_t)ty * tiles_x + tx] = s;
        for (uint32_t py = ty * th; py < std::min((ty + 1) * th, H); py++)
          for (uint32_t px = tx * tw; px < std::min((tx + 1) * tw, W); px++) {
            uint32_t stk[8];
            const uint64_t it0 = g_walk.iter;
            const uint4 r = trace_pixel(tp, px, py, stk, 1, s);
            tile_max = std::max<uint64_t>(tile_max, g_walk.iter - it0);
            svd_hit& h = out[(size_t)py * W + px];
            h.xy = r.x;
            h.zf = r.y;
            memcpy(&h.t, &r.z, 4);
            h.chunk = r.w;
          }
        mine[kEvents] += tile_max;
        mine[kEvents + 1] += 1;
      }
    }
    memcpy(mine, &g_walk, sizeof(WalkCounts));
  };
  std::vector<std::thread> pool;
  for (uint32_t t = 0; t < nt; t++) pool.emplace_back(run_rows, t);
  for (auto& t : pool) t.join();
  if (counts) {
    for (int e = 0; e < kEvents + 2; e++) {
      counts[e] = 0;
      for (uint32_t t = 0; t < nt; t++) counts[e] += part[(size_t)t * (kEvents + 2) + e];
    }
  }
  return SVD_OK;
}

// The per-view trace's row-interleaved tile queues: every tile of queue 0,
// then of queue 1, ... into `out` (room for tiles_x * tiles_y); returns the
// count.
extern "C" uint32_t hk_row_queue_tiles(uint32_t tiles_x, uint32_t tiles_y, uint32_t* out) {
  uint32_t n = 0;
  for (uint32_t q = 0; q < kQueues; q++)
    for (uint32_t j = 0; j < row_queue_tiles(q, tiles_x, tiles_y); j++) out[n++] = row_queue_tile(q, j, tiles_x);
  return n;
}

// The beam pass's cone test and distance for one tile and one cube, as the
// kernels evaluate them: returns -1 for a degenerate cone, else 1 when the
// cube [lo, lo + s] is dropped as outside the cone; *dist gets the cube's
// distance bound in voxels.
extern "C" int hk_beam_cube(const int64_t O[3], const int64_t A[3], const int64_t BX[3], const int64_t BY[3],
                            uint32_t x0, uint32_t y0, uint32_t x1, uint32_t y1, const int32_t lo[3], int32_t s,
                            uint32_t* dist) {
  BeamParams bp;
  memset(&bp, 0, sizeof(bp));
  memcpy(bp.O, O, sizeof(bp.O));
  memcpy(bp.A, A, sizeof(bp.A));
  memcpy(bp.BX, BX, sizeof(bp.BX));
  memcpy(bp.BY, BY, sizeof(bp.BY));
  BeamCone q;
  if (!beam_cone(bp, x0, y0, x1, y1, q)) return -1;
  *dist = beam_dist(q, lo, s);
  return beam_outside(q, lo, s) ? 1 : 0;
}

// The GPU scene generator's element functions (column heights, cave lattice
// tables, voxels) run on the host over one chunk; arguments as sgg_gen_chunk,
// with host memory.  Returns 0, or -1 on bad arguments.
extern "C" int hk_scene_chunk(const int64_t ip[6], const double dp[2], uint64_t seed, uint32_t chunk_log2,
                              uint32_t cx, uint32_t cy, uint32_t cz, const int32_t* boxes, uint32_t nbox,
                              uint8_t* out, int threads) {
  sgg::Params p{};
  if (!sgg::params_from(p, ip, dp, seed, chunk_log2, cx, cy, cz, nbox)) return -1;
  const int64_t S = (int64_t)1 << chunk_log2;
  std::vector<int32_t> hh((size_t)(S * S));
  for (int64_t i = 0; i < S * S; i++) hh[(size_t)i] = sgg::column_height(p, i);
  std::vector<double> V[sgg::kCaveOctaves];
  for (int o = 0; o < sgg::kCaveOctaves; o++) {
    V[o].resize((size_t)(p.n[o] * p.n[o] * p.n[o]));
    for (size_t i = 0; i < V[o].size(); i++) V[o][i] = sgg::lattice_entry(p, o, (int64_t)i);
  }
  const int nt = std::max(1, std::min(threads, (int)S));
  std::vector<std::thread> th;
  for (int t = 0; t < nt; t++)
    th.emplace_back([&, t] {
      for (int64_t z = S * t / nt; z < S * (t + 1) / nt; z++)
        for (int64_t i = z * S * S; i < (z + 1) * S * S; i++)
          out[i] = sgg::voxel_value(p, hh.data(), V[0].data(), V[1].data(), boxes, i);
    });
  for (auto& x : th) x.join();
  return 0;
}
