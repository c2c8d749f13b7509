// Internal declarations shared by the host runtime and the HIP kernels of
// libsvdag.  Nothing here is part of the public ABI (include/svdag.h).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstddef>
#include <cstdint>
#include <map>
#include <vector>

#include "svdag.h"

namespace svd {

// Device descriptor of one (chunk, LOD) DAG: 64 bytes, one per (chunk, LOD)
// slot in the world's table.
//
// Device node layout (derived from the canonical node format of Section
// 3.2): a node with k children is k consecutive u32 "child words",
// child word = (mask of the child << 24) | pointer, in ascending octant.
// The pointer of an internal child is the child's word offset; for the
// children of a level-3 node it indexes the u64 leaf bitmaps, and the "mask"
// is the leaf's 8-bit summary (bit i: 2^3 sub-block i is non-empty).  Keeping
// the child's mask in its parent makes every descent one 4-byte load.  A parallel
// u32 array `pre` holds, at the same offsets, the solid count of the earlier
// siblings (the DFS prefix of Section 3.3), read only once per hit.
struct alignas(64) DevDag {
  uint64_t nodes;      // device address: u32 child words
  uint64_t leaves;     // device address: u64 leaf bitmaps
  uint64_t pre;        // device address: u32 prefix counts, parallel to nodes
  uint64_t rle_start;  // device address: u32 run starts (DFS index), then the u8 run materials
  uint64_t rle_dir;    // device address: u32 run directory (see kRunDir)
  uint32_t rle_n;      // number of runs
  uint32_t root;       // child word of the root: (root mask << 24) | 0
  uint32_t solid;      // solid cells at this LOD (0 = empty)
  uint16_t lo[3];      // tight box of solid cells, LOD cells, inclusive
  uint16_t hi[3];
};
static_assert(sizeof(DevDag) == 64, "DevDag must stay 64 bytes");

// Run directory: with B = max(0, clz(rle_n) - clz(solid)), entry j is the
// last run starting at or before DFS index j * 2^B, for j = 0 .. (solid-1) >> B,
// followed by one more entry, rle_n - 1.  The run holding DFS index i lies
// between entries i >> B and (i >> B) + 1, inclusive, and there are at most
// 2 rle_n + 2 entries.
__host__ __device__ inline uint32_t run_dir_shift(uint32_t rle_n, uint32_t solid) {
  const int b = __builtin_clz(rle_n) - __builtin_clz(solid);
  return b > 0 ? (uint32_t)b : 0u;
}

constexpr uint32_t kPtrBits = 24;
constexpr uint32_t kPtrMask = (1u << kPtrBits) - 1;

// Per-chunk entry of the per-view table written by the chunk stage.
constexpr uint32_t kViewLodMask = 3u;
constexpr uint32_t kViewCulled = 4u;
constexpr uint32_t kViewEmpty = 8u;
constexpr uint32_t kViewMissing = 16u;  // needed, but its DAG is not resident (nodes == 0)

struct LodData {
  uint32_t R = 0;
  uint32_t root_level = 0;
  // canonical form (paper's node format)
  std::vector<uint32_t> words;
  std::vector<uint64_t> leaves;
  std::vector<uint32_t> rle_start;
  std::vector<uint8_t> rle_mat;
  uint32_t n_solid = 0;
  uint32_t level_nodes[16] = {};
  uint16_t lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  // device image sections, byte offsets inside the blob's image
  uint64_t off_nodes = 0, off_pre = 0, off_leaves = 0, off_rle_start = 0, off_rle_dir = 0;
  uint64_t off_begin = 0, off_end = 0;
  uint32_t dev_words = 0;
  uint32_t root_word = 0;
};

// Kernel parameters of one traced view.
struct TraceParams {
  int64_t O[3];
  int64_t A[3], BX[3], BY[3];
  uint32_t W, H;
  uint32_t grid[3];
  uint32_t chunk_log2;
  uint32_t tile_w;        // wave tile: tile_w x 64/tile_w pixels, tile_w in {8, 16, 32, 64}
  uint32_t tiles_x;       // wave tiles per image row
  uint32_t total_tiles;
  uint32_t* queue;        // tile queues (see kQueues); all zero between launches
  const uint32_t* view;   // per-chunk view entry
  const DevDag* desc;     // [chunk * 4 + lod]
  svd_hit* out;
  uint32_t beam;          // 1: each tile's first record holds its start bound
};
constexpr uint32_t kViewTileW = 16;  // default per-view wave tile: 16 x 4 pixels

// Tile queues of the persistent traces: one per XCD (a block's home queue is
// blockIdx % kQueues, which follows the round-robin placement of blocks on
// XCDs), each over a contiguous band of the tiles, so that the counters'
// atomics stay in separate cache lines and a band's rays share one L2.  A
// wave whose queue runs dry takes tiles from the next queues.  Counter q is
// word q * kQueueStride of the queue block; word kQueues * kQueueStride
// counts finished waves (per-view trace).
constexpr uint32_t kQueues = 8;
constexpr uint32_t kQueueStride = 32;  // u32 words: one 128-byte line per counter
constexpr size_t kQueueBlockBytes = 2048;

// Start bound of a tile, written by the beam pass into the first word of the
// tile's first record (the trace reads it before writing the tile): whole
// voxels of Chebyshev distance from the camera within which no ray of the
// tile meets a cell it could hit (or a chunk whose LOD is not loaded).
// kBeamNone: no ray of the tile meets one at all.
constexpr uint32_t kBeamNone = 0xFFFFFFFFu;

struct BeamParams {
  int64_t O[3], A[3], BX[3], BY[3];
  uint32_t W, H;
  uint32_t tiles_x, total_tiles, tile_w;
  uint32_t grid[3];
  uint32_t chunk_log2;
  const uint32_t* view;
  const DevDag* desc;
  svd_hit* out;
};

struct StageParams {
  int64_t O[3];
  int64_t n[4][3];        // cull planes through O (inward normals); zero = none
  uint32_t grid[3];
  uint32_t chunk_log2;
  uint32_t lod_count;
  uint32_t thr[3];
  uint32_t cull;          // 0 = keep every non-empty chunk
  uint32_t nchunks;
  const DevDag* desc;
  uint32_t* view;
};

// One view of a batch (device memory, 256 bytes).
struct alignas(256) BatchView {
  int64_t O[3], A[3], BX[3], BY[3];
  int64_t n[4][3];        // cull planes (zero = none)
  uint64_t out;           // device address of this view's first record
  uint32_t W, H;
  uint32_t tiles_x;       // tiles per image row
  uint32_t tile_base;     // first global tile index of this view
  uint32_t cull;
};
static_assert(sizeof(BatchView) == 256, "BatchView must stay 256 bytes");

// Batch header (device memory): rewritten by each svd_batch_trace call, so
// that one captured graph serves every batch.
struct alignas(64) BatchHeader {
  uint32_t nviews;
  uint32_t total_tiles;
  uint32_t unused;
  uint32_t tile_w;        // tile width in pixels (tile = tile_w x 64/tile_w)
  uint32_t claim;         // tiles a wave takes per queue access
  uint32_t beam;          // 1: run the beam pass (tile start bounds)
  uint32_t pad[10];
};
static_assert(sizeof(BatchHeader) == 64, "BatchHeader must stay 64 bytes");

struct BatchParams {
  const BatchView* views;
  BatchHeader* hdr;
  uint32_t max_views;
  uint32_t grid[3];
  uint32_t chunk_log2;
  uint32_t lod_count;
  uint32_t thr[3];
  uint32_t nchunks;
  const DevDag* desc;
  uint32_t* view_tables;  // [view * nchunks + chunk]
  uint32_t* queue;        // tile queues (kQueueBlockBytes), cleared by a kernel at each launch
};

// runtime.cpp: inward normals of the view cone's side planes (false = degenerate)
bool cull_planes(const svd_ray_frame* f, int64_t n[4][3]);
int check_frame(const svd_ray_frame* f);

// kernels.hip
int launch_chunk_stage(const StageParams& p, void* stream);
uint32_t host_stage_chunk(const StageParams& p, uint32_t ci);  // the stage's decision, on the host
// `start` / `stop` (hipEvent_t, may be null): events that take their
// timestamps from the kernel's own dispatch, not from marker commands
int launch_trace(const TraceParams& p, uint32_t blocks, void* stream, void* start = nullptr, void* stop = nullptr);
int launch_beam(const BeamParams& p, void* stream, void* start = nullptr);
int trace_occupancy(uint32_t* blocks_per_cu);
int launch_set_desc(DevDag* dst, const DevDag* src4, uint32_t n, void* stream);
// batched views: queue reset, per-(view, chunk) stage, persistent trace
int launch_batch(const BatchParams& p, uint32_t trace_blocks, void* stream);
int batch_trace_occupancy(uint32_t* blocks_per_cu);
// zero a queue block's counters and its done counter (a per-view trace on it
// then starts from zero and clears it again when it ends)
int launch_queue_clear(uint32_t* queue, void* stream);

// Allocation-free batches (svd_batch_trace_frames_static): one file-scope
// device array per GPU holds a call's queue block, header, views and view
// tables, laid out as a batch's pool area.
constexpr size_t kStaticScratchBytes = (size_t)1 << 20;
struct StaticDevice {
  uint8_t* scratch;  // device address of this GPU's copy of the array
  uint32_t cus;      // compute units
  uint32_t per_cu;   // batch trace blocks that fit a CU
};
// Set-up of the current device on its first use (symbol address, CU count,
// occupancy), cached per device afterwards.
int static_device(StaticDevice* out);
// Write views[first, first + count) (count <= kPackViews) and, when hdr is
// not null, the header, by a kernel whose arguments carry them.
constexpr uint32_t kPackViews = 8;
int launch_set_views(BatchView* dst, const BatchView* src, uint32_t count, BatchHeader* hdr_dst,
                     const BatchHeader* hdr, void* stream);
// The batch kernels (queue reset, stage, beam when `beam`, trace) with
// `trace_blocks` persistent trace blocks, outside any graph.
int launch_batch_direct(const BatchParams& p, uint32_t views, uint32_t trace_blocks, bool beam, void* stream);

}  // namespace svd

struct svd_blob {
  uint32_t chunk_log2 = 0;
  uint32_t lod_count = 0;
  std::vector<svd::LodData> lod;
  std::vector<uint8_t> image;  // device image of every LOD (256-byte sections)
};

// Thread-local error message; returns `code` for convenient `return fail(...)`.
int svd_fail(int code, const char* fmt, ...);

// Default persistent grid of the per-view trace: 6 blocks per CU (the most
// that fit).  With per-XCD tile queues, 1440p views of the 16x16-chunk map
// take 0.716 / 0.718 / 0.736 / 0.818 ms at 6 / 5 / 4 / 3 blocks per CU.
constexpr uint32_t kViewBlocksPerCu = 6;

// A world: the device descriptor table, the per-view table and queue, and a
// first-fit sub-allocator over the rest of the caller's pool.  Residency is
// kept per (chunk, LOD) slot:
//   absent     nothing known (a plain trace refuses to run while any is);
//   described  the blob's box and solid count are in the descriptor, but no
//              DAG (addresses zero): a view that needs it gets records
//              marked "not loaded" instead of reading it;
//   resident   the LOD's device image is in the pool.
struct svd_world {
  enum : uint8_t { kAbsent = 0, kDescribed = 1, kResident = 2 };
  struct Slot {
    size_t off = 0, bytes = 0;
    uint8_t state = kAbsent;
  };
  svd_world_desc desc;
  uint32_t nchunks = 0;
  uint8_t* pool = nullptr;
  size_t pool_bytes = 0;
  svd::DevDag* d_desc = nullptr;
  uint32_t* d_view = nullptr;
  uint32_t* d_queue = nullptr;  // per-view trace work queue (256-byte control block)
  uint32_t cus = 0;             // compute units of the device
  uint32_t max_per_cu = 0;      // resident trace blocks per CU at full occupancy
  uint32_t per_cu = 0;          // trace blocks per CU in use (persistent grid = per_cu x cus)
  uint32_t tile_w = svd::kViewTileW;  // per-view wave tile width (tile = tile_w x 64/tile_w pixels)
  size_t data_begin = 0;
  std::map<size_t, size_t> free_blocks;  // offset -> bytes
  std::vector<Slot> slot;                // [chunk * 4 + lod]
  std::vector<svd::DevDag> h_desc;       // host copy of the device descriptor table
  uint32_t absent = 0;                   // absent slots with lod < lod_count
  size_t used = 0;
  svd_ray_frame staged;  // frame of the last chunk stage (its view table)
  bool has_staged = false;
  bool staged_beam = false;  // the trace of the staged view runs the beam pass
  const svd_hit* beamed = nullptr;  // output that already holds the staged view's tile bounds
  // Timing of the next trace passes (svd_world_time_traces): a start and a
  // stop event per armed pass, stamped by the kernels' own dispatches.
  std::vector<hipEvent_t> timing;  // [2 * pass + 0/1]
  uint32_t timed = 0;              // passes recorded so far
  bool timing_started = false;     // the current pass's start was stamped by its beam launch

  uint32_t timing_slots() const { return (uint32_t)(timing.size() / 2); }
  void drop_timing() {
    for (uint32_t i = 0; i < timed; i++) (void)hipEventSynchronize(timing[2 * i + 1]);
    for (hipEvent_t e : timing) (void)hipEventDestroy(e);
    timing.clear();
    timed = 0;
    timing_started = false;
  }
  ~svd_world() { drop_timing(); }

  bool alloc(size_t bytes, size_t* off) {
    bytes = (bytes + 255) / 256 * 256;
    for (auto it = free_blocks.begin(); it != free_blocks.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t roff = it->first + bytes;
      free_blocks.erase(it);
      if (rest) free_blocks[roff] = rest;
      used += bytes;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + 255) / 256 * 256;
    used -= bytes;
    auto it = free_blocks.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_blocks.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_blocks.erase(nx);
    }
    if (it != free_blocks.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_blocks.erase(it);
      }
    }
  }
};

// Stage parameters of a frame over the world (cull planes unless no_cull),
// with `desc` pointing at the given table (device or host copy).
svd::StageParams world_stage_params(const svd_world* w, const svd_ray_frame* f, bool no_cull,
                                    const svd::DevDag* desc);
// Make LODs `mask` of chunk ci resident from b and describe the others from b
// (descriptor writes on `stream`); all or nothing (SVD_ENOMEM if the pool has
// no room).  Evict: LODs `mask` go back to described (descriptor writes on
// `stream`), their memory to the pool.
int world_upload_lods(svd_world* w, uint32_t ci, const svd_blob* b, uint32_t mask, hipStream_t stream);
int world_evict_lods(svd_world* w, uint32_t ci, uint32_t mask, hipStream_t stream);

// A batch: device memory from the world's pool,
//   [tile queues 2048 B][BatchHeader 64 B | pad to 256][BatchView x max_views][view tables: max_views x nchunks u32],
// pinned host staging (header + views) guarded by an event, and the captured
// graph (reset + stage + persistent trace) that every launch replays.
struct svd_batch {
  svd_world* w = nullptr;
  uint32_t max_views = 0;
  size_t off = 0, bytes = 0;
  uint32_t* d_queue = nullptr;
  svd::BatchHeader* d_hdr = nullptr;
  svd::BatchView* d_views = nullptr;
  uint32_t* d_tables = nullptr;
  uint8_t* h_stage = nullptr;      // pinned: header + views
  size_t stage_bytes = 0;
  hipEvent_t staged = nullptr;     // the last upload of h_stage has been consumed
  hipEvent_t finished = nullptr;   // the last graph launch has completed
  bool stage_pending = false;
  bool launched = false;
  hipStream_t cap = nullptr;       // capture stream (default priority)
  hipGraphExec_t exec = nullptr;
  uint32_t cus = 0, max_per_cu = 0, per_cu = 0;  // persistent grid = per_cu x cus blocks
  uint32_t tile_w = 8, claim = 1;
};

// Enqueue a batch whose view v writes its records at outs[v] (validated
// like svd_batch_trace_frames, except the capacity of each output, which is
// the caller's).
int batch_enqueue(svd_batch* b, const svd_ray_frame* frames, svd_hit* const* outs, uint32_t n, uint32_t flags,
                  hipStream_t stream);
// One view on a batch's own view table and queue block, without the graph:
// queue clear, the per-view stage, beam (with SVD_BEAM) and trace kernels,
// parameters as kernel arguments.  Same records as a one-view batch; for a
// launch that holds a single view it skips the header upload.
int batch_enqueue_single(svd_batch* b, const svd_ray_frame* frame, svd_hit* out, uint32_t flags, hipStream_t stream);
