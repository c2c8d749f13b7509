/*
 * svdag.h — C ABI of libsvdag: chunked Sparse Voxel DAGs with LODs, traced
 * per pixel on an AMD Instinct MI355X (gfx950).
 *
 * Method: Fang, Wang, Wang, "Aokana: A GPU-Driven Voxel Rendering Framework
 * for Open World Games", PACMCGIT 2025.  The world is cut into cubic chunks,
 * each stored as a shallow SVDAG (Section 3.1) whose nodes follow the format
 * of Section 3.2, with colours (here: material IDs) decoupled into a DFS-order
 * array compressed into blocks (Section 3.3) and a per-chunk LOD pyramid
 * (Section 3.4).  Per view, a GPU chunk stage culls chunks to the frustum and
 * picks each chunk's LOD by distance (Section 3.5, Eq. 1), and a GPU trace
 * finds, per pixel, the first solid voxel along the primary ray (Section 3.5,
 * ray marching and colour resolve).
 *
 * Conventions
 *  - Every function returns SVD_OK (0) or a negative SVD_E* code; the message
 *    of the last failure on the calling thread is svd_last_error().
 *  - Argument errors are reported before anything is enqueued.  Device
 *    errors (launch or copy failures) are returned as SVD_EDEVICE.
 *  - "stream" arguments are hipStream_t values passed as void* (NULL = the
 *    null stream).  Enqueue-only functions return before the device work
 *    completes; the caller synchronises the stream.
 *  - Pointers named *_dev are device addresses; all others are host.
 *  - No exceptions cross this boundary.  Not thread-safe per world: use one
 *    world from one thread and one stream at a time.
 */
#ifndef SVDAG_H
#define SVDAG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SVD_OK 0
#define SVD_EINVAL (-1)    /* bad argument */
#define SVD_ENOMEM (-2)    /* pool or host memory exhausted */
#define SVD_EDEVICE (-3)   /* HIP runtime error */
#define SVD_EFORMAT (-4)   /* malformed blob bytes */
#define SVD_ERANGE (-5)    /* value outside the exact-integer range */
#define SVD_ENOTFOUND (-6) /* chunk not resident */
#define SVD_EIO (-7)       /* a file could not be written */

/* Trace flags (results are identical with any of them) */
#define SVD_NO_CULL 1u     /* skip frustum culling */
#define SVD_BEAM 2u        /* run the beam pass first (rays start at their tile's bound) */

/* Message of the last failure on this thread (static storage, never NULL). */
const char* svd_last_error(void);

/* ------------------------------------------------------------------------
 * World description.
 *   chunk_log2     S = 2^chunk_log2 voxels per chunk edge, 3..10.
 *   grid[3]        chunks per axis; grid[a] * S <= 32768.
 *   lod_count      1..4 LODs per chunk; requires chunk_log2 - (lod_count-1) >= 3
 *                  (the coarsest LOD grid is at least 8^3).
 *   lod_threshold  voxel distances (ascending); a chunk's LOD is the number of
 *                  the first lod_count-1 thresholds that the camera-to-chunk-
 *                  centre distance reaches (Eq. 1 distance term).
 * World coordinates are voxels; chunk (cx,cy,cz) covers [c*S, (c+1)*S) per
 * axis; +z is up.
 * ------------------------------------------------------------------------ */
typedef struct {
  uint32_t chunk_log2;
  uint32_t grid[3];
  uint32_t lod_count;
  uint32_t lod_threshold[3];
} svd_world_desc;

/* Pinhole camera (float32, voxel units): vertical FOV in degrees (0, 180);
 * pixel (px, py) looks through its centre; row 0 is the top of the image. */
typedef struct {
  float pos[3];
  float target[3];
  float up[3];
  float vfov_deg;
  uint32_t width;
  uint32_t height;
} svd_camera;

/* Exact integer ray frame of a camera: origin O in voxels * 2^16 and pixel
 * direction D(px,py) = A + px*BX + py*BY with every component below 2^31 in
 * magnitude.  The ray is p(t) = (O + t D) / 2^16, t >= 0. */
typedef struct {
  int64_t O[3];
  int64_t A[3];
  int64_t BX[3];
  int64_t BY[3];
  int32_t G;        /* directions are scaled by 2^G */
  uint32_t width, height;
} svd_ray_frame;

/* Per-pixel result, 16 bytes, written for every pixel (row-major, py*W+px).
 *   xy     x | y<<16: LOD-0 voxel of the hit cell's minimum corner
 *   zf     z | lod<<16 | face<<20 | hit<<23 | material<<24
 *          face: 0 none, else 1 + 2*axis + (ray component < 0) of the cell
 *          side the ray entered through (lowest axis on ties)
 *   t      Euclidean distance in voxels from the camera to where the ray
 *          enters the hit cell (float32); +inf on a miss
 *   chunk  linear chunk index cx + gx*(cy + gy*cz); 0xFFFFFFFF on a miss;
 *          SVD_CHUNK_NOT_LOADED (below) when the ray reached a chunk whose
 *          picked LOD is described but not resident; 0xFFFFFFFE if the chunk
 *          walk's iteration guard fired (a ray crosses at most 3 x 4096
 *          chunks, so it never fires; the walk inside a chunk ends by
 *          construction)
 * A miss has xy = zf = 0. */
typedef struct {
  uint32_t xy;
  uint32_t zf;
  float t;
  uint32_t chunk;
} svd_hit;

/* ------------------------------------------------------------------------
 * Host-side chunk build (the paper's offline preprocessing, Sections 3.1-3.4).
 * ------------------------------------------------------------------------ */
typedef struct svd_blob svd_blob;

/* Builds every LOD of one chunk from a dense grid.
 *   dense       S^3 bytes, index x + S*(y + S*z); 0 = empty, 1..255 = material.
 *               Read only during the call; the caller keeps ownership.
 *   chunk_log2  3..10;  lod_count 1..4 with chunk_log2-(lod_count-1) >= 3.
 * LOD k+1 voxel = aggregate of 8 LOD-k voxels: solid iff >= 2 are solid
 * (density, Section 3.4), material = most frequent, ties to the smallest ID.
 * Each LOD becomes an SVDAG (isomorphic subtrees merged, 4^3 leaf bitmaps,
 * Section 3.2) plus lossless DFS-order material runs (Section 3.3).
 * Errors: SVD_EINVAL (arguments), SVD_ENOMEM, SVD_ERANGE (a DAG needs more
 * than 2^24 node words or leaves).  *out is owned by the caller
 * (svd_blob_free). */
int svd_chunk_build(const uint8_t* dense, uint32_t chunk_log2, uint32_t lod_count,
                    svd_blob** out);

/* Serialise a blob (versioned, canonical: identical geometry gives identical
 * bytes).  *bytes is allocated by the library; release with svd_free. */
int svd_blob_to_bytes(const svd_blob* b, void** bytes, size_t* n);
/* Parse and fully validate serialised bytes (SVD_EFORMAT on any
 * inconsistency: sizes, pointers, levels, counts, runs).  Caller owns *out. */
int svd_blob_from_bytes(const void* bytes, size_t n, svd_blob** out);
void svd_blob_free(svd_blob* b);
void svd_free(void* p);

/* Statistics of LOD `lod` of a blob. */
typedef struct {
  uint32_t R;              /* grid edge at this LOD */
  uint32_t n_words;        /* node words in the paper's format */
  uint32_t n_leaves;       /* unique 4^3 leaf bitmaps */
  uint32_t n_rle;          /* material run blocks */
  uint32_t n_solid;        /* solid voxels */
  uint32_t level_nodes[16];/* unique nodes per level (2 = leaves, log2(R) = root) */
  uint16_t aabb_lo[3], aabb_hi[3]; /* tight box of solid cells (inclusive), if n_solid */
  uint64_t device_bytes;   /* bytes this LOD occupies in the pool */
} svd_blob_stats;
int svd_blob_stats_get(const svd_blob* b, uint32_t lod, svd_blob_stats* out);
/* Canonical arrays of LOD `lod` (paper's node format: per node u32 mask,
 * u32 solid count, one u32 pointer per child; leaf bitmaps; run starts and
 * materials).  Pointers into blob memory, valid until svd_blob_free. */
int svd_blob_canonical(const svd_blob* b, uint32_t lod, const uint32_t** words,
                       const uint64_t** leaves, const uint32_t** rle_start,
                       const uint8_t** rle_mat);

/* ------------------------------------------------------------------------
 * Device world: chunk DAGs resident in a caller-owned HBM pool.
 * ------------------------------------------------------------------------ */
typedef struct svd_world svd_world;

/* pool_dev: caller-owned device buffer (e.g. a torch uint8 tensor), 256-byte
 * aligned, that must outlive the world; the library only sub-allocates it.
 * The world's tables take nchunks*4*64 + round256(nchunks*4) + 2048 bytes at
 * its start.  Must be called with the pool's device current.  Errors:
 * SVD_EINVAL, SVD_ENOMEM (pool too small for the tables), SVD_EDEVICE. */
int svd_world_create(const svd_world_desc* desc, void* pool_dev, size_t pool_bytes,
                     svd_world** out);
void svd_world_destroy(svd_world* w);
/* Pool bytes currently allocated to chunk data. */
int svd_world_pool_used(const svd_world* w, size_t* used);

/* Upload all LODs of `b` as chunk c (replacing what was there).  Enqueues an
 * H2D copy from the blob's memory on `stream`: the blob must stay alive and
 * unchanged until the stream has passed this point.  Replacing a resident
 * chunk releases its old space at once, so the caller orders this call after
 * every trace that still reads the chunk (same stream, or an event wait).
 * SVD_ENOMEM if the pool has no room (nothing is changed then); SVD_EINVAL if
 * the blob's chunk size or LOD count differ from the world's. */
int svd_chunk_upload(svd_world* w, const uint32_t c[3], const svd_blob* b, void* stream);
/* Release chunk c's pool space; the chunk counts as never uploaded again
 * (traces refuse to run until it is).  No device work is enqueued: traces
 * already enqueued still read the old data, so the caller orders later
 * uploads that may reuse the space after them (as for svd_chunk_evict_lods). */
int svd_chunk_evict(svd_world* w, const uint32_t c[3]);

/* Per-LOD residency, for streaming (Section 3.4: LODs are loaded and
 * unloaded by camera distance).  A (chunk, LOD) slot is never uploaded,
 * described (its tight box and solid count are known, its DAG is not in the
 * pool) or resident.
 * svd_chunk_upload_lods: makes the LODs in lod_mask (bit k = LOD k) resident
 *   from b and describes every LOD of the chunk from b; LODs outside the mask
 *   that are resident stay so (they must hold the same chunk content).  All
 *   or nothing: SVD_ENOMEM leaves the world unchanged.  lod_mask 0 only
 *   describes the chunk.  H2D copies and descriptor writes on `stream`.
 * svd_chunk_evict_lods: the LODs in lod_mask go back to described and their
 *   pool space is released; descriptor writes on `stream`.  The caller
 *   orders later uploads that may reuse the space after every trace that
 *   still reads it.
 * A view traced while a LOD it needs (picked, not culled, not empty) is only
 * described writes, for every ray that reaches that chunk, a record with
 * hit = 0, t = +inf and chunk = SVD_CHUNK_NOT_LOADED instead of reading it. */
#define SVD_CHUNK_NOT_LOADED 0xFFFFFFFDu
int svd_chunk_upload_lods(svd_world* w, const uint32_t c[3], const svd_blob* b, uint32_t lod_mask,
                          void* stream);
int svd_chunk_evict_lods(svd_world* w, const uint32_t c[3], uint32_t lod_mask, void* stream);

/* Exact integer frame of a camera (host, FP64 with fixed operation order).
 * SVD_EINVAL for a degenerate camera, SVD_ERANGE if the position is outside
 * (-32768, 65536) voxels on some axis. */
int svd_camera_frame(const svd_camera* cam, svd_ray_frame* out);

/* Trace one view: enqueue the chunk stage (LOD pick and frustum cull per
 * chunk) and the per-pixel trace on `stream`.
 *   out_dev  width*height svd_hit records (device, caller-owned).
 *   flags    SVD_NO_CULL, SVD_BEAM or 0.
 * Errors: SVD_EINVAL, SVD_ERANGE (camera), SVD_ENOTFOUND (some (chunk, LOD)
 * was never uploaded nor described), SVD_EDEVICE. */
int svd_trace_view(svd_world* w, const svd_camera* cam, svd_hit* out_dev, uint32_t flags,
                   void* stream);
/* Same, from an integer frame (directions must satisfy |D| < 2^31 over the
 * image and the origin the camera range above).  Equivalent to
 * svd_view_stage followed by svd_view_trace. */
int svd_trace_frame(svd_world* w, const svd_ray_frame* frame, svd_hit* out_dev, uint32_t flags,
                    void* stream);

/* The parts of a traced view, for callers that time or schedule them
 * separately.
 * svd_view_stage: the chunk stage (Section 3.5 chunk selection pass): per
 *   chunk, the LOD by camera distance (Eq. 1) and a conservative frustum
 *   cull of its tight box at that LOD, written to the world's view table.
 *   Errors as svd_trace_frame.  flags: SVD_NO_CULL, SVD_BEAM.
 * svd_view_beam (optional): the beam pass (ESVO's beam optimisation, Section
 *   2.2: a coarse distance pass that moves the rays' starting points; here
 *   made exact, so records do not change): per wave tile (the world's
 *   tiling, svd_world_set_tiling), a
 *   distance within which no ray of the tile can meet a cell it could hit,
 *   parked in the tile's first record of out_dev.  The next svd_view_trace
 *   into the same out_dev then starts each ray there instead of running the
 *   pass itself.  Nothing is done unless the view was staged with SVD_BEAM.
 * svd_view_trace: the per-pixel trace (Section 3.5 ray marching and colour
 *   resolve) over the view table of the last svd_view_stage, which must have
 *   been given an identical frame (else SVD_EINVAL); with SVD_BEAM staged,
 *   runs the beam pass first unless svd_view_beam did.
 * The beam pass is off by default: on MI355X it cuts the trace's time by
 * about a fifth, but its own search (one serial chain of dependent loads
 * per tile) costs about twice the trace. */
int svd_view_stage(svd_world* w, const svd_ray_frame* frame, uint32_t flags, void* stream);
int svd_view_beam(svd_world* w, const svd_ray_frame* frame, svd_hit* out_dev, void* stream);
int svd_view_trace(svd_world* w, const svd_ray_frame* frame, svd_hit* out_dev, void* stream);

/* Kernel time of trace passes, for measurement (the duration of the
 * per-pixel trace kernel of Section 3.5 ray marching, with the beam kernel
 * when the pass runs one).
 * svd_world_time_traces: arms the world to time its next n trace passes
 *   (svd_view_trace, svd_trace_frame, svd_trace_view; batches and served
 *   requests are not timed).  A pass's start and stop timestamps come from
 *   the dispatch packets of its first and last kernel, so no marker command
 *   is put on the stream and back-to-back launches keep their spacing
 *   (event markers between kernels each add a few microseconds of idle
 *   time).  Passes after the n-th run untimed.  n = 0 disarms; arming again
 *   drops earlier records.  Both calls wait for passes already recorded.
 *   Errors: SVD_EINVAL for n > SVD_MAX_TIMED_PASSES (nothing changes),
 *   SVD_EDEVICE if the events cannot be created (the world is then
 *   disarmed).
 * svd_world_trace_times: waits for the recorded passes and writes the
 *   durations of the first min(n, recorded) of them, in milliseconds and in
 *   launch order, to host array ms; *count gets how many were written.
 *   Errors: SVD_EINVAL for null arguments, SVD_EDEVICE if a pass failed
 *   (*count then holds the durations written before it). */
#define SVD_MAX_TIMED_PASSES 65536u
int svd_world_time_traces(svd_world* w, uint32_t n);
int svd_world_trace_times(svd_world* w, float* ms, uint32_t n, uint32_t* count);

/* Occupancy of the per-view persistent trace: the grid is blocks_per_cu x
 * (compute units) blocks of 4 waves, but never more waves than the view has
 * 64-pixel tiles.  0 selects the default, 6 blocks per CU (or the most that
 * fit, if fewer); more than fit is SVD_EINVAL.  Results do not depend on it. */
int svd_world_set_occupancy(svd_world* w, uint32_t blocks_per_cu);
int svd_world_get_occupancy(const svd_world* w, uint32_t* blocks_per_cu, uint32_t* max_per_cu);

/* Wave tile of the per-view beam and trace passes: tile_w x (64/tile_w)
 * pixels, tile_w in {8, 16, 32, 64} (0 selects the default, 16); anything
 * else is SVD_EINVAL.  Results do not depend on it. */
int svd_world_set_tiling(svd_world* w, uint32_t tile_w);
int svd_world_get_tiling(const svd_world* w, uint32_t* tile_w);

/* Outcome of an autotuning call. */
typedef struct svd_tune_result {
  uint32_t tile_w;         /* wave tile width (tile = tile_w x 64/tile_w pixels) */
  uint32_t claim;          /* tiles per queue access (always 1 for the per-view trace) */
  uint32_t blocks_per_cu;  /* occupancy of the persistent grid */
  uint32_t from_cache;     /* 1: taken from the cache file, nothing was timed */
  float ms;                /* median time of the chosen configuration when it was timed */
  uint32_t configs_timed;  /* configurations this call timed (0 from the cache) */
  char key[384];           /* the cache key: device, kernel source hash, workload shape */
} svd_tune_result;

/* Per-view autotuner: times the whole per-view pass (svd_trace_frame with
 * `flags`: stage, beam with SVD_BEAM, trace) of every frame in turn, median
 * of `reps` (1..64) runs after one warm-up, HIP events on `stream`
 * (synchronises it), for every tile width at the current occupancy, then
 * every occupancy from the most that fit down to 2 blocks per CU at the best
 * width; keeps the fastest in the world (svd_world_set_tiling and
 * svd_world_set_occupancy), so that every later per-view call uses it.
 * out_dev holds out_records records (at least the largest frame); its
 * contents are overwritten.
 *   cache_path (NULL or "" = no cache): a text file of earlier choices keyed
 *   by this device (architecture, CUs, peak clock), the kernel source hash
 *   (svd_kernel_hash) and the workload shape (chunk grid, chunk size, LOD
 *   count, flags, the frames' resolutions and count).  A matching entry is
 *   applied without timing anything (res->from_cache = 1); otherwise the
 *   choice is timed and stored (the file is rewritten through a temporary
 *   and a rename; the directory must exist).  Errors as svd_trace_frame,
 *   plus SVD_EIO if the cache cannot be written (the tuned configuration is
 *   applied all the same).  On any other error the world keeps its previous
 *   tiling and occupancy. */
int svd_world_tune(svd_world* w, const svd_ray_frame* frames, uint32_t n, svd_hit* out_dev, uint64_t out_records,
                   uint32_t flags, uint32_t reps, const char* cache_path, void* stream, svd_tune_result* res);

/* The cache file of svd_world_tune and svd_batch_tune_cached, directly.
 * Lookup: the last entry for `key` into *res (from_cache = 1,
 * configs_timed = 0); SVD_ENOTFOUND if the file or the entry is missing.
 * Store: res->key (no tab or line break), tile_w (8/16/32/64), claim
 * (1..16), blocks_per_cu (>= 1) and ms, replacing any entry of that key;
 * SVD_EINVAL for a bad entry, SVD_EIO if the file cannot be written.  Other
 * lines of the file are kept. */
int svd_tune_cache_lookup(const char* cache_path, const char* key, svd_tune_result* res);
int svd_tune_cache_store(const char* cache_path, const svd_tune_result* res);

/* Hash of the trace kernels' source this library was built from: the first
 * 16 hex digits of SHA-256 over kernels.hip followed by svdag_internal.h
 * ("unknown" if the build did not supply it).  Static string. */
const char* svd_kernel_hash(void);

/* Per-chunk LOD (bits 0-1), culled (bit 2) and empty (bit 3) flags of the
 * last traced view, copied to host (synchronises `stream`). */
int svd_view_table(svd_world* w, uint32_t* out, uint32_t n, void* stream);

/* ------------------------------------------------------------------------
 * Batches of views: many cameras of uneven resolution traced in one graph
 * launch (a per-(view, chunk) chunk stage and one persistent trace whose
 * waves take 64-pixel tiles of any view from a shared work queue).  Each
 * view's records are identical to what svd_trace_view writes for it alone.
 * ------------------------------------------------------------------------ */
typedef struct svd_batch svd_batch;

/* Takes 2304 + 256*max_views + 4*max_views*nchunks bytes (rounded to 256)
 * from the world's pool and captures the batch's graph.  The batch must be
 * destroyed before its world.  Errors: SVD_EINVAL (max_views 1..65535),
 * SVD_ENOMEM (pool), SVD_EDEVICE. */
int svd_batch_create(svd_world* w, uint32_t max_views, svd_batch** out);
void svd_batch_destroy(svd_batch* b);

/* Trace n <= max_views cameras.  Records of view v start at the sum of the
 * pixel counts of views 0..v-1 in out_dev (row-major per view); out_records
 * is the capacity of out_dev.  Enqueue-only on `stream`.  The camera array
 * is read during the call only.  Errors as svd_trace_view, plus SVD_EINVAL
 * when the views need more than out_records records. */
int svd_batch_trace(svd_batch* b, const svd_camera* cams, uint32_t n, svd_hit* out_dev,
                    uint64_t out_records, uint32_t flags, void* stream);
int svd_batch_trace_frames(svd_batch* b, const svd_ray_frame* frames, uint32_t n, svd_hit* out_dev,
                           uint64_t out_records, uint32_t flags, void* stream);

/* Allocation-free form of svd_batch_trace_frames, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  No batch object is needed, and the call
 * allocates nothing (no device or pinned memory, stream, event, graph or
 * host heap).  The queue block, batch header, views and per-(view, chunk)
 * view tables of the call live in one static device array of the library,
 * 1 MiB per GPU, held by each GPU the library runs on until the process
 * ends; the views reach it as kernel arguments.  The kernels (view writes,
 * queue clear, stage, beam with SVD_BEAM, persistent trace with 16x4-pixel
 * tiles) are enqueued on `stream`, and can be captured into a graph.
 *   Layout and capacity: 2304 + 256*n + 4*n*nchunks (rounded up to 256)
 *   bytes must fit 1 MiB (SVD_ENOMEM otherwise, before anything is
 *   enqueued); n <= 65535.  Output and errors otherwise as
 *   svd_batch_trace_frames.
 * The array is shared by every call on the same GPU and keeps the last
 * call's contents (the queue counters are cleared by each call): calls that
 * overlap on one GPU (different streams, or other threads) race and must be
 * serialised by the caller.  The first call on a device also looks up the
 * array's address there (once per device). */
int svd_batch_trace_frames_static(svd_world* w, const svd_ray_frame* frames, uint32_t n, svd_hit* out_dev,
                                  uint64_t out_records, uint32_t flags, void* stream);

/* Work shape of the persistent trace: a wave's tile is tile_w x (64/tile_w)
 * pixels (tile_w in {8, 16, 32, 64}); a wave takes `claim` (1..16)
 * consecutive tiles per queue access.  Results do not depend on it. */
int svd_batch_set_tiling(svd_batch* b, uint32_t tile_w, uint32_t claim);

/* Persistent grid of the batch trace: blocks_per_cu x (compute units) blocks
 * of 4 waves; 0 selects the most that fit a CU (the default), more is
 * SVD_EINVAL.  A change re-captures the batch's graph, after waiting for the
 * batch's last launch to finish.  Results do not depend on it. */
int svd_batch_set_occupancy(svd_batch* b, uint32_t blocks_per_cu);
int svd_batch_get_tiling(const svd_batch* b, uint32_t* tile_w, uint32_t* claim, uint32_t* blocks_per_cu);

/* Autotuner: times every tiling candidate (tile width 8/16/32/64 x claim
 * 1/2/4) at the current occupancy, then every occupancy from the maximum
 * down to 2 blocks per CU at the best tiling, on this batch of cameras
 * (median of `reps` launches after one warm-up, HIP events on `stream`;
 * synchronises it); keeps the fastest and returns its time in *best_ms
 * (may be NULL). */
int svd_batch_tune(svd_batch* b, const svd_camera* cams, uint32_t n, svd_hit* out_dev,
                   uint64_t out_records, uint32_t reps, void* stream, float* best_ms);

/* svd_batch_tune through the cache of svd_world_tune (kind "batch", keyed by
 * the cameras' resolutions and count): a matching entry sets the batch's
 * tiling and occupancy without timing; otherwise the batch is tuned and the
 * choice stored.  Errors as svd_batch_tune, plus SVD_EIO as in
 * svd_world_tune. */
int svd_batch_tune_cached(svd_batch* b, const svd_camera* cams, uint32_t n, svd_hit* out_dev,
                          uint64_t out_records, uint32_t reps, const char* cache_path, void* stream,
                          svd_tune_result* res);

/* ------------------------------------------------------------------------
 * Serving: view requests of any resolution, arriving at any time, over a
 * world whose pool may hold only part of the map (Section 3.4 streaming:
 * chunk LODs are loaded by camera distance and unloaded when space is
 * needed).  A worker thread owns the world while the server lives (the
 * caller makes no other call on it meanwhile):
 *   - requests are admitted in arrival order; the (chunk, LOD) slots a view
 *     reads (the chunk stage's LOD pick and cull, evaluated on the host) are
 *     pinned, missing ones uploaded from the chunk's source blob on an
 *     upload stream, evicting unpinned slots least recently used first; a
 *     request waits while in-flight work holds the memory it needs and
 *     fails with SVD_ENOMEM if it does not fit the idle pool;
 *   - SVD_SERVE_BATCHED packs admitted requests (same flags, up to max_views
 *     views and max_rays rays) into captured batch launches, up to
 *     `inflight` of them on the device at once, each on its own stream;
 *     requests arriving meanwhile join the next launch as soon as a launch
 *     slot frees (continuous batching); a launch that holds one request runs
 *     the per-view kernels on its batch's tables instead of the graph (no
 *     upload first);
 *   - SVD_SERVE_PLAIN traces each request with its own stage + trace launch
 *     pair, all on one stream, up to `inflight` queued (the per-request
 *     comparison, serial);
 *   - SVD_SERVE_PLAIN_CONCURRENT traces each request with its own stage +
 *     trace launch pair too, but up to `inflight` of them run at once, each
 *     on its own stream with its own view table and queue block (the
 *     per-request comparison, concurrent; takes inflight x
 *     svd_batch_create(w, 1) pool space);
 *   - with streaming_factor f > 0, the streaming policy of Section 3.4 runs
 *     whenever a request's camera enters a chunk not among the last 8 seen:
 *     an implicit octree over the chunk grid is walked from the root, a node
 *     (a cube of 2^n chunks) being split while its LOD error (Eq. 1: the
 *     distance at which its LOD gives way to a finer one, times max(f, 1),
 *     minus its distance from the camera) is positive; the chunks of the
 *     nodes where it stops are wanted at the LOD Eq. 1 picks with every
 *     threshold stretched by f, and at the LOD it picks now.  Wanted slots
 *     are uploaded, coarse LODs first and nearer first, into free pool space
 *     while no request waits (1/8 of the pool stays free for demand), and
 *     eviction takes unwanted slots before wanted ones.  Records never
 *     depend on it.
 * Each request's records equal those of svd_trace_view of the same camera
 * on a world with every chunk resident.
 * ------------------------------------------------------------------------ */
typedef struct svd_server svd_server;

#define SVD_SERVE_BATCHED 0u
#define SVD_SERVE_PLAIN 1u
#define SVD_SERVE_PLAIN_CONCURRENT 2u

typedef struct {
  uint32_t mode;           /* SVD_SERVE_BATCHED, SVD_SERVE_PLAIN or SVD_SERVE_PLAIN_CONCURRENT */
  uint32_t max_views;      /* batched: requests per launch, 1..1024 */
  uint32_t inflight;       /* launches on the device at once, 1..8 */
  uint32_t tile_w, claim;  /* batched: tiling (0 = the batch default) */
  uint32_t blocks_per_cu;  /* batched: persistent grid (0 = the batch default) */
  uint64_t max_rays;       /* batched: rays per launch (a larger request goes alone) */
  float streaming_factor;  /* > 0: prefetch by the streaming policy (below); 0: demand only */
  uint32_t reserved;       /* 0 */
} svd_server_desc;

typedef struct {
  uint64_t tag;            /* the caller's tag of the request */
  int32_t status;          /* SVD_OK, or the error that failed the request */
  uint32_t batch_views;    /* requests in the launch that traced it (0 if none) */
  double t_submit, t_launch, t_done;  /* seconds on the server's clock: submit call,
                                         launch enqueued, completion seen by the worker */
} svd_request_done;

typedef struct {
  uint64_t submitted, completed, failed, launches;
  uint64_t uploads, upload_bytes, evictions, evict_bytes;
  uint64_t memory_waits;   /* requests that waited for in-flight work to release memory */
  uint64_t pool_used;      /* pool bytes holding chunk LODs */
  uint64_t prefetches, prefetch_bytes;  /* uploads made by the streaming policy */
} svd_server_stats;

/* Batched mode takes inflight x svd_batch_create(w, max_views) pool space.
 * Errors: SVD_EINVAL, SVD_ENOMEM, SVD_EDEVICE. */
int svd_server_create(svd_world* w, const svd_server_desc* d, svd_server** out);
/* Source of chunk c's LODs (kept alive by the caller until the server is
 * destroyed); describes the chunk in the world.  Every chunk needs one
 * before the first submit; none may change after it (SVD_EINVAL). */
int svd_server_set_chunk(svd_server* s, const uint32_t c[3], const svd_blob* b);
/* Queue a request; returns at once.  out_dev: width*height records (device),
 * with no pending work of the caller's (the server's streams do not wait
 * for other streams) and untouched until the request is reported done.  flags:
 * SVD_NO_CULL, SVD_BEAM or 0.  Camera errors as svd_camera_frame, synchronously.
 * Thread-safe. */
int svd_server_submit(svd_server* s, const svd_camera* cam, svd_hit* out_dev, uint32_t flags, uint64_t tag);
/* Up to `max` finished requests (oldest first) into out, their count in *n;
 * waits up to wait_us microseconds for the first.  Thread-safe. */
int svd_server_poll(svd_server* s, svd_request_done* out, uint32_t max, uint32_t* n, uint32_t wait_us);
int svd_server_stats_get(svd_server* s, svd_server_stats* st);
/* Completes every submitted request, then frees the server (not the world). */
void svd_server_destroy(svd_server* s);

#ifdef __cplusplus
}
#endif
#endif /* SVDAG_H */
