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

/* svd_trace_view flags */
#define SVD_NO_CULL 1u     /* skip frustum culling (results are identical) */

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
 *   chunk  linear chunk index cx + gx*(cy + gy*cz); 0xFFFFFFFF on a miss
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
 * The world's tables take nchunks*4*64 + round256(nchunks*4) + 256 bytes at
 * its start.  Must be called with the pool's device current.  Errors:
 * SVD_EINVAL, SVD_ENOMEM (pool too small for the tables), SVD_EDEVICE. */
int svd_world_create(const svd_world_desc* desc, void* pool_dev, size_t pool_bytes,
                     svd_world** out);
void svd_world_destroy(svd_world* w);
/* Pool bytes currently allocated to chunk data. */
int svd_world_pool_used(const svd_world* w, size_t* used);

/* Upload all LODs of `b` as chunk c (replacing what was there).  Enqueues an
 * H2D copy from the blob's memory on `stream`: the blob must stay alive and
 * unchanged until the stream has passed this point.  SVD_ENOMEM if the pool
 * has no room (nothing is changed then); SVD_EINVAL if the blob's chunk size
 * or LOD count differ from the world's. */
int svd_chunk_upload(svd_world* w, const uint32_t c[3], const svd_blob* b, void* stream);
/* Release chunk c's pool space.  Work already enqueued on the world's stream
 * still sees the old data (stream order). */
int svd_chunk_evict(svd_world* w, const uint32_t c[3]);

/* Exact integer frame of a camera (host, FP64 with fixed operation order).
 * SVD_EINVAL for a degenerate camera, SVD_ERANGE if the position is outside
 * (-32768, 65536) voxels on some axis. */
int svd_camera_frame(const svd_camera* cam, svd_ray_frame* out);

/* Trace one view: enqueue the chunk stage (LOD pick and frustum cull per
 * chunk) and the per-pixel trace on `stream`.
 *   out_dev  width*height svd_hit records (device, caller-owned).
 *   flags    SVD_NO_CULL or 0.
 * Errors: SVD_EINVAL, SVD_ERANGE (camera), SVD_ENOTFOUND (a chunk was never
 * uploaded), SVD_EDEVICE. */
int svd_trace_view(svd_world* w, const svd_camera* cam, svd_hit* out_dev, uint32_t flags,
                   void* stream);
/* Same, from an integer frame (directions must satisfy |D| < 2^31 over the
 * image and the origin the camera range above).  Equivalent to
 * svd_view_stage followed by svd_view_trace. */
int svd_trace_frame(svd_world* w, const svd_ray_frame* frame, svd_hit* out_dev, uint32_t flags,
                    void* stream);

/* The two halves of a traced view, for callers that time or schedule them
 * separately.
 * svd_view_stage: the chunk stage (Section 3.5 chunk selection pass): per
 *   chunk, the LOD by camera distance (Eq. 1) and a conservative frustum
 *   cull of its tight box at that LOD, written to the world's view table.
 *   Errors as svd_trace_frame.
 * svd_view_trace: the per-pixel trace (Section 3.5 ray marching and colour
 *   resolve) over the view table of the last svd_view_stage, which must have
 *   been given an identical frame (else SVD_EINVAL). */
int svd_view_stage(svd_world* w, const svd_ray_frame* frame, uint32_t flags, void* stream);
int svd_view_trace(svd_world* w, const svd_ray_frame* frame, svd_hit* out_dev, void* stream);

/* Occupancy of the per-view persistent trace: the grid is blocks_per_cu x
 * (compute units) blocks of 4 waves, but never more waves than the view has
 * 64-pixel tiles.  0 selects the default, 4 blocks per CU (or the most that
 * fit, if fewer); more than fit is SVD_EINVAL.  Results do not depend on it. */
int svd_world_set_occupancy(svd_world* w, uint32_t blocks_per_cu);
int svd_world_get_occupancy(const svd_world* w, uint32_t* blocks_per_cu, uint32_t* max_per_cu);

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

/* Takes 256 + 256*max_views + 4*max_views*nchunks bytes (rounded to 256)
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

/* Autotuner: times every tiling candidate (tile width 8/16/32 x claim
 * 1/2/4) at the current occupancy, then every occupancy from the maximum
 * down to 2 blocks per CU at the best tiling, on this batch of cameras
 * (median of `reps` launches after one warm-up, HIP events on `stream`;
 * synchronises it); keeps the fastest and returns its time in *best_ms
 * (may be NULL). */
int svd_batch_tune(svd_batch* b, const svd_camera* cams, uint32_t n, svd_hit* out_dev,
                   uint64_t out_records, uint32_t reps, void* stream, float* best_ms);

#ifdef __cplusplus
}
#endif
#endif /* SVDAG_H */
