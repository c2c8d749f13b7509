/*
 * CPU oracle for chunked-SVDAG primary-ray traversal.
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the GPU library; only
 * the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * load it.  It shares no code with the GPU library.
 *
 * Every function is a plain, slow restatement of a definition:
 *   - LOD pyramid: a coarse voxel is solid iff at least `density` = 2 of its
 *     8 finer voxels are solid (Section 3.4); its material is the most
 *     frequent material among them, ties to the smallest ID (the paper
 *     averages colours; material IDs cannot be averaged).
 *   - Sparse voxel octree with the three deepest levels as 4x4x4 leaf
 *     bitmaps, merged into a DAG by identical subtrees, serialised in the
 *     node format of Section 3.2: u32 header (child mask in bits 0..7), u32
 *     solid-voxel count of the subtree, one u32 pointer per set mask bit.
 *   - DFS-order material array and its lossless run blocks (Section 3.3
 *     with error threshold 0), looked up by binary search.
 *   - LOD pick by exact camera-to-chunk-centre distance (Eq. 1 distance term).
 *   - Traversal: the first visited cell (half-open cells, fixed tie rule)
 *     that is solid in its chunk's picked LOD grid, found by stepping cell
 *     by cell with exact integer (128-bit) comparisons.
 */
#ifndef SVDAG_ORACLE_H
#define SVDAG_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- camera -> integer ray frame --------------------------------------- */
typedef struct {
  int64_t O[3];              /* origin, voxels * 2^16 */
  int64_t A[3], BX[3], BY[3];/* D(px,py) = A + px*BX + py*BY, |D_a| < 2^31 */
  int32_t G;                 /* direction scale exponent */
  uint32_t W, H;
} or_frame;

/* Returns 0, or -1 (degenerate camera), -2 (origin outside the guard band). */
int or_camera_frame(const float pos[3], const float target[3], const float up[3],
                    float vfov_deg, uint32_t W, uint32_t H, or_frame* out);

/* ---- LOD pyramid --------------------------------------------------------- */
/* dst[(R/2)^3] from src[R^3] (index x + R*(y + R*z)). */
void or_downsample(const uint8_t* src, uint32_t R, uint8_t* dst);

/* ---- DAG ------------------------------------------------------------------ */
typedef struct {
  uint32_t R;           /* grid edge in cells (power of two, >= 8) */
  uint32_t root_level;  /* log2(R) */
  uint32_t n_words;     /* node words (0 when the grid is empty) */
  uint32_t* words;
  uint32_t n_leaves;
  uint64_t* leaves;
  uint32_t n_solid;
  uint32_t n_rle;
  uint32_t* rle_start;
  uint8_t* rle_mat;
  uint32_t level_nodes[16]; /* unique nodes per level (index = level; 2 = leaves) */
} or_dag;

/* Build from a dense R^3 grid.  Returns NULL on bad arguments. */
or_dag* or_dag_build(const uint8_t* grid, uint32_t R);
void or_dag_free(or_dag* d);
/* 1 if cell (x,y,z) is solid; then *dfs = its DFS index.  0 if empty; then
 * *empty_level = level of the largest empty cube containing the cell
 * (root_level for an empty grid). */
int or_dag_lookup(const or_dag* d, uint32_t x, uint32_t y, uint32_t z, uint32_t* dfs,
                  uint32_t* empty_level);
uint8_t or_dag_material(const or_dag* d, uint32_t dfs);
/* Expand back to a dense grid (materials included). */
void or_dag_expand(const or_dag* d, uint8_t* out);

/* ---- world ----------------------------------------------------------------- */
typedef struct or_world or_world;
or_world* or_world_new(uint32_t chunk_log2, const uint32_t grid[3], uint32_t lod_count);
void or_world_free(or_world* w);
/* Takes ownership of `d` (may be NULL = empty).  lod < lod_count. */
int or_world_set_dag(or_world* w, uint32_t chunk, uint32_t lod, or_dag* d);
/* Optional dense LOD grid ((S>>lod)^3 bytes, copied) used instead of the DAG
 * when `use_dense` is set on trace. */
int or_world_set_dense(or_world* w, uint32_t chunk, uint32_t lod, const uint8_t* g);

void or_lod_pick(const or_world* w, const int64_t O[3], const uint32_t thr[3], uint8_t* lods);

typedef struct {
  int32_t x, y, z;      /* LOD-0 voxel of the hit cell's min corner */
  int32_t hit;          /* 1 hit, 0 miss */
  int32_t lod;
  int32_t face;         /* 0 none, else 1 + 2*axis + (D_axis < 0) */
  int32_t material;
  int32_t chunk;        /* linear chunk index, -1 on miss */
  double t;             /* Euclidean distance in voxels to the cell entry; inf on miss */
  double t_num;         /* hit time as the rational t_num / t_den (exact in double */
  double t_den;         /*   only when small; for diagnostics) */
} or_hit;

/* Trace n rays sharing origin O, directions D[3*i..3*i+2].
 * mode bit 0: skip empty DAG subtrees (1) or step every cell (0);
 * mode bit 1: use the dense grids instead of the DAGs. */
void or_trace(const or_world* w, const uint8_t* lods, const int64_t O[3], const int32_t* D,
              uint32_t n, or_hit* out, int mode, int nthreads);
/* Per-ray visit counts of the hierarchical traversal (DAG modes only):
 * chunks the ray passes through, non-empty chunk DAGs it enters, non-empty
 * internal-node cubes (levels 3 .. root-1) and leaf cubes (level 2) it
 * enters up to and including its hit; at a hit, the preceding set siblings
 * summed over the internal levels of the hit cell's path (the subtree counts
 * its DFS index adds up, Section 3.3) and the run starts the material search
 * compares.  Used to state algorithmic memory traffic. */
typedef struct {
  int32_t chunk_visits, chunk_entries, node_cubes, leaf_cubes;
  int32_t preceding_siblings, run_probes;
} or_counts;

/* Trace the pixels idx[0..n) (idx = px + W*py; all pixels if idx is NULL)
 * of a frame; `counts` (n entries) may be NULL. */
void or_trace_frame(const or_world* w, const uint8_t* lods, const or_frame* f,
                    const uint32_t* idx, uint32_t n, or_hit* out, int mode, int nthreads,
                    or_counts* counts);

/* Counting instrumentation for the compulsory-traffic figure: trace every
 * pixel of a frame (mode 1) and count, each once, the parts of the device
 * layout its rays touch: child words read on descents, leaf bitmaps,
 * prefix counts and run starts read by hits, run materials, the view-table
 * entries of the chunks visited and the descriptors of the chunk DAGs
 * entered. */
typedef struct {
  uint64_t rays, hits;
  uint64_t child_words, leaves, prefixes, run_starts, run_materials, chunks, dags;
} or_touched;
void or_touch_frame(const or_world* w, const uint8_t* lods, const or_frame* f, int nthreads,
                    or_touched* out);

#ifdef __cplusplus
}
#endif
#endif
