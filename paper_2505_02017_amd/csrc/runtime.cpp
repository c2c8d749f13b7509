// Host runtime of libsvdag: errors, camera frame, world and pool management,
// chunk upload/evict, and the per-view entry points that enqueue the GPU
// chunk stage and trace.  Compile with -ffp-contract=off: the camera frame is
// defined by a fixed sequence of IEEE double operations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "svdag_internal.h"

using namespace svd;

// ------------------------------------------------------------------ errors
static thread_local char g_err[512] = "no error";

int svd_fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

extern "C" const char* svd_last_error(void) { return g_err; }

#define HIP_OK(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) return svd_fail(SVD_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// ------------------------------------------------------------ camera frame
// Pinhole camera, vertical FOV, pixel centres, row 0 on top.  The direction of
// pixel (px, py) is fwd + ((2(px+.5)/W - 1) tau a) right + ((1 - 2(py+.5)/H) tau) up',
// i.e. affine: A + px BX + py BY.  A, BX, BY are rounded to integers at 2^G,
// G maximal with every corner component below 2^31; O is rounded at 2^16.
namespace {
void cross(const double a[3], const double b[3], double r[3]) {
  r[0] = a[1] * b[2] - a[2] * b[1];
  r[1] = a[2] * b[0] - a[0] * b[2];
  r[2] = a[0] * b[1] - a[1] * b[0];
}
}  // namespace

extern "C" int svd_camera_frame(const svd_camera* cam, svd_ray_frame* out) {
  if (!cam || !out) return svd_fail(SVD_EINVAL, "svd_camera_frame: null argument");
  const uint32_t W = cam->width, H = cam->height;
  if (W == 0 || H == 0) return svd_fail(SVD_EINVAL, "camera: empty image");
  if ((uint64_t)W * H > (1ull << 31)) return svd_fail(SVD_EINVAL, "camera: image larger than 2^31 pixels");
  if (!(cam->vfov_deg > 0.0f && cam->vfov_deg < 180.0f)) return svd_fail(SVD_EINVAL, "camera: FOV outside (0,180)");
  double f[3], up[3], fn[3], r[3], rn[3], u[3];
  for (int i = 0; i < 3; i++) {
    f[i] = (double)cam->target[i] - (double)cam->pos[i];
    up[i] = (double)cam->up[i];
  }
  const double fl = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
  if (!(fl > 0.0)) return svd_fail(SVD_EINVAL, "camera: target equals position");
  for (int i = 0; i < 3; i++) fn[i] = f[i] / fl;
  cross(fn, up, r);
  const double rl = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  if (!(rl > 0.0)) return svd_fail(SVD_EINVAL, "camera: up is parallel to the view direction");
  for (int i = 0; i < 3; i++) rn[i] = r[i] / rl;
  cross(rn, fn, u);
  const double tau = std::tan((double)cam->vfov_deg * (M_PI / 360.0));
  const double aspect = (double)W / (double)H;
  const double sx0 = ((1.0 / (double)W - 1.0) * tau) * aspect;
  const double sy0 = (1.0 - 1.0 / (double)H) * tau;
  const double sbx = ((2.0 / (double)W) * tau) * aspect;
  const double sby = -((2.0 / (double)H) * tau);
  double A[3], BX[3], BY[3];
  for (int i = 0; i < 3; i++) {
    A[i] = (fn[i] + sx0 * rn[i]) + sy0 * u[i];
    BX[i] = sbx * rn[i];
    BY[i] = sby * u[i];
  }
  const int64_t lim = (int64_t)1 << 31;
  int G = 40;
  for (; G >= 0; G--) {
    int64_t qa[3], qx[3], qy[3];
    for (int i = 0; i < 3; i++) {
      qa[i] = (int64_t)std::rint(std::ldexp(A[i], G));
      qx[i] = (int64_t)std::rint(std::ldexp(BX[i], G));
      qy[i] = (int64_t)std::rint(std::ldexp(BY[i], G));
    }
    bool fits = true;
    for (int cpx = 0; cpx < 2 && fits; cpx++)
      for (int cpy = 0; cpy < 2 && fits; cpy++) {
        const int64_t px = cpx ? (int64_t)W - 1 : 0, py = cpy ? (int64_t)H - 1 : 0;
        for (int i = 0; i < 3; i++) {
          const int64_t d = qa[i] + px * qx[i] + py * qy[i];
          if (d >= lim || d <= -lim) fits = false;
        }
      }
    if (fits) {
      memcpy(out->A, qa, sizeof(qa));
      memcpy(out->BX, qx, sizeof(qx));
      memcpy(out->BY, qy, sizeof(qy));
      break;
    }
  }
  if (G < 0) return svd_fail(SVD_EINVAL, "camera: no direction scale fits");
  out->G = G;
  out->width = W;
  out->height = H;
  for (int i = 0; i < 3; i++) {
    const int64_t o = (int64_t)std::rint(std::ldexp((double)cam->pos[i], 16));
    if (o <= -((int64_t)1 << 31) || o >= ((int64_t)1 << 32))
      return svd_fail(SVD_ERANGE, "camera: position outside (-32768, 65536) voxels");
    out->O[i] = o;
  }
  return SVD_OK;
}

// ------------------------------------------------------------------ world
static int check_desc(const svd_world_desc* d) {
  if (d->chunk_log2 < 3 || d->chunk_log2 > 10) return svd_fail(SVD_EINVAL, "world: chunk_log2 must be 3..10");
  if (d->lod_count < 1 || d->lod_count > 4 || (int)d->chunk_log2 - (int)(d->lod_count - 1) < 3)
    return svd_fail(SVD_EINVAL, "world: lod_count must be 1..4 with coarsest grid >= 8^3");
  for (int a = 0; a < 3; a++)
    if (d->grid[a] < 1 || ((uint64_t)d->grid[a] << d->chunk_log2) > 32768)
      return svd_fail(SVD_EINVAL, "world: grid must be >= 1 and at most 32768 voxels per axis");
  return SVD_OK;
}

extern "C" int svd_world_create(const svd_world_desc* desc, void* pool_dev, size_t pool_bytes,
                                svd_world** out) {
  if (!desc || !pool_dev || !out) return svd_fail(SVD_EINVAL, "svd_world_create: null argument");
  *out = nullptr;
  int rc = check_desc(desc);
  if (rc) return rc;
  if ((uintptr_t)pool_dev % 256) return svd_fail(SVD_EINVAL, "world: pool must be 256-byte aligned");
  const uint64_t n = (uint64_t)desc->grid[0] * desc->grid[1] * desc->grid[2];
  const size_t desc_bytes = (size_t)n * 4 * sizeof(DevDag);
  const size_t view_bytes = ((size_t)n * 4 + 255) / 256 * 256;
  const size_t ctl_bytes = kQueueBlockBytes;
  if (pool_bytes < desc_bytes + view_bytes + ctl_bytes)
    return svd_fail(SVD_ENOMEM, "world: pool smaller than its tables");
  uint32_t per_cu = 0;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return svd_fail(SVD_EDEVICE, "world: cannot query the device");
  rc = trace_occupancy(&per_cu);
  if (rc) return rc;
  try {
    svd_world* w = new svd_world();
    w->desc = *desc;
    w->nchunks = (uint32_t)n;
    w->pool = (uint8_t*)pool_dev;
    w->pool_bytes = pool_bytes;
    w->d_desc = (DevDag*)pool_dev;
    w->d_view = (uint32_t*)(w->pool + desc_bytes);
    w->d_queue = (uint32_t*)(w->pool + desc_bytes + view_bytes);
    w->cus = (uint32_t)cus;
    w->max_per_cu = per_cu;
    w->per_cu = std::min(per_cu, kViewBlocksPerCu);
    w->data_begin = desc_bytes + view_bytes + ctl_bytes;
    if (pool_bytes > w->data_begin) w->free_blocks[w->data_begin] = (pool_bytes - w->data_begin) / 256 * 256;
    w->slot.resize((size_t)n * 4);
    w->h_desc.assign((size_t)n * 4, DevDag());
    memset(w->h_desc.data(), 0, w->h_desc.size() * sizeof(DevDag));
    w->absent = (uint32_t)n * desc->lod_count;
    hipError_t e = hipMemset(pool_dev, 0, w->data_begin);
    if (e != hipSuccess) {
      delete w;
      return svd_fail(SVD_EDEVICE, "world: hipMemset: %s", hipGetErrorString(e));
    }
    *out = w;
    return SVD_OK;
  } catch (const std::bad_alloc&) {
    return svd_fail(SVD_ENOMEM, "world: out of host memory");
  }
}

extern "C" void svd_world_destroy(svd_world* w) { delete w; }

extern "C" int svd_world_pool_used(const svd_world* w, size_t* used) {
  if (!w || !used) return svd_fail(SVD_EINVAL, "svd_world_pool_used: null argument");
  *used = w->used;
  return SVD_OK;
}

static int chunk_index(const svd_world* w, const uint32_t c[3], uint32_t* ci) {
  if (!c) return svd_fail(SVD_EINVAL, "null chunk coordinates");
  for (int a = 0; a < 3; a++)
    if (c[a] >= w->desc.grid[a]) return svd_fail(SVD_EINVAL, "chunk (%u,%u,%u) outside the grid", c[0], c[1], c[2]);
  *ci = c[0] + w->desc.grid[0] * (c[1] + w->desc.grid[1] * c[2]);
  return SVD_OK;
}

// Descriptor of LOD k of blob b whose device image section starts at pool
// offset `off` (addresses zero when the LOD is only described).
static DevDag lod_desc(const svd_world* w, const svd_blob* b, uint32_t k, bool loaded, size_t off) {
  DevDag d;
  memset(&d, 0, sizeof(d));
  const LodData& L = b->lod[k];
  if (loaded) {
    const uint64_t base = (uint64_t)(uintptr_t)(w->pool + off) - L.off_begin;
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
  return d;
}

int world_upload_lods(svd_world* w, uint32_t ci, const svd_blob* b, uint32_t mask, hipStream_t s) {
  if (b->chunk_log2 != w->desc.chunk_log2 || b->lod_count != w->desc.lod_count)
    return svd_fail(SVD_EINVAL, "upload: blob chunk size or LOD count differs from the world's");
  const uint32_t nl = w->desc.lod_count;
  if (mask >> nl) return svd_fail(SVD_EINVAL, "upload: LOD mask 0x%x beyond %u LODs", mask, nl);
  size_t off[4] = {0, 0, 0, 0}, bytes[4] = {0, 0, 0, 0};
  for (uint32_t k = 0; k < nl; k++) {
    if (!((mask >> k) & 1)) continue;
    bytes[k] = b->lod[k].off_end - b->lod[k].off_begin;
    if (bytes[k] && !w->alloc(bytes[k], &off[k])) {
      for (uint32_t j = 0; j < k; j++)
        if (bytes[j]) w->release(off[j], bytes[j]);
      return svd_fail(SVD_ENOMEM, "upload: pool full (%zu bytes requested, %zu used of %zu)", bytes[k], w->used,
                      w->pool_bytes - w->data_begin);
    }
  }
  hipError_t e = hipSuccess;
  for (uint32_t k = 0; k < nl && e == hipSuccess; k++)
    if (bytes[k])
      e = hipMemcpyAsync(w->pool + off[k], b->image.data() + b->lod[k].off_begin, bytes[k], hipMemcpyHostToDevice, s);
  DevDag d[4];
  memset(d, 0, sizeof(d));
  const size_t base = (size_t)ci * 4;
  for (uint32_t k = 0; k < nl; k++) {
    const bool load = (mask >> k) & 1;
    d[k] = lod_desc(w, b, k, load, off[k]);
    if (!load && w->slot[base + k].state == svd_world::kResident) {  // keep what is loaded
      d[k].nodes = w->h_desc[base + k].nodes;
      d[k].leaves = w->h_desc[base + k].leaves;
      d[k].pre = w->h_desc[base + k].pre;
      d[k].rle_start = w->h_desc[base + k].rle_start;
      d[k].rle_dir = w->h_desc[base + k].rle_dir;
    }
  }
  int rc = e == hipSuccess ? launch_set_desc(w->d_desc + base, d, 4, s)
                           : svd_fail(SVD_EDEVICE, "upload: hipMemcpyAsync: %s", hipGetErrorString(e));
  if (rc) {
    for (uint32_t k = 0; k < nl; k++)
      if (bytes[k]) w->release(off[k], bytes[k]);
    return rc;
  }
  for (uint32_t k = 0; k < nl; k++) {
    svd_world::Slot& sl = w->slot[base + k];
    if (sl.state == svd_world::kAbsent) w->absent--;
    if ((mask >> k) & 1) {
      if (sl.state == svd_world::kResident && sl.bytes) w->release(sl.off, sl.bytes);
      sl.off = off[k];
      sl.bytes = bytes[k];
      sl.state = svd_world::kResident;
    } else if (sl.state == svd_world::kAbsent) {
      sl.state = svd_world::kDescribed;
    }
    w->h_desc[base + k] = d[k];
  }
  return SVD_OK;
}

int world_evict_lods(svd_world* w, uint32_t ci, uint32_t mask, hipStream_t s) {
  const uint32_t nl = w->desc.lod_count;
  if (mask >> nl) return svd_fail(SVD_EINVAL, "evict: LOD mask 0x%x beyond %u LODs", mask, nl);
  const size_t base = (size_t)ci * 4;
  DevDag d[4];
  bool change = false;
  for (uint32_t k = 0; k < 4; k++) {
    d[k] = w->h_desc[base + k];
    if (k < nl && ((mask >> k) & 1) && w->slot[base + k].state == svd_world::kResident) {
      d[k].nodes = d[k].leaves = d[k].pre = d[k].rle_start = d[k].rle_dir = 0;
      change = true;
    }
  }
  if (!change) return SVD_OK;
  int rc = launch_set_desc(w->d_desc + base, d, 4, s);
  if (rc) return rc;
  for (uint32_t k = 0; k < nl; k++) {
    svd_world::Slot& sl = w->slot[base + k];
    if (((mask >> k) & 1) && sl.state == svd_world::kResident) {
      if (sl.bytes) w->release(sl.off, sl.bytes);
      sl.off = sl.bytes = 0;
      sl.state = svd_world::kDescribed;
    }
    w->h_desc[base + k] = d[k];
  }
  return SVD_OK;
}

extern "C" int svd_chunk_upload_lods(svd_world* w, const uint32_t c[3], const svd_blob* b, uint32_t lod_mask,
                                     void* stream) {
  if (!w || !b) return svd_fail(SVD_EINVAL, "svd_chunk_upload_lods: null argument");
  uint32_t ci;
  int rc = chunk_index(w, c, &ci);
  if (rc) return rc;
  return world_upload_lods(w, ci, b, lod_mask, (hipStream_t)stream);
}

extern "C" int svd_chunk_upload(svd_world* w, const uint32_t c[3], const svd_blob* b, void* stream) {
  if (!w || !b) return svd_fail(SVD_EINVAL, "svd_chunk_upload: null argument");
  return svd_chunk_upload_lods(w, c, b, (1u << w->desc.lod_count) - 1, stream);
}

extern "C" int svd_chunk_evict_lods(svd_world* w, const uint32_t c[3], uint32_t lod_mask, void* stream) {
  if (!w) return svd_fail(SVD_EINVAL, "svd_chunk_evict_lods: null world");
  uint32_t ci;
  int rc = chunk_index(w, c, &ci);
  if (rc) return rc;
  return world_evict_lods(w, ci, lod_mask, (hipStream_t)stream);
}

extern "C" int svd_chunk_evict(svd_world* w, const uint32_t c[3]) {
  if (!w) return svd_fail(SVD_EINVAL, "svd_chunk_evict: null world");
  uint32_t ci;
  int rc = chunk_index(w, c, &ci);
  if (rc) return rc;
  bool any = false;
  for (uint32_t k = 0; k < w->desc.lod_count; k++) {
    svd_world::Slot& sl = w->slot[(size_t)ci * 4 + k];
    if (sl.state == svd_world::kAbsent) continue;
    any = true;
    if (sl.state == svd_world::kResident && sl.bytes) w->release(sl.off, sl.bytes);
    sl = svd_world::Slot();
    w->absent++;
  }
  if (!any) return svd_fail(SVD_ENOTFOUND, "evict: chunk not resident");
  return SVD_OK;
}

// ------------------------------------------------------------------ trace
typedef __int128 i128;

// Inward normals of the four side planes of the cone spanned by the corner
// rays (pixel-centre rays of the image corners).  Every pixel direction is a
// convex combination of the corners.  Returns false when the cone is
// degenerate; then culling is disabled for the view.
bool svd::cull_planes(const svd_ray_frame* f, int64_t n[4][3]) {
  int64_t C[4][3];
  const int64_t W1 = (int64_t)f->width - 1, H1 = (int64_t)f->height - 1;
  const int64_t px[4] = {0, W1, W1, 0}, py[4] = {0, 0, H1, H1};
  for (int i = 0; i < 4; i++)
    for (int a = 0; a < 3; a++) C[i][a] = f->A[a] + px[i] * f->BX[a] + py[i] * f->BY[a];
  for (int i = 0; i < 4; i++) {
    const int64_t* p = C[i];
    const int64_t* q = C[(i + 1) % 4];
    int64_t m[3] = {p[1] * q[2] - p[2] * q[1], p[2] * q[0] - p[0] * q[2], p[0] * q[1] - p[1] * q[0]};
    i128 s0 = 0, s1 = 0;
    for (int a = 0; a < 3; a++) {
      s0 += (i128)m[a] * C[(i + 2) % 4][a];
      s1 += (i128)m[a] * C[(i + 3) % 4][a];
    }
    int sgn;
    if (s0 >= 0 && s1 >= 0 && (s0 > 0 || s1 > 0)) sgn = 1;
    else if (s0 <= 0 && s1 <= 0 && (s0 < 0 || s1 < 0)) sgn = -1;
    else return false;
    for (int a = 0; a < 3; a++) n[i][a] = sgn * m[a];
  }
  return true;
}

int svd::check_frame(const svd_ray_frame* f) {
  const uint32_t W = f->width, H = f->height;
  if (W == 0 || H == 0 || (uint64_t)W * H > (1ull << 31)) return svd_fail(SVD_EINVAL, "trace: bad image size");
  for (int a = 0; a < 3; a++)
    if (f->O[a] <= -((int64_t)1 << 31) || f->O[a] >= ((int64_t)1 << 32))
      return svd_fail(SVD_ERANGE, "trace: origin outside (-32768, 65536) voxels");
  const i128 lim = (i128)1 << 31;
  for (int cpx = 0; cpx < 2; cpx++)
    for (int cpy = 0; cpy < 2; cpy++)
      for (int a = 0; a < 3; a++) {
        const i128 d = (i128)f->A[a] + (i128)(cpx ? W - 1 : 0) * f->BX[a] + (i128)(cpy ? H - 1 : 0) * f->BY[a];
        if (d >= lim || d <= -lim) return svd_fail(SVD_ERANGE, "trace: direction component >= 2^31");
      }
  return SVD_OK;
}

static bool same_frame(const svd_ray_frame& a, const svd_ray_frame& b) {
  return memcmp(a.O, b.O, sizeof(a.O)) == 0 && memcmp(a.A, b.A, sizeof(a.A)) == 0 &&
         memcmp(a.BX, b.BX, sizeof(a.BX)) == 0 && memcmp(a.BY, b.BY, sizeof(a.BY)) == 0 &&
         a.width == b.width && a.height == b.height;
}

StageParams world_stage_params(const svd_world* w, const svd_ray_frame* f, bool no_cull, const DevDag* desc) {
  StageParams sp;
  memset(&sp, 0, sizeof(sp));
  memcpy(sp.O, f->O, sizeof(sp.O));
  sp.cull = !no_cull && cull_planes(f, sp.n);
  memcpy(sp.grid, w->desc.grid, sizeof(sp.grid));
  sp.chunk_log2 = w->desc.chunk_log2;
  sp.lod_count = w->desc.lod_count;
  memcpy(sp.thr, w->desc.lod_threshold, sizeof(sp.thr));
  sp.nchunks = w->nchunks;
  sp.desc = desc;
  return sp;
}

// Per-view beam and trace parameters: the world's wave tiles (tile_w x
// 64/tile_w pixels) over the frame, the given view table (per-chunk LOD and
// flags) and, for the trace, the given queue block.
static BeamParams view_beam_params(const svd_world* w, const svd_ray_frame* f, const uint32_t* view, svd_hit* out) {
  BeamParams bp;
  memset(&bp, 0, sizeof(bp));
  memcpy(bp.O, f->O, sizeof(bp.O));
  memcpy(bp.A, f->A, sizeof(bp.A));
  memcpy(bp.BX, f->BX, sizeof(bp.BX));
  memcpy(bp.BY, f->BY, sizeof(bp.BY));
  bp.W = f->width;
  bp.H = f->height;
  bp.tile_w = w->tile_w;
  bp.tiles_x = (f->width + bp.tile_w - 1) / bp.tile_w;
  const uint64_t th = 64 / bp.tile_w;
  bp.total_tiles = (uint32_t)((uint64_t)bp.tiles_x * ((f->height + th - 1) / th));
  memcpy(bp.grid, w->desc.grid, sizeof(bp.grid));
  bp.chunk_log2 = w->desc.chunk_log2;
  bp.view = view;
  bp.desc = w->d_desc;
  bp.out = out;
  return bp;
}

static TraceParams view_trace_params(const svd_world* w, const svd_ray_frame* f, uint32_t* queue,
                                     const uint32_t* view, svd_hit* out, bool beam) {
  TraceParams tp;
  memset(&tp, 0, sizeof(tp));
  memcpy(tp.O, f->O, sizeof(tp.O));
  memcpy(tp.A, f->A, sizeof(tp.A));
  memcpy(tp.BX, f->BX, sizeof(tp.BX));
  memcpy(tp.BY, f->BY, sizeof(tp.BY));
  tp.W = f->width;
  tp.H = f->height;
  memcpy(tp.grid, w->desc.grid, sizeof(tp.grid));
  tp.chunk_log2 = w->desc.chunk_log2;
  tp.tile_w = w->tile_w;
  tp.tiles_x = (f->width + tp.tile_w - 1) / tp.tile_w;
  const uint64_t th = 64 / tp.tile_w;
  tp.total_tiles = (uint32_t)((uint64_t)tp.tiles_x * ((f->height + th - 1) / th));
  tp.queue = queue;
  tp.view = view;
  tp.desc = w->d_desc;
  tp.out = out;
  tp.beam = beam;
  return tp;
}

// A persistent grid at the world's occupancy, but no more waves (4 per
// block) than there are tiles.
static uint32_t view_trace_blocks(const svd_world* w, const TraceParams& tp) {
  return (uint32_t)std::min<uint64_t>((uint64_t)w->per_cu * w->cus, (tp.total_tiles + 3) / 4);
}

extern "C" int svd_view_stage(svd_world* w, const svd_ray_frame* f, uint32_t flags, void* stream) {
  if (!w || !f) return svd_fail(SVD_EINVAL, "svd_view_stage: null argument");
  if (flags & ~(SVD_NO_CULL | SVD_BEAM)) return svd_fail(SVD_EINVAL, "stage: unknown flags");
  int rc = check_frame(f);
  if (rc) return rc;
  if (w->absent) return svd_fail(SVD_ENOTFOUND, "stage: %u (chunk, LOD) slots were never uploaded", w->absent);
  StageParams sp = world_stage_params(w, f, flags & SVD_NO_CULL, w->d_desc);
  sp.view = w->d_view;
  rc = launch_chunk_stage(sp, stream);
  if (rc) return rc;
  w->staged = *f;
  w->has_staged = true;
  w->staged_beam = (flags & SVD_BEAM) != 0;
  w->beamed = nullptr;
  w->timing_started = false;
  return SVD_OK;
}

extern "C" int svd_view_beam(svd_world* w, const svd_ray_frame* f, svd_hit* out_dev, void* stream) {
  if (!w || !f || !out_dev) return svd_fail(SVD_EINVAL, "svd_view_beam: null argument");
  if (!w->has_staged || !same_frame(w->staged, *f))
    return svd_fail(SVD_EINVAL, "beam: the frame was not staged by the last svd_view_stage");
  if (w->absent) return svd_fail(SVD_ENOTFOUND, "beam: %u (chunk, LOD) slots were never uploaded", w->absent);
  if (!w->staged_beam) return SVD_OK;
  // an armed pass starts at its beam launch
  void* start = (w->timed < w->timing_slots() && !w->timing_started) ? w->timing[2 * w->timed] : nullptr;
  const int rc = launch_beam(view_beam_params(w, f, w->d_view, out_dev), stream, start);
  if (rc == SVD_OK) w->beamed = out_dev;
  if (rc == SVD_OK && start) w->timing_started = true;
  return rc;
}

extern "C" int svd_view_trace(svd_world* w, const svd_ray_frame* f, svd_hit* out_dev, void* stream) {
  if (!w || !f || !out_dev) return svd_fail(SVD_EINVAL, "svd_view_trace: null argument");
  if (!w->has_staged || !same_frame(w->staged, *f))
    return svd_fail(SVD_EINVAL, "trace: the frame was not staged by the last svd_view_stage");
  if (w->absent) return svd_fail(SVD_ENOTFOUND, "trace: %u (chunk, LOD) slots were never uploaded", w->absent);
  const TraceParams tp = view_trace_params(w, f, w->d_queue, w->d_view, out_dev, w->staged_beam);
  if (tp.beam && w->beamed != out_dev) {  // per-tile start bounds, parked in each tile's first record
    const int rc = svd_view_beam(w, f, out_dev, stream);
    if (rc) return rc;
  }
  w->beamed = nullptr;
  void *start = nullptr, *stop = nullptr;
  if (w->timed < w->timing_slots()) {
    if (!w->timing_started) start = w->timing[2 * w->timed];
    stop = w->timing[2 * w->timed + 1];
  }
  const int rc = launch_trace(tp, view_trace_blocks(w, tp), stream, start, stop);
  if (stop) {
    if (rc == SVD_OK) w->timed++;
    w->timing_started = false;
  }
  return rc;
}

extern "C" int svd_world_time_traces(svd_world* w, uint32_t n) {
  if (!w) return svd_fail(SVD_EINVAL, "svd_world_time_traces: null world");
  if (n > SVD_MAX_TIMED_PASSES)
    return svd_fail(SVD_EINVAL, "time_traces: at most %u passes, asked for %u", (unsigned)SVD_MAX_TIMED_PASSES, n);
  w->drop_timing();
  w->timing.reserve(2 * (size_t)n);
  for (uint32_t i = 0; i < 2 * n; i++) {
    hipEvent_t e = nullptr;
    const hipError_t err = hipEventCreate(&e);
    if (err != hipSuccess) {
      w->drop_timing();
      return svd_fail(SVD_EDEVICE, "time_traces: %s", hipGetErrorString(err));
    }
    w->timing.push_back(e);
  }
  return SVD_OK;
}

extern "C" int svd_world_trace_times(svd_world* w, float* ms, uint32_t n, uint32_t* count) {
  if (!w || !count || (n && !ms)) return svd_fail(SVD_EINVAL, "svd_world_trace_times: null argument");
  *count = 0;
  const uint32_t m = std::min(n, w->timed);
  for (uint32_t i = 0; i < m; i++) {
    hipError_t err = hipEventSynchronize(w->timing[2 * i + 1]);
    if (err == hipSuccess) err = hipEventElapsedTime(&ms[i], w->timing[2 * i], w->timing[2 * i + 1]);
    if (err != hipSuccess) return svd_fail(SVD_EDEVICE, "trace_times: pass %u: %s", i, hipGetErrorString(err));
    *count = i + 1;
  }
  return SVD_OK;
}

extern "C" int svd_world_set_occupancy(svd_world* w, uint32_t blocks_per_cu) {
  if (!w) return svd_fail(SVD_EINVAL, "svd_world_set_occupancy: null world");
  if (blocks_per_cu > w->max_per_cu)
    return svd_fail(SVD_EINVAL, "occupancy: at most %u trace blocks per CU", w->max_per_cu);
  w->per_cu = blocks_per_cu ? blocks_per_cu : std::min(w->max_per_cu, kViewBlocksPerCu);
  return SVD_OK;
}

extern "C" int svd_world_get_occupancy(const svd_world* w, uint32_t* blocks_per_cu, uint32_t* max_per_cu) {
  if (!w || !blocks_per_cu || !max_per_cu) return svd_fail(SVD_EINVAL, "svd_world_get_occupancy: null argument");
  *blocks_per_cu = w->per_cu;
  *max_per_cu = w->max_per_cu;
  return SVD_OK;
}

extern "C" int svd_world_set_tiling(svd_world* w, uint32_t tile_w) {
  if (!w) return svd_fail(SVD_EINVAL, "svd_world_set_tiling: null world");
  if (tile_w == 0) tile_w = kViewTileW;
  if (!(tile_w == 8 || tile_w == 16 || tile_w == 32 || tile_w == 64))
    return svd_fail(SVD_EINVAL, "tiling: tile width must be 8, 16, 32 or 64");
  w->tile_w = tile_w;
  return SVD_OK;
}

extern "C" int svd_world_get_tiling(const svd_world* w, uint32_t* tile_w) {
  if (!w || !tile_w) return svd_fail(SVD_EINVAL, "svd_world_get_tiling: null argument");
  *tile_w = w->tile_w;
  return SVD_OK;
}

extern "C" int svd_trace_frame(svd_world* w, const svd_ray_frame* f, svd_hit* out_dev, uint32_t flags,
                               void* stream) {
  if (!w || !f || !out_dev) return svd_fail(SVD_EINVAL, "svd_trace_frame: null argument");
  int rc = svd_view_stage(w, f, flags, stream);
  if (rc) return rc;
  return svd_view_trace(w, f, out_dev, stream);
}

extern "C" int svd_trace_view(svd_world* w, const svd_camera* cam, svd_hit* out_dev, uint32_t flags,
                              void* stream) {
  if (!w || !cam || !out_dev) return svd_fail(SVD_EINVAL, "svd_trace_view: null argument");
  svd_ray_frame f;
  int rc = svd_camera_frame(cam, &f);
  if (rc) return rc;
  return svd_trace_frame(w, &f, out_dev, flags, stream);
}

extern "C" int svd_view_table(svd_world* w, uint32_t* out, uint32_t n, void* stream) {
  if (!w || !out || n < w->nchunks) return svd_fail(SVD_EINVAL, "svd_view_table: bad argument");
  hipStream_t s = (hipStream_t)stream;
  HIP_OK(hipMemcpyAsync(out, w->d_view, (size_t)w->nchunks * 4, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  return SVD_OK;
}

// ------------------------------------------------------------ view batches
// Capture reset + stage + persistent trace as the batch's graph (again after
// an occupancy change); every batch reuses it.
static int batch_capture(svd_batch* b) {
  svd_world* w = b->w;
  BatchParams p;
  memset(&p, 0, sizeof(p));
  p.views = b->d_views;
  p.hdr = b->d_hdr;
  p.max_views = b->max_views;
  memcpy(p.grid, w->desc.grid, sizeof(p.grid));
  p.chunk_log2 = w->desc.chunk_log2;
  p.lod_count = w->desc.lod_count;
  memcpy(p.thr, w->desc.lod_threshold, sizeof(p.thr));
  p.nchunks = w->nchunks;
  p.desc = w->d_desc;
  p.view_tables = b->d_tables;
  p.queue = b->d_queue;
  if (b->exec) {
    (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  hipGraph_t g = nullptr;
  int rc = SVD_OK;
  hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    rc = launch_batch(p, b->per_cu * b->cus, b->cap);
    hipError_t e2 = hipStreamEndCapture(b->cap, &g);
    if (rc == SVD_OK && e2 != hipSuccess) rc = svd_fail(SVD_EDEVICE, "batch capture: %s", hipGetErrorString(e2));
  } else {
    rc = svd_fail(SVD_EDEVICE, "batch capture: %s", hipGetErrorString(e));
  }
  if (rc == SVD_OK) {
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) rc = svd_fail(SVD_EDEVICE, "batch graph: %s", hipGetErrorString(e));
  }
  if (g) (void)hipGraphDestroy(g);
  return rc;
}

static int batch_release(svd_batch* b) {
  if (!b) return SVD_OK;
  int rc = SVD_OK;
  if (b->launched && b->finished && hipEventSynchronize(b->finished) != hipSuccess)
    rc = svd_fail(SVD_EDEVICE, "batch destroy: waiting for the last launch failed");
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->staged) (void)hipEventDestroy(b->staged);
  if (b->finished) (void)hipEventDestroy(b->finished);
  if (b->h_stage) (void)hipHostFree(b->h_stage);
  if (b->w && b->bytes) b->w->release(b->off, b->bytes);
  delete b;
  return rc;
}

extern "C" int svd_batch_create(svd_world* w, uint32_t max_views, svd_batch** out) {
  if (!w || !out || max_views == 0 || max_views > 65535) return svd_fail(SVD_EINVAL, "svd_batch_create: bad argument");
  *out = nullptr;
  svd_batch* b = new (std::nothrow) svd_batch();
  if (!b) return svd_fail(SVD_ENOMEM, "batch: out of host memory");
  b->w = w;
  b->max_views = max_views;
  const size_t views_bytes = (size_t)max_views * sizeof(BatchView);
  const size_t tables_bytes = ((size_t)max_views * w->nchunks * 4 + 255) / 256 * 256;
  b->bytes = kQueueBlockBytes + 256 + views_bytes + tables_bytes;
  if (!w->alloc(b->bytes, &b->off)) {
    b->bytes = 0;
    batch_release(b);
    return svd_fail(SVD_ENOMEM, "batch: pool has no room for %u views", max_views);
  }
  b->d_queue = (uint32_t*)(w->pool + b->off);
  b->d_hdr = (BatchHeader*)(w->pool + b->off + kQueueBlockBytes);
  b->d_views = (BatchView*)(w->pool + b->off + kQueueBlockBytes + 256);
  b->d_tables = (uint32_t*)(w->pool + b->off + kQueueBlockBytes + 256 + views_bytes);
  b->stage_bytes = 256 + views_bytes;
  hipError_t e = hipHostMalloc((void**)&b->h_stage, b->stage_bytes, hipHostMallocDefault);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->staged, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->finished, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
  uint32_t per_cu = 0;
  int dev = 0, cus = 0;
  if (e == hipSuccess) e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) {
    batch_release(b);
    return svd_fail(SVD_EDEVICE, "batch: %s", hipGetErrorString(e));
  }
  int rc = batch_trace_occupancy(&per_cu);
  if (rc) { batch_release(b); return rc; }
  b->cus = (uint32_t)cus;
  b->max_per_cu = b->per_cu = per_cu;
  memset(b->h_stage, 0, b->stage_bytes);
  rc = batch_capture(b);
  if (rc) { batch_release(b); return rc; }
  *out = b;
  return SVD_OK;
}

extern "C" int svd_batch_set_occupancy(svd_batch* b, uint32_t blocks_per_cu) {
  if (!b) return svd_fail(SVD_EINVAL, "svd_batch_set_occupancy: null batch");
  if (blocks_per_cu > b->max_per_cu)
    return svd_fail(SVD_EINVAL, "occupancy: at most %u trace blocks per CU", b->max_per_cu);
  const uint32_t n = blocks_per_cu ? blocks_per_cu : b->max_per_cu;
  if (n == b->per_cu && b->exec) return SVD_OK;
  if (b->launched) {  // a launch of the old graph may still run; its exec must outlive it
    hipError_t e = hipEventSynchronize(b->finished);
    if (e != hipSuccess) return svd_fail(SVD_EDEVICE, "batch: %s", hipGetErrorString(e));
  }
  b->per_cu = n;
  return batch_capture(b);
}

extern "C" void svd_batch_destroy(svd_batch* b) { batch_release(b); }

extern "C" int svd_batch_set_tiling(svd_batch* b, uint32_t tile_w, uint32_t claim) {
  if (!b || !(tile_w == 8 || tile_w == 16 || tile_w == 32 || tile_w == 64) || claim < 1 || claim > 16)
    return svd_fail(SVD_EINVAL, "batch tiling: tile width 8/16/32/64 and claim 1..16");
  b->tile_w = tile_w;
  b->claim = claim;
  return SVD_OK;
}

extern "C" int svd_batch_get_tiling(const svd_batch* b, uint32_t* tile_w, uint32_t* claim,
                                    uint32_t* blocks_per_cu) {
  if (!b || !tile_w || !claim || !blocks_per_cu) return svd_fail(SVD_EINVAL, "svd_batch_get_tiling: null argument");
  *tile_w = b->tile_w;
  *claim = b->claim;
  *blocks_per_cu = b->per_cu;
  return SVD_OK;
}

int batch_enqueue(svd_batch* b, const svd_ray_frame* frames, svd_hit* const* outs, uint32_t n, uint32_t flags,
                  hipStream_t s) {
  if (n == 0 || n > b->max_views) return svd_fail(SVD_EINVAL, "batch: %u views, 1..%u allowed", n, b->max_views);
  if (flags & ~(SVD_NO_CULL | SVD_BEAM)) return svd_fail(SVD_EINVAL, "batch: unknown flags");
  svd_world* w = b->w;
  if (w->absent) return svd_fail(SVD_ENOTFOUND, "batch: %u (chunk, LOD) slots were never uploaded", w->absent);
  const uint32_t tw = b->tile_w, th = 64 / tw;
  uint64_t tiles = 0;
  for (uint32_t v = 0; v < n; v++) {
    int rc = check_frame(&frames[v]);
    if (rc) return rc;
    if (!outs[v]) return svd_fail(SVD_EINVAL, "batch: null output for view %u", v);
    tiles += (uint64_t)((frames[v].width + tw - 1) / tw) * ((frames[v].height + th - 1) / th);
  }
  if (tiles >= (1ull << 31)) return svd_fail(SVD_EINVAL, "batch: too many tiles");
  // the previous upload must have left the staging buffer before it is rewritten
  if (b->stage_pending) {
    hipError_t e = hipEventSynchronize(b->staged);
    if (e != hipSuccess) return svd_fail(SVD_EDEVICE, "batch: %s", hipGetErrorString(e));
    b->stage_pending = false;
  }
  BatchHeader* h = (BatchHeader*)b->h_stage;
  BatchView* vs = (BatchView*)(b->h_stage + 256);
  memset(h, 0, sizeof(*h));
  h->nviews = n;
  h->total_tiles = (uint32_t)tiles;
  h->tile_w = tw;
  h->claim = b->claim;
  h->beam = (flags & SVD_BEAM) != 0;
  uint32_t tbase = 0;
  for (uint32_t v = 0; v < n; v++) {
    const svd_ray_frame& f = frames[v];
    BatchView& bv = vs[v];
    memset(&bv, 0, sizeof(bv));
    memcpy(bv.O, f.O, sizeof(bv.O));
    memcpy(bv.A, f.A, sizeof(bv.A));
    memcpy(bv.BX, f.BX, sizeof(bv.BX));
    memcpy(bv.BY, f.BY, sizeof(bv.BY));
    bv.cull = !(flags & SVD_NO_CULL) && cull_planes(&f, bv.n);
    bv.out = (uint64_t)(uintptr_t)outs[v];
    bv.W = f.width;
    bv.H = f.height;
    bv.tiles_x = (f.width + tw - 1) / tw;
    bv.tile_base = tbase;
    tbase += bv.tiles_x * ((f.height + th - 1) / th);
  }
  HIP_OK(hipMemcpyAsync(b->d_hdr, b->h_stage, 256 + (size_t)n * sizeof(BatchView), hipMemcpyHostToDevice, s));
  HIP_OK(hipEventRecord(b->staged, s));
  b->stage_pending = true;
  HIP_OK(hipGraphLaunch(b->exec, s));
  HIP_OK(hipEventRecord(b->finished, s));
  b->launched = true;
  return SVD_OK;
}

int batch_enqueue_single(svd_batch* b, const svd_ray_frame* f, svd_hit* out, uint32_t flags, hipStream_t s) {
  if (flags & ~(SVD_NO_CULL | SVD_BEAM)) return svd_fail(SVD_EINVAL, "batch: unknown flags");
  if (!out) return svd_fail(SVD_EINVAL, "batch: null output");
  svd_world* w = b->w;
  if (w->absent) return svd_fail(SVD_ENOTFOUND, "batch: %u (chunk, LOD) slots were never uploaded", w->absent);
  int rc = check_frame(f);
  if (rc) return rc;
  // the graph's trace leaves its counters where they ended: start from zero
  rc = launch_queue_clear(b->d_queue, s);
  if (rc) return rc;
  StageParams sp = world_stage_params(w, f, flags & SVD_NO_CULL, w->d_desc);
  sp.view = b->d_tables;
  rc = launch_chunk_stage(sp, s);
  if (rc) return rc;
  const bool beam = (flags & SVD_BEAM) != 0;
  if (beam) {
    rc = launch_beam(view_beam_params(w, f, b->d_tables, out), s);
    if (rc) return rc;
  }
  const TraceParams tp = view_trace_params(w, f, b->d_queue, b->d_tables, out, beam);
  rc = launch_trace(tp, view_trace_blocks(w, tp), s);
  if (rc) return rc;
  HIP_OK(hipEventRecord(b->finished, s));
  b->launched = true;
  return SVD_OK;
}

extern "C" int svd_batch_trace_frames(svd_batch* b, const svd_ray_frame* frames, uint32_t n,
                                      svd_hit* out_dev, uint64_t out_records, uint32_t flags, void* stream) {
  if (!b || !frames || !out_dev || n == 0) return svd_fail(SVD_EINVAL, "svd_batch_trace: bad argument");
  if (n > b->max_views) return svd_fail(SVD_EINVAL, "batch: %u views > max %u", n, b->max_views);
  std::vector<svd_hit*> outs(n);
  uint64_t px_total = 0;
  for (uint32_t v = 0; v < n; v++) {
    outs[v] = out_dev + px_total;
    px_total += (uint64_t)frames[v].width * frames[v].height;
  }
  if (px_total > out_records) return svd_fail(SVD_EINVAL, "batch: output holds %llu records, views need %llu",
                                              (unsigned long long)out_records, (unsigned long long)px_total);
  return batch_enqueue(b, frames, outs.data(), n, flags, (hipStream_t)stream);
}

extern "C" int svd_batch_trace(svd_batch* b, const svd_camera* cams, uint32_t n, svd_hit* out_dev,
                               uint64_t out_records, uint32_t flags, void* stream) {
  if (!b || !cams || n == 0) return svd_fail(SVD_EINVAL, "svd_batch_trace: bad argument");
  if (n > b->max_views) return svd_fail(SVD_EINVAL, "batch: %u views > max %u", n, b->max_views);
  std::vector<svd_ray_frame> f(n);
  for (uint32_t v = 0; v < n; v++) {
    int rc = svd_camera_frame(&cams[v], &f[v]);
    if (rc) return rc;
  }
  return svd_batch_trace_frames(b, f.data(), n, out_dev, out_records, flags, stream);
}

// ------------------------------------------------- allocation-free batches
// svd_batch_trace_frames without a batch object: the queue block, header,
// views and view tables live in the library's static per-GPU array (laid out
// like a batch's pool area), the views reach it as kernel arguments, and the
// kernels run directly on the caller's stream.  Nothing is allocated: no
// device or pinned memory, no stream, event or graph, no host heap.
extern "C" int svd_batch_trace_frames_static(svd_world* w, const svd_ray_frame* frames, uint32_t n,
                                             svd_hit* out_dev, uint64_t out_records, uint32_t flags,
                                             void* stream) {
  if (!w || !frames || !out_dev || n == 0) return svd_fail(SVD_EINVAL, "svd_batch_trace_frames_static: bad argument");
  if (flags & ~(SVD_NO_CULL | SVD_BEAM)) return svd_fail(SVD_EINVAL, "static batch: unknown flags");
  if (w->absent) return svd_fail(SVD_ENOTFOUND, "static batch: %u (chunk, LOD) slots were never uploaded", w->absent);
  const size_t tables = ((size_t)n * w->nchunks * 4 + 255) / 256 * 256;
  const size_t need = kQueueBlockBytes + 256 + (size_t)n * sizeof(BatchView) + tables;
  if (n > 65535 || need > kStaticScratchBytes)
    return svd_fail(SVD_ENOMEM, "static batch: %u views over %u chunks need %zu bytes of scratch; the limit is %zu",
                    n, w->nchunks, need, kStaticScratchBytes);
  constexpr uint32_t tw = kViewTileW, th = 64 / kViewTileW;
  uint64_t tiles = 0, px_total = 0;
  for (uint32_t v = 0; v < n; v++) {
    const int rc = check_frame(&frames[v]);
    if (rc) return rc;
    tiles += (uint64_t)((frames[v].width + tw - 1) / tw) * ((frames[v].height + th - 1) / th);
    px_total += (uint64_t)frames[v].width * frames[v].height;
  }
  if (tiles >= (1ull << 31)) return svd_fail(SVD_EINVAL, "static batch: too many tiles");
  if (px_total > out_records)
    return svd_fail(SVD_EINVAL, "static batch: output holds %llu records, views need %llu",
                    (unsigned long long)out_records, (unsigned long long)px_total);
  StaticDevice dev;
  int rc = static_device(&dev);
  if (rc) return rc;
  BatchParams p;
  memset(&p, 0, sizeof(p));
  p.queue = (uint32_t*)dev.scratch;
  p.hdr = (BatchHeader*)(dev.scratch + kQueueBlockBytes);
  BatchView* d_views = (BatchView*)(dev.scratch + kQueueBlockBytes + 256);
  p.views = d_views;
  p.view_tables = (uint32_t*)(dev.scratch + kQueueBlockBytes + 256 + (size_t)n * sizeof(BatchView));
  p.max_views = n;
  memcpy(p.grid, w->desc.grid, sizeof(p.grid));
  p.chunk_log2 = w->desc.chunk_log2;
  p.lod_count = w->desc.lod_count;
  memcpy(p.thr, w->desc.lod_threshold, sizeof(p.thr));
  p.nchunks = w->nchunks;
  p.desc = w->d_desc;
  BatchHeader h;
  memset(&h, 0, sizeof(h));
  h.nviews = n;
  h.total_tiles = (uint32_t)tiles;
  h.tile_w = tw;
  h.claim = 1;
  h.beam = (flags & SVD_BEAM) != 0;
  BatchView pack[kPackViews];
  uint32_t tbase = 0;
  uint64_t rec = 0;
  for (uint32_t v0 = 0; v0 < n; v0 += kPackViews) {
    const uint32_t cnt = std::min(kPackViews, n - v0);
    for (uint32_t i = 0; i < cnt; i++) {
      const svd_ray_frame& f = frames[v0 + i];
      BatchView& bv = pack[i];
      memset(&bv, 0, sizeof(bv));
      memcpy(bv.O, f.O, sizeof(bv.O));
      memcpy(bv.A, f.A, sizeof(bv.A));
      memcpy(bv.BX, f.BX, sizeof(bv.BX));
      memcpy(bv.BY, f.BY, sizeof(bv.BY));
      bv.cull = !(flags & SVD_NO_CULL) && cull_planes(&f, bv.n);
      bv.out = (uint64_t)(uintptr_t)(out_dev + rec);
      bv.W = f.width;
      bv.H = f.height;
      bv.tiles_x = (f.width + tw - 1) / tw;
      bv.tile_base = tbase;
      tbase += bv.tiles_x * ((f.height + th - 1) / th);
      rec += (uint64_t)f.width * f.height;
    }
    rc = launch_set_views(d_views + v0, pack, cnt, v0 == 0 ? p.hdr : nullptr, v0 == 0 ? &h : nullptr, stream);
    if (rc) return rc;
  }
  const uint32_t blocks = (uint32_t)std::min<uint64_t>((uint64_t)dev.per_cu * dev.cus, (tiles + 3) / 4);
  return launch_batch_direct(p, n, blocks, (flags & SVD_BEAM) != 0, stream);
}
