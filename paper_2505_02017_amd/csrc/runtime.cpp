// Host runtime of libsvdag: errors, camera frame, world and pool management,
// chunk upload/evict, and the per-view entry points that enqueue the GPU
// chunk stage and trace.  Compile with -ffp-contract=off: the camera frame is
// defined by a fixed sequence of IEEE double operations.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>

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
struct svd_world {
  svd_world_desc desc;
  uint32_t nchunks = 0;
  uint8_t* pool = nullptr;
  size_t pool_bytes = 0;
  DevDag* d_desc = nullptr;
  uint32_t* d_view = nullptr;
  size_t data_begin = 0;
  std::map<size_t, size_t> free_blocks;  // offset -> bytes
  struct Region { size_t off = 0, bytes = 0; bool resident = false; };
  std::vector<Region> region;
  uint32_t missing = 0;  // chunks never uploaded or evicted
  size_t used = 0;
  svd_ray_frame staged;  // frame of the last chunk stage (its view table)
  bool has_staged = false;

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
  if (pool_bytes < desc_bytes + view_bytes) return svd_fail(SVD_ENOMEM, "world: pool smaller than its tables");
  try {
    svd_world* w = new svd_world();
    w->desc = *desc;
    w->nchunks = (uint32_t)n;
    w->pool = (uint8_t*)pool_dev;
    w->pool_bytes = pool_bytes;
    w->d_desc = (DevDag*)pool_dev;
    w->d_view = (uint32_t*)(w->pool + desc_bytes);
    w->data_begin = desc_bytes + view_bytes;
    if (pool_bytes > w->data_begin) w->free_blocks[w->data_begin] = (pool_bytes - w->data_begin) / 256 * 256;
    w->region.resize(n);
    w->missing = (uint32_t)n;
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

extern "C" int svd_chunk_upload(svd_world* w, const uint32_t c[3], const svd_blob* b, void* stream) {
  if (!w || !b) return svd_fail(SVD_EINVAL, "svd_chunk_upload: null argument");
  uint32_t ci;
  int rc = chunk_index(w, c, &ci);
  if (rc) return rc;
  if (b->chunk_log2 != w->desc.chunk_log2 || b->lod_count != w->desc.lod_count)
    return svd_fail(SVD_EINVAL, "upload: blob chunk size or LOD count differs from the world's");
  size_t off = 0;
  const size_t bytes = b->image.size();
  if (bytes && !w->alloc(bytes, &off))
    return svd_fail(SVD_ENOMEM, "upload: pool full (%zu bytes requested, %zu used of %zu)", bytes, w->used,
                    w->pool_bytes - w->data_begin);
  hipStream_t s = (hipStream_t)stream;
  if (bytes) {
    hipError_t e = hipMemcpyAsync(w->pool + off, b->image.data(), bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) {
      w->release(off, bytes);
      return svd_fail(SVD_EDEVICE, "upload: hipMemcpyAsync: %s", hipGetErrorString(e));
    }
  }
  DevDag d[4];
  memset(d, 0, sizeof(d));
  const uint64_t base = (uint64_t)(uintptr_t)(w->pool + off);
  for (uint32_t k = 0; k < b->lod_count; k++) {
    const LodData& L = b->lod[k];
    d[k].nodes = base + L.off_nodes;
    d[k].leaves = base + L.off_leaves;
    d[k].pre = base + L.off_pre;
    d[k].rle_start = base + L.off_rle_start;
    d[k].rle_mat = base + L.off_rle_mat;
    d[k].rle_n = (uint32_t)L.rle_start.size();
    d[k].root = L.root_word;
    d[k].solid = L.n_solid;
    for (int a = 0; a < 3; a++) {
      d[k].lo[a] = L.lo[a];
      d[k].hi[a] = L.hi[a];
    }
  }
  rc = launch_set_desc(w->d_desc + (size_t)ci * 4, d, 4, stream);
  if (rc) {
    if (bytes) w->release(off, bytes);
    return rc;
  }
  svd_world::Region& r = w->region[ci];
  if (r.resident) {
    if (r.bytes) w->release(r.off, r.bytes);
  } else {
    w->missing--;
  }
  r.off = off;
  r.bytes = bytes;
  r.resident = true;
  return SVD_OK;
}

extern "C" int svd_chunk_evict(svd_world* w, const uint32_t c[3]) {
  if (!w) return svd_fail(SVD_EINVAL, "svd_chunk_evict: null world");
  uint32_t ci;
  int rc = chunk_index(w, c, &ci);
  if (rc) return rc;
  svd_world::Region& r = w->region[ci];
  if (!r.resident) return svd_fail(SVD_ENOTFOUND, "evict: chunk not resident");
  if (r.bytes) w->release(r.off, r.bytes);
  r = svd_world::Region();
  w->missing++;
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

static int check_frame(const svd_ray_frame* f) {
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

extern "C" int svd_view_stage(svd_world* w, const svd_ray_frame* f, uint32_t flags, void* stream) {
  if (!w || !f) return svd_fail(SVD_EINVAL, "svd_view_stage: null argument");
  if (flags & ~SVD_NO_CULL) return svd_fail(SVD_EINVAL, "stage: unknown flags");
  int rc = check_frame(f);
  if (rc) return rc;
  if (w->missing) return svd_fail(SVD_ENOTFOUND, "stage: %u chunks are not resident", w->missing);
  StageParams sp;
  memset(&sp, 0, sizeof(sp));
  memcpy(sp.O, f->O, sizeof(sp.O));
  sp.cull = !(flags & SVD_NO_CULL) && cull_planes(f, sp.n);
  memcpy(sp.grid, w->desc.grid, sizeof(sp.grid));
  sp.chunk_log2 = w->desc.chunk_log2;
  sp.lod_count = w->desc.lod_count;
  memcpy(sp.thr, w->desc.lod_threshold, sizeof(sp.thr));
  sp.nchunks = w->nchunks;
  sp.desc = w->d_desc;
  sp.view = w->d_view;
  rc = launch_chunk_stage(sp, stream);
  if (rc) return rc;
  w->staged = *f;
  w->has_staged = true;
  return SVD_OK;
}

extern "C" int svd_view_trace(svd_world* w, const svd_ray_frame* f, svd_hit* out_dev, void* stream) {
  if (!w || !f || !out_dev) return svd_fail(SVD_EINVAL, "svd_view_trace: null argument");
  if (!w->has_staged || !same_frame(w->staged, *f))
    return svd_fail(SVD_EINVAL, "trace: the frame was not staged by the last svd_view_stage");
  if (w->missing) return svd_fail(SVD_ENOTFOUND, "trace: %u chunks are not resident", w->missing);
  const uint32_t W = f->width, H = f->height;
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
  tp.tiles_x = (W + 15) / 16;
  tp.nblocks = tp.tiles_x * ((H + 15) / 16);
  tp.view = w->d_view;
  tp.desc = w->d_desc;
  tp.out = out_dev;
  return launch_trace(tp, stream);
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
