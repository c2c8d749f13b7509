// Autotuning of the persistent traces' work shape, and a file cache of the
// choices.  The per-view trace is tuned over its wave tile (8x8, 16x4, 32x2
// or 64x1 pixels) and its occupancy, the batched trace over its tile, claim
// and occupancy.  The work shape only decides which wave traces which pixel,
// and when, never a record, so every configuration is correct; the fastest
// depends on the device, the kernels and the workload, which make the key:
//   dev=<arch>/<CUs>cu/<clock>mhz kernel=<source hash> kind=view|batch
//   cl=<chunk log2> grid=<gx>x<gy>x<gz> lods=<n> flags=<f> views=<n> res=<WxH*count,...>
// The cache is a text file, one line per key: the key, a tab, then
// "tile_w claim blocks_per_cu ms".  A store rewrites the whole file through
// a temporary and a rename, so a reader never sees half a file; of two
// processes storing at once one entry may be lost (and is tuned again).
#include <hip/hip_runtime.h>

#include <unistd.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "svdag_internal.h"

#ifndef SVD_KERNEL_HASH
#define SVD_KERNEL_HASH "unknown"
#endif

using namespace svd;

extern "C" const char* svd_kernel_hash(void) { return SVD_KERNEL_HASH; }

namespace {

using Res = std::vector<std::pair<uint32_t, uint32_t>>;

bool valid_tile(uint32_t tw) { return tw == 8 || tw == 16 || tw == 32 || tw == 64; }

// Device part of the key: architecture (with its target features), compute
// units and peak clock.  The device's marketing name is not used: it is
// generic on some systems and reads empty under some profilers.
int device_key(std::string* out) {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return svd_fail(SVD_EDEVICE, "tune: cannot query the device");
  std::string arch(prop.gcnArchName);
  for (char& c : arch)
    if (c == ' ' || c == '\t' || c == '\n' || c == '\r') c = '_';
  *out = "dev=" + arch + "/" + std::to_string(prop.multiProcessorCount) + "cu/" +
         std::to_string(prop.clockRate / 1000) + "mhz";
  return SVD_OK;
}

// Resolutions of a workload: the distinct WxH with their counts, ascending;
// a list longer than 120 characters becomes its view count, pixel total and
// an FNV-1a hash of the sorted list.
std::string res_key(Res wh) {
  std::sort(wh.begin(), wh.end());
  std::string s;
  for (size_t i = 0; i < wh.size();) {
    size_t j = i;
    while (j < wh.size() && wh[j] == wh[i]) j++;
    s += (s.empty() ? "" : ",") + std::to_string(wh[i].first) + "x" + std::to_string(wh[i].second) + "*" +
         std::to_string(j - i);
    i = j;
  }
  if (s.size() <= 120) return "res=" + s;
  uint64_t px = 0, h = 1469598103934665603ull;
  auto mix = [&h](uint32_t v) {
    for (int i = 0; i < 4; i++) {
      h ^= (v >> (8 * i)) & 0xFFu;
      h *= 1099511628211ull;
    }
  };
  for (const auto& p : wh) {
    px += (uint64_t)p.first * p.second;
    mix(p.first);
    mix(p.second);
  }
  char buf[96];
  snprintf(buf, sizeof(buf), "res=%zu:%llu:%016llx", wh.size(), (unsigned long long)px, (unsigned long long)h);
  return buf;
}

int workload_key(const svd_world* w, const char* kind, uint32_t flags, const Res& wh, std::string* key) {
  std::string dev;
  const int rc = device_key(&dev);
  if (rc) return rc;
  char buf[192];
  snprintf(buf, sizeof(buf), " kernel=%s kind=%s cl=%u grid=%ux%ux%u lods=%u flags=%u views=%zu ", SVD_KERNEL_HASH,
           kind, w->desc.chunk_log2, w->desc.grid[0], w->desc.grid[1], w->desc.grid[2], w->desc.lod_count, flags,
           wh.size());
  *key = dev + buf + res_key(wh);
  if (key->size() >= sizeof(svd_tune_result::key)) return svd_fail(SVD_EINVAL, "tune: cache key too long");
  return SVD_OK;
}

// Every line of the file (without the newline); false if it cannot be read.
bool read_lines(const char* path, std::vector<std::string>* lines) {
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char* buf = nullptr;
  size_t cap = 0;
  ssize_t n;
  while ((n = getline(&buf, &cap, f)) >= 0) {
    while (n > 0 && (buf[n - 1] == '\n' || buf[n - 1] == '\r')) n--;
    lines->emplace_back(buf, (size_t)n);
  }
  free(buf);
  fclose(f);
  return true;
}

bool has_key(const std::string& line, const std::string& key) {
  return line.size() > key.size() && line[key.size()] == '\t' && line.compare(0, key.size(), key) == 0;
}

// The last entry for `key`: v = {tile_w, claim, blocks_per_cu}.
bool cache_find(const char* path, const std::string& key, uint32_t v[3], float* ms) {
  std::vector<std::string> lines;
  if (!read_lines(path, &lines)) return false;
  bool found = false;
  for (const std::string& l : lines) {
    uint32_t t[3];
    float m;
    if (has_key(l, key) && sscanf(l.c_str() + key.size() + 1, "%u %u %u %f", &t[0], &t[1], &t[2], &m) == 4) {
      memcpy(v, t, sizeof(t));
      *ms = m;
      found = true;
    }
  }
  return found;
}

int cache_store(const char* path, const std::string& key, uint32_t tw, uint32_t claim, uint32_t occ, float ms) {
  std::vector<std::string> lines;
  read_lines(path, &lines);  // a missing file starts empty
  const std::string tmp = std::string(path) + ".tmp." + std::to_string((long)getpid());
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return svd_fail(SVD_EIO, "tune cache: cannot create %s", tmp.c_str());
  bool ok = true;
  if (lines.empty() || lines[0].rfind("#", 0) != 0)
    ok = fputs("# libsvdag tuning cache: key<TAB>tile_w claim blocks_per_cu ms\n", f) >= 0;
  for (const std::string& l : lines)
    if (ok && !has_key(l, key) && !l.empty()) ok = fprintf(f, "%s\n", l.c_str()) >= 0;
  if (ok) ok = fprintf(f, "%s\t%u %u %u %.4f\n", key.c_str(), tw, claim, occ, ms) >= 0;
  if (fclose(f) != 0) ok = false;
  if (!ok || rename(tmp.c_str(), path) != 0) {
    unlink(tmp.c_str());
    return svd_fail(SVD_EIO, "tune cache: cannot write %s", path);
  }
  return SVD_OK;
}

struct Events {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ~Events() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
  int create() {
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
      return svd_fail(SVD_EDEVICE, "tune: event create failed");
    return SVD_OK;
  }
};

// Median over `reps` timed runs (after one warm-up run) of `run`, HIP events
// on `s`.
template <class F>
int median_time(F run, uint32_t reps, hipStream_t s, const Events& ev, float* med) {
  std::vector<float> t;
  for (uint32_t r = 0; r <= reps; r++) {
    if (hipEventRecord(ev.e0, s) != hipSuccess) return svd_fail(SVD_EDEVICE, "tune: event record failed");
    const int rc = run();
    if (rc) return rc;
    if (hipEventRecord(ev.e1, s) != hipSuccess || hipEventSynchronize(ev.e1) != hipSuccess)
      return svd_fail(SVD_EDEVICE, "tune: sync failed");
    float ms = 0;
    if (hipEventElapsedTime(&ms, ev.e0, ev.e1) != hipSuccess) return svd_fail(SVD_EDEVICE, "tune: event timing failed");
    if (r > 0) t.push_back(ms);
  }
  std::sort(t.begin(), t.end());
  *med = t[t.size() / 2];
  return SVD_OK;
}

// Batch autotuner: every (tile width, claim) at the current occupancy, then
// every occupancy from the maximum down to 2 blocks per CU at the best
// tiling; keeps the fastest.
int batch_tune(svd_batch* b, const svd_camera* cams, uint32_t n, svd_hit* out_dev, uint64_t out_records,
               uint32_t reps, hipStream_t s, float* best_ms, uint32_t* timed) {
  Events ev;
  int rc = ev.create();
  if (rc) return rc;
  auto run = [&] { return svd_batch_trace(b, cams, n, out_dev, out_records, 0, s); };
  const uint32_t widths[] = {8, 16, 32, 64};
  const uint32_t claims[] = {1, 2, 4};
  uint32_t bw = b->tile_w, bc = b->claim, bo = b->per_cu, count = 0;
  float best = 3.4e38f;
  for (uint32_t tw : widths) {
    for (uint32_t cl : claims) {
      if (rc) break;
      b->tile_w = tw;
      b->claim = cl;
      float med = 0;
      rc = median_time(run, reps, s, ev, &med);
      count++;
      if (rc == SVD_OK && med < best) {
        best = med;
        bw = tw;
        bc = cl;
      }
    }
  }
  b->tile_w = bw;
  b->claim = bc;
  const uint32_t start = b->per_cu;
  for (uint32_t occ = b->max_per_cu; occ >= 2 && rc == SVD_OK; occ--) {
    if (occ == start) continue;  // already timed above
    rc = svd_batch_set_occupancy(b, occ);
    float med = 0;
    if (rc == SVD_OK) rc = median_time(run, reps, s, ev, &med);
    count++;
    if (rc == SVD_OK && med < best) {
      best = med;
      bo = occ;
    }
  }
  const int rc2 = svd_batch_set_occupancy(b, bo);
  if (rc == SVD_OK) rc = rc2;
  if (best_ms) *best_ms = best;
  if (timed) *timed = count;
  return rc;
}

void fill(svd_tune_result* res, const std::string& key, uint32_t tw, uint32_t claim, uint32_t occ, float ms,
          uint32_t from_cache, uint32_t timed) {
  res->tile_w = tw;
  res->claim = claim;
  res->blocks_per_cu = occ;
  res->from_cache = from_cache;
  res->ms = ms;
  res->configs_timed = timed;
  snprintf(res->key, sizeof(res->key), "%s", key.c_str());
}

}  // namespace

extern "C" int svd_tune_cache_lookup(const char* cache_path, const char* key, svd_tune_result* res) {
  if (!cache_path || !*cache_path || !key || !*key || !res)
    return svd_fail(SVD_EINVAL, "svd_tune_cache_lookup: null or empty argument");
  memset(res, 0, sizeof(*res));
  const std::string k(key);
  if (k.size() >= sizeof(res->key)) return svd_fail(SVD_EINVAL, "tune cache: key too long");
  uint32_t v[3];
  float ms = 0;
  if (!cache_find(cache_path, k, v, &ms)) return svd_fail(SVD_ENOTFOUND, "tune cache: no entry for the key");
  fill(res, k, v[0], v[1], v[2], ms, 1, 0);
  return SVD_OK;
}

extern "C" int svd_tune_cache_store(const char* cache_path, const svd_tune_result* res) {
  if (!cache_path || !*cache_path || !res) return svd_fail(SVD_EINVAL, "svd_tune_cache_store: null or empty argument");
  const size_t n = strnlen(res->key, sizeof(res->key));
  if (n == 0 || n == sizeof(res->key)) return svd_fail(SVD_EINVAL, "tune cache: key empty or not terminated");
  if (strpbrk(res->key, "\t\n\r")) return svd_fail(SVD_EINVAL, "tune cache: key holds a tab or a line break");
  if (!valid_tile(res->tile_w) || res->claim < 1 || res->claim > 16 || res->blocks_per_cu < 1)
    return svd_fail(SVD_EINVAL, "tune cache: tile_w must be 8/16/32/64, claim 1..16, blocks_per_cu >= 1");
  return cache_store(cache_path, std::string(res->key, n), res->tile_w, res->claim, res->blocks_per_cu, res->ms);
}

extern "C" int svd_batch_tune(svd_batch* b, const svd_camera* cams, uint32_t n, svd_hit* out_dev,
                              uint64_t out_records, uint32_t reps, void* stream, float* best_ms) {
  if (!b || !cams || n == 0 || reps == 0 || reps > 64) return svd_fail(SVD_EINVAL, "svd_batch_tune: bad argument");
  return batch_tune(b, cams, n, out_dev, out_records, reps, (hipStream_t)stream, best_ms, nullptr);
}

extern "C" int svd_batch_tune_cached(svd_batch* b, const svd_camera* cams, uint32_t n, svd_hit* out_dev,
                                     uint64_t out_records, uint32_t reps, const char* cache_path, void* stream,
                                     svd_tune_result* res) {
  if (!b || !cams || n == 0 || !out_dev || !res || reps == 0 || reps > 64)
    return svd_fail(SVD_EINVAL, "svd_batch_tune_cached: bad argument");
  if (n > b->max_views) return svd_fail(SVD_EINVAL, "batch: %u views > max %u", n, b->max_views);
  memset(res, 0, sizeof(*res));
  Res wh(n);
  for (uint32_t v = 0; v < n; v++) wh[v] = {cams[v].width, cams[v].height};
  std::string key;
  int rc = workload_key(b->w, "batch", 0, wh, &key);
  if (rc) return rc;
  if (cache_path && *cache_path) {
    uint32_t v[3];
    float ms = 0;
    if (cache_find(cache_path, key, v, &ms) && valid_tile(v[0]) && v[1] >= 1 && v[1] <= 16 && v[2] >= 1 &&
        v[2] <= b->max_per_cu) {
      rc = svd_batch_set_tiling(b, v[0], v[1]);
      if (rc == SVD_OK) rc = svd_batch_set_occupancy(b, v[2]);
      if (rc) return rc;
      fill(res, key, v[0], v[1], v[2], ms, 1, 0);
      return SVD_OK;
    }
  }
  float best = 0;
  uint32_t timed = 0;
  rc = batch_tune(b, cams, n, out_dev, out_records, reps, (hipStream_t)stream, &best, &timed);
  if (rc) return rc;
  fill(res, key, b->tile_w, b->claim, b->per_cu, best, 0, timed);
  if (cache_path && *cache_path) return cache_store(cache_path, key, b->tile_w, b->claim, b->per_cu, best);
  return SVD_OK;
}

// Per-view autotuner: every tile width at the current occupancy, then every
// occupancy from the maximum down to 2 blocks per CU at the best width; the
// time of a configuration is the median over `reps` runs of the whole
// per-view pass (stage, beam with SVD_BEAM, trace) of every frame in turn.
extern "C" int svd_world_tune(svd_world* w, const svd_ray_frame* frames, uint32_t n, svd_hit* out_dev,
                              uint64_t out_records, uint32_t flags, uint32_t reps, const char* cache_path,
                              void* stream, svd_tune_result* res) {
  if (!w || !frames || n == 0 || !out_dev || !res || reps == 0 || reps > 64)
    return svd_fail(SVD_EINVAL, "svd_world_tune: bad argument");
  if (flags & ~(SVD_NO_CULL | SVD_BEAM)) return svd_fail(SVD_EINVAL, "tune: unknown flags");
  memset(res, 0, sizeof(*res));
  Res wh(n);
  for (uint32_t v = 0; v < n; v++) {
    const int rc = check_frame(&frames[v]);
    if (rc) return rc;
    if ((uint64_t)frames[v].width * frames[v].height > out_records)
      return svd_fail(SVD_EINVAL, "tune: output holds %llu records, frame %u needs %llu",
                      (unsigned long long)out_records, v, (unsigned long long)frames[v].width * frames[v].height);
    wh[v] = {frames[v].width, frames[v].height};
  }
  if (w->absent) return svd_fail(SVD_ENOTFOUND, "tune: %u (chunk, LOD) slots were never uploaded", w->absent);
  std::string key;
  int rc = workload_key(w, "view", flags, wh, &key);
  if (rc) return rc;
  if (cache_path && *cache_path) {
    uint32_t v[3];
    float ms = 0;
    if (cache_find(cache_path, key, v, &ms) && valid_tile(v[0]) && v[1] == 1 && v[2] >= 1 && v[2] <= w->max_per_cu) {
      w->tile_w = v[0];
      w->per_cu = v[2];
      fill(res, key, v[0], 1, v[2], ms, 1, 0);
      return SVD_OK;
    }
  }
  Events ev;
  rc = ev.create();
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  auto run = [&] {
    for (uint32_t v = 0; v < n; v++) {
      const int r = svd_trace_frame(w, &frames[v], out_dev, flags, s);
      if (r) return r;
    }
    return SVD_OK;
  };
  const uint32_t tw0 = w->tile_w, oc0 = w->per_cu;
  uint32_t bw = tw0, bo = oc0, timed = 0;
  float best = 3.4e38f;
  for (uint32_t tw : {8u, 16u, 32u, 64u}) {
    w->tile_w = tw;
    float med = 0;
    rc = median_time(run, reps, s, ev, &med);
    timed++;
    if (rc) break;
    if (med < best) {
      best = med;
      bw = tw;
    }
  }
  w->tile_w = bw;
  for (uint32_t occ = w->max_per_cu; occ >= 2 && rc == SVD_OK; occ--) {
    if (occ == oc0) continue;  // already timed above
    w->per_cu = occ;
    float med = 0;
    rc = median_time(run, reps, s, ev, &med);
    timed++;
    if (rc == SVD_OK && med < best) {
      best = med;
      bo = occ;
    }
  }
  if (rc) {  // leave the world as it was
    w->tile_w = tw0;
    w->per_cu = oc0;
    return rc;
  }
  w->tile_w = bw;
  w->per_cu = bo;
  fill(res, key, bw, 1, bo, best, 0, timed);
  if (cache_path && *cache_path) return cache_store(cache_path, key, bw, 1, bo, best);
  return SVD_OK;
}
