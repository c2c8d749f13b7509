// Request server of libsvdag: view requests of any size, arriving at any
// time, over a world whose pool holds only part of the map.
//
// One worker thread owns the world while the server lives.  It
//   - admits pending requests in arrival order: the chunk stage's decision
//     is evaluated on the host (the same function the GPU stage runs) to get
//     the (chunk, LOD) slots the view reads; resident ones are pinned,
//     missing ones are uploaded on the upload stream, evicting unpinned
//     slots in least-recently-used order when the pool is full.  A request
//     that does not fit while other work holds memory waits; one that does
//     not fit an idle pool fails with SVD_ENOMEM;
//   - packs admitted requests into launches (batched mode: up to max_views
//     requests and max_rays rays per captured batch graph; plain modes: one
//     stage + trace launch pair per request, serial on one stream or
//     concurrent on the flights' own streams and view tables) and keeps up to
//     `inflight` launches on the device, so requests that arrive while others
//     run are admitted as soon as a launch slot and memory free up
//     (continuous batching);
//   - reaps finished launches (event query), unpins their slots and reports
//     each request's submit, launch and completion times;
//   - optionally runs the streaming policy of Section 3.4 (an implicit chunk
//     octree cut by the LOD error of Eq. 1) on the recent camera positions,
//     prefetches the slots it wants into free pool space while nothing
//     waits, and evicts slots it does not want first.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "svdag_internal.h"

using namespace svd;

namespace {
using Clock = std::chrono::steady_clock;

struct Request {
  uint64_t tag = 0;
  svd_ray_frame frame;
  svd_hit* out = nullptr;
  uint32_t flags = 0;
  double t_submit = 0;
  std::vector<uint32_t> need;  // slots (chunk * 4 + lod) the view reads
  bool staged = false;         // `need` is computed
  bool waited = false;         // has waited for memory
};

struct Flight {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  svd_batch* batch = nullptr;  // batched mode
  std::vector<Request> reqs;
  double t_launch = 0;
  bool busy = false;
};

enum { kAdmitted = 0, kWait = 1 };  // admit(): or a negative SVD error
}  // namespace

struct svd_server {
  svd_world* w = nullptr;
  svd_server_desc d;
  int device = 0;
  Clock::time_point t0;
  std::vector<const svd_blob*> src;  // per chunk: where its LODs are uploaded from
  uint32_t sources = 0;
  std::vector<uint32_t> pins;        // per slot: in-flight or admitted requests reading it
  std::vector<uint64_t> last_use;    // per slot: admission sequence of its last reader
  uint64_t use_seq = 0;
  uint64_t data_bytes = 0;           // pool bytes of resident chunk LODs
  hipStream_t up = nullptr;          // uploads and descriptor writes
  hipEvent_t up_done = nullptr;      // recorded on `up` before a launch that follows new uploads
  bool up_dirty = false;             // uploads enqueued since up_done was last recorded
  bool up_pending = false;           // up_done has been recorded
  hipStream_t plain = nullptr;       // serial plain mode: every launch (on the world's view table)
  std::vector<Flight> fl;
  // streaming policy
  std::deque<std::array<int64_t, 4>> recent;  // last camera positions (2^16 units) and their chunk
  std::vector<uint8_t> wanted;               // per slot
  std::vector<uint32_t> want_order;          // wanted slots: coarse LODs first, then nearer first
  size_t want_next = 0;
  bool want_dirty = false;

  std::mutex mu;                     // guards everything below
  std::condition_variable wake;      // worker: submissions, stop
  std::condition_variable done_cv;   // pollers
  std::deque<Request> inbox;
  std::deque<svd_request_done> done;
  svd_server_stats st;
  bool started = false, stop = false;
  std::thread th;

  std::deque<Request> pending;       // worker-owned

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

static bool any_busy(const svd_server* s) {
  for (const Flight& f : s->fl)
    if (f.busy) return true;
  return false;
}

static void finish(svd_server* s, const Request& r, int status, uint32_t views, double t_launch, double t_done) {
  svd_request_done x;
  memset(&x, 0, sizeof(x));
  x.tag = r.tag;
  x.status = status;
  x.batch_views = views;
  x.t_submit = r.t_submit;
  x.t_launch = t_launch;
  x.t_done = t_done;
  std::lock_guard<std::mutex> lk(s->mu);
  s->done.push_back(x);
  if (status == SVD_OK) s->st.completed++;
  else s->st.failed++;
}

static void unpin(svd_server* s, const std::vector<uint32_t>& slots) {
  for (uint32_t sl : slots) s->pins[sl]--;
}

// Evict the least recently used resident slot that nobody pins, taking slots
// the streaming policy does not want before those it wants; false if there
// is none.
static bool evict_one(svd_server* s) {
  svd_world* w = s->w;
  size_t best = SIZE_MAX;
  for (int pass = 0; pass < 2 && best == SIZE_MAX; pass++) {
    for (size_t i = 0; i < w->slot.size(); i++) {
      if (w->slot[i].state != svd_world::kResident || !w->slot[i].bytes || s->pins[i]) continue;
      if (pass == 0 && !s->wanted.empty() && s->wanted[i]) continue;
      if (best == SIZE_MAX || s->last_use[i] < s->last_use[best]) best = i;
    }
  }
  if (best == SIZE_MAX) return false;
  const size_t bytes = w->slot[best].bytes;
  if (world_evict_lods(w, (uint32_t)(best / 4), 1u << (best % 4), s->up) != SVD_OK) return false;
  std::lock_guard<std::mutex> lk(s->mu);
  s->data_bytes -= bytes;
  s->st.evictions++;
  s->st.evict_bytes += bytes;
  s->st.pool_used = s->data_bytes;
  return true;
}

// Streaming policy (Section 3.4): walk an implicit octree over the chunk
// grid from each recent camera.  A node at level n covers 2^n chunks per
// axis.  LODs are per-chunk pyramids here, chosen by Eq. 1's distance rule,
// so the policy's LOD for a chunk at centre distance d is
//   LOD_f(d) = number of thresholds T with d >= T f   (f = streaming factor),
// the chunk's Eq. 1 LOD with every threshold stretched by f (f > 1 loads
// finer LODs farther out, ahead of a camera that approaches).  A node is
// split while a chunk in it could still get an LOD finer than the node's
// own (its LOD error, threshold x f - distance to the node, is positive);
// the chunks of a node that is not split are wanted at LOD_f and at their
// exact current LOD.  Wanted slots are ordered coarse LODs first, then
// nearer chunks first.
static uint32_t lod_at(const svd_world* w, double d, double f) {
  uint32_t k = 0;
  for (uint32_t j = 0; j + 1 < w->desc.lod_count; j++)
    if (d >= (double)w->desc.lod_threshold[j] * f) k++;
  return k;
}

static void policy_node(svd_server* s, const double cam[3], int n, const int64_t c[3],
                        std::vector<std::pair<double, uint32_t>>& out) {
  const svd_world* w = s->w;
  const int64_t span = (int64_t)1 << n;
  for (int a = 0; a < 3; a++)
    if (c[a] >= (int64_t)w->desc.grid[a]) return;
  const double S = (double)((int64_t)1 << w->desc.chunk_log2);
  const double f = s->d.streaming_factor;
  const int nl = (int)w->desc.lod_count;
  const int own = std::min(n, nl - 1);  // the LOD a node of this size stands for
  bool split = false;
  if (n > 0) {
    if (n > nl - 1) {
      split = true;  // no LOD this coarse: always refine
    } else {
      double d2 = 0;  // camera to the node's box (clipped to the grid)
      for (int a = 0; a < 3; a++) {
        const int64_t hi = std::min<int64_t>(c[a] + span, w->desc.grid[a]);
        const double lo_v = (double)c[a] * S, hi_v = (double)hi * S;
        const double e = cam[a] < lo_v ? lo_v - cam[a] : (cam[a] > hi_v ? cam[a] - hi_v : 0.0);
        d2 += e * e;
      }
      split = (double)w->desc.lod_threshold[own - 1] * std::max(f, 1.0) - std::sqrt(d2) > 0;  // LOD error
    }
  }
  if (split) {
    const int64_t h = span / 2;
    for (int o = 0; o < 8; o++) {
      const int64_t cc[3] = {c[0] + ((o & 1) ? h : 0), c[1] + ((o & 2) ? h : 0), c[2] + ((o & 4) ? h : 0)};
      policy_node(s, cam, n - 1, cc, out);
    }
    return;
  }
  for (int64_t z = c[2]; z < std::min<int64_t>(c[2] + span, w->desc.grid[2]); z++)
    for (int64_t y = c[1]; y < std::min<int64_t>(c[1] + span, w->desc.grid[1]); y++)
      for (int64_t x = c[0]; x < std::min<int64_t>(c[0] + span, w->desc.grid[0]); x++) {
        const uint32_t ci = (uint32_t)(x + w->desc.grid[0] * (y + w->desc.grid[1] * z));
        const double dx = (x + 0.5) * S - cam[0], dy = (y + 0.5) * S - cam[1], dz = (z + 0.5) * S - cam[2];
        const double d = std::sqrt(dx * dx + dy * dy + dz * dz);
        const uint32_t ks[2] = {lod_at(w, d, f), lod_at(w, d, 1.0)};
        for (uint32_t k : ks) {
          const uint32_t sl = ci * 4 + k;
          if (s->wanted[sl] || !s->src[ci]->lod[k].n_solid) continue;
          s->wanted[sl] = 1;
          out.push_back({(double)(nl - 1 - (int)k) * 1e12 + d, sl});
        }
      }
}

static void run_policy(svd_server* s) {
  const svd_world* w = s->w;
  std::fill(s->wanted.begin(), s->wanted.end(), 0);
  std::vector<std::pair<double, uint32_t>> list;
  int levels = 0;
  while (((int64_t)1 << levels) < (int64_t)std::max({w->desc.grid[0], w->desc.grid[1], w->desc.grid[2]})) levels++;
  for (const auto& r : s->recent) {
    const double cam[3] = {r[0] / 65536.0, r[1] / 65536.0, r[2] / 65536.0};
    const int64_t root[3] = {0, 0, 0};
    policy_node(s, cam, levels, root, list);
  }
  std::sort(list.begin(), list.end());
  s->want_order.clear();
  for (const auto& e : list) s->want_order.push_back(e.second);
  s->want_next = 0;
  s->want_dirty = false;
}

// Note the camera of an admitted request; a chunk not among the last 8
// cameras' chunks re-runs the policy.
static void note_camera(svd_server* s, const svd_ray_frame& f) {
  if (!(s->d.streaming_factor > 0)) return;
  const svd_world* w = s->w;
  int64_t cc[3];
  for (int a = 0; a < 3; a++) cc[a] = (f.O[a] >> 16) >> w->desc.chunk_log2;
  const int64_t key = cc[0] + 65536 * (cc[1] + 65536 * cc[2]);
  for (const auto& r : s->recent)
    if (r[3] == key) return;
  s->recent.push_back({f.O[0], f.O[1], f.O[2], key});
  if (s->recent.size() > 8) s->recent.pop_front();
  s->want_dirty = true;
}

// Upload up to 4 wanted slots into free space; false when there is nothing
// left to do.
static bool prefetch(svd_server* s) {
  if (!(s->d.streaming_factor > 0)) return false;
  if (s->want_dirty) run_policy(s);
  svd_world* w = s->w;
  size_t free_bytes = 0, largest = 0;
  for (const auto& fb : w->free_blocks) {
    free_bytes += fb.second;
    largest = std::max(largest, fb.second);
  }
  const size_t reserve = (w->pool_bytes - w->data_begin) / 8;
  int n = 0;
  while (s->want_next < s->want_order.size() && n < 4) {
    const uint32_t sl = s->want_order[s->want_next];
    if (w->slot[sl].state == svd_world::kResident) {
      s->want_next++;
      continue;
    }
    const LodData& L = s->src[sl / 4]->lod[sl % 4];
    const size_t bytes = L.off_end - L.off_begin;
    if (free_bytes < reserve + bytes || largest < bytes) {  // full: stop until the policy changes
      s->want_next = s->want_order.size();
      break;
    }
    if (world_upload_lods(w, sl / 4, s->src[sl / 4], 1u << (sl % 4), s->up) != SVD_OK) {
      s->want_next = s->want_order.size();
      break;
    }
    s->want_next++;
    s->last_use[sl] = ++s->use_seq;
    free_bytes -= bytes;
    n++;
    std::lock_guard<std::mutex> lk(s->mu);
    s->data_bytes += bytes;
    s->st.prefetches++;
    s->st.prefetch_bytes += bytes;
    s->st.pool_used = s->data_bytes;
  }
  if (n) s->up_dirty = true;
  return n > 0;
}

// Make every slot of r resident and pinned.  `others` = launches or
// already admitted requests hold pins, so waiting can free memory.  When
// nothing else holds memory and the slots still do not fit (the free space is
// fragmented), the pool is cleared and the view's slots are loaded into it
// largest first.
static int admit(svd_server* s, Request& r, bool others) {
  svd_world* w = s->w;
  if (!r.staged) {
    const StageParams sp = world_stage_params(w, &r.frame, r.flags & SVD_NO_CULL, w->h_desc.data());
    for (uint32_t ci = 0; ci < w->nchunks; ci++) {
      const uint32_t v = host_stage_chunk(sp, ci);
      if (!(v & (kViewCulled | kViewEmpty))) r.need.push_back(ci * 4 + (v & kViewLodMask));
    }
    r.staged = true;
  }
  bool uploaded = false;
  int rc = SVD_OK;
  for (int pass = 0; pass < 2; pass++) {
    std::vector<uint32_t> pinned, miss;
    for (uint32_t sl : r.need) {
      if (w->slot[sl].state == svd_world::kResident) {
        s->pins[sl]++;
        pinned.push_back(sl);
      } else {
        miss.push_back(sl);
      }
    }
    std::sort(miss.begin(), miss.end(), [&](uint32_t a, uint32_t b) {
      const LodData& la = s->src[a / 4]->lod[a % 4];
      const LodData& lb = s->src[b / 4]->lod[b % 4];
      return la.off_end - la.off_begin > lb.off_end - lb.off_begin;
    });
    rc = SVD_OK;
    for (uint32_t sl : miss) {
      const uint32_t ci = sl / 4, k = sl % 4;
      for (;;) {
        rc = world_upload_lods(w, ci, s->src[ci], 1u << k, s->up);
        if (rc != SVD_ENOMEM || !evict_one(s)) break;
      }
      if (rc) break;
      s->pins[sl]++;
      pinned.push_back(sl);
      uploaded = true;
      std::lock_guard<std::mutex> lk(s->mu);
      s->data_bytes += w->slot[sl].bytes;
      s->st.uploads++;
      s->st.upload_bytes += w->slot[sl].bytes;
      s->st.pool_used = s->data_bytes;
    }
    if (rc == SVD_OK) break;
    unpin(s, pinned);
    if (rc != SVD_ENOMEM || others) break;
    while (evict_one(s)) {  // nobody pins anything: start from an empty pool
    }
  }
  if (uploaded) s->up_dirty = true;  // the next launch waits for these copies
  if (rc == SVD_ENOMEM) return others ? kWait : svd_fail(SVD_ENOMEM, "serve: the view needs more than the whole pool");
  if (rc) return rc;
  for (uint32_t sl : r.need) s->last_use[sl] = ++s->use_seq;
  return kAdmitted;
}

static bool reap(svd_server* s) {
  bool progress = false;
  for (Flight& f : s->fl) {
    if (!f.busy) continue;
    const hipError_t e = hipEventQuery(f.done);
    if (e == hipErrorNotReady) continue;
    const double t = s->now();
    const int status = e == hipSuccess ? SVD_OK : SVD_EDEVICE;
    for (const Request& r : f.reqs) {
      unpin(s, r.need);
      finish(s, r, status, (uint32_t)f.reqs.size(), f.t_launch, t);
    }
    f.reqs.clear();
    f.busy = false;
    progress = true;
  }
  if (progress) s->done_cv.notify_all();
  return progress;
}

static int enqueue(svd_server* s, Flight& f) {
  if (s->up_dirty) {  // every upload enqueued so far lands before this launch reads the pool
    if (hipEventRecord(s->up_done, s->up) != hipSuccess) return svd_fail(SVD_EDEVICE, "serve: upload event");
    s->up_dirty = false;
    s->up_pending = true;
  }
  if (s->up_pending && hipStreamWaitEvent(f.stream, s->up_done, 0) != hipSuccess)
    return svd_fail(SVD_EDEVICE, "serve: stream wait");
  int rc = SVD_OK;
  if (f.batch && f.reqs.size() == 1) {  // nothing to pack: the batch's tables without the graph
    rc = batch_enqueue_single(f.batch, &f.reqs[0].frame, f.reqs[0].out, f.reqs[0].flags, f.stream);
  } else if (f.batch) {
    std::vector<svd_ray_frame> frames;
    std::vector<svd_hit*> outs;
    for (const Request& r : f.reqs) {
      frames.push_back(r.frame);
      outs.push_back(r.out);
    }
    rc = batch_enqueue(f.batch, frames.data(), outs.data(), (uint32_t)frames.size(), f.reqs[0].flags, f.stream);
  } else {
    rc = svd_trace_frame(s->w, &f.reqs[0].frame, f.reqs[0].out, f.reqs[0].flags, f.stream);
  }
  if (rc) return rc;
  if (hipEventRecord(f.done, f.stream) != hipSuccess) return svd_fail(SVD_EDEVICE, "serve: launch event");
  return SVD_OK;
}

static bool launch(svd_server* s) {
  bool progress = false;
  const uint32_t per_launch = s->d.mode == SVD_SERVE_BATCHED ? s->d.max_views : 1;
  for (Flight& f : s->fl) {
    if (f.busy) continue;
    if (s->pending.empty()) break;
    std::vector<Request> take;
    uint64_t rays = 0;
    while (!s->pending.empty() && take.size() < per_launch) {
      Request& r = s->pending.front();
      const uint64_t px = (uint64_t)r.frame.width * r.frame.height;
      if (!take.empty() && (rays + px > s->d.max_rays || r.flags != take[0].flags)) break;
      const int a = admit(s, r, !take.empty() || any_busy(s));
      if (a == kWait) {
        if (!r.waited) {
          r.waited = true;
          std::lock_guard<std::mutex> lk(s->mu);
          s->st.memory_waits++;
        }
        break;
      }
      if (a != kAdmitted) {  // cannot be served: report and drop
        finish(s, r, a, 0, 0, s->now());
        s->pending.pop_front();
        progress = true;
        continue;
      }
      rays += px;
      note_camera(s, r.frame);
      take.push_back(std::move(r));
      s->pending.pop_front();
    }
    if (take.empty()) break;
    f.reqs = std::move(take);
    f.t_launch = s->now();
    const int rc = enqueue(s, f);
    if (rc) {
      for (const Request& r : f.reqs) {
        unpin(s, r.need);
        finish(s, r, rc, 0, f.t_launch, s->now());
      }
      f.reqs.clear();
    } else {
      f.busy = true;
      std::lock_guard<std::mutex> lk(s->mu);
      s->st.launches++;
    }
    progress = true;
  }
  if (progress) s->done_cv.notify_all();
  return progress;
}

static bool stopping(svd_server* s) {
  std::lock_guard<std::mutex> lk(s->mu);
  return s->stop;
}

static void worker(svd_server* s) {
  if (hipSetDevice(s->device) != hipSuccess) {
    // no device on this thread: every request fails until the server stops
    for (;;) {
      std::deque<Request> got;
      {
        std::unique_lock<std::mutex> lk(s->mu);
        s->wake.wait(lk, [s] { return s->stop || !s->inbox.empty(); });
        got.swap(s->inbox);
        if (got.empty() && s->stop) return;
      }
      for (const Request& r : got) finish(s, r, SVD_EDEVICE, 0, 0.0, s->now());
      s->done_cv.notify_all();
    }
  }
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(s->mu);
      while (!s->inbox.empty()) {
        s->pending.push_back(std::move(s->inbox.front()));
        s->inbox.pop_front();
      }
      const bool prefetch_left = !s->stop && s->d.streaming_factor > 0 &&
                                 (s->want_dirty || s->want_next < s->want_order.size());
      if (s->pending.empty() && !any_busy(s) && !prefetch_left) {
        if (s->stop) break;
        s->wake.wait(lk, [s] { return s->stop || !s->inbox.empty(); });
        continue;
      }
    }
    const bool a = reap(s);
    const bool b = launch(s);
    const bool c = s->pending.empty() && !stopping(s) && prefetch(s);  // streaming policy, while nothing waits
    if (!a && !b && !c) std::this_thread::yield();  // launches in flight: poll their events
  }
}

static void server_release(svd_server* s) {
  for (Flight& f : s->fl) {
    if (f.batch) svd_batch_destroy(f.batch);
    if (f.done) (void)hipEventDestroy(f.done);
    if (f.stream && f.stream != s->plain) (void)hipStreamDestroy(f.stream);
  }
  if (s->plain) (void)hipStreamDestroy(s->plain);
  if (s->up_done) (void)hipEventDestroy(s->up_done);
  if (s->up) (void)hipStreamDestroy(s->up);
  delete s;
}

extern "C" int svd_server_create(svd_world* w, const svd_server_desc* d, svd_server** out) {
  if (!w || !d || !out) return svd_fail(SVD_EINVAL, "svd_server_create: null argument");
  *out = nullptr;
  if (d->mode != SVD_SERVE_BATCHED && d->mode != SVD_SERVE_PLAIN && d->mode != SVD_SERVE_PLAIN_CONCURRENT)
    return svd_fail(SVD_EINVAL, "serve: unknown mode");
  if (d->inflight < 1 || d->inflight > 8) return svd_fail(SVD_EINVAL, "serve: inflight must be 1..8");
  if (d->mode == SVD_SERVE_BATCHED && (d->max_views < 1 || d->max_views > 1024 || d->max_rays < 1))
    return svd_fail(SVD_EINVAL, "serve: max_views must be 1..1024 and max_rays >= 1");
  if (!(d->streaming_factor >= 0.0f && d->streaming_factor <= 1e6f) || d->reserved)
    return svd_fail(SVD_EINVAL, "serve: streaming_factor must be in [0, 1e6] and reserved 0");
  svd_server* s = new (std::nothrow) svd_server();
  if (!s) return svd_fail(SVD_ENOMEM, "serve: out of host memory");
  s->w = w;
  s->d = *d;
  s->t0 = Clock::now();
  memset(&s->st, 0, sizeof(s->st));
  for (const svd_world::Slot& sl : w->slot)
    if (sl.state == svd_world::kResident) s->data_bytes += sl.bytes;
  s->st.pool_used = s->data_bytes;
  s->src.assign(w->nchunks, nullptr);
  s->wanted.assign(w->slot.size(), 0);
  s->pins.assign(w->slot.size(), 0);
  s->last_use.assign(w->slot.size(), 0);
  hipError_t e = hipGetDevice(&s->device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->up, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&s->up_done, hipEventDisableTiming);
  if (e == hipSuccess && d->mode == SVD_SERVE_PLAIN) e = hipStreamCreateWithFlags(&s->plain, hipStreamNonBlocking);
  s->fl.resize(d->inflight);
  for (Flight& f : s->fl) {
    if (e != hipSuccess) break;
    if (d->mode == SVD_SERVE_PLAIN) f.stream = s->plain;
    else e = hipStreamCreateWithFlags(&f.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&f.done, hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    server_release(s);
    return svd_fail(SVD_EDEVICE, "serve: %s", hipGetErrorString(e));
  }
  if (d->mode == SVD_SERVE_BATCHED || d->mode == SVD_SERVE_PLAIN_CONCURRENT) {
    // concurrent plain launches each trace one request on their flight's own
    // view table and queue block (a one-view batch area), on its own stream
    const uint32_t views = d->mode == SVD_SERVE_BATCHED ? d->max_views : 1u;
    for (Flight& f : s->fl) {
      int rc = svd_batch_create(w, views, &f.batch);
      if (rc == SVD_OK && d->tile_w) rc = svd_batch_set_tiling(f.batch, d->tile_w, d->claim ? d->claim : 1);
      if (rc == SVD_OK && d->blocks_per_cu) rc = svd_batch_set_occupancy(f.batch, d->blocks_per_cu);
      if (rc) {
        server_release(s);
        return rc;
      }
    }
  }
  s->th = std::thread(worker, s);
  *out = s;
  return SVD_OK;
}

extern "C" int svd_server_set_chunk(svd_server* s, const uint32_t c[3], const svd_blob* b) {
  if (!s || !c || !b) return svd_fail(SVD_EINVAL, "svd_server_set_chunk: null argument");
  svd_world* w = s->w;
  for (int a = 0; a < 3; a++)
    if (c[a] >= w->desc.grid[a]) return svd_fail(SVD_EINVAL, "serve: chunk outside the grid");
  const uint32_t ci = c[0] + w->desc.grid[0] * (c[1] + w->desc.grid[1] * c[2]);
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->started) return svd_fail(SVD_EINVAL, "serve: chunk sources are fixed once requests arrive");
  const int rc = world_upload_lods(w, ci, b, 0, s->up);  // describe only
  if (rc) return rc;
  if (!s->src[ci]) s->sources++;
  s->src[ci] = b;
  return SVD_OK;
}

extern "C" int svd_server_submit(svd_server* s, const svd_camera* cam, svd_hit* out_dev, uint32_t flags,
                                 uint64_t tag) {
  if (!s || !cam || !out_dev) return svd_fail(SVD_EINVAL, "svd_server_submit: null argument");
  if (flags & ~(SVD_NO_CULL | SVD_BEAM)) return svd_fail(SVD_EINVAL, "serve: unknown flags");
  Request r;
  int rc = svd_camera_frame(cam, &r.frame);
  if (rc) return rc;
  rc = check_frame(&r.frame);
  if (rc) return rc;
  r.tag = tag;
  r.out = out_dev;
  r.flags = flags;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return svd_fail(SVD_EINVAL, "serve: server is stopping");
  if (s->sources != s->w->nchunks)
    return svd_fail(SVD_EINVAL, "serve: %u of %u chunks have no source", s->w->nchunks - s->sources, s->w->nchunks);
  if (!s->started) {
    // chunk descriptions are on the device before any launch
    if (hipStreamSynchronize(s->up) != hipSuccess) return svd_fail(SVD_EDEVICE, "serve: upload stream failed");
    s->started = true;
  }
  r.t_submit = s->now();
  s->inbox.push_back(std::move(r));
  s->st.submitted++;
  s->wake.notify_one();
  return SVD_OK;
}

extern "C" int svd_server_poll(svd_server* s, svd_request_done* out, uint32_t max, uint32_t* n, uint32_t wait_us) {
  if (!s || !n || (max && !out)) return svd_fail(SVD_EINVAL, "svd_server_poll: null argument");
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->done.empty() && wait_us)
    s->done_cv.wait_for(lk, std::chrono::microseconds(wait_us), [s] { return !s->done.empty(); });
  uint32_t k = 0;
  while (k < max && !s->done.empty()) {
    out[k++] = s->done.front();
    s->done.pop_front();
  }
  *n = k;
  return SVD_OK;
}

extern "C" int svd_server_stats_get(svd_server* s, svd_server_stats* st) {
  if (!s || !st) return svd_fail(SVD_EINVAL, "svd_server_stats_get: null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *st = s->st;
  return SVD_OK;
}

extern "C" void svd_server_destroy(svd_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->wake.notify_one();
  if (s->th.joinable()) s->th.join();
  server_release(s);
}
