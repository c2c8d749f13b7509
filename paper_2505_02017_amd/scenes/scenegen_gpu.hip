// Seeded synthetic terrain chunks, generated on the GPU.
//
// The same scenes as the host generator (scenegen.c), kinds 1..4: heightfield
// from 2D fBm value noise, caves carved by 3D fBm below h - 4, materials
// banded by height, then seeded boxes painted in order.  It produces INPUTS
// only and holds no part of the SVDAG method.  A 1024^3 chunk takes tens of
// milliseconds here against tens of core-seconds on the host, which is what
// makes the 32x32-chunk map practical to build.
//
// Every value is computed with the host code's operations in the host code's
// order, in double precision with contraction off (division and floor are
// correctly rounded on both sides), so the bytes equal the host generator's.
// Integer lattice hashing is splitmix64 (Steele, Lea, Flood 2014).
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace sgg {

__host__ __device__ inline uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

__host__ __device__ inline double lattice(uint64_t seed, int64_t i, int64_t j, int64_t k) {
  uint64_t h = splitmix64(seed ^ (uint64_t)i);
  h = splitmix64(h ^ (uint64_t)j);
  h = splitmix64(h ^ (uint64_t)k);
  return (double)(h >> 11) * 0x1p-53;
}

__host__ __device__ inline double fade(double t) { return t * t * (3.0 - 2.0 * t); }
__host__ __device__ inline double lerp(double a, double b, double t) { return a + (b - a) * t; }

__host__ __device__ inline int64_t floordiv(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) q--;
  return q;
}

__host__ __device__ inline int ilog2(int64_t v) {
  int l = 0;
  while (((int64_t)1 << (l + 1)) <= v) l++;
  return l;
}

struct Params {
  uint64_t terrain_seed, cave_seed;
  int64_t X0, Y0, Z0;
  int64_t centre, zmax, terrain_lam, cave_lam;
  double amp, cave_tau;
  uint32_t chunk_log2, nbox;
  // cave lattice tables: octave o covers lattice points [i0, i0 + n) per axis
  int64_t i0[2], j0[2], k0[2], n[2];
};

constexpr int kCaveOctaves = 2;
constexpr int kTerrainOctaves = 6;

__host__ __device__ double vnoise2(uint64_t seed, int64_t x, int64_t y, int64_t lam) {
  const int64_t i = floordiv(x, lam), j = floordiv(y, lam);
  const double fx = fade((double)(x - i * lam) / (double)lam);
  const double fy = fade((double)(y - j * lam) / (double)lam);
  const double a = lerp(lattice(seed, i, j, 0), lattice(seed, i + 1, j, 0), fx);
  const double b = lerp(lattice(seed, i, j + 1, 0), lattice(seed, i + 1, j + 1, 0), fx);
  return lerp(a, b, fy);
}

__host__ __device__ int64_t terrain_h(const Params& p, int64_t x, int64_t y) {
  double s = 0.0, w = 0.0, amp = 1.0;
  for (int o = 0; o < kTerrainOctaves; o++) {
    s += amp * vnoise2(p.terrain_seed + 0x1000ull * (uint64_t)o, x, y, p.terrain_lam >> o);
    w += amp;
    amp *= 0.5;
  }
  const double f = s / w;
  int64_t h = (int64_t)floor((double)p.centre + p.amp * (f - 0.5));
  if (h > p.zmax - 1) h = p.zmax - 1;
  if (h < 0) h = 0;
  return h;
}

// Terrain height of column idx = x + S*y of the chunk.
__host__ __device__ inline int32_t column_height(const Params& p, int64_t idx) {
  const int64_t S = (int64_t)1 << p.chunk_log2;
  const int64_t x = idx & (S - 1), y = idx >> p.chunk_log2;
  return (int32_t)terrain_h(p, p.X0 + x, p.Y0 + y);
}

// Lattice value idx = a + n*(b + n*c) of cave octave o's table.
__host__ __device__ inline double lattice_entry(const Params& p, int o, int64_t idx) {
  const int64_t n = p.n[o];
  const int64_t a = idx % n, b = (idx / n) % n, c = idx / (n * n);
  return lattice(p.cave_seed + 0x1000ull * (uint64_t)o, p.i0[o] + a, p.j0[o] + b, p.k0[o] + c);
}

// The cave fBm at one voxel, from the tabulated lattice values.
__host__ __device__ double cave(const Params& p, const double* const V[2], int64_t X, int64_t Y, int64_t Z) {
  double v = 0.0, w = 0.0, amp = 1.0;
  for (int o = 0; o < kCaveOctaves; o++) {
    const int64_t lam = p.cave_lam >> o;
    const int sh = ilog2(lam);
    const int64_t j = Y >> sh, k = Z >> sh, n = p.n[o];
    const double fy = fade((double)(Y - (j << sh)) / (double)lam);
    const double fz = fade((double)(Z - (k << sh)) / (double)lam);
    const int64_t jb = j - p.j0[o], kb = k - p.k0[o];
    const double* T = V[o];
    double s[2];
    for (int e = 0; e < 2; e++) {
      const int64_t ia = (X >> sh) - p.i0[o] + e;
      const double a = lerp(T[ia + n * (jb + n * kb)], T[ia + n * (jb + 1 + n * kb)], fy);
      const double b = lerp(T[ia + n * (jb + n * (kb + 1))], T[ia + n * (jb + 1 + n * (kb + 1))], fy);
      s[e] = lerp(a, b, fz);
    }
    const double fx = fade((double)(X & (lam - 1)) / (double)lam);
    v += amp * lerp(s[0], s[1], fx);
    w += amp;
    amp *= 0.5;
  }
  return v / w;
}

// Material of voxel idx = x + S*(y + S*z).  hh: the chunk's column heights;
// V0, V1: the cave octaves' lattice tables; boxes: nbox records {x0, y0, z0,
// x1, y1, z1, material, 0} (half-open bounds), at least those meeting this
// chunk, in paint order.
__host__ __device__ inline uint8_t voxel_value(const Params& p, const int32_t* hh, const double* V0,
                                               const double* V1, const int32_t* boxes, int64_t idx) {
  const uint32_t cl = p.chunk_log2;
  const int64_t S = (int64_t)1 << cl;
  const int64_t x = idx & (S - 1), y = (idx >> cl) & (S - 1), z = idx >> (2 * cl);
  const int64_t X = p.X0 + x, Y = p.Y0 + y, Z = p.Z0 + z;
  const int64_t h = hh[(y << cl) + x];
  uint8_t m = 0;
  if (Z <= h) {
    m = (uint8_t)(1 + (8 * Z) / p.zmax);
    if (Z < h - 4) {
      const double* const V[2] = {V0, V1};
      if (cave(p, V, X, Y, Z) > p.cave_tau) m = 0;
    }
  }
  for (uint32_t b = 0; b < p.nbox; b++) {
    const int32_t* r = boxes + 8 * b;
    if (X >= r[0] && X < r[3] && Y >= r[1] && Y < r[4] && Z >= r[2] && Z < r[5]) m = (uint8_t)r[6];
  }
  return m;
}

// One thread per column of the chunk.
__global__ void heights_kernel(Params p, int32_t* hh) {
  const int64_t S = (int64_t)1 << p.chunk_log2;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < S * S) hh[idx] = column_height(p, idx);
}

// One thread per lattice point of one cave octave.
__global__ void lattice_kernel(Params p, int o, double* V) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < p.n[o] * p.n[o] * p.n[o]) V[idx] = lattice_entry(p, o, idx);
}

// One thread per voxel, x fastest.
__global__ void voxel_kernel(Params p, const int32_t* hh, const double* V0, const double* V1,
                             const int32_t* boxes, uint8_t* out) {
  const uint32_t cl = p.chunk_log2;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < ((int64_t)1 << (3 * cl))) out[idx] = voxel_value(p, hh, V0, V1, boxes, idx);
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

void octave_tables(Params& p) {
  const int64_t S = (int64_t)1 << p.chunk_log2;
  for (int o = 0; o < kCaveOctaves; o++) {
    const int sh = ilog2(p.cave_lam >> o);
    p.n[o] = ((S - 1) >> sh) + 3;
    p.i0[o] = p.X0 >> sh;
    p.j0[o] = p.Y0 >> sh;
    p.k0[o] = p.Z0 >> sh;
  }
}

size_t work_bytes(const Params& p) {
  const size_t S = (size_t)1 << p.chunk_log2;
  size_t b = align256(S * S * sizeof(int32_t));
  for (int o = 0; o < kCaveOctaves; o++) b += align256((size_t)(p.n[o] * p.n[o] * p.n[o]) * sizeof(double));
  return b;
}

bool params_from(Params& p, const int64_t ip[6], const double dp[2], uint64_t seed, uint32_t chunk_log2,
                 uint32_t cx, uint32_t cy, uint32_t cz, uint32_t nbox) {
  // ip = {terrain, centre, zmax, terrain_lam, cave_lam, nbox-of-world}; dp = {amp, cave_tau}
  if (!ip || !dp || ip[0] != 1 || chunk_log2 < 3 || chunk_log2 > 10) return false;
  const int64_t tl = ip[3], cl = ip[4];
  if (tl < (1 << (kTerrainOctaves - 1)) || cl < (1 << (kCaveOctaves - 1)) || (cl & (cl - 1)) != 0) return false;
  if (ip[2] <= 0 || ((int64_t)cz << chunk_log2) >= ip[2]) return false;
  p.terrain_seed = seed ^ 0x7E44A1Cull;
  p.cave_seed = seed ^ 0xCA7ECA7Eull;
  p.X0 = (int64_t)cx << chunk_log2;
  p.Y0 = (int64_t)cy << chunk_log2;
  p.Z0 = (int64_t)cz << chunk_log2;
  p.centre = ip[1];
  p.zmax = ip[2];
  p.terrain_lam = tl;
  p.cave_lam = cl;
  p.amp = dp[0];
  p.cave_tau = dp[1];
  p.chunk_log2 = chunk_log2;
  p.nbox = nbox;
  octave_tables(p);
  return true;
}

}  // namespace sgg

extern "C" {

// Workspace (device bytes) that sgg_gen_chunk needs for chunks of this world:
// the column heights and the two cave lattice tables.  0 on bad parameters.
__attribute__((visibility("default"))) size_t sgg_work_bytes(const int64_t ip[6], const double dp[2],
                                                             uint32_t chunk_log2) {
  sgg::Params p{};
  if (!sgg::params_from(p, ip, dp, 0, chunk_log2, 0, 0, 0, 0)) return 0;
  return sgg::work_bytes(p);
}

// Enqueue the generation of chunk (cx, cy, cz) of a terrain world on `stream`.
// ip/dp: the world's parameters as sg_world_params returns them; seed: the
// world's seed.  boxes_dev: nbox device records of 8 int32 {x0, y0, z0, x1,
// y1, z1, material, 0} in paint order (at least the boxes that meet the
// chunk).  out_dev: S^3 device bytes (x fastest).  work_dev: work_bytes of
// device memory, 256-byte aligned.  All device memory is the caller's and must
// stay valid until the stream has run the work.  Returns 0, -1 on bad
// arguments (nothing enqueued), -2 on a HIP launch error.
__attribute__((visibility("default"))) int sgg_gen_chunk(const int64_t ip[6], const double dp[2], uint64_t seed,
                                                         uint32_t chunk_log2, uint32_t cx, uint32_t cy,
                                                         uint32_t cz, const int32_t* boxes_dev, uint32_t nbox,
                                                         uint8_t* out_dev, void* work_dev, size_t work_bytes,
                                                         void* stream) {
  sgg::Params p{};
  if (!sgg::params_from(p, ip, dp, seed, chunk_log2, cx, cy, cz, nbox)) return -1;
  if (!out_dev || !work_dev || (nbox && !boxes_dev) || ((uintptr_t)work_dev & 255)) return -1;
  if (work_bytes < sgg::work_bytes(p)) return -1;
  const int64_t S = (int64_t)1 << chunk_log2;
  if (((cx + 1ull) << chunk_log2) > 32768ull || ((cy + 1ull) << chunk_log2) > 32768ull) return -1;
  hipStream_t s = (hipStream_t)stream;
  uint8_t* w = (uint8_t*)work_dev;
  int32_t* hh = (int32_t*)w;
  w += sgg::align256((size_t)(S * S) * sizeof(int32_t));
  double* V[2];
  for (int o = 0; o < sgg::kCaveOctaves; o++) {
    V[o] = (double*)w;
    w += sgg::align256((size_t)(p.n[o] * p.n[o] * p.n[o]) * sizeof(double));
  }
  constexpr int kB = 256;
  hipLaunchKernelGGL(sgg::heights_kernel, dim3((unsigned)((S * S + kB - 1) / kB)), dim3(kB), 0, s, p, hh);
  for (int o = 0; o < sgg::kCaveOctaves; o++) {
    const int64_t n3 = p.n[o] * p.n[o] * p.n[o];
    hipLaunchKernelGGL(sgg::lattice_kernel, dim3((unsigned)((n3 + kB - 1) / kB)), dim3(kB), 0, s, p, o, V[o]);
  }
  const int64_t nv = S * S * S;
  hipLaunchKernelGGL(sgg::voxel_kernel, dim3((unsigned)((nv + kB - 1) / kB)), dim3(kB), 0, s, p, hh, V[0], V[1],
                     boxes_dev, out_dev);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // extern "C"
