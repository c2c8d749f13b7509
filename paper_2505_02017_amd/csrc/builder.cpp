// Host-side chunk build for libsvdag: LOD pyramid, SVDAG per LOD, DFS-order
// material runs, canonical serialisation and the device image.
//
// Method sections (Fang, Wang, Wang, PACMCGIT 2025):
//   3.4  LOD chunks: a level-n voxel aggregates 8 level-(n-1) voxels, solid
//        iff at least density = 2 of them are solid.
//   3.2  SVDAG: isomorphic subtrees merged; the three deepest levels are one
//        4x4x4 leaf chunk stored as a 64-bit bitmap; node = u32 header with
//        the child mask in bits 0..7, u32 count of solid voxels below, one
//        u32 pointer per set mask bit.
//   3.3  Colours (material IDs here) in DFS order, compressed into blocks of
//        equal value (error threshold 0), found by binary search.
//
// The build is bottom-up: every 4^3 block of the grid becomes a bitmap,
// deduplicated by value; every level above is built from the ids of the
// level below, deduplicated by (mask, child ids).  Empty and full blocks take
// fast paths.  The canonical node order is fixed (levels from the root; in a
// level, first reference when the level above is scanned in order), so equal
// geometry always serialises to equal bytes.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "svdag_internal.h"

namespace svd {
namespace {

inline uint64_t mix64(uint64_t h) {
  h ^= h >> 31;
  h *= 0x7fb5d329728ea185ull;
  h ^= h >> 27;
  h *= 0x81dadef4bc2dd44dull;
  h ^= h >> 33;
  return h;
}

// ---------------------------------------------------------------- LOD step
inline uint8_t aggregate8(const uint8_t v[8]) {
  int solid = 0;
  for (int i = 0; i < 8; i++) solid += v[i] != 0;
  if (solid < 2) return 0;
  uint8_t best = 0;
  int best_n = 0;
  for (int i = 0; i < 8; i++) {
    if (!v[i]) continue;
    int n = 0;
    for (int j = 0; j < 8; j++) n += v[j] == v[i];
    if (n > best_n || (n == best_n && v[i] < best)) {
      best_n = n;
      best = v[i];
    }
  }
  return best;
}

void downsample(const uint8_t* src, uint32_t R, uint8_t* dst) {
  const size_t h = R / 2, r = R;
  for (size_t z = 0; z < h; z++)
    for (size_t y = 0; y < h; y++) {
      const uint8_t* a = src + r * ((2 * y) + r * (2 * z));
      const uint8_t* b = a + r;          // y+1
      const uint8_t* c = a + r * r;      // z+1
      const uint8_t* d = c + r;          // y+1, z+1
      uint8_t* o = dst + h * (y + h * z);
      for (size_t x = 0; x < h; x++) {
        if ((x & 3) == 0 && x + 4 <= h) {  // 4 coarse cells whose 32 voxels share one value
          uint64_t qa, qb, qc, qd;
          memcpy(&qa, a + 2 * x, 8);
          memcpy(&qb, b + 2 * x, 8);
          memcpy(&qc, c + 2 * x, 8);
          memcpy(&qd, d + 2 * x, 8);
          if (qa == qb && qa == qc && qa == qd && qa == 0x0101010101010101ull * (qa & 0xFF)) {
            memset(o + x, (int)(qa & 0xFF), 4);
            x += 3;
            continue;
          }
        }
        uint16_t wa, wb, wc, wd;
        memcpy(&wa, a + 2 * x, 2);
        memcpy(&wb, b + 2 * x, 2);
        memcpy(&wc, c + 2 * x, 2);
        memcpy(&wd, d + 2 * x, 2);
        if (wa == wb && wa == wc && wa == wd && (wa & 0xFF) == (wa >> 8)) {
          o[x] = (uint8_t)(wa & 0xFF);  // 8 equal voxels (empty or full)
          continue;
        }
        const uint8_t v[8] = {a[2 * x], a[2 * x + 1], b[2 * x], b[2 * x + 1],
                              c[2 * x], c[2 * x + 1], d[2 * x], d[2 * x + 1]};
        o[x] = aggregate8(v);
      }
    }
}

// ------------------------------------------------------ leaf bitmap tables
// Cell (x,y,z) of a 4^3 leaf maps to bit 8*oct(x>>1,y>>1,z>>1) + oct(x&1,y&1,z&1).
struct LeafTables {
  uint8_t bit[64];        // indexed by x + 4y + 16z
  uint8_t lx[64], ly[64], lz[64];  // inverse: local coordinates of bit b
  uint64_t axis_mask[3][4];        // bits whose local coordinate on an axis is i
  LeafTables() {
    memset(axis_mask, 0, sizeof(axis_mask));
    for (int z = 0; z < 4; z++)
      for (int y = 0; y < 4; y++)
        for (int x = 0; x < 4; x++) {
          int o1 = (x >> 1) | ((y >> 1) << 1) | ((z >> 1) << 2);
          int o0 = (x & 1) | ((y & 1) << 1) | ((z & 1) << 2);
          int b = 8 * o1 + o0;
          bit[x + 4 * y + 16 * z] = (uint8_t)b;
          lx[b] = (uint8_t)x;
          ly[b] = (uint8_t)y;
          lz[b] = (uint8_t)z;
          axis_mask[0][x] |= 1ull << b;
          axis_mask[1][y] |= 1ull << b;
          axis_mask[2][z] |= 1ull << b;
        }
  }
};
const LeafTables& leaf_tables() {
  static const LeafTables t;
  return t;
}

// ------------------------------------------------------ dedup hash tables
struct LeafTable {
  std::vector<uint64_t> vals;
  std::vector<uint32_t> slot;  // id + 1, 0 = free
  uint32_t intern(uint64_t v) {
    if (2 * (vals.size() + 1) > slot.size()) grow();
    size_t m = slot.size() - 1, h = mix64(v) & m;
    while (slot[h]) {
      if (vals[slot[h] - 1] == v) return slot[h] - 1;
      h = (h + 1) & m;
    }
    vals.push_back(v);
    slot[h] = (uint32_t)vals.size();
    return (uint32_t)vals.size() - 1;
  }
  void grow() {
    size_t n = slot.empty() ? 4096 : slot.size() * 2;
    slot.assign(n, 0);
    for (size_t i = 0; i < vals.size(); i++) {
      size_t h = mix64(vals[i]) & (n - 1);
      while (slot[h]) h = (h + 1) & (n - 1);
      slot[h] = (uint32_t)i + 1;
    }
  }
};

struct TNode {
  uint32_t mask;
  uint32_t child[8];  // ids one level down, ~0u when absent
  uint32_t count;
  uint64_t hash() const {
    uint64_t h = mix64(mask ^ 0x51ed2701ull);
    for (int i = 0; i < 8; i++) h = mix64(h + child[i] * 0x9e3779b97f4a7c15ull + (uint64_t)i);
    return h;
  }
  bool same(const TNode& o) const {
    return mask == o.mask && memcmp(child, o.child, sizeof(child)) == 0;
  }
};

struct NodeTable {
  std::vector<TNode> nodes;
  std::vector<uint32_t> slot;
  uint32_t intern(const TNode& t) {
    if (2 * (nodes.size() + 1) > slot.size()) grow();
    size_t m = slot.size() - 1, h = t.hash() & m;
    while (slot[h]) {
      if (nodes[slot[h] - 1].same(t)) return slot[h] - 1;
      h = (h + 1) & m;
    }
    nodes.push_back(t);
    slot[h] = (uint32_t)nodes.size();
    return (uint32_t)nodes.size() - 1;
  }
  void grow() {
    size_t n = slot.empty() ? 1024 : slot.size() * 2;
    slot.assign(n, 0);
    for (size_t i = 0; i < nodes.size(); i++) {
      size_t h = nodes[i].hash() & (n - 1);
      while (slot[h]) h = (h + 1) & (n - 1);
      slot[h] = (uint32_t)i + 1;
    }
  }
};

int ilog2(uint32_t v) {
  int l = 0;
  while ((1u << (l + 1)) <= v) l++;
  return l;
}

// ------------------------------------------------------------ DFS materials
struct RunBuilder {
  std::vector<uint32_t>* start;
  std::vector<uint8_t>* mat;
  uint32_t i = 0;
  void push(uint8_t m) {
    if (mat->empty() || mat->back() != m) {
      start->push_back(i);
      mat->push_back(m);
    }
    i++;
  }
};

// uni[l] (per cube of 2^l cells of the grid, x fastest, l >= 2): m when
// every cell of the cube holds material m, else 0.  Such a cube adds at most
// one run, whatever its size.
void dfs_runs(const LodData& L, const uint8_t* g, const std::vector<std::vector<uint8_t>>& uni, uint32_t off,
              int lev, uint32_t x0, uint32_t y0, uint32_t z0, RunBuilder& rb) {
  const LeafTables& T = leaf_tables();
  const size_t R = L.R;
  const uint32_t mask = L.words[off];
  const uint32_t h = 1u << (lev - 1);
  const size_t nc = R >> (lev - 1);  // child cubes per axis
  const std::vector<uint8_t>& cu = uni[lev - 1];
  uint32_t slot = 0;
  for (int o = 0; o < 8; o++) {
    if (!((mask >> o) & 1)) continue;
    const uint32_t p = L.words[off + 2 + slot++];
    const uint32_t cx = x0 + ((o & 1) ? h : 0), cy = y0 + ((o & 2) ? h : 0), cz = z0 + ((o & 4) ? h : 0);
    const uint8_t m = cu[(cx >> (lev - 1)) + nc * ((cy >> (lev - 1)) + nc * (cz >> (lev - 1)))];
    if (m) {
      rb.push(m);
      rb.i += (lev > 3 ? L.words[p + 1] : 64u) - 1;
      continue;
    }
    if (lev > 3) {
      dfs_runs(L, g, uni, p, lev - 1, cx, cy, cz, rb);
      continue;
    }
    uint64_t bits = L.leaves[p];
    while (bits) {
      const int b = __builtin_ctzll(bits);
      bits &= bits - 1;
      const size_t x = cx + T.lx[b], y = cy + T.ly[b], z = cz + T.lz[b];
      rb.push(g[x + R * (y + R * z)]);
    }
  }
}

}  // namespace

// Count and tight box of every canonical node, bottom-up (children follow
// their parents in canonical order, so a reverse scan sees children first).
// Returns false if the structure is inconsistent.
bool node_boxes(const LodData& L, std::vector<uint32_t>* level_of, uint16_t lo[3], uint16_t hi[3]);

// Builds the canonical DAG of grid g (R^3) into L (R set by caller).
int build_lod(const uint8_t* g, uint32_t R, LodData& L) {
  const LeafTables& T = leaf_tables();
  const int Lr = ilog2(R);
  L.R = R;
  L.root_level = (uint32_t)Lr;
  const size_t r = R;
  // level 2: 4^3 leaf bitmaps
  size_t n = R / 4;
  std::vector<uint32_t> cur(n * n * n, ~0u);
  LeafTable lt;
  uint32_t base_bit[4][4];
  for (int z = 0; z < 4; z++)
    for (int y = 0; y < 4; y++) base_bit[y][z] = T.bit[4 * y + 16 * z];
  std::vector<std::vector<uint8_t>> unis(Lr + 1);
  unis[2].assign(n * n * n, 0);
  std::vector<uint8_t>& uni = unis[2];
  uint64_t last_bits = 0;
  uint32_t last_id = 0;
  for (size_t bz = 0; bz < n; bz++)
    for (size_t by = 0; by < n; by++)
      for (size_t bx = 0; bx < n; bx++) {
        if ((bx & 3) == 0 && bx + 4 <= n) {  // 4 blocks whose 256 voxels share one value
          const uint8_t v = g[4 * bx + r * (4 * by + r * 4 * bz)];
          const uint64_t v8 = 0x0101010101010101ull * v;
          bool one = true;
          for (int z = 0; z < 4 && one; z++)
            for (int y = 0; y < 4 && one; y++) {
              uint64_t q[2];
              memcpy(q, g + 4 * bx + r * ((4 * by + y) + r * (4 * bz + z)), 16);
              one = q[0] == v8 && q[1] == v8;
            }
          if (one) {
            if (v) {
              if (last_bits != ~0ull) {
                last_bits = ~0ull;
                last_id = lt.intern(~0ull);
              }
              for (size_t i = 0; i < 4; i++) {
                cur[bx + i + n * (by + n * bz)] = last_id;
                uni[bx + i + n * (by + n * bz)] = v;
              }
            }
            bx += 3;
            continue;
          }
        }
        uint64_t bits = 0;
        const uint32_t m4 = 0x01010101u * g[4 * bx + r * (4 * by + r * 4 * bz)];
        bool same = m4 != 0;
        for (int z = 0; z < 4; z++)
          for (int y = 0; y < 4; y++) {
            uint32_t row;
            memcpy(&row, g + 4 * bx + r * ((4 * by + y) + r * (4 * bz + z)), 4);
            same = same && row == m4;
            if (!row) continue;
            const uint32_t b = base_bit[y][z];
            if (!((row - 0x01010101u) & ~row & 0x80808080u)) {  // no zero byte: 4 solid voxels
              bits |= 0x303ull << b;
              continue;
            }
            if (row & 0x000000FFu) bits |= 1ull << b;
            if (row & 0x0000FF00u) bits |= 1ull << (b + 1);
            if (row & 0x00FF0000u) bits |= 1ull << (b + 8);
            if (row & 0xFF000000u) bits |= 1ull << (b + 9);
          }
        if (!bits) continue;
        if (same) uni[bx + n * (by + n * bz)] = (uint8_t)m4;
        if (bits != last_bits) {  // neighbouring leaves are often equal (full, or one pattern)
          last_bits = bits;
          last_id = lt.intern(bits);
        }
        cur[bx + n * (by + n * bz)] = last_id;
      }
  // levels 3 .. root
  std::vector<NodeTable> tabs(Lr + 1);
  for (int lev = 3; lev <= Lr; lev++) {
    const size_t m = R >> lev, cn = 2 * m;
    std::vector<uint32_t> next(m * m * m, ~0u);
    NodeTable& tab = tabs[lev];
    unis[lev].assign(m * m * m, 0);
    const std::vector<uint8_t>& cu = unis[lev - 1];
    for (size_t z = 0; z < m; z++)
      for (size_t y = 0; y < m; y++)
        for (size_t x = 0; x < m; x++) {
          TNode t;
          t.mask = 0;
          t.count = 0;
          uint8_t u = cu[2 * x + cn * (2 * y + cn * 2 * z)];
          for (int o = 0; o < 8; o++) {
            const size_t cx = 2 * x + (o & 1), cy = 2 * y + ((o >> 1) & 1), cz = 2 * z + ((o >> 2) & 1);
            if (cu[cx + cn * (cy + cn * cz)] != u) u = 0;
            const uint32_t id = cur[cx + cn * (cy + cn * cz)];
            t.child[o] = id;
            if (id == ~0u) continue;
            t.mask |= 1u << o;
            t.count += (lev == 3) ? (uint32_t)__builtin_popcountll(lt.vals[id]) : tabs[lev - 1].nodes[id].count;
          }
          unis[lev][x + m * (y + m * z)] = u;
          if (t.mask) next[x + m * (y + m * z)] = tab.intern(t);
        }
    cur.swap(next);
  }
  L.words.clear();
  L.leaves.clear();
  L.rle_start.clear();
  L.rle_mat.clear();
  memset(L.level_nodes, 0, sizeof(L.level_nodes));
  L.n_solid = 0;
  const uint32_t root = cur[0];
  if (root == ~0u) return SVD_OK;

  // canonical order: level by level from the root
  std::vector<std::vector<uint32_t>> order(Lr + 1);
  std::vector<std::vector<uint32_t>> woff(Lr + 1);
  std::vector<uint32_t> leaf_index(lt.vals.size(), ~0u);
  std::vector<uint32_t> leaf_order;
  std::vector<uint8_t> seen;
  order[Lr].push_back(root);
  for (int lev = Lr; lev >= 3; lev--) {
    if (lev > 3) seen.assign(tabs[lev - 1].nodes.size(), 0);
    for (uint32_t id : order[lev]) {
      const TNode& t = tabs[lev].nodes[id];
      for (int o = 0; o < 8; o++) {
        const uint32_t c = t.child[o];
        if (c == ~0u) continue;
        if (lev > 3) {
          if (!seen[c]) { seen[c] = 1; order[lev - 1].push_back(c); }
        } else if (leaf_index[c] == ~0u) {
          leaf_index[c] = (uint32_t)leaf_order.size();
          leaf_order.push_back(c);
        }
      }
    }
  }
  uint64_t off = 0;
  for (int lev = Lr; lev >= 3; lev--) {
    woff[lev].assign(tabs[lev].nodes.size(), ~0u);
    for (uint32_t id : order[lev]) {
      woff[lev][id] = (uint32_t)off;
      off += 2 + (uint32_t)__builtin_popcount(tabs[lev].nodes[id].mask);
    }
    L.level_nodes[lev] = (uint32_t)order[lev].size();
  }
  if (off > 0xFFFFFFFFull) return svd_fail(SVD_ERANGE, "DAG too large (%llu words)", (unsigned long long)off);
  L.level_nodes[2] = (uint32_t)leaf_order.size();
  L.words.resize(off);
  for (int lev = Lr; lev >= 3; lev--)
    for (uint32_t id : order[lev]) {
      const TNode& t = tabs[lev].nodes[id];
      uint32_t* w = &L.words[woff[lev][id]];
      w[0] = t.mask;
      w[1] = t.count;
      uint32_t s = 2;
      for (int o = 0; o < 8; o++) {
        if (t.child[o] == ~0u) continue;
        w[s++] = (lev > 3) ? woff[lev - 1][t.child[o]] : leaf_index[t.child[o]];
      }
    }
  L.leaves.resize(leaf_order.size());
  for (size_t i = 0; i < leaf_order.size(); i++) L.leaves[i] = lt.vals[leaf_order[i]];
  L.n_solid = L.words[1];
  RunBuilder rb{&L.rle_start, &L.rle_mat};
  dfs_runs(L, g, unis, 0, Lr, 0, 0, 0, rb);
  if (rb.i != L.n_solid) return svd_fail(SVD_EINVAL, "internal: DFS count mismatch");
  if (!node_boxes(L, nullptr, L.lo, L.hi)) return svd_fail(SVD_EINVAL, "internal: bad DAG");
  return SVD_OK;
}

bool node_boxes(const LodData& L, std::vector<uint32_t>* level_out, uint16_t lo_out[3],
                uint16_t hi_out[3]) {
  const LeafTables& T = leaf_tables();
  const size_t nw = L.words.size();
  if (nw == 0) return true;
  // node starts and levels (root at L.root_level; children one level down)
  std::vector<uint32_t> starts;
  std::vector<int8_t> level(nw, -1);
  size_t i = 0;
  while (i < nw) {
    if (i + 2 > nw) return false;
    const uint32_t mask = L.words[i];
    if (mask == 0 || (mask & ~0xFFu)) return false;
    const size_t k = (size_t)__builtin_popcount(mask);
    if (i + 2 + k > nw) return false;
    starts.push_back((uint32_t)i);
    i += 2 + k;
  }
  std::vector<uint8_t> is_start(nw, 0);
  for (uint32_t s : starts) is_start[s] = 1;
  level[0] = (int8_t)L.root_level;
  for (uint32_t s : starts) {
    const int lev = level[s];
    if (lev < 3) return false;  // unreachable node or bad level
    const uint32_t mask = L.words[s];
    const int k = __builtin_popcount(mask);
    for (int j = 0; j < k; j++) {
      const uint32_t p = L.words[s + 2 + j];
      if (lev == 3) {
        if (p >= L.leaves.size()) return false;
      } else {
        if (p >= nw || !is_start[p] || p <= s) return false;
        if (level[p] == -1) level[p] = (int8_t)(lev - 1);
        else if (level[p] != lev - 1) return false;
      }
    }
  }
  // counts and boxes bottom-up (box coordinates relative to the node's cube)
  struct Box { uint16_t lo[3], hi[3]; };
  std::vector<Box> lbox(L.leaves.size());
  for (size_t q = 0; q < L.leaves.size(); q++) {
    const uint64_t b = L.leaves[q];
    if (!b) return false;
    for (int a = 0; a < 3; a++) {
      int mn = 0, mx = 3;
      while (!(b & T.axis_mask[a][mn])) mn++;
      while (!(b & T.axis_mask[a][mx])) mx--;
      lbox[q].lo[a] = (uint16_t)mn;
      lbox[q].hi[a] = (uint16_t)mx;
    }
  }
  std::vector<Box> nbox(nw);
  std::vector<uint32_t> count(nw, 0);
  for (size_t si = starts.size(); si-- > 0;) {
    const uint32_t s = starts[si];
    const int lev = level[s];
    const uint32_t mask = L.words[s];
    const uint32_t h = 1u << (lev - 1);
    uint64_t cnt = 0;
    Box bx = {{0xFFFF, 0xFFFF, 0xFFFF}, {0, 0, 0}};
    uint32_t slot = 0;
    for (int o = 0; o < 8; o++) {
      if (!((mask >> o) & 1)) continue;
      const uint32_t p = L.words[s + 2 + slot++];
      const Box& cb = (lev == 3) ? lbox[p] : nbox[p];
      cnt += (lev == 3) ? (uint64_t)__builtin_popcountll(L.leaves[p]) : count[p];
      const uint32_t off[3] = {(o & 1) ? h : 0u, (o & 2) ? h : 0u, (o & 4) ? h : 0u};
      for (int a = 0; a < 3; a++) {
        bx.lo[a] = (uint16_t)std::min<uint32_t>(bx.lo[a], cb.lo[a] + off[a]);
        bx.hi[a] = (uint16_t)std::max<uint32_t>(bx.hi[a], cb.hi[a] + off[a]);
      }
    }
    if (cnt != L.words[s + 1]) return false;
    count[s] = (uint32_t)cnt;
    nbox[s] = bx;
  }
  if (count[0] != L.n_solid) return false;
  for (int a = 0; a < 3; a++) {
    lo_out[a] = nbox[0].lo[a];
    hi_out[a] = nbox[0].hi[a];
  }
  if (level_out) {
    level_out->assign(16, 0);
    for (uint32_t s : starts) (*level_out)[level[s]]++;
  }
  return true;
}

// Device image of one LOD appended to `image` (sections 256-byte aligned).
int derive_device(LodData& L, std::vector<uint8_t>& image) {
  auto align = [&](size_t a) { image.resize((image.size() + a - 1) / a * a, 0); };
  align(256);
  L.off_begin = image.size();
  const size_t nw = L.words.size();
  std::vector<uint32_t> dev_off(nw, 0);
  uint64_t dw = 0;
  size_t i = 0;
  std::vector<uint32_t> starts;
  while (i < nw) {
    starts.push_back((uint32_t)i);
    dev_off[i] = (uint32_t)dw;
    const uint32_t k = (uint32_t)__builtin_popcount(L.words[i]);
    dw += k;
    i += 2 + k;
  }
  if (dw > kPtrMask || L.leaves.size() > kPtrMask)
    return svd_fail(SVD_ERANGE, "DAG exceeds 2^24 device words or leaves");
  L.dev_words = (uint32_t)dw;
  std::vector<uint32_t> nodes(dw), pre(dw);
  // a node whose pointers index leaves is one at level 3: its children are
  // not node starts; the root level tells which nodes those are
  std::vector<uint32_t> level_of(nw, 0);
  if (nw) level_of[0] = L.root_level;
  for (uint32_t s : starts) {
    const uint32_t mask = L.words[s];
    const uint32_t lev = level_of[s];
    const uint32_t k = (uint32_t)__builtin_popcount(mask);
    uint32_t acc = 0;
    for (uint32_t j = 0; j < k; j++) {
      const uint32_t p = L.words[s + 2 + j];
      uint32_t cw, cc;
      if (lev == 3) {
        // a leaf's "mask" is its 8-bit summary: bit i set iff 2^3 sub-block i is non-empty
        uint32_t summary = 0;
        for (int s = 0; s < 8; s++)
          if ((L.leaves[p] >> (8 * s)) & 0xFFu) summary |= 1u << s;
        cw = (summary << kPtrBits) | p;
        cc = (uint32_t)__builtin_popcountll(L.leaves[p]);
      } else {
        level_of[p] = lev - 1;
        cw = (L.words[p] << kPtrBits) | dev_off[p];
        cc = L.words[p + 1];
      }
      nodes[dev_off[s] + j] = cw;
      pre[dev_off[s] + j] = acc;
      acc += cc;
    }
  }
  L.root_word = nw ? (L.words[0] << kPtrBits) : 0u;
  auto put = [&](const void* p, size_t bytes) {
    align(256);
    const size_t o = image.size();
    image.resize(o + bytes);
    if (bytes) memcpy(image.data() + o, p, bytes);
    return (uint64_t)o;
  };
  L.off_nodes = put(nodes.data(), nodes.size() * 4);
  L.off_pre = put(pre.data(), pre.size() * 4);
  L.off_leaves = put(L.leaves.data(), L.leaves.size() * 8);
  // runs: starts then materials, one section; then the run directory
  const size_t nr = L.rle_start.size();
  std::vector<uint8_t> runs(nr * 5);
  if (nr) {
    memcpy(runs.data(), L.rle_start.data(), nr * 4);
    memcpy(runs.data() + nr * 4, L.rle_mat.data(), nr);
  }
  L.off_rle_start = put(runs.data(), runs.size());
  std::vector<uint32_t> dir;
  if (nr) {
    const uint32_t B = run_dir_shift((uint32_t)nr, L.n_solid);
    const uint32_t nd = ((L.n_solid - 1) >> B) + 1;
    dir.resize((size_t)nd + 1);
    uint32_t q = 0;
    for (uint32_t j = 0; j < nd; j++) {
      const uint64_t first = (uint64_t)j << B;
      while (q + 1 < nr && L.rle_start[q + 1] <= first) q++;
      dir[j] = q;
    }
    dir[nd] = (uint32_t)nr - 1;
  }
  L.off_rle_dir = put(dir.data(), dir.size() * 4);
  align(256);
  L.off_end = image.size();
  return SVD_OK;
}

}  // namespace svd

using namespace svd;

extern "C" int svd_chunk_build(const uint8_t* dense, uint32_t chunk_log2, uint32_t lod_count,
                               svd_blob** out) {
  if (!dense || !out) return svd_fail(SVD_EINVAL, "svd_chunk_build: null argument");
  *out = nullptr;
  if (chunk_log2 < 3 || chunk_log2 > 10) return svd_fail(SVD_EINVAL, "chunk_log2 must be 3..10");
  if (lod_count < 1 || lod_count > 4 || (int)chunk_log2 - (int)(lod_count - 1) < 3)
    return svd_fail(SVD_EINVAL, "lod_count must be 1..4 with coarsest grid >= 8^3");
  try {
    svd_blob* b = new svd_blob();
    b->chunk_log2 = chunk_log2;
    b->lod_count = lod_count;
    b->lod.resize(lod_count);
    const uint32_t S = 1u << chunk_log2;
    std::vector<uint8_t> prev, next;
    const uint8_t* g = dense;
    for (uint32_t k = 0; k < lod_count; k++) {
      const uint32_t R = S >> k;
      if (k > 0) {
        next.resize((size_t)R * R * R);
        downsample(g, R * 2, next.data());
        prev.swap(next);
        g = prev.data();
      }
      int rc = build_lod(g, R, b->lod[k]);
      if (rc != SVD_OK) { delete b; return rc; }
      rc = derive_device(b->lod[k], b->image);
      if (rc != SVD_OK) { delete b; return rc; }
    }
    *out = b;
    return SVD_OK;
  } catch (const std::bad_alloc&) {
    return svd_fail(SVD_ENOMEM, "svd_chunk_build: out of host memory");
  }
}

extern "C" void svd_blob_free(svd_blob* b) { delete b; }
extern "C" void svd_free(void* p) { free(p); }

// ---------------------------------------------------------------- bytes
namespace {
constexpr uint32_t kMagic = 0x42445653u;  // "SVDB"
constexpr uint32_t kVersion = 1;

struct Writer {
  std::vector<uint8_t> v;
  void u32(uint32_t x) { raw(&x, 4); }
  void raw(const void* p, size_t n) {
    const size_t o = v.size();
    v.resize(o + n);
    if (n) memcpy(v.data() + o, p, n);
  }
  void pad8() { v.resize((v.size() + 7) / 8 * 8, 0); }
};

struct Reader {
  const uint8_t* p;
  size_t n, o = 0;
  bool u32(uint32_t* x) { return raw(x, 4); }
  bool raw(void* d, size_t k) {
    if (k > n - o) return false;
    if (k) memcpy(d, p + o, k);
    o += k;
    return true;
  }
  bool pad8() {  // padding must be zero: serialisations stay canonical
    size_t q = (o + 7) / 8 * 8;
    if (q > n) return false;
    for (; o < q; o++)
      if (p[o]) return false;
    return true;
  }
};
}  // namespace

extern "C" int svd_blob_to_bytes(const svd_blob* b, void** bytes, size_t* n) {
  if (!b || !bytes || !n) return svd_fail(SVD_EINVAL, "svd_blob_to_bytes: null argument");
  try {
    Writer w;
    w.u32(kMagic);
    w.u32(kVersion);
    w.u32(b->chunk_log2);
    w.u32(b->lod_count);
    for (const LodData& L : b->lod) {
      w.u32(L.R);
      w.u32((uint32_t)L.words.size());
      w.u32((uint32_t)L.leaves.size());
      w.u32((uint32_t)L.rle_start.size());
      w.u32(L.n_solid);
      w.u32(0);
      w.raw(L.words.data(), L.words.size() * 4);
      w.pad8();
      w.raw(L.leaves.data(), L.leaves.size() * 8);
      w.raw(L.rle_start.data(), L.rle_start.size() * 4);
      w.raw(L.rle_mat.data(), L.rle_mat.size());
      w.pad8();
    }
    void* p = malloc(w.v.size() ? w.v.size() : 1);
    if (!p) return svd_fail(SVD_ENOMEM, "svd_blob_to_bytes: out of memory");
    memcpy(p, w.v.data(), w.v.size());
    *bytes = p;
    *n = w.v.size();
    return SVD_OK;
  } catch (const std::bad_alloc&) {
    return svd_fail(SVD_ENOMEM, "svd_blob_to_bytes: out of memory");
  }
}

extern "C" int svd_blob_from_bytes(const void* bytes, size_t n, svd_blob** out) {
  if (!bytes || !out) return svd_fail(SVD_EINVAL, "svd_blob_from_bytes: null argument");
  *out = nullptr;
  Reader r{(const uint8_t*)bytes, n};
  uint32_t magic, ver, cl, lc;
  if (!r.u32(&magic) || !r.u32(&ver) || !r.u32(&cl) || !r.u32(&lc))
    return svd_fail(SVD_EFORMAT, "blob: truncated header");
  if (magic != kMagic || ver != kVersion) return svd_fail(SVD_EFORMAT, "blob: bad magic/version");
  if (cl < 3 || cl > 10 || lc < 1 || lc > 4 || (int)cl - (int)(lc - 1) < 3)
    return svd_fail(SVD_EFORMAT, "blob: bad chunk size or LOD count");
  try {
    svd_blob* b = new svd_blob();
    b->chunk_log2 = cl;
    b->lod_count = lc;
    b->lod.resize(lc);
    for (uint32_t k = 0; k < lc; k++) {
      LodData& L = b->lod[k];
      uint32_t R, nw, nl, nr, ns, zero;
      if (!r.u32(&R) || !r.u32(&nw) || !r.u32(&nl) || !r.u32(&nr) || !r.u32(&ns) || !r.u32(&zero)) {
        delete b;
        return svd_fail(SVD_EFORMAT, "blob: truncated LOD header");
      }
      const uint64_t need = (uint64_t)nw * 4 + (uint64_t)nl * 8 + (uint64_t)nr * 5;  // before padding
      if (R != (1u << (cl - k)) || zero != 0 || need > n - r.o) {
        delete b;
        return svd_fail(SVD_EFORMAT, "blob: bad LOD %u sizes", k);
      }
      L.R = R;
      L.root_level = (uint32_t)ilog2(R);
      L.n_solid = ns;
      L.words.resize(nw);
      L.leaves.resize(nl);
      L.rle_start.resize(nr);
      L.rle_mat.resize(nr);
      bool ok = r.raw(L.words.data(), (size_t)nw * 4) && r.pad8() &&
                r.raw(L.leaves.data(), (size_t)nl * 8) && r.raw(L.rle_start.data(), (size_t)nr * 4) &&
                r.raw(L.rle_mat.data(), nr) && r.pad8();
      if (!ok) { delete b; return svd_fail(SVD_EFORMAT, "blob: truncated LOD %u", k); }
      // structure: empty, or a consistent DAG with runs covering every voxel
      bool valid;
      if (nw == 0) {
        valid = nl == 0 && nr == 0 && ns == 0;
      } else {
        std::vector<uint32_t> lev_count;
        valid = ns > 0 && nr > 0 && node_boxes(L, &lev_count, L.lo, L.hi);
        if (valid) {
          for (int q = 0; q < 16; q++) L.level_nodes[q] = lev_count[q];
          L.level_nodes[2] = nl;
          valid = L.rle_start[0] == 0 && L.rle_start[nr - 1] < ns;
          for (uint32_t q = 0; valid && q < nr; q++) {
            valid = L.rle_mat[q] != 0;
            if (q > 0) valid = valid && L.rle_start[q] > L.rle_start[q - 1] && L.rle_mat[q] != L.rle_mat[q - 1];
          }
          for (int a = 0; valid && a < 3; a++) valid = L.hi[a] < R;
        }
      }
      if (!valid) { delete b; return svd_fail(SVD_EFORMAT, "blob: inconsistent DAG at LOD %u", k); }
      int rc = derive_device(L, b->image);
      if (rc != SVD_OK) { delete b; return rc == SVD_ERANGE ? rc : SVD_EFORMAT; }
    }
    if (r.o != n) { delete b; return svd_fail(SVD_EFORMAT, "blob: trailing bytes"); }
    *out = b;
    return SVD_OK;
  } catch (const std::bad_alloc&) {
    return svd_fail(SVD_ENOMEM, "svd_blob_from_bytes: out of memory");
  }
}

extern "C" int svd_blob_stats_get(const svd_blob* b, uint32_t lod, svd_blob_stats* out) {
  if (!b || !out || lod >= b->lod_count) return svd_fail(SVD_EINVAL, "svd_blob_stats_get: bad argument");
  const LodData& L = b->lod[lod];
  memset(out, 0, sizeof(*out));
  out->R = L.R;
  out->n_words = (uint32_t)L.words.size();
  out->n_leaves = (uint32_t)L.leaves.size();
  out->n_rle = (uint32_t)L.rle_start.size();
  out->n_solid = L.n_solid;
  for (int i = 0; i < 16; i++) out->level_nodes[i] = L.level_nodes[i];
  for (int a = 0; a < 3; a++) {
    out->aabb_lo[a] = L.lo[a];
    out->aabb_hi[a] = L.hi[a];
  }
  out->device_bytes = L.off_end - L.off_begin;
  return SVD_OK;
}

extern "C" int svd_blob_canonical(const svd_blob* b, uint32_t lod, const uint32_t** words,
                                  const uint64_t** leaves, const uint32_t** rle_start,
                                  const uint8_t** rle_mat) {
  if (!b || lod >= b->lod_count || !words || !leaves || !rle_start || !rle_mat)
    return svd_fail(SVD_EINVAL, "svd_blob_canonical: bad argument");
  const LodData& L = b->lod[lod];
  *words = L.words.data();
  *leaves = L.leaves.data();
  *rle_start = L.rle_start.data();
  *rle_mat = L.rle_mat.data();
  return SVD_OK;
}
