// lb_analysis.hip -- droplet-level observables of a lattice state: connected
// components of the dispersed phase (droplet count, volumes, centroids, the
// number of droplet rows) and the vorticity of the flow (Results: droplet
// arrangements and their flow, vorticity after break-up).
//
// Droplets.  The dispersed phase is the set of fluid nodes with
// psi = (rho1 - rho2)/(rho1 + rho2) > 0, evaluated in FP64 from the fields
// that the lattice pass in FIELDS mode writes.  Components under face
// adjacency are found by union-find in two passes: inside 64-wide tiles in
// LDS (x-runs from wavefront ballots, then the remaining tile edges), then
// across tile faces on a parent array in HBM.  Every parent points to a
// smaller node index of the same component and links are made with atomicMin
// on a root, so the root of each final tree is the smallest node index of its
// component -- the canonical label, independent of the order in which the
// wavefronts run.  Volumes and centroid offsets are integer sums (exact,
// order-independent); droplets are listed in ascending label order through a
// block count / scan / write sequence.
//
// Vorticity: central differences of the FP64 velocity between nearest nodes.
#include "lb_internal.hpp"

#include <hip/hip_runtime.h>
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

using namespace lbk;
using namespace lbi;

namespace {

constexpr int TPB = 256;           // threads per block of the node-parallel kernels
constexpr int CHUNK = 4 * TPB;     // nodes per block of the root enumeration

struct Geo {
  int nx, ny, nz, walls;
  int32_t N;
};

__device__ __forceinline__ void coords(const Geo &g, int32_t n, int &x, int &y, int &z) {
  x = n % g.nx;
  const int32_t r = n / g.nx;
  y = r % g.ny;
  z = r / g.ny;
}

__device__ __forceinline__ bool wall_row(const Geo &g, int y) {
  return g.walls && (y == 0 || y == g.ny - 1);
}

// Tile of the local labelling pass: 64 x TY x TZ nodes per block of TPB
// threads (a whole number of nodes per thread).
#ifndef LBA_TY3
#define LBA_TY3 4
#endif
#ifndef LBA_TZ3
#define LBA_TZ3 4
#endif
template <int D>
struct Tile {
  static constexpr int TX = 64, TY = (D == 2) ? 16 : LBA_TY3, TZ = (D == 2) ? 1 : LBA_TZ3;
  static constexpr int NODES = TX * TY * TZ;
  static_assert(NODES % TPB == 0, "whole nodes per thread");
};

template <int D>
__host__ __device__ __forceinline__ int tiles_x(const Geo &g) { return (g.nx + Tile<D>::TX - 1) / Tile<D>::TX; }
template <int D>
__host__ __device__ __forceinline__ int tiles_y(const Geo &g) { return (g.ny + Tile<D>::TY - 1) / Tile<D>::TY; }
template <int D>
__host__ __device__ __forceinline__ int tiles_z(const Geo &g) { return (g.nz + Tile<D>::TZ - 1) / Tile<D>::TZ; }

// Parent reads during linking see other threads' links (any value read is an
// ancestor of the node, since links only ever lower a parent).
__device__ __forceinline__ int32_t load_parent(const int32_t *parent, int32_t x) {
  return __hip_atomic_load(parent + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t load_local(const int32_t *lp, int32_t x) {
  return __hip_atomic_load(lp + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

template <bool LOCAL>
__device__ __forceinline__ int32_t find_root(const int32_t *parent, int32_t x) {
  int32_t p = LOCAL ? load_local(parent, x) : load_parent(parent, x);
  while (p != x) {
    x = p;
    p = LOCAL ? load_local(parent, x) : load_parent(parent, x);
  }
  return x;
}

// Joins the trees of a and b: the larger root is linked below the smaller
// one.  A link only succeeds on a node that is still a root; otherwise the
// atomic returns that node's new parent and the walk continues from there.
// Each failed round lowers a + b, so the loop ends.  Works on the LDS copy of
// a tile (LOCAL) or on the parent array in HBM.
template <bool LOCAL>
__device__ __forceinline__ void unite(int32_t *parent, int32_t a, int32_t b) {
  for (;;) {
    a = find_root<LOCAL>(parent, a);
    b = find_root<LOCAL>(parent, b);
    if (a == b) return;
    if (a > b) {
      const int32_t t = a;
      a = b;
      b = t;
    }
    const int32_t old = atomicMin(parent + b, a);
    if (old == b) return;
    b = old;
  }
}

template <int D>
__device__ __forceinline__ void tile_origin(const Geo &g, int &x0, int &y0, int &z0) {
  const int tx = tiles_x<D>(g), ty = tiles_y<D>(g);
  x0 = (blockIdx.x % tx) * Tile<D>::TX;
  y0 = ((blockIdx.x / tx) % ty) * Tile<D>::TY;
  z0 = (blockIdx.x / (tx * ty)) * Tile<D>::TZ;
}

// Local pass over one tile: the dispersed-phase mask (psi > 0 in FP64, wall
// rows excluded), components over the edges inside the tile (no wrap) by
// union-find in LDS, then parent[n] = global index of the node's local root
// (-1 outside the dispersed phase).  Local and global node order agree, so a
// local root is also the smallest global index of its local component.  The
// four result counters are cleared here.
template <int D>
__global__ __launch_bounds__(TPB) void k_cc_local(const double *__restrict__ r1,
                                                  const double *__restrict__ r2, int32_t *parent,
                                                  unsigned long long *counters, Geo g) {
  using T = Tile<D>;
  if (blockIdx.x == 0 && threadIdx.x < 4) counters[threadIdx.x] = 0ull;
  __shared__ int32_t lp[T::NODES];
  int x0, y0, z0;
  tile_origin<D>(g, x0, y0, z0);
  constexpr int PER = T::NODES / TPB;
  for (int k = 0; k < PER; ++k) {
    const int li = threadIdx.x + TPB * k;
    const int x = x0 + (li % T::TX), y = y0 + (li / T::TX) % T::TY, z = z0 + li / (T::TX * T::TY);
    bool m = false;
    if (x < g.nx && y < g.ny && z < g.nz) {
      const int32_t n = x + g.nx * (y + g.ny * z);
      if (!wall_row(g, y)) {
        const double a = r1[n], b = r2[n], rho = a + b;
        const double psi = rho > 0.0 ? (a - b) / rho : -1.0;
        m = psi > 0.0;
      }
    }
    // one tile row is one wavefront (lane = x offset): a dispersed node points
    // at the first node of its run along x, which joins the run without atomics
    const uint64_t M = __ballot(m);
    const int xl = li % T::TX;
    const uint64_t gaps = ~M & ((1ull << xl) - 1ull);
    const int start = gaps ? 64 - __clzll(gaps) : 0;
    lp[li] = m ? li - xl + start : -1;
  }
  __syncthreads();
  // +y and +z edges inside the tile; of a run of such edges along x whose end
  // nodes are joined by their x-runs, only the first is needed
  for (int k = 0; k < PER; ++k) {
    const int li = threadIdx.x + TPB * k;
    if (lp[li] < 0) continue;
    const int xl = li % T::TX, yl = (li / T::TX) % T::TY, zl = li / (T::TX * T::TY);
    const bool left = xl > 0 && lp[li - 1] >= 0;
    if (yl + 1 < T::TY && lp[li + T::TX] >= 0 && !(left && lp[li - 1 + T::TX] >= 0))
      unite<true>(lp, li, li + T::TX);
    constexpr int PZ = T::TX * T::TY;
    if (D == 3 && zl + 1 < T::TZ && lp[li + PZ] >= 0 && !(left && lp[li - 1 + PZ] >= 0))
      unite<true>(lp, li, li + PZ);
  }
  __syncthreads();
  for (int k = 0; k < PER; ++k) {
    const int li = threadIdx.x + TPB * k;
    const int x = x0 + (li % T::TX), y = y0 + (li / T::TX) % T::TY, z = z0 + li / (T::TX * T::TY);
    if (x >= g.nx || y >= g.ny || z >= g.nz) continue;
    int32_t p = -1;
    if (lp[li] >= 0) {
      const int r = find_root<true>(lp, li);
      p = (x0 + r % T::TX) + g.nx * ((y0 + (r / T::TX) % T::TY) + g.ny * (z0 + r / (T::TX * T::TY)));
    }
    parent[x + g.nx * (y + g.ny * z)] = p;
  }
}

// Global pass: the edges that leave a tile in +x, +y, +z (wrapping along the
// periodic axes), joined by union-find on the parent array in HBM.  Along a
// tile face, consecutive crossing edges whose end nodes are linked inside
// their own tiles join the same two local components: only the first edge of
// each such run is taken (the run runs along x on the y and z faces, along y
// on the x face, and never leaves the tile).
template <int D>
__global__ __launch_bounds__(TPB) void k_cc_border(int32_t *parent, Geo g) {
  using T = Tile<D>;
  const int32_t n = blockIdx.x * TPB + threadIdx.x;
  if (n >= g.N) return;
  int x, y, z;
  coords(g, n, x, y, z);
  const bool fx = (x % T::TX == T::TX - 1) || x + 1 == g.nx;
  const bool fy = (y % T::TY == T::TY - 1) || y + 1 == g.ny;
  const bool fz = D == 3 && ((z % T::TZ == T::TZ - 1) || z + 1 == g.nz);
  if (!(fx || fy || fz) || parent[n] < 0) return;
  // run predecessor along x (same tile row on both sides) / along y
  const bool has_xm = x % T::TX != 0;
  const bool has_ym = y % T::TY != 0;
  if (fx && g.nx > 1) {
    const int32_t m = (x + 1 == g.nx) ? n - x : n + 1;
    // predecessor pair one row down, inside both tiles (m's tile row starts
    // at the same y as n's)
    const bool skip = has_ym && parent[n - g.nx] >= 0 && parent[m - g.nx] >= 0;
    if (!skip && parent[m] >= 0) unite<false>(parent, n, m);
  }
  if (fy) {
    int32_t m = -1;
    if (y + 1 < g.ny) m = n + g.nx;
    else if (!g.walls && g.ny > 1) m = n - (g.ny - 1) * g.nx;
    if (m >= 0) {
      const bool skip = has_xm && parent[n - 1] >= 0 && parent[m - 1] >= 0;
      if (!skip && parent[m] >= 0) unite<false>(parent, n, m);
    }
  }
  if (fz && g.nz > 1) {
    const int32_t plane = g.nx * g.ny;
    const int32_t m = (z + 1 == g.nz) ? n - z * plane : n + plane;
    const bool skip = has_xm && parent[n - 1] >= 0 && parent[m - 1] >= 0;
    if (!skip && parent[m] >= 0) unite<false>(parent, n, m);
  }
}

// parent[n] = root of n (the canonical label); the trees are final here.
// Roots clear their slots of the per-root sums of the stats pass.
__global__ __launch_bounds__(TPB) void k_cc_flatten(int32_t *parent, uint32_t *vol,
                                                    unsigned long long *sums, Geo g) {
  const int32_t n = blockIdx.x * TPB + threadIdx.x;
  if (n >= g.N) return;
  int32_t p = parent[n];
  if (p < 0) return;
  if (p == n) {
    vol[n] = 0u;
    sums[n] = 0ull;
    sums[(size_t)g.N + n] = 0ull;
    sums[2 * (size_t)g.N + n] = 0ull;
    return;
  }
  int32_t q = parent[p];
  while (q != p) {
    p = q;
    q = parent[p];
  }
  parent[n] = p;
}

// Offset of coordinate c from the root's coordinate rc: in periodic directions
// the image in [-floor(L/2), L - 1 - floor(L/2)].
__device__ __forceinline__ int offset(int c, int rc, int L, bool periodic) {
  int d = c - rc;
  if (periodic) {
    const int h = L / 2;
    d += h;
    if (d < 0) d += L;
    else if (d >= L) d -= L;
    d -= h;
  }
  return d;
}

__device__ __forceinline__ long long wave_sum(long long v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Per-root volume and coordinate-offset sums, and the dispersed-node count.
// Each wavefront walks STATS_ITER consecutive 64-node chunks; within a chunk
// the lanes are grouped by root, each group summed across the wave, and the
// sums carried while the root stays the same.  A change of root flushes the
// carry with atomics; the final carries of the block's wavefronts (in node
// order) are merged where they share a root before their atomics, so a
// droplet costs one set of atomics per block it spans rather than per node.
constexpr int STATS_ITER = 4, STATS_TPB = 1024, STATS_WAVES = STATS_TPB / 64;
__global__ __launch_bounds__(STATS_TPB) void k_cc_stats(const int32_t *__restrict__ label, uint32_t *vol,
                                                        unsigned long long *sums, Geo g,
                                                        unsigned long long *dispersed) {
  __shared__ int32_t s_root[STATS_WAVES];
  __shared__ long long s_acc[STATS_WAVES][4];
  __shared__ long long s_total[STATS_WAVES];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t wave = (int64_t)blockIdx.x * STATS_WAVES + wv;
  int32_t cur = -1;
  long long acc[4] = {0, 0, 0, 0};
  long long total = 0;
  auto flush = [&](int32_t r, const long long *v) {
    atomicAdd(vol + r, (uint32_t)v[0]);
    for (int d = 0; d < 3; ++d)
      if (v[d + 1]) atomicAdd(sums + (size_t)d * g.N + r, (unsigned long long)v[d + 1]);
  };
  for (int it = 0; it < STATS_ITER; ++it) {
    const int64_t n = (wave * STATS_ITER + it) * 64 + lane;
    const int32_t r = n < g.N ? label[n] : -1;
    long long o[3] = {0, 0, 0};
    if (r >= 0) {
      int x, y, z, rx, ry, rz;
      coords(g, (int32_t)n, x, y, z);
      coords(g, r, rx, ry, rz);
      o[0] = offset(x, rx, g.nx, true);
      o[1] = offset(y, ry, g.ny, !g.walls);
      o[2] = offset(z, rz, g.nz, true);
    }
    bool todo = r >= 0;
    total += __popcll(__ballot(todo));
    for (;;) {
      const uint64_t m = __ballot(todo);
      if (!m) break;
      const int leader = __ffsll((unsigned long long)m) - 1;
      const int32_t R = __shfl(r, leader);
      const bool mine = todo && r == R;
      const long long c = __popcll(__ballot(mine));
      long long sm[3];
      for (int d = 0; d < 3; ++d) sm[d] = wave_sum(mine ? o[d] : 0ll);
      if (R != cur) {
        if (cur >= 0 && lane == 0) flush(cur, acc);
        cur = R;
        acc[0] = acc[1] = acc[2] = acc[3] = 0;
      }
      acc[0] += c;
      for (int d = 0; d < 3; ++d) acc[d + 1] += sm[d];
      todo = todo && !mine;
    }
  }
  if (lane == 0) {
    s_root[wv] = cur;
    for (int d = 0; d < 4; ++d) s_acc[wv][d] = acc[d];
    s_total[wv] = total;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t r = -1;
    long long v[4] = {0, 0, 0, 0};
    long long t = 0;
    for (int w = 0; w < STATS_WAVES; ++w) {
      t += s_total[w];
      if (s_root[w] < 0) continue;
      if (s_root[w] != r) {
        if (r >= 0) flush(r, v);
        r = s_root[w];
        v[0] = v[1] = v[2] = v[3] = 0;
      }
      for (int d = 0; d < 4; ++d) v[d] += s_acc[w][d];
    }
    if (r >= 0) flush(r, v);
    if (t) atomicAdd(dispersed, (unsigned long long)t);
  }
}

// Roots among the CHUNK nodes of each block.
__global__ __launch_bounds__(TPB) void k_root_count(const int32_t *__restrict__ label, int32_t *cnt,
                                                    Geo g) {
  int total = 0;
  for (int k = 0; k < CHUNK / TPB; ++k) {
    const int64_t n = (int64_t)blockIdx.x * CHUNK + k * TPB + threadIdx.x;
    total += __syncthreads_count(n < g.N && label[n] == (int32_t)n);
  }
  if (threadIdx.x == 0) cnt[blockIdx.x] = total;
}

// Exclusive scan of nb block counts (one block of 1024 threads), total into *count.
__global__ __launch_bounds__(1024) void k_scan(const int32_t *cnt, int32_t *off, int nb,
                                               unsigned long long *count) {
  __shared__ int32_t s[1024];
  int32_t carry = 0;
  for (int base = 0; base < nb; base += 1024) {
    const int i = base + threadIdx.x;
    const int32_t v = i < nb ? cnt[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
      const int32_t t = threadIdx.x >= d ? s[threadIdx.x - d] : 0;
      __syncthreads();
      s[threadIdx.x] += t;
      __syncthreads();
    }
    if (i < nb) off[i] = carry + s[threadIdx.x] - v;
    carry += s[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) *count = (unsigned long long)carry;
}

// Writes the droplet table in ascending root order: root, volume, centroid.
__global__ __launch_bounds__(TPB) void k_root_write(const int32_t *__restrict__ label,
                                                    const int32_t *__restrict__ off,
                                                    const uint32_t *__restrict__ vol,
                                                    const unsigned long long *__restrict__ sums, Geo g,
                                                    int64_t *root, int64_t *volume, double *centroid) {
  __shared__ int32_t wsum[TPB / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int32_t carry = off[blockIdx.x];
  for (int k = 0; k < CHUNK / TPB; ++k) {
    const int64_t n = (int64_t)blockIdx.x * CHUNK + k * TPB + threadIdx.x;
    const bool is_root = n < g.N && label[n] == (int32_t)n;
    const uint64_t mask = __ballot(is_root);
    const int rank = __popcll(mask & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wave] = __popcll(mask);
    __syncthreads();
    int before = 0, total = 0;
    for (int w = 0; w < TPB / 64; ++w) {
      before += w < wave ? wsum[w] : 0;
      total += wsum[w];
    }
    if (is_root) {
      const int32_t d = carry + before + rank;
      const int32_t r = (int32_t)n;
      int rc[3];
      coords(g, r, rc[0], rc[1], rc[2]);
      const uint32_t v = vol[r];
      root[d] = r;
      volume[d] = v;
      const int L[3] = {g.nx, g.ny, g.nz};
      const bool per[3] = {true, !g.walls, true};
      for (int a = 0; a < 3; ++a) {
        const long long s = (long long)sums[(size_t)a * g.N + r];
        double c = (double)rc[a] + (double)s / (double)v;
        if (per[a]) {
          if (c < 0.0) c += (double)L[a];
          else if (c >= (double)L[a]) c -= (double)L[a];
        }
        centroid[3 * (size_t)d + a] = c;
      }
    }
    carry += total;
    __syncthreads();
  }
}

// omega = curl u by central differences; u rows of walls count as 0.
template <int D>
__global__ __launch_bounds__(TPB) void k_vorticity(const double *__restrict__ u, double *w, Geo g) {
  const int32_t n = blockIdx.x * TPB + threadIdx.x;
  if (n >= g.N) return;
  int x, y, z;
  coords(g, n, x, y, z);
  const size_t N = (size_t)g.N;
  if (wall_row(g, y)) {
    for (int c = 0; c < (D == 3 ? 3 : 1); ++c) w[c * N + n] = 0.0;
    return;
  }
  const int32_t xp = (x + 1 == g.nx) ? n - x : n + 1;
  const int32_t xm = (x == 0) ? n + (g.nx - 1) : n - 1;
  const int32_t yp = (y + 1 == g.ny) ? n - (g.ny - 1) * g.nx : n + g.nx;
  const int32_t ym = (y == 0) ? n + (g.ny - 1) * g.nx : n - g.nx;
  // a neighbour on a wall row contributes u = 0
  const bool yp_wall = wall_row(g, y + 1 == g.ny ? 0 : y + 1);
  const bool ym_wall = wall_row(g, y == 0 ? g.ny - 1 : y - 1);
  auto at = [&](int c, int32_t m) { return u[c * N + m]; };
  auto aty = [&](int c, int32_t m, bool wall) { return wall ? 0.0 : u[c * N + m]; };
  const double dvy_dx = 0.5 * (at(1, xp) - at(1, xm));
  const double dux_dy = 0.5 * (aty(0, yp, yp_wall) - aty(0, ym, ym_wall));
  if constexpr (D == 2) {
    w[n] = dvy_dx - dux_dy;
  } else {
    const int32_t plane = g.nx * g.ny;
    const int32_t zp = (z + 1 == g.nz) ? n - z * plane : n + plane;
    const int32_t zm = (z == 0) ? n + (g.nz - 1) * plane : n - plane;
    const double duz_dy = 0.5 * (aty(2, yp, yp_wall) - aty(2, ym, ym_wall));
    const double duy_dz = 0.5 * (at(1, zp) - at(1, zm));
    const double dux_dz = 0.5 * (at(0, zp) - at(0, zm));
    const double duz_dx = 0.5 * (at(2, xp) - at(2, xm));
    w[n] = duz_dy - duy_dz;
    w[N + n] = dux_dz - duz_dx;
    w[2 * N + n] = dvy_dx - dux_dy;
  }
}

// Arena layout (byte offsets, each 256-aligned).
struct Arena {
  double *r1, *r2, *u, *w;
  int32_t *parent, *cnt, *off;
  uint32_t *vol;
  unsigned long long *sums, *counters;
  int64_t *root, *volume;
  double *centroid;
  size_t bytes;
};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

Arena layout(const lb_handle *h, char *base) {
  const size_t N = (size_t)h->N, nb = (N + CHUNK - 1) / CHUNK, maxd = N / 2 + 1;
  Arena a{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    char *p = base ? base + o : nullptr;
    o += align256(bytes);
    return p;
  };
  a.r1 = (double *)take(8 * N);
  a.r2 = (double *)take(8 * N);
  a.u = (double *)take(8 * (size_t)h->D * N);
  a.w = (double *)take(8 * 3 * N);
  a.parent = (int32_t *)take(4 * N);
  a.vol = (uint32_t *)take(4 * N);
  a.sums = (unsigned long long *)take(8 * 3 * N);
  a.cnt = (int32_t *)take(4 * nb);
  a.off = (int32_t *)take(4 * nb);
  a.counters = (unsigned long long *)take(8 * 4);
  a.root = (int64_t *)take(8 * maxd);
  a.volume = (int64_t *)take(8 * maxd);
  a.centroid = (double *)take(8 * 3 * maxd);
  a.bytes = o;
  return a;
}

int ensure_arena(lb_handle *h, Arena &a) {
  const size_t need = layout(h, nullptr).bytes;
  if (!h->ana) {
    hipError_t e = hipMalloc(&h->ana, need);
    if (e != hipSuccess) {
      h->ana = nullptr;
      return fail(LB_ENOMEM, "hipMalloc(%zu): %s", need, hipGetErrorString(e));
    }
    h->ana_bytes = need;
    h->bytes += (int64_t)need;
    for (int k = 0; k < 2; ++k) HIP_TRY(hipEventCreate(&h->ana_ev[k]));
  }
  a = layout(h, (char *)h->ana);
  return LB_OK;
}

Geo geo_of(const lb_handle *h) {
  return Geo{h->p.nx, h->p.ny, h->p.nz, h->p.walls_y, (int32_t)h->N};
}

// The FIELDS pass of the lattice kernels into the arena.  It writes every
// fluid node; the analysis kernels never read wall rows, but with a node-type
// geometry the other non-fluid nodes must read as zero (no phase, u = 0).
int fields_to_arena(lb_handle *h, const Arena &a) {
  if (h->geom) {
    const size_t N = (size_t)h->N;
    HIP_TRY(hipMemsetAsync(a.r1, 0, 8 * N, h->stream));
    HIP_TRY(hipMemsetAsync(a.r2, 0, 8 * N, h->stream));
    HIP_TRY(hipMemsetAsync(a.u, 0, 8 * (size_t)h->D * N, h->stream));
  }
  return dispatch(h, FIELDS, a.r1, a.r2, a.u, nullptr);
}

int check(lb_handle *h, const char *what) {
  if (!h) return fail(LB_EINVAL, "%s: NULL handle", what);
  if (!h->initialised) return fail(LB_ESTATE, "%s before initialisation", what);
  if (h->N >= ((int64_t)1 << 31)) return fail(LB_EINVAL, "%s: more than 2^31 - 1 nodes", what);
  return LB_OK;
}

// Rows across the channel: droplets of at least a quarter of the mean volume,
// sorted by centroid y; a gap above half the equivalent diameter of their
// median volume starts a new row.
int32_t count_rows(const std::vector<double> &cy, const std::vector<int64_t> &vol, int D) {
  if (vol.empty()) return 0;
  double sum = 0.0;
  for (int64_t v : vol) sum += (double)v;
  const double mean = sum / (double)vol.size();
  std::vector<double> y, v;
  for (size_t i = 0; i < vol.size(); ++i)
    if ((double)vol[i] >= 0.25 * mean) {
      y.push_back(cy[i]);
      v.push_back((double)vol[i]);
    }
  std::sort(y.begin(), y.end());
  std::sort(v.begin(), v.end());
  const size_t m = v.size();
  const double vm = (m % 2) ? v[m / 2] : (v[m / 2 - 1] + v[m / 2]) / 2.0;
  const double d_eq = 2.0 * (D == 2 ? std::sqrt(vm / M_PI) : std::pow(3.0 * vm / (4.0 * M_PI), 1.0 / 3.0));
  int32_t rows = 1;
  for (size_t i = 1; i < y.size(); ++i)
    if (y[i] - y[i - 1] > 0.5 * d_eq) ++rows;
  return rows;
}

}  // namespace

namespace lbi {
void analysis_free(lb_handle *h) {
  (void)hipFree(h->ana);
  h->ana = nullptr;
  for (int k = 0; k < 2; ++k)
    if (h->ana_ev[k]) (void)hipEventDestroy(h->ana_ev[k]);
}
}  // namespace lbi

extern "C" {

int lb_droplets(lb_handle *h, lb_droplet_stats *stats, int32_t *label, int64_t cap, int64_t *root,
                int64_t *volume, double *centroid) {
  int rc = check(h, "lb_droplets");
  if (rc) return rc;
  if (cap < 0) return fail(LB_EINVAL, "lb_droplets: cap < 0");
  Arena a;
  rc = ensure_arena(h, a);
  if (rc) return rc;
  const Geo g = geo_of(h);
  const int nb_nodes = (int)((h->N + TPB - 1) / TPB);
  const int nb = (int)((h->N + CHUNK - 1) / CHUNK);
  HIP_TRY(hipEventRecord(h->ana_ev[0], h->stream));
  rc = fields_to_arena(h, a);
  if (rc) return rc;
  const int tiles = h->D == 2 ? tiles_x<2>(g) * tiles_y<2>(g) : tiles_x<3>(g) * tiles_y<3>(g) * tiles_z<3>(g);
  if (h->D == 2) {
    hipLaunchKernelGGL(k_cc_local<2>, dim3(tiles), dim3(TPB), 0, h->stream, a.r1, a.r2, a.parent, a.counters, g);
    hipLaunchKernelGGL(k_cc_border<2>, dim3(nb_nodes), dim3(TPB), 0, h->stream, a.parent, g);
  } else {
    hipLaunchKernelGGL(k_cc_local<3>, dim3(tiles), dim3(TPB), 0, h->stream, a.r1, a.r2, a.parent, a.counters, g);
    hipLaunchKernelGGL(k_cc_border<3>, dim3(nb_nodes), dim3(TPB), 0, h->stream, a.parent, g);
  }
  hipLaunchKernelGGL(k_cc_flatten, dim3(nb_nodes), dim3(TPB), 0, h->stream, a.parent, a.vol, a.sums, g);
  const int64_t per_block = (int64_t)64 * STATS_ITER * STATS_WAVES;
  hipLaunchKernelGGL(k_cc_stats, dim3((int)((h->N + per_block - 1) / per_block)), dim3(STATS_TPB), 0,
                     h->stream, a.parent, a.vol, a.sums, g, a.counters + 1);
  hipLaunchKernelGGL(k_root_count, dim3(nb), dim3(TPB), 0, h->stream, a.parent, a.cnt, g);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, h->stream, a.cnt, a.off, nb, a.counters);
  hipLaunchKernelGGL(k_root_write, dim3(nb), dim3(TPB), 0, h->stream, a.parent, a.off, a.vol, a.sums, g,
                     a.root, a.volume, a.centroid);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipEventRecord(h->ana_ev[1], h->stream));
  unsigned long long cnt[2] = {0, 0};
  HIP_TRY(hipMemcpyAsync(cnt, a.counters, sizeof cnt, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, h->ana_ev[0], h->ana_ev[1]));
  h->ana_ms[0] = ms;
  const size_t count = (size_t)cnt[0];
  std::vector<int64_t> vol(count);
  std::vector<double> cen(3 * count);
  // copies on the handle's stream only, so that handles on other streams keep running
  if (count) {
    HIP_TRY(hipMemcpyAsync(vol.data(), a.volume, 8 * count, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipMemcpyAsync(cen.data(), a.centroid, 8 * 3 * count, hipMemcpyDeviceToHost, h->stream));
  }
  const size_t ncopy = std::min(count, (size_t)cap);
  if (label) HIP_TRY(hipMemcpyAsync(label, a.parent, 4 * (size_t)h->N, hipMemcpyDeviceToHost, h->stream));
  if (root && ncopy) HIP_TRY(hipMemcpyAsync(root, a.root, 8 * ncopy, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  if (volume && ncopy) std::memcpy(volume, vol.data(), 8 * ncopy);
  if (centroid && ncopy) std::memcpy(centroid, cen.data(), 8 * 3 * ncopy);
  if (stats) {
    std::vector<double> cy(count);
    for (size_t i = 0; i < count; ++i) cy[i] = cen[3 * i + 1];
    stats->count = (int64_t)count;
    stats->dispersed = (int64_t)cnt[1];
    stats->rows = count_rows(cy, vol, h->D);
  }
  return LB_OK;
}

int lb_vorticity(lb_handle *h, double *omega) {
  int rc = check(h, "lb_vorticity");
  if (rc) return rc;
  if (!omega) return fail(LB_EINVAL, "lb_vorticity: omega is NULL");
  Arena a;
  rc = ensure_arena(h, a);
  if (rc) return rc;
  const Geo g = geo_of(h);
  const int nb_nodes = (int)((h->N + TPB - 1) / TPB);
  HIP_TRY(hipEventRecord(h->ana_ev[0], h->stream));
  rc = fields_to_arena(h, a);
  if (rc) return rc;
  if (h->D == 2)
    hipLaunchKernelGGL(k_vorticity<2>, dim3(nb_nodes), dim3(TPB), 0, h->stream, a.u, a.w, g);
  else
    hipLaunchKernelGGL(k_vorticity<3>, dim3(nb_nodes), dim3(TPB), 0, h->stream, a.u, a.w, g);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipEventRecord(h->ana_ev[1], h->stream));
  const size_t n = (size_t)(h->D == 2 ? 1 : 3) * (size_t)h->N;
  HIP_TRY(hipMemcpyAsync(omega, a.w, 8 * n, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, h->ana_ev[0], h->ana_ev[1]));
  h->ana_ms[1] = ms;
  return LB_OK;
}

int lb_analysis_times(const lb_handle *h, double *ms_droplets, double *ms_vorticity) {
  if (!h) return fail(LB_EINVAL, "NULL handle");
  if (ms_droplets) *ms_droplets = h->ana_ms[0];
  if (ms_vorticity) *ms_vorticity = h->ana_ms[1];
  return LB_OK;
}

}  // extern "C"
