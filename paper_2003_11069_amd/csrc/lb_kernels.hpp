// lb_kernels.hpp -- HIP kernels (gfx950) of the colour-gradient + NCI lattice
// Boltzmann update.  Method: Materials and Methods of Montessori et al. (2019),
// Eq. (CGLBE) for the two-population stream/collide, the three-part collision
// (BGK relaxation, perturbation, recolouring), Eq. (near_c) for the
// near-contact force, exact-difference forcing.
//
// State representation (exact rewrite of the two-population state).
// After recolouring, f1*_i = a f'_i + w_i (c_i.B)/|c_i| and f2*_i = f'_i - f1*_i
// with a = rho1/rho and B = beta (rho1 rho2/rho) G^ (Latva-Kokko form), so the
// post-collision state of a node is fully described by the total populations
// f'_i and the per-node colour scalars (a, B).  The library stores
//     s_i = f'_i / w_i - 1        Q values per node, storage type S
//     a   = rho1 / rho            1 value per node, compute type R
//     B   = beta rho1 rho2/rho G^ D values per node, FP32
// in structure-of-arrays layout s[i][n], a[n], B[d][n] (n = x + nx(y + ny z)),
// and rebuilds f_i^k(x, t+1) = f_i^k*(x - c_i, t) while pulling.  D3Q27 moves
// 27 + 1 + 3 values per node instead of 54; all moment sums use the
// deviations s_i (j = sum_i w_i c_i s_i exactly), which keeps small velocities
// well conditioned.
//
// Walls (rows y = 0 and ny-1) use half-way bounce-back.  After its collision a
// fluid node next to a wall also writes each population heading into the wall
// into the wall row, in the slot of the reflected direction, so every pull is
// a plain shifted load; only the colour scalars need the reflection rule.
//
// Kernels of one step t -> t+1:
//   k_phase : pull the state, rho1 and psi(t) at every fluid node (colour
//             scalars of the sources staged in LDS)
//   k_main  : LDS tile of psi (+halo) -> G, n, delta_I, NCI probe -> pull the
//             total populations, BGK + EDM + perturbation + recolouring ->
//             store (or FP64 observables, fields or populations instead)
// Indexing is 32-bit (the library limits N to 2^29 nodes) so that loads use a
// uniform base register plus a 32-bit per-lane offset; the stored deviations
// take one 64-bit base per direction.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>
#include <stdint.h>
#include <type_traits>

namespace lbk {

// ---------------------------------------------------------------------------
// Lattices.  Direction i <-> c = (i%3 - 1, (i/3)%3 - 1, i/9 - 1); the opposite
// direction is Q-1-i and the rest direction is Q/2.
template <int D>
struct Lat {
  static constexpr int Q = (D == 2) ? 9 : 27;
  static constexpr int REST = Q / 2;
  __host__ __device__ static constexpr int cx(int i) { return i % 3 - 1; }
  __host__ __device__ static constexpr int cy(int i) { return (i / 3) % 3 - 1; }
  __host__ __device__ static constexpr int cz(int i) { return D == 2 ? 0 : i / 9 - 1; }
  __host__ __device__ static constexpr int c2(int i) {
    return cx(i) * cx(i) + cy(i) * cy(i) + cz(i) * cz(i);
  }
  __host__ __device__ static constexpr int opp(int i) { return Q - 1 - i; }
  __host__ __device__ static constexpr double w(int i) {
    return D == 2 ? (c2(i) == 0 ? 4.0 / 9.0 : c2(i) == 1 ? 1.0 / 9.0 : 1.0 / 36.0)
                  : (c2(i) == 0 ? 8.0 / 27.0
                                : c2(i) == 1 ? 2.0 / 27.0 : c2(i) == 2 ? 1.0 / 54.0 : 1.0 / 216.0);
  }
  // 1/|c_i| (0 for the rest direction)
  __host__ __device__ static constexpr double inv_norm(int i) {
    return c2(i) == 0 ? 0.0
                      : c2(i) == 1 ? 1.0
                                   : c2(i) == 2 ? 0.70710678118654752440 : 0.57735026918962576451;
  }
};

// ---------------------------------------------------------------------------
// Storage codec of s_i.
__device__ __forceinline__ float to_f(float v) { return v; }
__device__ __forceinline__ float to_f(__half v) { return __half2float(v); }
__device__ __forceinline__ float to_f(__hip_bfloat16 v) { return __bfloat162float(v); }
template <typename S> __device__ __forceinline__ S from_f(float v);
template <> __device__ __forceinline__ float from_f<float>(float v) { return v; }
template <> __device__ __forceinline__ __half from_f<__half>(float v) { return __float2half_rn(v); }
template <> __device__ __forceinline__ __hip_bfloat16 from_f<__hip_bfloat16>(float v) {
  return __float2bfloat16(v);
}
// a * b + c as a fused multiply-add, stored as S.  For FP16 a mixed-precision
// FMA that reads b as FP16 and rounds its result once, to FP16 (the form the
// compiler itself emits for this expression within one basic block); written
// out so that b need not be converted to FP32 first when it was loaded in
// another block.  Other types round the FP32 result to S.
template <typename S>
__device__ __forceinline__ S fma_to(float a, S b, float c) {
  if constexpr (std::is_same<S, __half>::value) {
    _Float16 r;
    asm("v_fma_mixlo_f16 %0, %1, %2, %3 op_sel_hi:[0,1,0]"
        : "=v"(r)
        : "v"(a), "v"(__builtin_bit_cast(_Float16, b)), "v"(c));
    return __builtin_bit_cast(__half, r);
  } else {
    return from_f<S>(a * to_f(b) + c);
  }
}

// (R)a + (R)b of two stored deviations.  For FP16 pairs with FP32 moments a
// single mixed-precision FMA (a x 1 + b, both read as FP16) gives the same
// value as two conversions and an add: the sum of two FP16 values is rounded
// once to FP32 either way.
template <typename R, typename S>
__device__ __forceinline__ R pair_sum(S a, S b) {
  if constexpr (std::is_same<S, __half>::value && std::is_same<R, float>::value) {
    float r;
    asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel_hi:[1,0,1]"
        : "=v"(r)
        : "v"(__builtin_bit_cast(_Float16, a)), "v"(__builtin_bit_cast(_Float16, b)));
    return r;
  } else {
    return (R)to_f(a) + (R)to_f(b);
  }
}

template <typename S> struct is_fp32 { static constexpr bool value = false; };
template <> struct is_fp32<float> { static constexpr bool value = true; };

// 32-bit element offset from a uniform base pointer.
template <typename T>
__device__ __forceinline__ T ld(const T *base, uint32_t idx) {
  return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) +
                                      (size_t)(idx * (uint32_t)sizeof(T)));
}
template <typename T>
__device__ __forceinline__ void st(T *base, uint32_t idx, T v) {
  *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + (size_t)(idx * (uint32_t)sizeof(T))) = v;
}

// ---------------------------------------------------------------------------
// Kernel arguments (plain pointers; sizes in nodes).
template <typename S, typename R>
struct State {
  S *s;      // Q * N
  float *s0; // N, rest direction when S is a 16-bit type (exact mass closure)
  R *a;      // N
  float *B;  // D * N
};

template <typename S, typename R>
struct Args {
  int nx, ny, nz, walls;
  uint32_t N;
  R tau_inv, half_As, beta, A, h_min, h_max;
  R tau2_inv;         // component 2 (two_tau): 1/tau_mix = (rho1/rho)/tau + (rho2/rho)/tau2
  int two_tau;
  R F[3];
  int smax;           // floor(h_max)
  int smaxc;          // ceil(h_max), probe steps of the continuous-NCI variant
  int dr_on;          // density-ratio variant
  R dr_gamma;         // rho_1^0 / rho_2^0
  R dr_g1, dr_g2;     // (1 - alpha_k)/(1 - w_0) - 1 (0 for equal densities)
  State<S, R> in, out;
  const double *xt;   // explicit first-step state: f_i/w_i - 1 (Q*N) or null
  const double *xc;   // explicit first-step state: f1_i/w_i (Q*N)
  R *psi;             // N
  R *r1;              // N, rho1 of the current state (written by k_phase)
  double *partials;   // per-block observables (8 per block)
  double *f_out0, *f_out1, *f_out2; // FIELDS/POPS/DIAG outputs
  int32_t *i_out;     // DIAG: hit distance
  int xcd_remap;      // 1: contiguous tile ranges per XCD
  const uint32_t *nbm; // node-type geometry (GEOM kernels): bit i set when the
                       // source x - c_i is solid; GEO_SOLID, GEO_NONFLUID flags
};

// Flags of the geometry mask word.
constexpr uint32_t GEO_SOLID = 1u << 30, GEO_NONFLUID = 1u << 31;
// outlet nodes: GEO_OUTLET, and bits 0-2 hold the axis direction of the
// feeder (0..5 for -x, +x, -y, +y, -z, +z)
constexpr uint32_t GEO_OUTLET = 1u << 29, GEO_FEEDER = 7u;

enum Mode { STEP = 0, STEP_OBS = 1, OBSERVE = 2, FIELDS = 3, POPS = 4, DIAG = 5 };
enum Src { PULL = 0, EXPLICIT = 1 };
enum Col { COL_NONE = 0, COL_GLOBAL = 1, COL_LDS = 2 };

__device__ __forceinline__ int wrapi(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

// periodic wrap of v in [-n, 2n) (one step outside the lattice at most)
__device__ __forceinline__ int wrap_near(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Maps the hardware block id to a logical tile id so that the tiles of one
// XCD (blocks are dealt round-robin over the 8 XCDs) form a contiguous range.
__device__ __forceinline__ int logical_block(int b, int nb, int remap) {
  if (!remap) return b;
  const int q = nb >> 3, r = nb & 7;
  const int k = b & 7, idx = b >> 3;
  return k * q + (k < r ? k : r) + idx;
}

// Source node x - c of fluid node (x,y,z), periodic in x and z, and in y
// without walls (with walls a fluid row's sources stay inside [0, ny-1]):
// n - (cx + cy nx + cz nx ny) plus a wrap correction that is nonzero only on
// the first/last plane of a periodic direction (precomputed per thread).
struct Wrap {
  uint32_t xp, xm, yp, ym, zp, zm;  // corrections for c = +1 / -1 per axis
  uint32_t sy, sz;                   // strides nx and nx*ny
};

__device__ __forceinline__ Wrap make_wrap(int nx, int ny, int nz, int walls, int x, int y, int z) {
  Wrap w;
  const uint32_t sy = (uint32_t)nx, sz = (uint32_t)nx * (uint32_t)ny;
  w.sy = sy;
  w.sz = sz;
  w.xp = (x == 0) ? (uint32_t)nx : 0u;                 // source x-1 wraps to nx-1
  w.xm = (x == nx - 1) ? (uint32_t)(-nx) : 0u;         // source x+1 wraps to 0
  w.yp = (!walls && y == 0) ? sz : 0u;
  w.ym = (!walls && y == ny - 1) ? (uint32_t)0 - sz : 0u;
  const uint32_t szz = sz * (uint32_t)nz;
  w.zp = (z == 0) ? szz : 0u;
  w.zm = (z == nz - 1) ? (uint32_t)0 - szz : 0u;
  return w;
}

// Byte offsets (relative to node n) of the source x - c along each axis, for
// c = -1, 0, +1, scaled by the element size; the stored deviations of all
// directions share one base pointer (direction stride N elements).
struct Offs {
  uint32_t x[3], y[3], z[3];
};

template <int D, uint32_t SB>
__device__ __forceinline__ Offs make_offs(int nx, int ny, int nz, int walls, int x, int y, int z) {
  Offs o;
  const uint32_t sy = (uint32_t)nx, sz = (uint32_t)nx * (uint32_t)ny;
  o.x[0] = (x == nx - 1 ? 0u - (uint32_t)(nx - 1) : 1u) * SB;  // c = -1: source x+1
  o.x[1] = 0u;
  o.x[2] = (x == 0 ? (uint32_t)(nx - 1) : 0u - 1u) * SB;       // c = +1: source x-1
  o.y[0] = (!walls && y == ny - 1 ? 0u - (uint32_t)(ny - 1) * sy : sy) * SB;
  o.y[1] = 0u;
  o.y[2] = (!walls && y == 0 ? (uint32_t)(ny - 1) * sy : 0u - sy) * SB;
  if (D == 3) {
    o.z[0] = (z == nz - 1 ? 0u - (uint32_t)(nz - 1) * sz : sz) * SB;
    o.z[2] = (z == 0 ? (uint32_t)(nz - 1) * sz : 0u - sz) * SB;
  } else {
    o.z[0] = 0u;
    o.z[2] = 0u;
  }
  o.z[1] = 0u;
  return o;
}

// Stores of k_main's outputs, optionally non-temporal (streamed past the
// caches): LBNCI_NT = 0 none, 1 the populations, 2 also the colour scalars.
#ifndef LBNCI_NT
#define LBNCI_NT 0
#endif
// The default path is a raw buffer store: the 64-bit base sits in a scalar
// descriptor and the 32-bit byte offset in the instruction's vector offset.  A
// global store would need a 64-bit vector address add per store whenever the
// offset's zero extension was computed in another basic block (every store of
// the collision loop follows a conditional wall store).  The descriptor's
// extent is the whole 32-bit offset range, so no in-range store is dropped.
template <int LEVEL, typename T>
__device__ __forceinline__ void stb_out(T *base, uint32_t byte_off, T v) {
  if constexpr (LBNCI_NT >= LEVEL) {
    char *p = reinterpret_cast<char *>(base) + (size_t)byte_off;
    if constexpr (sizeof(T) == 2) {
      __builtin_nontemporal_store(__builtin_bit_cast(uint16_t, v), reinterpret_cast<uint16_t *>(p));
    } else {
      __builtin_nontemporal_store(v, reinterpret_cast<T *>(p));
    }
  } else {
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(base, (short)0, -1, 0x00020000);
    if constexpr (sizeof(T) == 2) {
      __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, v), r, byte_off, 0, 0);
    } else if constexpr (sizeof(T) == 4) {
      __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, byte_off, 0, 0);
    } else {
      static_assert(sizeof(T) == 8, "stb_out: 2-, 4- or 8-byte elements");
      using u32x2 = uint32_t __attribute__((ext_vector_type(2)));
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, byte_off, 0, 0);
    }
  }
}

// Base of direction i's block of N stored deviations: a 64-bit pointer per
// direction, so every byte offset inside a direction stays 32-bit and the
// lattice needs only N * sizeof(S) < 4 GiB (not Q N sizeof(S)).
template <typename T>
__device__ __forceinline__ T *dir_base(T *s, uint32_t N, int i) {
  return s + (size_t)i * N;
}

template <typename T>
__device__ __forceinline__ T ldb(const T *base, uint32_t byte_off) {
  return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + (size_t)byte_off);
}
template <typename T>
__device__ __forceinline__ void stb(T *base, uint32_t byte_off, T v) {
  *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + (size_t)byte_off) = v;
}

template <int D>
__device__ __forceinline__ uint32_t source(const Wrap &w, uint32_t n, int cx, int cy, int cz) {
  uint32_t s = n;
  if (cx == 1) s += w.xp - 1u;
  if (cx == -1) s += w.xm + 1u;
  if (cy == 1) s += w.yp - w.sy;
  if (cy == -1) s += w.ym + w.sy;
  if (D == 3 && cz == 1) s += w.zp - w.sz;
  if (D == 3 && cz == -1) s += w.zm + w.sz;
  return s;
}

// ---------------------------------------------------------------------------
// Pull of the post-streaming state at fluid node (x,y,z): total deviations f[i]
// (units of w_i), rho - 1 = sum_i w_i f_i, j and (COL != COL_NONE) rho1.
// Colour scalars (a, B) of the sources come from global memory (COL_GLOBAL)
// or from an LDS tile with a one-node halo (COL_LDS; strides PX, PX*PY); a
// source in a wall row means bounce-back, i.e. the node's own scalars with the
// colour term's sign flipped (c_opp(i) = -c_i).
template <int D, typename S, typename R, int SRC, int COL, bool WANT_C1, int PX = 1, int PY = 1,
          int TS = 1, int GEOM = 0, typename FT = float>
__device__ __forceinline__ void pull(const Args<S, R> &A, int x, int y, int z, uint32_t n,
                                     const R *ta, const float *tB, int lidx, FT *f, R *c1out,
                                     R &dr, R &r1, R *j, uint32_t gm = 0u) {
  using L = Lat<D>;
  constexpr uint32_t SB = sizeof(S);
  dr = 0; r1 = 0;
  j[0] = j[1] = j[2] = 0;
  const Wrap wr = make_wrap(A.nx, A.ny, A.nz, A.walls, x, y, z);
  const Offs of = make_offs<D, SB>(A.nx, A.ny, A.nz, A.walls, x, y, z);
  const uint32_t nb = n * SB;
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    const int cx = L::cx(i), cy = L::cy(i), cz = L::cz(i);
    const R wi = (R)L::w(i);
    float sv;
    S raw{};
    R c1 = 0;
    if (SRC == EXPLICIT) {
      sv = (float)A.xt[(size_t)i * A.N + n];
      raw = from_f<S>(sv);
      if (COL != COL_NONE) c1 = (R)A.xc[(size_t)i * A.N + n];
    } else {
      if (!is_fp32<S>::value && i == L::REST) {
        sv = ld(A.in.s0, n);
      } else {
        raw = ldb(dir_base(A.in.s, A.N, i), nb + of.x[cx + 1] + of.y[cy + 1] + of.z[cz + 1]);
        sv = to_f(raw);
      }
      if (COL != COL_NONE) {
        const bool bb = GEOM ? ((gm >> i) & 1u) != 0u
                             : (A.walls && cy != 0 && (y - cy == 0 || y - cy == A.ny - 1));
        const R sgn = bb ? (R)-1 : (R)1;
        R av, Bx = 0, By = 0, Bz = 0;
        if (COL == COL_GLOBAL) {
          const uint32_t cs = bb ? n : source<D>(wr, n, cx, cy, cz);
          av = ld(A.in.a, cs);
          if (cx) Bx = (R)ld(A.in.B, cs);
          if (cy) By = (R)ld(A.in.B + A.N, cs);
          if (D == 3 && cz) Bz = (R)ld(A.in.B + 2 * (size_t)A.N, cs);
        } else {
          const int ls = bb ? lidx : lidx - cx - PX * cy - PX * PY * cz;
          av = ta[ls];
          if (cx) Bx = (R)tB[ls];
          if (cy) By = (R)tB[TS + ls];
          if (D == 3 && cz) Bz = (R)tB[2 * TS + ls];
        }
        R cB = 0;
        if (cx != 0 || cy != 0 || cz != 0)
          cB = ((R)cx * Bx + (R)cy * By + (R)cz * Bz) * ((R)L::inv_norm(i) * sgn);
        c1 = av * ((R)1 + (R)sv) + cB;
      }
    }
    // f: the deviations as loaded (FT = S keeps them in their stored type, so
    // that the collision converts each inside its own fused multiply-add; the
    // rest slot of 16-bit storage is then not returned)
    if constexpr (std::is_same<FT, float>::value) f[i] = sv;
    else f[i] = raw;
    if (WANT_C1) c1out[i] = c1;
    const R svr = (R)sv;
    dr += wi * svr;
    if (COL != COL_NONE) r1 += wi * c1;
    if (cx) j[0] += wi * (R)cx * svr;
    if (cy) j[1] += wi * (R)cy * svr;
    if (D == 3 && cz) j[2] += wi * (R)cz * svr;
  }
}

// ---------------------------------------------------------------------------
// Phase pass over one 64 x 4 x TZP tile (block of 64 x 4 threads): rho1 and
// psi(x,t) = (rho1 - rho2)/rho at every fluid node.  The sources' colour
// scalars are staged in LDS with a one-node halo (each is read by up to Q
// neighbours).  Safe to call repeatedly from one block (persistent kernels):
// it synchronises before reusing the LDS tile and never returns early.
// LDS staging of a tile of ROWS rows of 64 + 2H nodes (x fastest; tile slot
// lx + (64 + 2H) r) whose first column is node x0 - H.  Each wave loads whole
// rows: 64 consecutive nodes of row r = wave + k (NT / 64), its global row
// base computed once per row in scalar registers, so an element costs no
// vector index arithmetic; the 2H halo columns of every row are loaded by
// the first ROWS 2H threads.  All loads of a thread are issued before its
// LDS writes.  row(r) returns the global index of node x = 0 of tile row r;
// load(p, gx) reads the element(s) of node gx of the row that starts at
// global index p; store(slot, v) writes them to LDS.  near: every x
// coordinate lies within one period of the lattice (one-step wrap), else
// modulo.
template <int H, int ROWS, int NT, typename Row, typename Load, typename Store>
__device__ __forceinline__ void fill_rows(int tid, int x0, int nx, bool near, Row row, Load load,
                                          Store store) {
  constexpr int LXR = 64 + 2 * H, NWV = NT / 64, RIT = (ROWS + NWV - 1) / NWV;
  static_assert(NT % 64 == 0, "fill_rows: whole waves");
  static_assert(ROWS * 2 * H <= NT, "fill_rows: one halo element per thread");
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int gxi = near ? wrap_near(x0 + lane, nx) : wrapi(x0 + lane, nx);
  using V = decltype(load(0u, 0));
  V v[RIT];
#pragma unroll
  for (int k = 0; k < RIT; ++k) {
    const int r = wave + k * NWV;
    if (ROWS % NWV == 0 || r < ROWS) v[k] = load(row(r), gxi);
  }
  // halo columns: thread t < ROWS 2H takes row t / 2H, column j = t % 2H
  // (j < H: left halo, slot j; else right halo, slot 64 + j)
  const bool hal = tid < ROWS * 2 * H;
  const int hr = tid / (2 * H), hj = tid % (2 * H), hlx = hj < H ? hj : 64 + hj;
  V vh{};
  if (hal) {
    const int gxh = near ? wrap_near(x0 + hlx - H, nx) : wrapi(x0 + hlx - H, nx);
    vh = load(row(hr), gxh);
  }
#pragma unroll
  for (int k = 0; k < RIT; ++k) {
    const int r = wave + k * NWV;
    if (ROWS % NWV == 0 || r < ROWS) store(lane + H + LXR * r, v[k]);
  }
  if (hal) store(hlx + LXR * hr, vh);
}

template <int D, int TZP, int PBY = 4>
struct PhaseTile {
  static constexpr int PX = 66, PY = PBY + 2, PZ = (D == 3) ? TZP + 2 : 1;
  static constexpr int TS = PX * PY * PZ;
};

template <int D, typename S, typename R, int SRC, int TZP, int GEOM = 0, int PBY = 4>
__device__ __forceinline__ void phase_tile(const Args<S, R> &A, int bx, int by, int bz, R *ta,
                                           float *tB) {
  using PT = PhaseTile<D, TZP, PBY>;
  constexpr int PX = PT::PX, PY = PT::PY, PZ = PT::PZ;
  constexpr int TS = PT::TS;
  constexpr int NT = 64 * PBY;  // threads per block (64 x PBY)
  const int x0 = bx * 64, y0 = by * PBY, z0 = (D == 3) ? bz * TZP : 0;
  const int tid = threadIdx.x + 64 * threadIdx.y;
  // geometry: the first node's mask word is loaded before the LDS fill, so
  // its non-fluid test below waits for nothing (geometries have no wall rows)
  uint32_t gm0 = 0u;
  if constexpr (GEOM) {
    const int xg = x0 + threadIdx.x, yg = y0 + threadIdx.y;
    if (xg < A.nx && yg < A.ny) gm0 = ld(A.nbm, (uint32_t)xg + (uint32_t)A.nx * ((uint32_t)yg + (uint32_t)A.ny * z0));
  }
  if (SRC == PULL) {
    // all loads of a thread before its LDS writes; one-step wraps on lattices
    // at least a tile plus halo wide (block-uniform test), else modulo
    __syncthreads();
    const bool near = A.nx >= PX - 1 && A.ny >= PY - 1 && (D == 2 || A.nz >= PZ - 1);
    auto wrap = [&](int v, int n) { return near ? wrap_near(v, n) : wrapi(v, n); };
    struct AB {
      R a;
      float b[D];
    };
    fill_rows<1, PY * PZ, NT>(
        tid, x0, A.nx, near,
        [&](int r) -> uint32_t {
          const int gyy = wrap(y0 + r % PY - 1, A.ny);
          const int gzz = (D == 3) ? wrap(z0 + r / PY - 1, A.nz) : 0;
          return (uint32_t)A.nx * ((uint32_t)gyy + (uint32_t)A.ny * gzz);
        },
        [&](uint32_t p, int gx) {
          AB v;
          v.a = ld(A.in.a + p, (uint32_t)gx);
#pragma unroll
          for (int d = 0; d < D; ++d) v.b[d] = ld(A.in.B + (size_t)d * A.N + p, (uint32_t)gx);
          return v;
        },
        [&](int k, const AB &v) {
          ta[k] = v.a;
#pragma unroll
          for (int d = 0; d < D; ++d) tB[d * TS + k] = v.b[d];
        });
    __syncthreads();
  }
  const int x = x0 + threadIdx.x, y = y0 + threadIdx.y;
  if (x < A.nx && y < A.ny && !(A.walls && (y == 0 || y == A.ny - 1))) {
    for (int tz = 0; tz < ((D == 3) ? TZP : 1); ++tz) {
      const int z = z0 + tz;
      if (z >= A.nz) break;
      const uint32_t n = (uint32_t)x + (uint32_t)A.nx * ((uint32_t)y + (uint32_t)A.ny * z);
      const uint32_t gm = GEOM ? (tz == 0 ? gm0 : ld(A.nbm, n)) : 0u;
      if (GEOM && (gm & GEO_NONFLUID)) continue;
      const int lidx = (threadIdx.x + 1) + PX * ((threadIdx.y + 1) + PY * ((D == 3) ? tz + 1 : 0));
      float f[Lat<D>::Q];
      R dr, r1, j[3];
      pull<D, S, R, SRC, COL_LDS, false, PX, PY, TS, GEOM>(A, x, y, z, n, ta, tB, lidx, f, nullptr, dr, r1,
                                                           j, gm);
      const R rho = (R)1 + dr;
      if (A.dr_on)  // density-ratio variant: psi normalised by the reference densities
        st(A.psi, n, (r1 - A.dr_gamma * (rho - r1)) / (r1 + A.dr_gamma * (rho - r1)));
      else
        st(A.psi, n, ((R)2 * r1 - rho) / rho);
      st(A.r1, n, r1);
    }
  }
}

// Number of phase tiles of a lattice.
template <int D, int TZP, int PBY = 4>
__host__ __device__ __forceinline__ int phase_tiles(int nx, int ny, int nz) {
  return ((nx + 63) / 64) * ((ny + PBY - 1) / PBY) * ((D == 3) ? (nz + TZP - 1) / TZP : 1);
}

template <int D, int TZP, int PBY = 4>
__device__ __forceinline__ void phase_decode(int nx, int ny, int lb, int &bx, int &by, int &bz) {
  const int gx = (nx + 63) / 64, gy = (ny + PBY - 1) / PBY;
  bx = lb % gx;
  by = (lb / gx) % gy;
  bz = lb / (gx * gy);
}

// k_phase: one phase tile per block over a single lattice.
template <int D, typename S, typename R, int SRC, int TZP, int WPE = 1, int GEOM = 0, int PBY = 4>
__global__ __launch_bounds__(64 * PBY) __attribute__((amdgpu_waves_per_eu(WPE))) void k_phase(Args<S, R> A) {
  constexpr int TS = PhaseTile<D, TZP, PBY>::TS;
  constexpr bool STAGE = (SRC == PULL);
  __shared__ R ta[STAGE ? TS : 1];
  __shared__ float tB[STAGE ? D * TS : 1];
  int bx, by, bz;
  phase_decode<D, TZP, PBY>(A.nx, A.ny, logical_block(blockIdx.x, gridDim.x, A.xcd_remap), bx, by, bz);
  phase_tile<D, S, R, SRC, TZP, GEOM, PBY>(A, bx, by, bz, ta, tB);
}

// A_h: A below h_min, A (h_min/h)^3 up to h_max, 0 beyond (Eq. near_c text).
template <typename R>
__device__ __forceinline__ R strength(int h, R A, R hmin, R hmax) {
  const R hr = (R)h;
  if (hr <= hmin) return A;
  if (hr <= hmax) {
    const R q = hmin / hr;
    return A * q * q * q;
  }
  return (R)0;
}

// Continuous-NCI variant: A below h_min, A ((h_min/h)^3 - q)/(1 - q) with
// q = (h_min/h_max)^3 up to h_max (0 there), 0 beyond.
template <typename R>
__device__ __forceinline__ R strength_shifted(R h, R A, R hmin, R hmax) {
  if (h <= hmin) return A;
  if (h > hmax) return (R)0;
  const R r = (hmin / h) * (hmin / h) * (hmin / h);
  const R q = (hmin / hmax) * (hmin / hmax) * (hmin / hmax);
  return A * (r - q) / ((R)1 - q);
}

__device__ __forceinline__ double round_away(double v) { return round(v); }
__device__ __forceinline__ float round_away(float v) { return roundf(v); }

// ---------------------------------------------------------------------------
// Main pass over one 64 x BY x TZ tile (block of 64 x BY threads, TZ z-planes
// per thread in 3-D): psi staged in LDS with a halo of H nodes (with H = 4 the
// NCI probe reads only LDS; with a smaller halo it falls back to the global
// psi array beyond the halo), gradient, NCI, pull, collision and store (or the
// MODE's alternative output).  Observable partials go to partials[slot].  Safe
// to call repeatedly from one block; it never returns early.
template <int D, int BY, int TZ, int H>
struct MainTile {
  static constexpr int LX = 64 + 2 * H, LY = BY + 2 * H, LZ = (D == 3) ? TZ + 2 * H : 1;
  static constexpr int TS = LX * LY * LZ;
};

template <int D, int BY, int TZ>
__host__ __device__ __forceinline__ int main_tiles(int nx, int ny, int nz) {
  return ((nx + 63) / 64) * ((ny + BY - 1) / BY) * ((D == 3) ? (nz + TZ - 1) / TZ : 1);
}

template <int D, int BY>
__device__ __forceinline__ void main_decode(int nx, int ny, int lb, int &bx, int &by, int &bz) {
  const int gx = (nx + 63) / 64, gy = (ny + BY - 1) / BY;
  bx = lb % gx;
  by = (lb / gx) % gy;
  bz = lb / (gx * gy);
}

// integer probe: up to this many samples are read together (longer probes
// take the sample-by-sample loop, which with a geometry reads the tile's psi
// inside the halo)
constexpr int PROBE_MAX = 4;

template <int D, typename S, typename R, int SRC, int MODE, int BY, int TZ, int H, int NCI = 0,
          int GEOM = 0>
__device__ __forceinline__ void main_tile(const Args<S, R> &A, int bx, int by, int bz, int slot,
                                          R *tile, double (*red)[8]) {
  using L = Lat<D>;
  constexpr int Q = L::Q;
  constexpr int LX = MainTile<D, BY, TZ, H>::LX, LY = MainTile<D, BY, TZ, H>::LY;
  constexpr int LZ = MainTile<D, BY, TZ, H>::LZ;
  constexpr int NT = 64 * BY;
  const int x0 = bx * 64, y0 = by * BY, z0 = (D == 3) ? bz * TZ : 0;
  const int tid = threadIdx.x + 64 * threadIdx.y;
  // geometry: the first node's mask word is loaded before the psi fill, so
  // its non-fluid test below waits for nothing (geometries have no wall rows)
  uint32_t gm0 = 0u;
  if constexpr (GEOM) {
    const int xg = x0 + threadIdx.x, yg = y0 + threadIdx.y;
    if (xg < A.nx && yg < A.ny) gm0 = ld(A.nbm, (uint32_t)xg + (uint32_t)A.nx * ((uint32_t)yg + (uint32_t)A.ny * z0));
  }

  // stage psi(tile + halo); wall rows read their fluid neighbour (copy rule).
  // A thread issues all its loads before its LDS writes; on lattices at least
  // a tile plus halo wide in every direction a coordinate wraps at most once
  // (a block-uniform test picks the one-step wrap over integer modulo).
  __syncthreads();
  {
    const bool near = A.nx >= LX - H && A.ny >= LY - H && (D == 2 || A.nz >= LZ - H);
    auto wrap = [&](int v, int n) { return near ? wrap_near(v, n) : wrapi(v, n); };
    fill_rows<H, LY * LZ, NT>(
        tid, x0, A.nx, near,
        [&](int r) -> uint32_t {
          int gyy = y0 + r % LY - H;
          if (A.walls) gyy = gyy < 1 ? 1 : (gyy > A.ny - 2 ? A.ny - 2 : gyy);
          else gyy = wrap(gyy, A.ny);
          const int gzz = (D == 3) ? wrap(z0 + r / LY - H, A.nz) : 0;
          return (uint32_t)A.nx * ((uint32_t)gyy + (uint32_t)A.ny * gzz);
        },
        [&](uint32_t p, int gx) { return ld(A.psi + p, (uint32_t)gx); },
        [&](int k, R v) { tile[k] = v; });
  }
  __syncthreads();

  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int x = x0 + threadIdx.x, y = y0 + threadIdx.y;
  const bool xy_ok = x < A.nx && y < A.ny && !(A.walls && (y == 0 || y == A.ny - 1));

  for (int tz = 0; tz < ((D == 3) ? TZ : 1); ++tz) {
    const int z = z0 + tz;
    if (!xy_ok || z >= A.nz) continue;
    const uint32_t n = (uint32_t)x + (uint32_t)A.nx * ((uint32_t)y + (uint32_t)A.ny * z);
    const uint32_t gm = GEOM ? (tz == 0 ? gm0 : ld(A.nbm, n)) : 0u;
    if (GEOM && (gm & GEO_NONFLUID)) continue;
    const int lx = threadIdx.x + H, ly = threadIdx.y + H, lz = (D == 3) ? tz + H : 0;
    auto T = [&](int ox, int oy, int oz) -> R {
      return tile[(lx + ox) + LX * ((ly + oy) + LY * (lz + oz))];
    };

    // colour gradient G = 3 sum_i w_i c_i psi(x + c_i)
    R G[3] = {0, 0, 0};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int cx = L::cx(i), cy = L::cy(i), cz = L::cz(i);
      if (cx == 0 && cy == 0 && cz == 0) continue;
      const R v = (R)(3.0 * L::w(i)) * T(cx, cy, cz);
      if (cx) G[0] += (R)cx * v;
      if (cy) G[1] += (R)cy * v;
      if (D == 3 && cz) G[2] += (R)cz * v;
    }
    const R g = sqrt(G[0] * G[0] + G[1] * G[1] + G[2] * G[2]);
    R Gh[3] = {0, 0, 0};
    if (g > (R)0) {
      const R ig = (R)1 / g;
      Gh[0] = G[0] * ig; Gh[1] = G[1] * ig; Gh[2] = G[2] * ig;
    }

    // near-contact probe along n = -G^: first s with psi(x + round(s n)) >= psi(x)
    R Fr[3] = {0, 0, 0};
    int hit = 0;
    // probe samples lie within ceil(h_max) <= 4 nodes of x, so on lattices at
    // least that long in every direction a coordinate wraps by one period at
    // most (a block-uniform test; integer modulo otherwise)
    const bool wrap1 = A.nx >= A.smaxc + 1 && A.ny >= A.smaxc + 1 && (D == 2 || A.nz >= A.smaxc + 1);
    auto wrapp = [&](int v, int n) { return wrap1 ? wrap_near(v, n) : wrapi(v, n); };
    if (NCI == 1 && A.A > (R)0 && g > (R)0) {
      // continuous-NCI variant: psi at x + s n by multilinear interpolation
      // (lerp x, then y, then z), h at the linear crossing between samples
      // s-1 and s (h = 1 for s = 1), A_h shifted to reach 0 at h_max
      const R ps = T(0, 0, 0);
      const R nn[3] = {-Gh[0], -Gh[1], -Gh[2]};
      auto node_psi = [&](int ox, int oy, int oz) -> R {
        if (abs(ox) <= H && abs(oy) <= H && abs(oz) <= H) return T(ox, oy, oz);
        const int xt = wrapp(x + ox, A.nx);
        int yt = y + oy;
        if (A.walls) yt = yt < 1 ? 1 : (yt > A.ny - 2 ? A.ny - 2 : yt);
        else yt = wrapp(yt, A.ny);
        const int zt = (D == 3) ? wrapp(z + oz, A.nz) : 0;
        return ld(A.psi, (uint32_t)xt + (uint32_t)A.nx * ((uint32_t)yt + (uint32_t)A.ny * zt));
      };
      R prev = ps, hc = 0;
      for (int s = 1; s <= A.smaxc; ++s) {
        const R px = (R)s * nn[0], py = (R)s * nn[1], pz = (D == 3) ? (R)s * nn[2] : (R)0;
        const R fx = floor(px), fy = floor(py), fz = floor(pz);
        const int ix = (int)fx, iy = (int)fy, iz = (int)fz;
        const R tx = px - fx, ty = py - fy, tzz = pz - fz;
        R cz[2] = {0, 0};
        for (int kz = 0; kz < (D == 3 ? 2 : 1); ++kz) {
          R cy[2];
          for (int ky = 0; ky < 2; ++ky) {
            const R a0 = node_psi(ix, iy + ky, iz + kz), a1 = node_psi(ix + 1, iy + ky, iz + kz);
            cy[ky] = a0 + tx * (a1 - a0);
          }
          cz[kz] = cy[0] + ty * (cy[1] - cy[0]);
        }
        const R pv = (D == 3) ? cz[0] + tzz * (cz[1] - cz[0]) : cz[0];
        if (pv >= ps) {
          hit = s;
          hc = (s == 1) ? (R)1 : (R)(s - 1) + (ps - prev) / (pv - prev);
          break;
        }
        prev = pv;
      }
      if (hit) {
        const R Ah = strength_shifted<R>(hc, A.A, A.h_min, A.h_max);
        Fr[0] = -Ah * nn[0] * (R)0.5 * g;
        Fr[1] = -Ah * nn[1] * (R)0.5 * g;
        Fr[2] = -Ah * nn[2] * (R)0.5 * g;
      }
    } else if (NCI == 0 && A.A > (R)0 && g > (R)0 && A.smax <= PROBE_MAX) {
      // up to PROBE_MAX samples: all of them read at once from the global psi
      // array (L2-resident; the row index clamped into the lattice, so every
      // read is in bounds), with a geometry's node-type words, so the reads
      // do not wait for one another; then the first sample at or above psi(x)
      // before a wall, a non-fluid node (geometries) or smax is the hit
      const R ps = T(0, 0, 0);
      const R nn[3] = {-Gh[0], -Gh[1], -Gh[2]};
      // every sample up to PROBE_MAX is read (also those beyond smax), so the
      // one-step wrap needs lattices longer than PROBE_MAX in every periodic
      // direction (a block-uniform test; integer modulo otherwise)
      const bool wrapb = A.nx > PROBE_MAX && A.ny > PROBE_MAX && (D == 2 || A.nz > PROBE_MAX);
      auto wrapq = [&](int v, int n) { return wrapb ? wrap_near(v, n) : wrapi(v, n); };
      R pv[PROBE_MAX];
      bool ok[PROBE_MAX];
      uint32_t ms[PROBE_MAX] = {};
#pragma unroll
      for (int k = 0; k < PROBE_MAX; ++k) {
        const int s = k + 1;
        const int ox = (int)round_away((R)s * nn[0]);
        const int oy = (int)round_away((R)s * nn[1]);
        const int oz = (D == 3) ? (int)round_away((R)s * nn[2]) : 0;
        const int yt = y + oy;
        ok[k] = s <= A.smax && !(A.walls && (yt <= 0 || yt >= A.ny - 1));
        const int xt = wrapq(x + ox, A.nx);
        const int ytt = A.walls ? min(max(yt, 1), A.ny - 2) : wrapq(yt, A.ny);
        const int zt = (D == 3) ? wrapq(z + oz, A.nz) : 0;
        const uint32_t ns = (uint32_t)xt + (uint32_t)A.nx * ((uint32_t)ytt + (uint32_t)A.ny * zt);
        pv[k] = ld(A.psi, ns);
        if constexpr (GEOM) ms[k] = ld(A.nbm, ns);
      }
#pragma unroll
      for (int k = 0; k < PROBE_MAX; ++k) {
        if (!ok[k]) break;
        if (GEOM && (ms[k] & GEO_NONFLUID)) break;
        if (pv[k] >= ps) { hit = k + 1; break; }
      }
      if (hit) {
        const R Ah = strength<R>(hit, A.A, A.h_min, A.h_max);
        Fr[0] = -Ah * nn[0] * (R)0.5 * g;
        Fr[1] = -Ah * nn[1] * (R)0.5 * g;
        Fr[2] = -Ah * nn[2] * (R)0.5 * g;
      }
    } else if (NCI == 0 && A.A > (R)0 && g > (R)0) {
      const R ps = T(0, 0, 0);
      const R nn[3] = {-Gh[0], -Gh[1], -Gh[2]};
      for (int s = 1; s <= A.smax; ++s) {
        const int ox = (int)round_away((R)s * nn[0]);
        const int oy = (int)round_away((R)s * nn[1]);
        const int oz = (D == 3) ? (int)round_away((R)s * nn[2]) : 0;
        const int yt = y + oy;
        if (A.walls && (yt <= 0 || yt >= A.ny - 1)) break;
        R pv;
        if constexpr (GEOM) {
          // the probe stops at any node that is not fluid; the sample's mask
          // word and psi are loaded together (a geometry's extents exceed the
          // probe reach, so one wrap step suffices).  psi: the LDS value read
          // at clamped offsets, the global value only beyond the halo (keeps
          // the two loads apart)
          const int xt = wrap_near(x + ox, A.nx);
          const int zt = (D == 3) ? wrap_near(z + oz, A.nz) : 0;
          const uint32_t ns =
              (uint32_t)xt + (uint32_t)A.nx * ((uint32_t)wrap_near(yt, A.ny) + (uint32_t)A.ny * zt);
          const uint32_t ms = ld(A.nbm, ns);
          const bool inside = abs(ox) <= H && abs(oy) <= H && abs(oz) <= H;
          pv = T(min(max(ox, -H), H), min(max(oy, -H), H), min(max(oz, -H), H));
          if (!inside) pv = ld(A.psi, ns);
          if (ms & GEO_NONFLUID) break;
        } else if (abs(ox) <= H && abs(oy) <= H && abs(oz) <= H) {
          pv = T(ox, oy, oz);
        } else {
          const int xt = wrapp(x + ox, A.nx);
          const int ytt = A.walls ? yt : wrapp(yt, A.ny);
          const int zt = (D == 3) ? wrapp(z + oz, A.nz) : 0;
          pv = ld(A.psi, (uint32_t)xt + (uint32_t)A.nx * ((uint32_t)ytt + (uint32_t)A.ny * zt));
        }
        if (pv >= ps) { hit = s; break; }
      }
      if (hit) {
        const R Ah = strength<R>(hit, A.A, A.h_min, A.h_max);
        // F_rep = -A_h n delta_I, delta_I = g/2
        Fr[0] = -Ah * nn[0] * (R)0.5 * g;
        Fr[1] = -Ah * nn[1] * (R)0.5 * g;
        Fr[2] = -Ah * nn[2] * (R)0.5 * g;
      }
    }
    const R F[3] = {A.F[0] + Fr[0], A.F[1] + Fr[1], (D == 3) ? A.F[2] + Fr[2] : (R)0};

    if (MODE == DIAG) {
      A.f_out0[n] = (double)T(0, 0, 0);
      A.f_out1[n] = (double)Fr[0];
      A.f_out1[(size_t)A.N + n] = (double)Fr[1];
      if (D == 3) A.f_out1[2 * (size_t)A.N + n] = (double)Fr[2];
      A.i_out[n] = hit;
      continue;
    }

    // the collision takes the deviations in their stored type (see pull)
    using FT = std::conditional_t<(MODE == STEP || MODE == STEP_OBS) && SRC == PULL, S, float>;
    FT f[Q];
    R c1[Q], dr, r1, j[3];
    if (MODE == POPS)
      pull<D, S, R, SRC, COL_GLOBAL, true, 1, 1, 1, GEOM>(A, x, y, z, n, nullptr, nullptr, 0, f, c1, dr, r1,
                                                          j, gm);
    else
      pull<D, S, R, SRC, COL_NONE, false, 1, 1, 1, GEOM>(A, x, y, z, n, nullptr, nullptr, 0, f, c1, dr, r1,
                                                         j, gm);
    r1 = ld(A.r1, n);
    const R rho = (R)1 + dr;

    if (MODE == POPS) {
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const double wi = L::w(i);
        A.f_out0[(size_t)i * A.N + n] = wi * (double)c1[i];
        A.f_out1[(size_t)i * A.N + n] = wi * (1.0 + (double)f[i]) - wi * (double)c1[i];
      }
      continue;
    }
    if (MODE == FIELDS) {
      A.f_out0[n] = (double)r1;
      A.f_out1[n] = (double)(rho - r1);
      for (int d = 0; d < D; ++d)
        A.f_out2[(size_t)d * A.N + n] = (double)((j[d] + (R)0.5 * F[d]) / rho);
      continue;
    }
    if (MODE == STEP_OBS || MODE == OBSERVE) {
      const double rd = (double)rho;
      double ph[3], uu = 0;
      for (int d = 0; d < 3; ++d) {
        ph[d] = (double)j[d] + 0.5 * (double)F[d];
        uu += (ph[d] / rd) * (ph[d] / rd);
      }
      acc[0] += (double)r1;
      acc[1] += rd - (double)r1;
      acc[2] += ph[0];
      acc[3] += ph[1];
      acc[4] += ph[2];
      acc[5] += ph[0] / rd;
      acc[6] += (double)r1 / rd * (ph[0] / rd);
      acc[7] = fmax(acc[7], sqrt(uu));
    }
    if (MODE == STEP || MODE == STEP_OBS) {
      // BGK + exact difference forcing + perturbation, in units of w_i.  The
      // moments, velocity, gradient and colour scalars stay in R; the
      // per-direction update works on O(1e-2) deviations and runs in FP32
      // (its rounding is of the order of the FP32 storage rounding).
      const R irho = (R)1 / rho;
      const R u[3] = {j[0] * irho, j[1] * irho, j[2] * irho};
      const float uf[3] = {(float)u[0], (float)u[1], (float)u[2]};
      const float uFf[3] = {(float)(u[0] + F[0] * irho), (float)(u[1] + F[1] * irho),
                            (float)(u[2] + F[2] * irho)};
      const float uu = uf[0] * uf[0] + uf[1] * uf[1] + uf[2] * uf[2];
      const float uuF = uFf[0] * uFf[0] + uFf[1] * uFf[1] + uFf[2] * uFf[2];
      const float pg = (float)(A.half_As * g), tinv = (float)A.tau_inv;
      const float drf = (float)dr, rhof = (float)rho;
      const float Ghf[3] = {(float)Gh[0], (float)Gh[1], (float)Gh[2]};
      const bool low = A.walls && y == 1, high = A.walls && y == A.ny - 2;
      // Directions i and opp(i) share the even part of the update and negate
      // the odd part:  sn = (1-om) f + C +- O  with
      //   C = om dr + rho (AF + (om-1) A) + pg (cG^2 - 1/3),
      //   O = 3 rho (cuF + (om-1) cu),  A = 4.5 cu^2 - 1.5 u.u (likewise AF).
      // The rest slot is set from the pre-collision density deviation dr (R)
      // minus the stored other directions, so each node keeps its mass up to
      // one rounding of the rest slot (the collision conserves mass exactly;
      // this removes the FP32 update's and the storage's rounding of it).  a
      // is taken against the density of the stored populations so that the
      // component-1 mass is carried exactly.
      // relaxation rate: one mixture tau, or the phase-weighted harmonic mean
      // of the two components' relaxation times (viscosity-ratio variant)
      const float om = A.two_tau ? (float)(r1 * irho * (A.tau_inv - A.tau2_inv) + A.tau2_inv) : tinv;
      const float omc = 1.f - om, om1 = om - 1.f;
      // density-ratio variant: the composition part of the equilibrium adds
      // dnr = rho1 (g1 - 1) + rho2 (g2 - 1) to every non-rest direction (0
      // for equal densities; the rest slot follows from mass closure)
      // (FP32: with a density ratio the stored deviations of the lighter
      // phase are O(1 - 1/gamma), so this rounding matches their storage's)
      const float dnrf = (float)(r1 * A.dr_g1 + (rho - r1) * A.dr_g2);
      const float cdr = om * (drf + dnrf) - pg * (1.0f / 3.0f);
      // When the moments are FP32 (16-bit storage, whose main pass is close
      // to its instruction-issue bound, and the FP32-arithmetic variant) C is evaluated as
      // a constant plus a quadratic form in c and O as a linear form; the
      // FP64-moment path and device geometries keep the per-direction form
      // above (same values up to FP32 rounding):
      //   C = K + c^T M c,  K = cdr - 1.5 rho (uF.uF + (om-1) u.u),
      //   M = 4.5 rho (uF uF^T + (om-1) u u^T) + pg G^ G^T,
      //   O = c.V,  V = 3 rho (uF + (om-1) u).
      // M's diagonal Md, its doubled off-diagonal entries Mo (xy, xz, yz) and
      // V are formed once per node; a direction's C is K plus Md of its
      // nonzero components plus Mo with the sign c_a c_b, summed in a fixed
      // order so that pairs share their partial sums.
      const float hq = 4.5f * rhof, hqo = hq * om1, r3 = 3.f * rhof;
      const float K = cdr - 1.5f * rhof * (uuF + om1 * uu);
      auto mq = [&](int a, int b) {
        return hq * uFf[a] * uFf[b] + hqo * uf[a] * uf[b] + pg * Ghf[a] * Ghf[b];
      };
      const float Md[3] = {mq(0, 0), mq(1, 1), (D == 3) ? mq(2, 2) : 0.f};
      const float Mo[3] = {2.f * mq(0, 1), (D == 3) ? 2.f * mq(0, 2) : 0.f, (D == 3) ? 2.f * mq(1, 2) : 0.f};
      const float V[3] = {r3 * (uFf[0] + om1 * uf[0]), r3 * (uFf[1] + om1 * uf[1]),
                          (D == 3) ? r3 * (uFf[2] + om1 * uf[2]) : 0.f};
      const uint32_t nb = n * (uint32_t)sizeof(S);
      Offs go{};  // geometry: wrapped byte offsets of the neighbours (periodic)
      if constexpr (GEOM) go = make_offs<D, (uint32_t)sizeof(S)>(A.nx, A.ny, A.nz, 0, x, y, z);
      constexpr bool QF = std::is_same<R, float>::value && !GEOM;
      R sum_q = 0;
#pragma unroll
      for (int i = 0; i < L::REST; ++i) {
        const int io = L::opp(i);
        const int icx = L::cx(i), icy = L::cy(i), icz = L::cz(i);
        // c.v over the nonzero components only, left to right (a zero
        // component's product would still cost an instruction)
        auto cdot = [&](const float *v) -> float {
          float t = 0.f;
          bool any = false;
          if (icx) { t = icx > 0 ? v[0] : -v[0]; any = true; }
          if (icy) { t = any ? (icy > 0 ? t + v[1] : t - v[1]) : (icy > 0 ? v[1] : -v[1]); any = true; }
          if (icz) t = any ? (icz > 0 ? t + v[2] : t - v[2]) : (icz > 0 ? v[2] : -v[2]);
          return t;
        };
        S q_i, q_o;
        if constexpr (QF) {
          float C = K;
          if (icx) C += Md[0];
          if (icy) C += Md[1];
          if (icz) C += Md[2];
          if (icx && icy) C = (icx == icy) ? C + Mo[0] : C - Mo[0];
          if (icx && icz) C = (icx == icz) ? C + Mo[1] : C - Mo[1];
          if (icy && icz) C = (icy == icz) ? C + Mo[2] : C - Mo[2];
          const float O = cdot(V);
          // one fused multiply-add per direction (with 16-bit storage it also
          // converts the stored deviation and rounds the result to 16 bits)
          q_i = fma_to<S>(omc, f[i], C + O);
          q_o = fma_to<S>(omc, f[io], C - O);
        } else {
          const float cu = cdot(uf), cuF = cdot(uFf), cG = cdot(Ghf);
          const float Ae = 4.5f * cu * cu - 1.5f * uu;
          const float AF = 4.5f * cuF * cuF - 1.5f * uuF;
          const float C = cdr + rhof * (AF + om1 * Ae) + pg * (cG * cG);
          const float O = 3.f * rhof * (cuF + om1 * cu);
          q_i = from_f<S>(omc * to_f(f[i]) + C + O);
          q_o = from_f<S>(omc * to_f(f[io]) + C - O);
        }
        stb_out<1>(dir_base(A.out.s, A.N, i), nb, q_i);
        stb_out<1>(dir_base(A.out.s, A.N, io), nb, q_o);
        // populations heading into a wall: reflected copy into the wall row,
        // node x + c_d, slot opp(d) (direction i has c_y = icy, opp(i) -icy)
        auto ghost = [&](int d, int dcx, int dcy, int dcz, S q) {
          const Offs wo = make_offs<D, (uint32_t)sizeof(S)>(A.nx, A.ny, A.nz, 1, x, y, z);
          stb_out<1>(dir_base(A.out.s, A.N, L::opp(d)), nb + wo.x[1 - dcx] + wo.y[1 - dcy] + wo.z[1 - dcz], q);
        };
        if constexpr (GEOM) {
          // populations heading into a solid node x + c_d: reflected copy in
          // its slot opp(d) (bit k of gm: the source x - c_k is solid); x + c_d
          // is the pull source of -c_d, so its byte offset is go.*[1 - c_d]
          auto ghost_g = [&](int d, int dcx, int dcy, int dcz, S q) {
            const uint32_t nwb = nb + go.x[1 - dcx] + go.y[1 - dcy] + go.z[1 - dcz];
            stb_out<1>(dir_base(A.out.s, A.N, L::opp(d)), nwb, q);
          };
          if ((gm >> io) & 1u) ghost_g(i, icx, icy, icz, q_i);
          if ((gm >> i) & 1u) ghost_g(io, -icx, -icy, -icz, q_o);
        } else {
          if ((icy == -1 && low) || (icy == 1 && high)) ghost(i, icx, icy, icz, q_i);
          if ((icy == 1 && low) || (icy == -1 && high)) ghost(io, -icx, -icy, -icz, q_o);
        }
        sum_q += (R)L::w(i) * pair_sum<R>(q_i, q_o);
      }
      const float srest = (float)((dr - sum_q) * (R)(1.0 / L::w(L::REST)));
      if (is_fp32<S>::value) stb_out<1>(dir_base(A.out.s, A.N, L::REST), nb, from_f<S>(srest));
      else stb_out<1>(A.out.s0, n * 4u, srest);
      const R dr_t = sum_q + (R)L::w(L::REST) * (R)srest;
      stb_out<2>(A.out.a, n * (uint32_t)sizeof(R), r1 / ((R)1 + dr_t));
      // recolouring weight (rho1 phi^1 + rho2 phi^2)/(rho w) = 1 + dnr/rho
      const R b = A.beta * r1 * (rho - r1) * irho * ((R)1 + (R)dnrf * irho);
      stb_out<2>(A.out.B, n * 4u, (float)(b * Gh[0]));
      stb_out<2>(A.out.B + A.N, n * 4u, (float)(b * Gh[1]));
      if (D == 3) stb_out<2>(A.out.B + 2 * (size_t)A.N, n * 4u, (float)(b * Gh[2]));
    }
  }

  if (MODE == STEP_OBS || MODE == OBSERVE) {
    // wavefront reduction (fixed butterfly), then across the block's waves
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      double v = acc[k];
      for (int m = 32; m >= 1; m >>= 1) {
        const double o = __shfl_xor(v, m, 64);
        v = (k == 7) ? fmax(v, o) : v + o;
      }
      acc[k] = v;
    }
    const int wave = tid >> 6, lane = tid & 63;
    if (lane == 0)
      for (int k = 0; k < 8; ++k) red[wave][k] = acc[k];
    __syncthreads();
    if (tid < 8) {
      double v = red[0][tid];
      for (int wv = 1; wv < NT / 64; ++wv) v = (tid == 7) ? fmax(v, red[wv][tid]) : v + red[wv][tid];
      A.partials[(size_t)slot * 8 + tid] = v;
    }
  }
}

// k_main: one main tile per block over a single lattice (NCI: 0 the integer
// probe, 1 the continuous-NCI variant).
template <int D, typename S, typename R, int SRC, int MODE, int BY, int TZ, int H, int WPE = 1, int NCI = 0,
          int GEOM = 0>
__global__ __launch_bounds__(64 * BY) __attribute__((amdgpu_waves_per_eu(WPE))) void k_main(Args<S, R> A) {
  __shared__ R tile[MainTile<D, BY, TZ, H>::TS];
  __shared__ double red[BY][8];
  int bx, by, bz;
  main_decode<D, BY>(A.nx, A.ny, logical_block(blockIdx.x, gridDim.x, A.xcd_remap), bx, by, bz);
  main_tile<D, S, R, SRC, MODE, BY, TZ, H, NCI, GEOM>(A, bx, by, bz, blockIdx.x, tile, red);
}


// ---------------------------------------------------------------------------
// Observables: deterministic reduction of the per-block partials (fixed
// strided order, then a fixed tree), followed by the windowed flow-rate
// convergence test: the mean Q over a window of W samples is compared with the
// previous window's; converged after m consecutive windows with a relative
// change <= eps.  A recorded sample whose component masses moved from those of
// the first recorded sample by more than mass_tol times the total mass
// (mass_tol > 0) raises the mass-drift flag.
struct ObsDev {
  double v[8];        // M1, M2, Px, Py, Pz, Q (unnormalised), Qd, umax
  double win_sum;     // running sum of Q in the current window
  double win_prev;    // mean Q of the previous complete window
  double win_last;    // mean Q of the last complete window
  int32_t win_count;  // samples in the current window
  int32_t n_windows;  // complete windows so far
  int32_t consec;     // consecutive windows within eps
  int32_t converged;
  int32_t flags;      // bit 0: NaN/Inf seen; bit 1: component mass drifted
  int32_t n_rec;      // recorded samples since initialisation
  double m_ref[2];    // component masses of the first recorded sample
};

// One 256-thread block reduces nparts per-tile partials (fixed order) into o
// and, when record != 0, advances the windowed flow-rate test.
__device__ __forceinline__ void obs_reduce_block(const double *partials, int nparts, ObsDev *o,
                                                 double inv_nx, int W, int m, double eps,
                                                 double mass_tol, int record, double (*sh)[8]) {
  const int t = threadIdx.x + blockDim.x * threadIdx.y;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int p = t; p < nparts; p += 256)
    for (int k = 0; k < 8; ++k) acc[k] = (k == 7) ? fmax(acc[k], partials[(size_t)p * 8 + k])
                                                  : acc[k] + partials[(size_t)p * 8 + k];
  __syncthreads();
  for (int k = 0; k < 8; ++k) sh[t][k] = acc[k];
  __syncthreads();
  for (int s = 128; s >= 1; s >>= 1) {
    if (t < s)
      for (int k = 0; k < 8; ++k)
        sh[t][k] = (k == 7) ? fmax(sh[t][k], sh[t + s][k]) : sh[t][k] + sh[t + s][k];
    __syncthreads();
  }
  if (t == 0) {
    for (int k = 0; k < 8; ++k) o->v[k] = sh[0][k];
    o->v[5] *= inv_nx;
    o->v[6] *= inv_nx;
    bool bad = false;
    for (int k = 0; k < 8; ++k) bad |= !isfinite(o->v[k]);
    if (bad) o->flags |= 1;
    if (record) {
      if (o->n_rec == 0) {
        o->m_ref[0] = o->v[0];
        o->m_ref[1] = o->v[1];
      } else if (mass_tol > 0) {
        const double tol = mass_tol * (fabs(o->m_ref[0]) + fabs(o->m_ref[1]));
        if (!(fabs(o->v[0] - o->m_ref[0]) <= tol && fabs(o->v[1] - o->m_ref[1]) <= tol)) o->flags |= 2;
      }
      o->n_rec += 1;
    }
    if (record && W > 0) {
      o->win_sum += o->v[5];
      o->win_count += 1;
      if (o->win_count == W) {
        const double mean = o->win_sum / W;
        if (o->n_windows > 0) {
          const bool ok = fabs(mean - o->win_last) <= eps * fabs(mean);
          o->consec = ok ? o->consec + 1 : 0;
          if (o->consec >= m) o->converged = 1;
        }
        o->win_prev = o->win_last;
        o->win_last = mean;
        o->n_windows += 1;
        o->win_sum = 0;
        o->win_count = 0;
      }
    }
  }
}

static __global__ __launch_bounds__(256) void k_obs_reduce(const double *partials, int nparts,
                                                    ObsDev *o, double inv_nx, int W, int m,
                                                    double eps, double mass_tol, int record) {
  __shared__ double sh[256][8];
  obs_reduce_block(partials, nparts, o, inv_nx, W, m, eps, mass_tol, record, sh);
}

// Streaming copy used as the achievable-bandwidth reference: one 16-byte
// vector per thread, non-temporal loads and stores (the fastest plain copy
// pattern measured on MI355X); init != 0 fills the source instead.
static __global__ __launch_bounds__(256) void k_copy_probe(float4 *src, float4 *dst, int64_t n4, int init) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n4) return;
  if (init) {
    src[k] = make_float4((float)k, 1.f, 2.f, 3.f);
    return;
  }
  float4 v;
  v.x = __builtin_nontemporal_load(&src[k].x);
  v.y = __builtin_nontemporal_load(&src[k].y);
  v.z = __builtin_nontemporal_load(&src[k].z);
  v.w = __builtin_nontemporal_load(&src[k].w);
  __builtin_nontemporal_store(v.x, &dst[k].x);
  __builtin_nontemporal_store(v.y, &dst[k].y);
  __builtin_nontemporal_store(v.z, &dst[k].z);
  __builtin_nontemporal_store(v.w, &dst[k].w);
}


// ---------------------------------------------------------------------------
// Batched stepping of many independent lattices ("channels") of uneven size.
// Each channel keeps its own Args (two per channel: one per ping-pong parity);
// channels never synchronise with each other.

// Per-channel bookkeeping shared by the batched kernels.
struct ChanCtl {
  ObsDev *obs;          // the channel's observables record
  double *partials;     // the channel's per-tile partials
  int32_t n_main;       // main tiles (= partial slots)
  int32_t n_phase;      // phase tiles
  int32_t active;       // 0 once retired (converged)
  int32_t retire;       // retire when the convergence flag rises
  int64_t t;            // steps completed
  double inv_nx;
  int32_t W, m;
  double eps;
  double mass_tol;
  int32_t obs_every;
  int32_t parity;       // state copy holding the current state
};

// Tile of a batched launch: channel and tile index within it.
struct TileRef {
  int32_t chan, tile;
};

template <int D, typename S, typename R, int TZP>
__global__ __launch_bounds__(256) void k_phase_batch(const Args<S, R> *__restrict__ args,
                                                     ChanCtl *ctl, const TileRef *__restrict__ tiles) {
  constexpr int TS = PhaseTile<D, TZP>::TS;
  __shared__ R ta[TS];
  __shared__ float tB[D * TS];
  const TileRef tr = tiles[blockIdx.x];
  const ChanCtl &c = ctl[tr.chan];
  if (!c.active) return;  // uniform per block
  const Args<S, R> &A = args[2 * tr.chan + c.parity];
  int bx, by, bz;
  phase_decode<D, TZP>(A.nx, A.ny, tr.tile, bx, by, bz);
  phase_tile<D, S, R, PULL, TZP>(A, bx, by, bz, ta, tB);
}

template <int D, typename S, typename R, int BY, int TZ, int H>
__global__ __launch_bounds__(64 * BY) void k_main_batch(const Args<S, R> *__restrict__ args,
                                                        ChanCtl *ctl, const TileRef *__restrict__ tiles) {
  __shared__ R tile[MainTile<D, BY, TZ, H>::TS];
  __shared__ double red[BY][8];
  const TileRef tr = tiles[blockIdx.x];
  const ChanCtl &c = ctl[tr.chan];
  if (!c.active) return;  // uniform per block
  const Args<S, R> &A = args[2 * tr.chan + c.parity];
  int bx, by, bz;
  main_decode<D, BY>(A.nx, A.ny, tr.tile, bx, by, bz);
  const bool rec = c.obs_every > 0 && (c.t % c.obs_every) == 0;
  if (rec) main_tile<D, S, R, PULL, STEP_OBS, BY, TZ, H>(A, bx, by, bz, tr.tile, tile, red);
  else main_tile<D, S, R, PULL, STEP, BY, TZ, H>(A, bx, by, bz, tr.tile, tile, red);
}

// End of a batched step, one block per channel: observables when recorded,
// retirement, step count and parity flip.
static __global__ __launch_bounds__(256) void k_batch_end(ChanCtl *ctl) {
  __shared__ double sh[256][8];
  ChanCtl &c = ctl[blockIdx.x];
  if (!c.active) return;
  const bool rec = c.obs_every > 0 && (c.t % c.obs_every) == 0;
  if (rec) obs_reduce_block(c.partials, c.n_main, c.obs, c.inv_nx, c.W, c.m, c.eps, c.mass_tol, 1, sh);
  __syncthreads();
  if (threadIdx.x == 0) {
    c.t += 1;
    c.parity ^= 1;
    if (c.retire && c.obs->converged) c.active = 0;
  }
}

// Per-channel barrier of a persistent launch.  Every wave waits until its own
// stores are complete in L2, then one lane per block publishes the block's
// writes at agent scope (one L2 write-back), counts the block in and waits
// (bounded) until all `target` arrivals of the channel's group are in, then
// acquires at agent scope (one L1/L2 invalidation) before the block goes on.
// Returns false if the wait exceeded 2 s or another block failed;
// the caller then leaves its loop, so every wave exits.
__device__ __forceinline__ bool group_barrier(uint32_t *cnt, uint32_t target, int32_t *err,
                                              int *flag) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0 && threadIdx.y == 0) {
    __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    int ok = 1;
    uint32_t spins = 0;
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();  // 100 MHz constant clock
    // wrap-safe: arrivals grow by 2 g per step and may pass 2^32 in a long launch
    while ((int32_t)(__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - target) < 0) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > (1u << 26) || __builtin_amdgcn_s_memrealtime() - t0 > 200000000ull ||
          __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *flag = ok;
  }
  __syncthreads();
  return *flag != 0;
}

// Persistent batched stepping: block b works for channel chan_of[b] as rank
// rank_of[b] of a group of group[c] blocks (groups sized by channel work).
// Per step: phase tiles, channel barrier, retirement check, main tiles,
// channel barrier; then the group's rank 0 reduces the observables of a
// recorded step and advances the channel record (step count, parity, active),
// which the other blocks read only after the next phase barrier.  Parity is
// tracked locally from the value read before the first barrier.  Must be
// launched cooperatively (all blocks resident).
template <int D, typename S, typename R, int TZP, int BY, int TZ, int H>
__global__ __launch_bounds__(256) void k_persistent(const Args<S, R> *__restrict__ args,
                                                    ChanCtl *ctl, const int32_t *__restrict__ chan_of,
                                                    const int32_t *__restrict__ rank_of,
                                                    const int32_t *__restrict__ group,
                                                    uint32_t *bar, int32_t *err, int nsteps) {
  static_assert(BY == 4, "persistent blocks are 64 x 4 threads");
  constexpr int PTS = PhaseTile<D, TZP>::TS, MTS = MainTile<D, BY, TZ, H>::TS;
  constexpr int PB = PTS * (int)sizeof(R) + D * PTS * 4, MB = MTS * (int)sizeof(R);
  constexpr int RB = 256 * 8 * 8;
  constexpr int LDS = PB > MB ? (PB > RB ? PB : RB) : (MB > RB ? MB : RB);
  __shared__ double lds[(LDS + 7) / 8];
  __shared__ double red[BY][8];
  __shared__ int flag;
  R *ta = reinterpret_cast<R *>(lds);
  float *tB = reinterpret_cast<float *>(reinterpret_cast<char *>(lds) + PTS * sizeof(R));
  R *tile = reinterpret_cast<R *>(lds);
  double(*sh)[8] = reinterpret_cast<double(*)[8]>(lds);
  const int ch = chan_of[blockIdx.x], rank = rank_of[blockIdx.x], g = group[ch];
  ChanCtl &c = ctl[ch];
  uint32_t *cnt = bar + ch;
  uint32_t arrivals = 0;
  const int par0 = c.parity;
  if (!c.active) return;  // retired before this launch: the same in every block
  for (int st = 0; st < nsteps; ++st) {
    const int par = par0 ^ (st & 1);
    const Args<S, R> &A = args[2 * ch + par];
    for (int k = rank; k < c.n_phase; k += g) {
      int bx, by, bz;
      phase_decode<D, TZP>(A.nx, A.ny, k, bx, by, bz);
      phase_tile<D, S, R, PULL, TZP>(A, bx, by, bz, ta, tB);
    }
    arrivals += g;
    if (!group_barrier(cnt, arrivals, err, &flag)) break;
    if (!c.active) break;  // retired at the end of the previous step
    const bool rec = c.obs_every > 0 && (c.t % c.obs_every) == 0;
    for (int k = rank; k < c.n_main; k += g) {
      int bx, by, bz;
      main_decode<D, BY>(A.nx, A.ny, k, bx, by, bz);
      if (rec) main_tile<D, S, R, PULL, STEP_OBS, BY, TZ, H>(A, bx, by, bz, k, tile, red);
      else main_tile<D, S, R, PULL, STEP, BY, TZ, H>(A, bx, by, bz, k, tile, red);
    }
    arrivals += g;
    if (!group_barrier(cnt, arrivals, err, &flag)) break;
    if (rank == 0) {
      if (rec) obs_reduce_block(c.partials, c.n_main, c.obs, c.inv_nx, c.W, c.m, c.eps, c.mass_tol, 1, sh);
      if (threadIdx.x == 0 && threadIdx.y == 0) {
        c.t += 1;
        c.parity = par ^ 1;
        if (c.retire && c.obs->converged) c.active = 0;
      }
    }
  }
}

// Fills n 32-bit words with v (used instead of a memset so the reset can sit
// inside a captured graph).
static __global__ __launch_bounds__(256) void k_fill_u32(uint32_t *p, int n, uint32_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace lbk
