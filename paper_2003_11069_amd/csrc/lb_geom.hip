// lb_geom.hip -- node-type geometry for device-scale runs (Results: droplet
// generation in a flow-focuser, Fig. 1): solid nodes with half-way
// bounce-back, velocity inlets and pressure outlets.
//
// A geometry handle runs the GEOM instantiations of k_phase and k_main: each
// node reads one mask word (bit i: the source x - c_i is solid; GEO_SOLID,
// GEO_NONFLUID), non-fluid nodes are skipped, pulls from solid sources use the
// bounce-back rule (the colliding fluid node writes its reflected populations
// into the solid node's slots, as for wall rows), and the NCI probe stops at
// non-fluid nodes.  Between k_phase and k_main one small kernel gives outlet
// nodes their feeder's psi and solid nodes the weighted mean psi of their
// non-solid neighbours; after k_main a second sets every inlet/outlet node's
// post-collision state from its feeder (the equilibrium of the boundary
// condition), so the next pull treats them like any node.
#include "lb_internal.hpp"

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <cmath>
#include <cstring>
#include <vector>

using namespace lbk;
using namespace lbi;

namespace {

template <int D>
__device__ __forceinline__ uint32_t neighbour(int nx, int ny, int nz, uint32_t n, int cx, int cy, int cz) {
  const int x = (int)(n % (uint32_t)nx);
  const int y = (int)((n / (uint32_t)nx) % (uint32_t)ny);
  const int z = (int)(n / ((uint32_t)nx * (uint32_t)ny));
  return (uint32_t)wrapi(x + cx, nx) +
         (uint32_t)nx * ((uint32_t)wrapi(y + cy, ny) + (uint32_t)ny * (D == 3 ? wrapi(z + cz, nz) : 0));
}

// psi of the boundary nodes, after k_phase, in one pass: an outlet takes its
// feeder's psi; a solid node the w_i-weighted mean over its non-solid
// neighbours, an outlet neighbour entering with its feeder's psi (the value
// it receives in the same pass), so no thread reads a slot another writes.
// Threads [0, n_out) handle the (outlet, feeder) pairs, the rest the solids.
template <int D, typename R>
__global__ __launch_bounds__(256) void k_psi_boundary(R *psi, const uint32_t *nbm, const int32_t *pairs,
                                                      int n_out, const int32_t *solids, int n_sol, int nx,
                                                      int ny, int nz) {
  using L = Lat<D>;
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k < n_out) {
    psi[pairs[2 * k]] = psi[pairs[2 * k + 1]];
    return;
  }
  if (k - n_out >= n_sol) return;
  const uint32_t s = (uint32_t)solids[k - n_out];
  R sw = 0, sp = 0;
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    if (i == L::REST) continue;
    uint32_t m = neighbour<D>(nx, ny, nz, s, L::cx(i), L::cy(i), L::cz(i));
    const uint32_t mm = nbm[m];
    if (mm & GEO_SOLID) continue;
    if (mm & GEO_OUTLET) {
      const int a = (int)(mm & GEO_FEEDER), sg = (a & 1) ? 1 : -1;
      m = neighbour<D>(nx, ny, nz, m, a < 2 ? sg : 0, (a >> 1) == 1 ? sg : 0, a >= 4 ? sg : 0);
    }
    sw += (R)L::w(i);
    sp += (R)L::w(i) * psi[m];
  }
  psi[s] = sw > (R)0 ? sp / sw : (R)0;
}

// Post-collision state of inlet/outlet nodes from their feeders' (copy out).
template <int D, typename S, typename R>
__global__ __launch_bounds__(256) void k_open_bc(Args<S, R> A, const BCNode *bc, int n) {
  using L = Lat<D>;
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= n) return;
  const BCNode b = bc[k];
  const uint32_t f = (uint32_t)b.feeder, node = (uint32_t)b.node;
  R dr = 0, j[3] = {0, 0, 0};
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    const float sv = (!is_fp32<S>::value && i == L::REST) ? ld(A.out.s0, f)
                                                          : to_f(A.out.s[(size_t)i * A.N + f]);
    const R wv = (R)L::w(i) * (R)sv;
    dr += wv;
    j[0] += (R)L::cx(i) * wv;
    j[1] += (R)L::cy(i) * wv;
    j[2] += (R)L::cz(i) * wv;
  }
  const R rho = (R)1 + dr;
  // composition: the inlet's prescribed fraction, or the feeder's own a, kept
  // exactly (a pure phase stays pure)
  R rb, frac, u[3];
  if (b.kind == LB_NODE_INLET) {
    rb = rho;
    frac = (R)b.frac1;
    for (int d = 0; d < 3; ++d) u[d] = (R)b.u[d];
  } else {
    rb = (R)b.rho;
    frac = ld(A.out.a, f);
    for (int d = 0; d < 3; ++d) u[d] = j[d] / rho;
  }
  const R uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    const R cu = (R)L::cx(i) * u[0] + (R)L::cy(i) * u[1] + (R)L::cz(i) * u[2];
    const float sv = (float)((rb - (R)1) + rb * ((R)3 * cu + (R)4.5 * cu * cu - (R)1.5 * uu));
    if (!is_fp32<S>::value && i == L::REST) st(A.out.s0, node, sv);
    else A.out.s[(size_t)i * A.N + node] = from_f<S>(sv);
  }
  st(A.out.a, node, frac);
  for (int d = 0; d < D; ++d) st(A.out.B + (size_t)d * A.N, node, 0.0f);
}

template <class K, class Ar>
void launch(K kernel, dim3 grid, dim3 block, hipStream_t st, hipEvent_t e0, hipEvent_t e1, const Ar &a) {
  if (e0) hipExtLaunchKernelGGL(kernel, grid, block, 0, st, e0, e1, 0, a);
  else hipLaunchKernelGGL(kernel, grid, block, 0, st, a);
}

template <int D, typename S, typename R, int SRC, int MODE>
void launch_main_geom(lb_handle *h, const Args<S, R> &a, hipEvent_t e0, hipEvent_t e1) {
  const int nb = blocks_main(h);
  if constexpr (D == 2)
    launch(k_main<D, S, R, SRC, MODE, BY2, TZ2, H2, 1, 0, 1>, dim3(nb), dim3(64, BY2), h->stream, e0, e1, a);
  else
    launch(k_main<D, S, R, SRC, MODE, BY3, TZ3, H3, LBNCI_WPE_MAIN3, 0, 1>, dim3(nb), dim3(64, BY3), h->stream,
           e0, e1, a);
}

template <int D, typename S, typename R, int SRC>
void launch_phase_geom(lb_handle *h, const Args<S, R> &a, hipEvent_t e0, hipEvent_t e1) {
  launch(k_phase<D, S, R, SRC, (D == 3 ? tzp3<S>() : 1), (D == 3 ? LBNCI_WPE_PHASE3 : 1), 1, (D == 3 ? PBY3 : 4)>,
         dim3(blocks_phase(h)), dim3(64, D == 3 ? PBY3 : 4), h->stream, e0, e1, a);
}

template <int D, typename S, typename R, int SRC>
void launch_main_mode(lb_handle *h, int mode, const Args<S, R> &a, hipEvent_t e0, hipEvent_t e1) {
  switch (mode) {
    case STEP: launch_main_geom<D, S, R, SRC, STEP>(h, a, e0, e1); break;
    case STEP_OBS: launch_main_geom<D, S, R, SRC, STEP_OBS>(h, a, e0, e1); break;
    case OBSERVE: launch_main_geom<D, S, R, SRC, OBSERVE>(h, a, nullptr, nullptr); break;
    case FIELDS: launch_main_geom<D, S, R, SRC, FIELDS>(h, a, nullptr, nullptr); break;
    case POPS: launch_main_geom<D, S, R, SRC, POPS>(h, a, nullptr, nullptr); break;
    default: launch_main_geom<D, S, R, SRC, DIAG>(h, a, nullptr, nullptr); break;
  }
}

template <int D, typename S, typename R>
int run_pass_geom(lb_handle *h, int mode, double *o0, double *o1, double *o2, int32_t *io) {
  const int in = h->cur, out = 1 - h->cur;
  Args<S, R> a = make_args<S, R>(h, in, out);
  a.f_out0 = o0; a.f_out1 = o1; a.f_out2 = o2; a.i_out = io;
  const bool step = mode == STEP || mode == STEP_OBS;
  const bool timed = h->profile && step;
  hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};
  if (timed)
    for (int k = 0; k < 4; ++k) HIP_TRY(hipEventCreate(&e[k]));
  if (h->explicit_src) launch_phase_geom<D, S, R, EXPLICIT>(h, a, e[0], e[1]);
  else launch_phase_geom<D, S, R, PULL>(h, a, e[0], e[1]);
  const int n_psi = h->n_psi_out + h->n_psi_solid;
  if (n_psi)
    hipLaunchKernelGGL((k_psi_boundary<D, R>), dim3((n_psi + 255) / 256), dim3(256), 0, h->stream, a.psi, h->nbm,
                       h->psi_out, h->n_psi_out, h->psi_solid, h->n_psi_solid, h->p.nx, h->p.ny, h->p.nz);
  if (h->explicit_src) launch_main_mode<D, S, R, EXPLICIT>(h, mode, a, e[2], e[3]);
  else launch_main_mode<D, S, R, PULL>(h, mode, a, e[2], e[3]);
  if (step && h->n_bc)
    hipLaunchKernelGGL((k_open_bc<D, S, R>), dim3((h->n_bc + 255) / 256), dim3(256), 0, h->stream, a,
                       (const BCNode *)h->bc, h->n_bc);
  HIP_TRY(hipGetLastError());
  if (timed)
    for (int k = 0; k < 4; ++k) h->ev.push_back(e[k]);
  if (step) {
    h->cur = out;
    h->explicit_src = 0;
  }
  return LB_OK;
}

int galloc(lb_handle *h, void **ptr, size_t bytes) {
  hipError_t e = hipMalloc(ptr, bytes);
  if (e != hipSuccess) return fail(LB_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
  h->bytes += (int64_t)bytes;
  return LB_OK;
}

}  // namespace

namespace lbi {

int dispatch_geom(lb_handle *h, int mode, double *o0, double *o1, double *o2, int32_t *io) {
  const bool d2 = h->D == 2;
  switch (h->store) {
    case LB_STORE_FP32:
      return d2 ? run_pass_geom<2, float, double>(h, mode, o0, o1, o2, io)
                : run_pass_geom<3, float, double>(h, mode, o0, o1, o2, io);
    case LB_STORE_FP16_DEV:
      return d2 ? run_pass_geom<2, __half, float>(h, mode, o0, o1, o2, io)
                : run_pass_geom<3, __half, float>(h, mode, o0, o1, o2, io);
    case LB_STORE_BF16_DEV:
      return d2 ? run_pass_geom<2, __hip_bfloat16, float>(h, mode, o0, o1, o2, io)
                : run_pass_geom<3, __hip_bfloat16, float>(h, mode, o0, o1, o2, io);
    default:
      return d2 ? run_pass_geom<2, float, float>(h, mode, o0, o1, o2, io)
                : run_pass_geom<3, float, float>(h, mode, o0, o1, o2, io);
  }
}

void geometry_free(lb_handle *h) {
  (void)hipFree(h->nbm);
  (void)hipFree(h->bc);
  (void)hipFree(h->psi_out);
  (void)hipFree(h->psi_solid);
  h->nbm = nullptr;
  h->bc = nullptr;
  h->psi_out = h->psi_solid = nullptr;
}

}  // namespace lbi

extern "C" {

int lb_set_geometry(lb_handle *h, const uint8_t *type, const double *rho1, const double *rho2,
                    const double *u) {
  if (!h || !type || !rho1 || !rho2) return fail(LB_EINVAL, "lb_set_geometry: NULL argument");
  if (h->geom) return fail(LB_EINVAL, "lb_set_geometry: the handle already has a geometry");
  if (h->p.walls_y) return fail(LB_EINVAL, "lb_set_geometry: walls_y must be 0 (walls are solid nodes)");
  if (h->p.nci_mode != 0) return fail(LB_EINVAL, "lb_set_geometry: needs nci_mode 0");
  if (h->p.rho_ratio != 0.0) return fail(LB_EINVAL, "lb_set_geometry: needs equal densities (rho_ratio 0)");
  const int nx = h->p.nx, ny = h->p.ny, nz = h->p.nz, Q = h->Q, D = h->D;
  const int64_t N = h->N;
  const int reach = (int)std::ceil(h->p.h_max);  // the probe wraps at most once
  if (h->p.A_nci > 0.0 && (nx <= reach || ny <= reach || (D == 3 && nz <= reach)))
    return fail(LB_EINVAL, "lb_set_geometry: every extent must exceed the probe reach h_max = %g", h->p.h_max);
  auto nbr = [&](int64_t n, int cx, int cy, int cz) -> int64_t {
    const int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((int64_t)nx * ny));
    const int xx = ((x + cx) % nx + nx) % nx, yy = ((y + cy) % ny + ny) % ny, zz = ((z + cz) % nz + nz) % nz;
    return xx + (int64_t)nx * (yy + (int64_t)ny * zz);
  };
  for (int64_t n = 0; n < N; ++n)
    if (type[n] > LB_NODE_OUTLET) return fail(LB_EINVAL, "lb_set_geometry: bad type %d at node %lld", type[n], (long long)n);
  std::vector<uint32_t> mask((size_t)N, 0u);
  std::vector<BCNode> bcs;
  std::vector<int32_t> pout, psol;
  std::vector<double> psi0((size_t)N, 0.0);
  static const int dirs[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
  for (int64_t n = 0; n < N; ++n) {
    const int t = type[n];
    uint32_t m = 0u;
    if (t != LB_NODE_FLUID) m |= GEO_NONFLUID;
    if (t == LB_NODE_SOLID) {
      m |= GEO_SOLID;
      bool any = false;
      for (int i = 0; i < Q && !any; ++i)
        if (h->c[i][0] || h->c[i][1] || h->c[i][2])
          any = type[nbr(n, h->c[i][0], h->c[i][1], h->c[i][2])] != LB_NODE_SOLID;
      if (any) psol.push_back((int32_t)n);
    } else if (t == LB_NODE_FLUID) {
      for (int i = 0; i < Q; ++i)
        if (type[nbr(n, -h->c[i][0], -h->c[i][1], -h->c[i][2])] == LB_NODE_SOLID) m |= 1u << i;
    } else {
      int64_t feeder = -1;
      uint32_t axis = 0;
      for (int k = 0; k < 6 && feeder < 0; ++k) {
        if (nz == 1 && dirs[k][2] != 0) continue;
        const int64_t f = nbr(n, dirs[k][0], dirs[k][1], dirs[k][2]);
        if (type[f] == LB_NODE_FLUID) {
          feeder = f;
          axis = (uint32_t)k;
        }
      }
      if (feeder < 0)
        return fail(LB_EINVAL, "lb_set_geometry: inlet/outlet node %lld has no fluid neighbour along an axis",
                    (long long)n);
      const double r1 = rho1[n], r2 = rho2[n];
      if (!(r1 >= 0.0 && r2 >= 0.0 && r1 + r2 > 0.0 && std::isfinite(r1 + r2)))
        return fail(LB_EINVAL, "lb_set_geometry: invalid prescribed densities at node %lld", (long long)n);
      BCNode b{};
      b.node = (int32_t)n;
      b.feeder = (int32_t)feeder;
      b.kind = t;
      b.frac1 = r1 / (r1 + r2);
      b.rho = r1 + r2;
      if (t == LB_NODE_INLET && u)
        for (int d = 0; d < D; ++d) {
          b.u[d] = u[(size_t)d * N + n];
          if (!std::isfinite(b.u[d])) return fail(LB_EINVAL, "lb_set_geometry: non-finite inlet velocity");
        }
      bcs.push_back(b);
      if (t == LB_NODE_INLET) psi0[(size_t)n] = (r1 - r2) / (r1 + r2);
      else {
        pout.push_back((int32_t)n);
        pout.push_back((int32_t)feeder);
        m |= GEO_OUTLET | axis;
      }
    }
    mask[(size_t)n] = m;
  }
  int rc = galloc(h, (void **)&h->nbm, sizeof(uint32_t) * (size_t)N);
  if (!rc && !bcs.empty()) rc = galloc(h, &h->bc, sizeof(BCNode) * bcs.size());
  if (!rc && !pout.empty()) rc = galloc(h, (void **)&h->psi_out, sizeof(int32_t) * pout.size());
  if (!rc && !psol.empty()) rc = galloc(h, (void **)&h->psi_solid, sizeof(int32_t) * psol.size());
  if (rc) {
    geometry_free(h);
    return rc;
  }
  HIP_TRY(hipMemcpy(h->nbm, mask.data(), sizeof(uint32_t) * (size_t)N, hipMemcpyHostToDevice));
  if (!bcs.empty()) HIP_TRY(hipMemcpy(h->bc, bcs.data(), sizeof(BCNode) * bcs.size(), hipMemcpyHostToDevice));
  if (!pout.empty())
    HIP_TRY(hipMemcpy(h->psi_out, pout.data(), sizeof(int32_t) * pout.size(), hipMemcpyHostToDevice));
  if (!psol.empty())
    HIP_TRY(hipMemcpy(h->psi_solid, psol.data(), sizeof(int32_t) * psol.size(), hipMemcpyHostToDevice));
  // inlet psi is constant (their composition); k_phase never writes non-fluid nodes
  if (h->r_elem == 8) {
    HIP_TRY(hipMemcpy(h->psi, psi0.data(), sizeof(double) * (size_t)N, hipMemcpyHostToDevice));
  } else {
    std::vector<float> pf(psi0.begin(), psi0.end());
    HIP_TRY(hipMemcpy(h->psi, pf.data(), sizeof(float) * (size_t)N, hipMemcpyHostToDevice));
  }
  h->n_bc = (int)bcs.size();
  h->n_psi_out = (int)(pout.size() / 2);
  h->n_psi_solid = (int)psol.size();
  h->type.assign(type, type + N);
  // graphs captured before the geometry would replay the plain kernels
  for (int k = 0; k < 2; ++k)
    if (h->graph[k]) {
      (void)hipGraphExecDestroy(h->graph[k]);
      h->graph[k] = nullptr;
    }
  h->geom = 1;
  return LB_OK;
}

}  // extern "C"
