// lb_internal.hpp -- handle layout and helpers shared by the single-lattice
// and the batched C-ABI translation units (not part of the public ABI).
#pragma once
#include "lbnci.h"
#include "lb_kernels.hpp"

#include <hip/hip_runtime.h>
#include <string>
#include <vector>

namespace lbi {

int fail(int code, const char *fmt, ...);

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) return ::lbi::fail(LB_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// Tile shapes (x extent is always one 64-wide wavefront); the defaults can be
// overridden at build time for tile sweeps.
#ifndef LBNCI_XCD_REMAP
#define LBNCI_XCD_REMAP 1
#endif
#ifndef LBNCI_BY2
#define LBNCI_BY2 4
#endif
#ifndef LBNCI_BY3
#define LBNCI_BY3 4
#endif
#ifndef LBNCI_TZ3
#define LBNCI_TZ3 1
#endif
#ifndef LBNCI_H3
#define LBNCI_H3 1
#endif
#ifndef LBNCI_TZP3
#define LBNCI_TZP3 2
#endif
#ifndef LBNCI_TZP3_16
#define LBNCI_TZP3_16 4
#endif
#ifndef LBNCI_PBY3
#define LBNCI_PBY3 8
#endif
#ifndef LBNCI_WPE_MAIN3
#define LBNCI_WPE_MAIN3 1
#endif
#ifndef LBNCI_WPE_PHASE3
#define LBNCI_WPE_PHASE3 1
#endif
constexpr int BY2 = LBNCI_BY2, TZ2 = 1, H2 = 4;  // D2Q9: halo 4, NCI probe from LDS only
constexpr int BY3 = LBNCI_BY3, TZ3 = LBNCI_TZ3, H3 = LBNCI_H3;  // D3Q27: probe beyond the halo from L2
constexpr int TZP3 = LBNCI_TZP3;                 // k_phase z-planes per block (3-D)
constexpr int TZP3_16 = LBNCI_TZP3_16;           // the same with 16-bit storage (measured faster)
constexpr int PBY3 = LBNCI_PBY3;                 // rows per single-lattice k_phase block (3-D)
// z-planes per single-lattice k_phase block for storage type S
template <typename S>
constexpr int tzp3() { return sizeof(S) == 2 ? TZP3_16 : TZP3; }

}  // namespace lbi

struct lb_handle {
  lb_params p;
  int D, Q;
  int64_t N;
  hipStream_t stream;
  int device = 0;    // HIP device current at lb_create
  int store;         // lb_storage
  size_t s_elem;     // bytes per stored s value
  size_t r_elem;     // bytes per compute-type value (a, psi)
  // state, two copies
  void *s[2] = {nullptr, nullptr};
  float *s0[2] = {nullptr, nullptr};
  void *a[2] = {nullptr, nullptr};
  float *B[2] = {nullptr, nullptr};
  void *psi = nullptr;
  void *r1 = nullptr;
  double *xt = nullptr, *xc = nullptr;  // explicit first-step state
  double *partials = nullptr;
  int nparts = 0;
  lbk::ObsDev *obs = nullptr;
  int32_t *hflags = nullptr;  // pinned host copy of obs->flags after each recorded step
  int cur = 0;
  int initialised = 0;
  int explicit_src = 0;
  int64_t t = 0;
  int xcd_remap = LBNCI_XCD_REMAP;
  int64_t bytes = 0;
  // replay of GRAPH_STEPS plain steps from a hipGraph, one per starting copy
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  int graphs_ok = 1;
  // node-type geometry (lb_set_geometry): mask words, open-boundary and
  // derived-psi lists on the device, the node types on the host
  int geom = 0;
  uint32_t *nbm = nullptr;
  void *bc = nullptr;           // lbi::BCNode[n_bc]
  int32_t *psi_out = nullptr;   // outlet node, feeder pairs
  int32_t *psi_solid = nullptr; // solid nodes with a non-solid neighbour
  int n_bc = 0, n_psi_out = 0, n_psi_solid = 0;
  std::vector<uint8_t> type;
  // droplet analysis and vorticity: one device arena, allocated on first use
  void *ana = nullptr;
  size_t ana_bytes = 0;
  hipEvent_t ana_ev[2] = {nullptr, nullptr};
  double ana_ms[2] = {0.0, 0.0};  // last lb_droplets, lb_vorticity device time
  // per-kernel event timing
  int profile = 0;
  std::vector<hipEvent_t> ev;  // quadruples: phase start/stop, main start/stop
  // lattice tables (host)
  int c[27][3];
  double w[27];
};

namespace lbi {
// One pass of the single-lattice kernels in the given mode (lbk::Mode);
// STEP modes advance the handle's state copy.
int dispatch(lb_handle *h, int mode, double *o0 = nullptr, double *o1 = nullptr,
             double *o2 = nullptr, int32_t *io = nullptr);
int validate(const lb_params *p);
// Releases the droplet-analysis arena and events of a handle.
void analysis_free(lb_handle *h);
// Grid sizes of the single-lattice kernels.
int blocks_main(const lb_handle *h);
int blocks_phase(const lb_handle *h);
// Releases the geometry buffers of a handle.
void geometry_free(lb_handle *h);
// One pass of the geometry kernels (handles with lb_set_geometry).
int dispatch_geom(lb_handle *h, int mode, double *o0, double *o1, double *o2, int32_t *io);
// Open-boundary node: inlet (velocity, composition prescribed) or outlet
// (density prescribed), refreshed from its feeder after every collision.
struct BCNode {
  int32_t node, feeder, kind, pad;  // kind: LB_NODE_INLET or LB_NODE_OUTLET
  double frac1;                     // inlet: rho1/rho; outlet: unused
  double rho;                       // outlet: density; inlet: unused
  double u[3];                      // inlet velocity
};
int reduce_obs(lb_handle *h, int record);
// Kernel arguments of a handle reading state copy `in` and writing `out`.
template <typename S, typename R>
inline lbk::Args<S, R> make_args(lb_handle *h, int in, int out) {
  lbk::Args<S, R> a{};
  const lb_params &p = h->p;
  a.nx = p.nx; a.ny = p.ny; a.nz = p.nz; a.walls = p.walls_y;
  a.N = (uint32_t)h->N;
  a.tau_inv = (R)(1.0 / p.tau);
  a.two_tau = p.tau2 > 0 ? 1 : 0;
  a.tau2_inv = (R)(p.tau2 > 0 ? 1.0 / p.tau2 : 1.0 / p.tau);
  a.half_As = (R)(0.5 * p.A_s);
  a.beta = (R)p.beta;
  a.A = (R)p.A_nci;
  a.h_min = (R)p.h_min;
  a.h_max = (R)p.h_max;
  for (int d = 0; d < 3; ++d) a.F[d] = (R)p.force[d];
  a.smax = (int)std::floor(p.h_max);
  a.smaxc = (int)std::ceil(p.h_max);
  a.dr_on = p.rho_ratio > 0 ? 1 : 0;
  a.dr_gamma = (R)(p.rho_ratio > 0 ? p.rho_ratio : 1.0);
  if (p.rho_ratio > 0) {
    const double w0 = h->D == 2 ? 4.0 / 9.0 : 8.0 / 27.0;
    const double a2 = 1.0 - p.rho_ratio * (1.0 - p.alpha1);
    a.dr_g1 = (R)((1.0 - p.alpha1) / (1.0 - w0) - 1.0);
    a.dr_g2 = (R)((1.0 - a2) / (1.0 - w0) - 1.0);
  } else {
    a.dr_g1 = a.dr_g2 = (R)0;
  }
  a.in = lbk::State<S, R>{(S *)h->s[in], h->s0[in], (R *)h->a[in], h->B[in]};
  a.out = lbk::State<S, R>{(S *)h->s[out], h->s0[out], (R *)h->a[out], h->B[out]};
  a.xt = h->xt;
  a.xc = h->xc;
  a.psi = (R *)h->psi;
  a.r1 = (R *)h->r1;
  a.partials = h->partials;
  a.xcd_remap = h->xcd_remap;
  a.nbm = h->nbm;
  return a;
}
}  // namespace lbi
