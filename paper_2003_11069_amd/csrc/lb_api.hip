// lb_api.hip -- C ABI of the colour-gradient + NCI lattice Boltzmann library
// (declarations and argument contracts in include/lbnci.h).
#include "lb_internal.hpp"

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

using namespace lbk;
using namespace lbi;

namespace lbi {
thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}
}  // namespace lbi

namespace lbi {

template <int D>
void fill_tables(lb_handle *h) {
  using L = Lat<D>;
  for (int i = 0; i < L::Q; ++i) {
    h->c[i][0] = L::cx(i);
    h->c[i][1] = L::cy(i);
    h->c[i][2] = L::cz(i);
    h->w[i] = L::w(i);
  }
}

int blocks_main(const lb_handle *h) {
  const lb_params &p = h->p;
  if (h->D == 2) return ((p.nx + 63) / 64) * ((p.ny + BY2 - 1) / BY2);
  return ((p.nx + 63) / 64) * ((p.ny + BY3 - 1) / BY3) * ((p.nz + TZ3 - 1) / TZ3);
}

int blocks_phase(const lb_handle *h) {
  const lb_params &p = h->p;
  const int tz = h->s_elem == 2 ? TZP3_16 : TZP3;
  const int gz = h->D == 3 ? (p.nz + tz - 1) / tz : 1;
  const int by = h->D == 3 ? PBY3 : 4;
  return ((p.nx + 63) / 64) * ((p.ny + by - 1) / by) * gz;
}


// Kernel launches; with events (profiling) the start/stop events travel in the
// kernel's own dispatch packet, so they time the kernel alone.
template <class K, class A>
void launch(K kernel, dim3 grid, dim3 block, hipStream_t st, hipEvent_t e0, hipEvent_t e1, const A &a) {
  if (e0) hipExtLaunchKernelGGL(kernel, grid, block, 0, st, e0, e1, 0, a);
  else hipLaunchKernelGGL(kernel, grid, block, 0, st, a);
}

template <int D, typename S, typename R, int SRC, int MODE, int NCI>
void launch_main_nci(lb_handle *h, const Args<S, R> &a, hipEvent_t e0, hipEvent_t e1) {
  const int nb = blocks_main(h);
  if constexpr (D == 2)
    launch(k_main<D, S, R, SRC, MODE, BY2, TZ2, H2, 1, NCI>, dim3(nb), dim3(64, BY2), h->stream, e0, e1, a);
  else
    launch(k_main<D, S, R, SRC, MODE, BY3, TZ3, H3, LBNCI_WPE_MAIN3, NCI>, dim3(nb), dim3(64, BY3),
           h->stream, e0, e1, a);
}

template <int D, typename S, typename R, int SRC, int MODE>
void launch_main(lb_handle *h, const Args<S, R> &a, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
  if (h->p.nci_mode == 1) launch_main_nci<D, S, R, SRC, MODE, 1>(h, a, e0, e1);
  else launch_main_nci<D, S, R, SRC, MODE, 0>(h, a, e0, e1);
}

template <int D, typename S, typename R, int SRC>
void launch_phase(lb_handle *h, const Args<S, R> &a, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
  launch(k_phase<D, S, R, SRC, (D == 3 ? tzp3<S>() : 1), (D == 3 ? LBNCI_WPE_PHASE3 : 1), 0, (D == 3 ? PBY3 : 4)>,
         dim3(blocks_phase(h)), dim3(64, D == 3 ? PBY3 : 4), h->stream, e0, e1, a);
}

// One pass over the lattice in the given mode; STEP modes write the other copy.
template <int D, typename S, typename R>
int run_pass(lb_handle *h, int mode, double *o0, double *o1, double *o2, int32_t *io) {
  const int in = h->cur, out = 1 - h->cur;
  Args<S, R> a = make_args<S, R>(h, in, out);
  a.f_out0 = o0; a.f_out1 = o1; a.f_out2 = o2; a.i_out = io;
  const bool timed = h->profile && (mode == STEP || mode == STEP_OBS);
  hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};
  if (timed)
    for (int k = 0; k < 4; ++k) HIP_TRY(hipEventCreate(&e[k]));
  if (h->explicit_src) {
    launch_phase<D, S, R, EXPLICIT>(h, a, e[0], e[1]);
    switch (mode) {
      case STEP: launch_main<D, S, R, EXPLICIT, STEP>(h, a, e[2], e[3]); break;
      case STEP_OBS: launch_main<D, S, R, EXPLICIT, STEP_OBS>(h, a, e[2], e[3]); break;
      case OBSERVE: launch_main<D, S, R, EXPLICIT, OBSERVE>(h, a); break;
      case FIELDS: launch_main<D, S, R, EXPLICIT, FIELDS>(h, a); break;
      case POPS: launch_main<D, S, R, EXPLICIT, POPS>(h, a); break;
      default: launch_main<D, S, R, EXPLICIT, DIAG>(h, a); break;
    }
  } else {
    launch_phase<D, S, R, PULL>(h, a, e[0], e[1]);
    switch (mode) {
      case STEP: launch_main<D, S, R, PULL, STEP>(h, a, e[2], e[3]); break;
      case STEP_OBS: launch_main<D, S, R, PULL, STEP_OBS>(h, a, e[2], e[3]); break;
      case OBSERVE: launch_main<D, S, R, PULL, OBSERVE>(h, a); break;
      case FIELDS: launch_main<D, S, R, PULL, FIELDS>(h, a); break;
      case POPS: launch_main<D, S, R, PULL, POPS>(h, a); break;
      default: launch_main<D, S, R, PULL, DIAG>(h, a); break;
    }
  }
  HIP_TRY(hipGetLastError());
  if (timed)
    for (int k = 0; k < 4; ++k) h->ev.push_back(e[k]);
  if (mode == STEP || mode == STEP_OBS) {
    h->cur = out;
    h->explicit_src = 0;
  }
  return LB_OK;
}

int dispatch(lb_handle *h, int mode, double *o0, double *o1, double *o2, int32_t *io) {
  if (h->geom) return dispatch_geom(h, mode, o0, o1, o2, io);
  const bool d2 = h->D == 2;
  switch (h->store) {
    case LB_STORE_FP32:
      return d2 ? run_pass<2, float, double>(h, mode, o0, o1, o2, io)
                : run_pass<3, float, double>(h, mode, o0, o1, o2, io);
    case LB_STORE_FP16_DEV:
      return d2 ? run_pass<2, __half, float>(h, mode, o0, o1, o2, io)
                : run_pass<3, __half, float>(h, mode, o0, o1, o2, io);
    case LB_STORE_BF16_DEV:
      return d2 ? run_pass<2, __hip_bfloat16, float>(h, mode, o0, o1, o2, io)
                : run_pass<3, __hip_bfloat16, float>(h, mode, o0, o1, o2, io);
    default:
      return d2 ? run_pass<2, float, float>(h, mode, o0, o1, o2, io)
                : run_pass<3, float, float>(h, mode, o0, o1, o2, io);
  }
}

int reduce_obs(lb_handle *h, int record) {
  hipLaunchKernelGGL(k_obs_reduce, dim3(1), dim3(256), 0, h->stream, h->partials, h->nparts,
                     h->obs, 1.0 / h->p.nx, h->p.conv_window, h->p.conv_m, h->p.conv_eps,
                     h->p.mass_tol, record);
  HIP_TRY(hipGetLastError());
  // the flags of a recorded step travel to pinned host memory behind it, so
  // lb_step can report them without synchronising
  if (record && h->hflags)
    HIP_TRY(hipMemcpyAsync(h->hflags, &h->obs->flags, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
  return LB_OK;
}

int validate(const lb_params *p) {
  if (!p) return fail(LB_EINVAL, "params is NULL");
  if (p->lattice != LB_D2Q9 && p->lattice != LB_D3Q27) return fail(LB_EINVAL, "unknown lattice %d", p->lattice);
  if (p->nx <= 0 || p->ny <= 0 || p->nz <= 0) return fail(LB_EINVAL, "sizes must be positive");
  if (p->lattice == LB_D2Q9 && p->nz != 1) return fail(LB_EINVAL, "D2Q9 needs nz == 1");
  if (p->walls_y && p->ny < 3) return fail(LB_EINVAL, "walls need ny >= 3");
  if ((int64_t)p->nx * p->ny * p->nz > (int64_t)1 << 29)
    return fail(LB_EINVAL, "lattice too large (at most 2^29 nodes)");
  if (!(p->tau > 0.5)) return fail(LB_EINVAL, "tau must exceed 1/2");
  if (!(p->tau2 == 0.0 || p->tau2 > 0.5)) return fail(LB_EINVAL, "tau2 must be 0 or exceed 1/2");
  if (p->nci_mode != 0 && p->nci_mode != 1) return fail(LB_EINVAL, "nci_mode must be 0 or 1");
  if (p->rho_ratio != 0.0) {
    const double a2 = 1.0 - p->rho_ratio * (1.0 - p->alpha1);
    if (!(p->rho_ratio > 0.0 && p->alpha1 > 0.0 && p->alpha1 < 1.0 && a2 > 0.0 && a2 < 1.0))
      return fail(LB_EINVAL, "density ratio: need rho_ratio > 0 and 0 < alpha1, 1 - rho_ratio (1 - alpha1) < 1");
  }
  if (!(p->beta >= 0.0 && p->beta <= 1.0)) return fail(LB_EINVAL, "beta must lie in [0,1]");
  if (!(p->A_s >= 0.0)) return fail(LB_EINVAL, "A_s must be >= 0");
  if (!(p->A_nci >= 0.0)) return fail(LB_EINVAL, "A_nci must be >= 0");
  if (!(p->h_min > 0.0 && p->h_min <= p->h_max && p->h_max <= 4.0))
    return fail(LB_EINVAL, "need 0 < h_min <= h_max <= 4");
  for (int d = 0; d < 3; ++d)
    if (!std::isfinite(p->force[d])) return fail(LB_EINVAL, "force must be finite");
  if (p->storage < LB_STORE_FP32 || p->storage > LB_STORE_FP32_F32)
    return fail(LB_EINVAL, "unknown storage %d", p->storage);
  if (p->obs_every < 0 || p->conv_window < 0 || p->conv_m < 0 || !(p->conv_eps >= 0))
    return fail(LB_EINVAL, "bad observable/convergence settings");
  if (!(p->mass_tol >= 0.0) || !std::isfinite(p->mass_tol)) return fail(LB_EINVAL, "mass_tol must be finite and >= 0");
  return LB_OK;
}

int alloc(lb_handle *h, void **ptr, size_t bytes) {
  hipError_t e = hipMalloc(ptr, bytes);
  if (e != hipSuccess) return fail(LB_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
  h->bytes += (int64_t)bytes;
  e = hipMemsetAsync(*ptr, 0, bytes, h->stream);
  if (e != hipSuccess) return fail(LB_EDEVICE, "hipMemsetAsync: %s", hipGetErrorString(e));
  return LB_OK;
}

bool is_wall(const lb_handle *h, int64_t n) {
  if (h->geom) return h->type[(size_t)n] != LB_NODE_FLUID;
  if (!h->p.walls_y) return false;
  const int y = (int)((n / h->p.nx) % h->p.ny);
  return y == 0 || y == h->p.ny - 1;
}

// Uploads an explicit two-population state given on the host in FP64.
int upload_explicit(lb_handle *h, const std::vector<double> &xt, const std::vector<double> &xc) {
  const size_t bytes = sizeof(double) * (size_t)h->Q * (size_t)h->N;
  if (!h->xt) {
    int rc = alloc(h, (void **)&h->xt, bytes);
    if (rc) return rc;
    rc = alloc(h, (void **)&h->xc, bytes);
    if (rc) return rc;
  }
  HIP_TRY(hipMemcpyAsync(h->xt, xt.data(), bytes, hipMemcpyHostToDevice, h->stream));
  HIP_TRY(hipMemcpyAsync(h->xc, xc.data(), bytes, hipMemcpyHostToDevice, h->stream));
  HIP_TRY(hipMemsetAsync(h->obs, 0, sizeof(ObsDev), h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  if (h->hflags) *h->hflags = 0;
  h->explicit_src = 1;
  h->initialised = 1;
  h->t = 0;
  return LB_OK;
}

}  // namespace

extern "C" {

int lb_lattice_tables(int32_t lattice, int32_t *c, double *w) {
  lb_handle tmp;
  if (lattice == LB_D2Q9) fill_tables<2>(&tmp);
  else if (lattice == LB_D3Q27) fill_tables<3>(&tmp);
  else return fail(LB_EINVAL, "unknown lattice %d", lattice);
  const int Q = lattice == LB_D2Q9 ? 9 : 27;
  for (int i = 0; i < Q; ++i) {
    if (c)
      for (int d = 0; d < 3; ++d) c[3 * i + d] = tmp.c[i][d];
    if (w) w[i] = tmp.w[i];
  }
  return Q;
}

int lb_create(const lb_params *p, void *hip_stream, lb_handle **out) {
  if (!out) return fail(LB_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate(p);
  if (rc) return rc;
  lb_handle *h = new (std::nothrow) lb_handle();
  if (!h) return fail(LB_ENOMEM, "host allocation failed");
  h->p = *p;
  h->D = p->lattice == LB_D2Q9 ? 2 : 3;
  h->Q = h->D == 2 ? 9 : 27;
  if (h->D == 2) fill_tables<2>(h); else fill_tables<3>(h);
  h->N = (int64_t)p->nx * p->ny * p->nz;
  h->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return fail(LB_EDEVICE, "hipGetDevice failed");
  }
  h->store = p->storage;
  h->s_elem = (p->storage == LB_STORE_FP16_DEV || p->storage == LB_STORE_BF16_DEV) ? 2 : 4;
  h->r_elem = (p->storage == LB_STORE_FP32) ? 8 : 4;
  const size_t N = (size_t)h->N;
  for (int k = 0; k < 2 && !rc; ++k) {
    rc = alloc(h, &h->s[k], h->s_elem * h->Q * N);
    if (!rc && h->s_elem == 2) rc = alloc(h, (void **)&h->s0[k], sizeof(float) * N);
    if (!rc) rc = alloc(h, &h->a[k], h->r_elem * N);
    if (!rc) rc = alloc(h, (void **)&h->B[k], sizeof(float) * h->D * N);
  }
  if (!rc) rc = alloc(h, &h->psi, h->r_elem * N);
  if (!rc) rc = alloc(h, &h->r1, h->r_elem * N);
  h->nparts = blocks_main(h);
  if (!rc) rc = alloc(h, (void **)&h->partials, sizeof(double) * 8 * (size_t)h->nparts);
  if (!rc) rc = alloc(h, (void **)&h->obs, sizeof(ObsDev));
  if (!rc) {
    hipError_t e = hipHostMalloc((void **)&h->hflags, sizeof(int32_t), hipHostMallocDefault);
    if (e != hipSuccess) rc = fail(LB_ENOMEM, "hipHostMalloc: %s", hipGetErrorString(e));
    else *h->hflags = 0;
  }
  if (!rc) {
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) rc = fail(LB_EDEVICE, "hipStreamSynchronize: %s", hipGetErrorString(e));
  }
  if (rc) {
    lb_destroy(h);
    return rc;
  }
  *out = h;
  return LB_OK;
}

void lb_destroy(lb_handle *h) {
  if (!h) return;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  else (void)hipDeviceSynchronize();
  for (int k = 0; k < 2; ++k) {
    (void)hipFree(h->s[k]);
    (void)hipFree(h->s0[k]);
    (void)hipFree(h->a[k]);
    (void)hipFree(h->B[k]);
  }
  (void)hipFree(h->psi);
  (void)hipFree(h->r1);
  (void)hipFree(h->xt);
  (void)hipFree(h->xc);
  (void)hipFree(h->partials);
  (void)hipFree(h->obs);
  if (h->hflags) (void)hipHostFree(h->hflags);
  analysis_free(h);
  geometry_free(h);
  for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
  for (int k = 0; k < 2; ++k)
    if (h->graph[k]) (void)hipGraphExecDestroy(h->graph[k]);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  delete h;
}

int lb_init_fields(lb_handle *h, const double *rho1, const double *rho2, const double *u) {
  if (!h || !rho1 || !rho2) return fail(LB_EINVAL, "NULL argument");
  const int Q = h->Q, D = h->D;
  const int64_t N = h->N;
  for (int64_t n = 0; n < N; ++n) {
    if (is_wall(h, n)) continue;
    if (!(rho1[n] >= 0.0) || !(rho2[n] >= 0.0) || !(rho1[n] + rho2[n] > 0.0) ||
        !std::isfinite(rho1[n] + rho2[n]))
      return fail(LB_EINVAL, "invalid densities at node %lld", (long long)n);
    if (u)
      for (int d = 0; d < D; ++d)
        if (!std::isfinite(u[d * N + n])) return fail(LB_EINVAL, "non-finite velocity at node %lld", (long long)n);
  }
  std::vector<double> xt((size_t)Q * N, 0.0), xc((size_t)Q * N, 0.0);
  for (int64_t n = 0; n < N; ++n) {
    if (is_wall(h, n)) continue;
    double v[3] = {0, 0, 0};
    if (u)
      for (int d = 0; d < D; ++d) v[d] = u[d * N + n];
    const double rho = rho1[n] + rho2[n];
    const double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    for (int i = 0; i < Q; ++i) {
      const double cu = h->c[i][0] * v[0] + h->c[i][1] * v[1] + h->c[i][2] * v[2];
      const double P = 3.0 * cu + 4.5 * cu * cu - 1.5 * vv;  // E_i = w_i rho (1 + P)
      // total deviation f_i/w_i - 1 and component-1 share f1_i/w_i
      if (h->p.rho_ratio > 0) {
        // density-ratio variant: E_i^k = rho_k (phi_i^k + w_i P), phi_i^k/w_i = g_i^k
        const bool rest = !h->c[i][0] && !h->c[i][1] && !h->c[i][2];
        const double w0 = D == 2 ? 4.0 / 9.0 : 8.0 / 27.0;
        const double a1 = h->p.alpha1, a2 = 1.0 - h->p.rho_ratio * (1.0 - a1);
        const double g1 = rest ? a1 / w0 : (1.0 - a1) / (1.0 - w0);
        const double g2 = rest ? a2 / w0 : (1.0 - a2) / (1.0 - w0);
        xt[(size_t)i * N + n] = (rho1[n] * g1 + rho2[n] * g2 - 1.0) + rho * P;
        xc[(size_t)i * N + n] = rho1[n] * (g1 + P);
      } else {
        xt[(size_t)i * N + n] = (rho - 1.0) + rho * P;
        xc[(size_t)i * N + n] = rho1[n] * (1.0 + P);
      }
    }
  }
  return upload_explicit(h, xt, xc);
}

int lb_set_populations(lb_handle *h, const double *f1, const double *f2) {
  if (!h || !f1 || !f2) return fail(LB_EINVAL, "NULL argument");
  const int Q = h->Q;
  const int64_t N = h->N;
  std::vector<double> xt((size_t)Q * N, 0.0), xc((size_t)Q * N, 0.0);
  for (int64_t n = 0; n < N; ++n) {
    if (is_wall(h, n)) continue;
    double r1 = 0, r2 = 0;
    for (int i = 0; i < Q; ++i) {
      const double a = f1[(size_t)i * N + n], b = f2[(size_t)i * N + n];
      if (!std::isfinite(a) || !std::isfinite(b))
        return fail(LB_EINVAL, "non-finite population at node %lld", (long long)n);
      r1 += a;
      r2 += b;
      xt[(size_t)i * N + n] = (a + b) / h->w[i] - 1.0;
      xc[(size_t)i * N + n] = a / h->w[i];
    }
    if (!(r1 >= 0.0) || !(r2 >= 0.0) || !(r1 + r2 > 0.0))
      return fail(LB_EINVAL, "invalid densities at node %lld", (long long)n);
  }
  return upload_explicit(h, xt, xc);
}

// Plain steps replayed from a graph: GRAPH_STEPS (even) kernel pairs captured
// once per starting copy on a private stream, launched on the handle's stream.
static constexpr int GRAPH_STEPS = 16;

// Captures and instantiates the graph of GRAPH_STEPS plain (pulling) steps
// starting from state copy c0, without running it.
static int graph_capture(lb_handle *h, int c0) {
  if (h->graph[c0]) return LB_OK;
  if (!h->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
  hipStream_t user = h->stream;
  const int cur = h->cur, xs = h->explicit_src;
  const int prof = h->profile;
  h->stream = h->cap_stream;
  h->cur = c0;
  h->explicit_src = 0;
  h->profile = 0;  // no timing events inside a graph
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal);
  int rc = LB_OK;
  for (int k = 0; k < GRAPH_STEPS && e == hipSuccess && rc == LB_OK; ++k) rc = dispatch(h, STEP);
  hipError_t e2 = hipStreamEndCapture(h->cap_stream, &g);
  h->stream = user;
  h->cur = cur;
  h->explicit_src = xs;
  h->profile = prof;
  if (e == hipSuccess) e = e2;
  if (e == hipSuccess && rc == LB_OK) e = hipGraphInstantiate(&h->graph[c0], g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (e != hipSuccess || rc != LB_OK) {
    (void)hipGetLastError();
    h->graph[c0] = nullptr;
    return fail(LB_EDEVICE, "graph capture: %s", hipGetErrorString(e));
  }
  return LB_OK;
}

static int graph_steps(lb_handle *h) {
  int rc = graph_capture(h, h->cur);
  if (rc) return rc;
  HIP_TRY(hipGraphLaunch(h->graph[h->cur], h->stream));
  return LB_OK;
}

int lb_step(lb_handle *h, int64_t n) {
  if (!h) return fail(LB_EINVAL, "NULL handle");
  if (n < 0) return fail(LB_EINVAL, "negative step count");
  if (!h->initialised) return fail(LB_ESTATE, "lb_step before initialisation");
  if (const int32_t fl = h->hflags ? *(volatile int32_t *)h->hflags : 0)
    return fail(LB_ENUMERIC, "a recorded step flagged %s", (fl & 1) ? "a NaN/Inf" : "a mass drift beyond mass_tol");
  const int64_t oe = h->p.obs_every;
  for (int64_t k = 0; k < n;) {
    // a window of plain steps (no recording step inside) goes through a graph
    const bool plain_window =
        oe <= 0 || (h->t % oe != 0 && (h->t / oe) == ((h->t + GRAPH_STEPS - 1) / oe));
    if (h->graphs_ok && !h->profile && !h->explicit_src && n - k >= GRAPH_STEPS && plain_window) {
      if (graph_steps(h) == LB_OK) {
        h->t += GRAPH_STEPS;
        k += GRAPH_STEPS;
        continue;
      }
      h->graphs_ok = 0;  // fall back to plain launches from now on
    }
    const bool rec = oe > 0 && (h->t % oe) == 0;
    const bool first = h->explicit_src != 0;
    int rc = dispatch(h, rec ? STEP_OBS : STEP);
    if (rc) return rc;
    if (first) {
      // the explicit initial state (2 Q FP64 values per node) has been
      // consumed: release it once that step is done (the next lb_init_fields
      // or lb_set_populations allocates it again)
      HIP_TRY(hipStreamSynchronize(h->stream));
      const int64_t bytes = (int64_t)(2 * sizeof(double) * (size_t)h->Q * (size_t)h->N);
      HIP_TRY(hipFree(h->xt));
      HIP_TRY(hipFree(h->xc));
      h->xt = h->xc = nullptr;
      h->bytes -= bytes;
    }
    if (rec) {
      rc = reduce_obs(h, 1);
      if (rc) return rc;
    }
    h->t += 1;
    k += 1;
  }
  return LB_OK;
}

int lb_step_timed(lb_handle *h, int64_t n, double *ms) {
  if (!h || !ms) return fail(LB_EINVAL, "NULL argument");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  hipError_t e = hipEventCreate(&e1);
  int rc = e == hipSuccess ? LB_OK : fail(LB_EDEVICE, "hipEventCreate: %s", hipGetErrorString(e));
  if (!rc) {
    e = hipEventRecord(e0, h->stream);
    if (e != hipSuccess) rc = fail(LB_EDEVICE, "hipEventRecord: %s", hipGetErrorString(e));
  }
  if (!rc) rc = lb_step(h, n);
  if (!rc) {
    e = hipEventRecord(e1, h->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float f = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&f, e0, e1);
    if (e != hipSuccess) rc = fail(LB_EDEVICE, "step timing: %s", hipGetErrorString(e));
    *ms = f;
  }
  (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return rc;
}

int lb_prepare(lb_handle *h) {
  if (!h) return fail(LB_EINVAL, "NULL handle");
  if (!h->graphs_ok) return LB_OK;
  for (int c = 0; c < 2; ++c) {
    const int rc = graph_capture(h, c);
    if (rc) {
      h->graphs_ok = 0;
      return rc;
    }
  }
  return LB_OK;
}

int lb_graphs(const lb_handle *h) { return h ? h->graphs_ok : -1; }

int lb_observables(lb_handle *h, lb_obs *out) {
  if (!h || !out) return fail(LB_EINVAL, "NULL argument");
  if (!h->initialised) return fail(LB_ESTATE, "lb_observables before initialisation");
  int rc = dispatch(h, OBSERVE);
  if (rc) return rc;
  rc = reduce_obs(h, 0);
  if (rc) return rc;
  ObsDev o;
  HIP_TRY(hipMemcpyAsync(&o, h->obs, sizeof o, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  out->step = h->t;
  out->mass[0] = o.v[0];
  out->mass[1] = o.v[1];
  for (int d = 0; d < 3; ++d) out->mom[d] = o.v[2 + d];
  out->Q = o.v[5];
  out->Q_d = o.v[6];
  out->umax = o.v[7];
  out->Q_window = o.n_windows > 0 ? o.win_last : 0.0;
  out->converged = o.converged;
  out->flags = o.flags;
  if (o.flags & 1) return fail(LB_ENUMERIC, "NaN/Inf in the observables");
  if (o.flags & 2) return fail(LB_ENUMERIC, "component mass drifted beyond mass_tol");
  return LB_OK;
}

static int fetch(lb_handle *h, int mode, size_t n0, size_t n1, size_t n2, size_t ni, double *h0,
                 double *h1, double *h2, int32_t *hi) {
  double *d0 = nullptr, *d1 = nullptr, *d2 = nullptr;
  int32_t *di = nullptr;
  int rc = LB_OK;
  auto get = [&](void **p, size_t bytes) {
    if (!bytes || rc) return;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) { rc = fail(LB_ENOMEM, "hipMalloc: %s", hipGetErrorString(e)); return; }
    e = hipMemsetAsync(*p, 0, bytes, h->stream);
    if (e != hipSuccess) rc = fail(LB_EDEVICE, "hipMemsetAsync: %s", hipGetErrorString(e));
  };
  get((void **)&d0, n0 * sizeof(double));
  get((void **)&d1, n1 * sizeof(double));
  get((void **)&d2, n2 * sizeof(double));
  get((void **)&di, ni * sizeof(int32_t));
  if (!rc) rc = dispatch(h, mode, d0, d1, d2, di);
  auto put = [&](void *dst, void *src, size_t bytes) {
    if (rc || !dst || !src) return;
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, h->stream);
    if (e != hipSuccess) rc = fail(LB_EDEVICE, "hipMemcpyAsync: %s", hipGetErrorString(e));
  };
  put(h0, d0, n0 * sizeof(double));
  put(h1, d1, n1 * sizeof(double));
  put(h2, d2, n2 * sizeof(double));
  put(hi, di, ni * sizeof(int32_t));
  if (!rc) {
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) rc = fail(LB_EDEVICE, "hipStreamSynchronize: %s", hipGetErrorString(e));
  }
  (void)hipFree(d0);
  (void)hipFree(d1);
  (void)hipFree(d2);
  (void)hipFree(di);
  return rc;
}

int lb_get_fields(lb_handle *h, double *rho1, double *rho2, double *u) {
  if (!h || !rho1 || !rho2 || !u) return fail(LB_EINVAL, "NULL argument");
  if (!h->initialised) return fail(LB_ESTATE, "lb_get_fields before initialisation");
  const size_t N = (size_t)h->N;
  return fetch(h, FIELDS, N, N, (size_t)h->D * N, 0, rho1, rho2, u, nullptr);
}

int lb_get_populations(lb_handle *h, double *f1, double *f2) {
  if (!h || !f1 || !f2) return fail(LB_EINVAL, "NULL argument");
  if (!h->initialised) return fail(LB_ESTATE, "lb_get_populations before initialisation");
  const size_t QN = (size_t)h->Q * (size_t)h->N;
  return fetch(h, POPS, QN, QN, 0, 0, f1, f2, nullptr, nullptr);
}

int lb_get_nci(lb_handle *h, double *psi, double *frep, int32_t *hit) {
  if (!h) return fail(LB_EINVAL, "NULL handle");
  if (!h->initialised) return fail(LB_ESTATE, "lb_get_nci before initialisation");
  const size_t N = (size_t)h->N;
  std::vector<double> ps(N), fr((size_t)h->D * N);
  std::vector<int32_t> ht(N);
  int rc = fetch(h, DIAG, N, (size_t)h->D * N, 0, N, ps.data(), fr.data(), nullptr, ht.data());
  if (rc) return rc;
  if (h->p.walls_y) {  // wall rows carry the adjacent fluid row's psi
    const int nx = h->p.nx, ny = h->p.ny;
    for (int z = 0; z < h->p.nz; ++z)
      for (int x = 0; x < nx; ++x) {
        const size_t b = x + (size_t)nx * ((size_t)ny * z);
        ps[b] = ps[b + nx];
        const size_t t = x + (size_t)nx * ((ny - 1) + (size_t)ny * z);
        ps[t] = ps[t - nx];
      }
  }
  if (psi) std::memcpy(psi, ps.data(), N * sizeof(double));
  if (frep) std::memcpy(frep, fr.data(), fr.size() * sizeof(double));
  if (hit) std::memcpy(hit, ht.data(), N * sizeof(int32_t));
  return LB_OK;
}

int lb_profile(lb_handle *h, int enable) {
  if (!h) return fail(LB_EINVAL, "NULL handle");
  h->profile = enable ? 1 : 0;
  return LB_OK;
}

int lb_kernel_times(lb_handle *h, double *ms_phase, double *ms_main, int64_t *launches) {
  if (!h) return fail(LB_EINVAL, "NULL handle");
  HIP_TRY(hipStreamSynchronize(h->stream));
  double a = 0, b = 0;
  int64_t n = 0;
  for (size_t k = 0; k + 3 < h->ev.size(); k += 4) {
    float t0 = 0, t1 = 0;
    HIP_TRY(hipEventElapsedTime(&t0, h->ev[k], h->ev[k + 1]));
    HIP_TRY(hipEventElapsedTime(&t1, h->ev[k + 2], h->ev[k + 3]));
    a += t0;
    b += t1;
    ++n;
  }
  for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
  h->ev.clear();
  if (ms_phase) *ms_phase = a;
  if (ms_main) *ms_main = b;
  if (launches) *launches = n;
  return LB_OK;
}

int lb_stream_create(void **stream) {
  if (!stream) return fail(LB_EINVAL, "lb_stream_create: NULL argument");
  hipStream_t st = nullptr;
  HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  *stream = (void *)st;
  return LB_OK;
}

int lb_stream_destroy(void *stream) {
  if (!stream) return fail(LB_EINVAL, "lb_stream_destroy: NULL stream");
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  HIP_TRY(hipStreamDestroy((hipStream_t)stream));
  return LB_OK;
}

int lb_copy_probe(int64_t bytes, int iters, void *hip_stream, double *ms, double *gbps) {
  if (bytes < 16 || iters < 1) return fail(LB_EINVAL, "bad copy-probe size");
  hipStream_t st = (hipStream_t)hip_stream;
  const int64_t n4 = bytes / 16;
  float4 *src = nullptr, *dst = nullptr;
  if (hipMalloc(&src, n4 * 16) != hipSuccess) return fail(LB_ENOMEM, "copy probe allocation");
  if (hipMalloc(&dst, n4 * 16) != hipSuccess) {
    (void)hipFree(src);
    return fail(LB_ENOMEM, "copy probe allocation");
  }
  int rc = LB_OK;
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  const int threads = 256;
  const int64_t nblk = (n4 + threads - 1) / threads;
  if (nblk > INT32_MAX) {
    (void)hipFree(src);
    (void)hipFree(dst);
    return fail(LB_EINVAL, "copy probe too large");
  }
  const int blocks = (int)nblk;
  hipLaunchKernelGGL(k_copy_probe, dim3(blocks), dim3(threads), 0, st, src, dst, n4, 1);
  hipLaunchKernelGGL(k_copy_probe, dim3(blocks), dim3(threads), 0, st, dst, src, n4, 0);
  (void)hipEventRecord(e0, st);
  for (int k = 0; k < iters; ++k)
    hipLaunchKernelGGL(k_copy_probe, dim3(blocks), dim3(threads), 0, st, src, dst, n4, 0);
  (void)hipEventRecord(e1, st);
  hipError_t e = hipEventSynchronize(e1);
  if (e != hipSuccess) rc = fail(LB_EDEVICE, "copy probe: %s", hipGetErrorString(e));
  float t = 0;
  (void)hipEventElapsedTime(&t, e0, e1);
  if (ms) *ms = t / iters;
  if (gbps) *gbps = 2.0 * (double)n4 * 16.0 / (t / iters * 1e-3) / 1e9;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(src);
  (void)hipFree(dst);
  return rc;
}

int64_t lb_time(const lb_handle *h) { return h ? h->t : -1; }

int64_t lb_device_bytes(const lb_handle *h) { return h ? h->bytes : -1; }

const char *lb_last_error(void) { return lbi::g_err.c_str(); }

}  // extern "C"
