// lb_batch.hip -- batched stepping of many independent lattices of uneven
// size (declarations in include/lbnci.h).
//
// Two execution modes over the same tile kernels:
//   LB_BATCH_LAUNCH      per step three launches over a flattened tile table of
//                        all channels (phase, main, end-of-step bookkeeping),
//                        recorded once into a hipGraph of LB_GRAPH_CHUNK steps
//                        and replayed;
//   LB_BATCH_PERSISTENT  one cooperative launch for all n steps: every block
//                        works for one channel, channels synchronise only within
//                        their own block group (channel barrier), and retire
//                        independently when their convergence flag rises.  The
//                        counter reset and the launch form a hipGraph with a
//                        cooperative kernel node.
#include "lb_internal.hpp"

#include <hip/hip_runtime.h>
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

using namespace lbk;
using namespace lbi;

namespace {
constexpr int LB_GRAPH_CHUNK = 32;
}

struct lb_batch {
  int n = 0, D = 2, store = 0;
  hipStream_t stream = nullptr;
  std::vector<lb_handle *> h;
  void *d_args = nullptr;        // Args<S,R>[2n]
  ChanCtl *d_ctl = nullptr;      // [n]
  std::vector<ChanCtl> ctl;      // host mirror
  TileRef *d_phase = nullptr, *d_main = nullptr;
  int n_phase = 0, n_main = 0;
  int32_t *d_chan_of = nullptr, *d_rank_of = nullptr, *d_group = nullptr;
  uint32_t *d_bar = nullptr;
  int32_t *d_err = nullptr;
  int32_t *d_flags = nullptr;    // [n] observable flags gathered after each lb_batch_step
  std::vector<int32_t> flags;    // host copy
  int grid_persistent = 0;
  std::vector<int32_t> group;    // blocks per channel (persistent mode)
  std::vector<int32_t> xcd_of;   // XCD of each channel (persistent mode)
  hipGraphExec_t launch_graph = nullptr;
  hipGraphExec_t pers_graph = nullptr;
  int64_t pers_graph_steps = -1;
  int graph_ok = 1;              // 0 once a graph path failed (direct launches used)
  int64_t bytes = 0;
  int own_stream = 0;            // stream created by the batch (caller passed NULL)
  // execution configuration (chosen by lb_batch_tune or lb_batch_set_config)
  int cfg_mode = LB_BATCH_LAUNCH;
  int cfg_order = 0;             // 0: tiles dealt so each XCD gets a contiguous range; 1: channel order
  int cfg_by = 0;                // main-tile height of the launch mode (0 = library default)
};

namespace {

// Copies the observable flags of every channel into one array.
__global__ __launch_bounds__(256) void k_gather_flags(const ChanCtl *__restrict__ ctl, int n,
                                                      int32_t *__restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) out[c] = ctl[c].obs->flags;
}

template <typename S, typename R>
int build_tables_t(lb_batch *b) {
  std::vector<Args<S, R>> args(2 * b->n);
  for (int c = 0; c < b->n; ++c)
    for (int par = 0; par < 2; ++par) args[2 * c + par] = make_args<S, R>(b->h[c], par, 1 - par);
  HIP_TRY(hipMalloc(&b->d_args, sizeof(Args<S, R>) * args.size()));
  HIP_TRY(hipMemcpy(b->d_args, args.data(), sizeof(Args<S, R>) * args.size(), hipMemcpyHostToDevice));
  b->bytes += sizeof(Args<S, R>) * args.size();
  return LB_OK;
}

int phase_count(const lb_batch *b, const lb_params &p) {
  return b->D == 2 ? phase_tiles<2, 1>(p.nx, p.ny, p.nz) : phase_tiles<3, TZP3>(p.nx, p.ny, p.nz);
}
int main_count(const lb_batch *b, const lb_params &p) {
  return b->D == 2 ? main_tiles<2, BY2, TZ2>(p.nx, p.ny, p.nz) : main_tiles<3, BY3, TZ3>(p.nx, p.ny, p.nz);
}
// main tiles of the launch mode with tile height `by` (2-D: 4, 8 or 16)
int main_count_by(const lb_batch *b, const lb_params &p, int by) {
  if (b->D == 3 || by == 0 || by == BY2) return main_count(b, p);
  return by == 8 ? main_tiles<2, 8, 1>(p.nx, p.ny, p.nz) : main_tiles<2, 16, 1>(p.nx, p.ny, p.nz);
}

// Tile table of all channels, ordered so that each XCD (blocks are dealt
// round-robin over the 8 XCDs) receives a contiguous range of the flat list.
std::vector<TileRef> tile_table(const lb_batch *b, bool phase, int order, int by) {
  std::vector<TileRef> flat;
  for (int c = 0; c < b->n; ++c) {
    const int nt = phase ? phase_count(b, b->h[c]->p) : main_count_by(b, b->h[c]->p, by);
    for (int k = 0; k < nt; ++k) flat.push_back(TileRef{c, k});
  }
  if (order == 1) return flat;
  const int nb = (int)flat.size();
  std::vector<TileRef> t(nb);
  const int q = nb >> 3, r = nb & 7;
  for (int blk = 0; blk < nb; ++blk) {
    const int k = blk & 7, idx = blk >> 3;
    t[blk] = flat[k * q + (k < r ? k : r) + idx];
  }
  return t;
}

template <int D, typename S, typename R>
const void *persistent_fn() {
  if constexpr (D == 2)
    return reinterpret_cast<const void *>(&k_persistent<2, S, R, 1, BY2, TZ2, H2>);
  else
    return reinterpret_cast<const void *>(&k_persistent<3, S, R, TZP3, BY3, TZ3, H3>);
}

const void *persistent_kernel(const lb_batch *b) {
  switch (b->store) {
    case LB_STORE_FP32:
      return b->D == 2 ? persistent_fn<2, float, double>() : persistent_fn<3, float, double>();
    case LB_STORE_FP16_DEV:
      return b->D == 2 ? persistent_fn<2, __half, float>() : persistent_fn<3, __half, float>();
    case LB_STORE_BF16_DEV:
      return b->D == 2 ? persistent_fn<2, __hip_bfloat16, float>()
                       : persistent_fn<3, __hip_bfloat16, float>();
    default:
      return b->D == 2 ? persistent_fn<2, float, float>() : persistent_fn<3, float, float>();
  }
}

// Groups for the persistent launch: channels are bin-packed onto the 8 XCDs by
// work (largest first), then each XCD's resident blocks are split among its
// channels in proportion to their main tiles (at least one block each).  The
// block ids of an XCD's share are those congruent to the XCD index mod 8.
int build_groups(lb_batch *b) {
  const void *fn = persistent_kernel(b);
  int per_cu = 0, n_cu = 0, dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, 0));
  if (per_cu < 1) return fail(LB_EDEVICE, "persistent kernel cannot be resident");
  int G = per_cu * n_cu;
  long total_tiles = 0;
  for (int c = 0; c < b->n; ++c) total_tiles += main_count(b, b->h[c]->p);
  G = (int)std::min<long>(G, std::max<long>(total_tiles, b->n));
  G -= G % 8;
  if (G < b->n || G < 8) return fail(LB_EINVAL, "more channels than resident blocks");
  const int per_xcd = G / 8;
  // bin-pack channels onto XCDs
  std::vector<int> order(b->n);
  std::iota(order.begin(), order.end(), 0);
  std::vector<long> work(b->n);
  for (int c = 0; c < b->n; ++c) work[c] = main_count(b, b->h[c]->p);
  std::sort(order.begin(), order.end(), [&](int x, int y) { return work[x] > work[y]; });
  std::vector<long> load(8, 0);
  std::vector<std::vector<int>> bins(8);
  b->xcd_of.assign(b->n, 0);
  for (int c : order) {
    int best = 0;
    for (int k = 1; k < 8; ++k)
      if (load[k] < load[best] || (load[k] == load[best] && bins[k].size() < bins[best].size())) best = k;
    if ((int)bins[best].size() >= per_xcd) {  // keep at least one block per channel
      for (int k = 0; k < 8; ++k)
        if ((int)bins[k].size() < per_xcd) { best = k; break; }
    }
    bins[best].push_back(c);
    load[best] += work[c];
    b->xcd_of[c] = best;
  }
  b->group.assign(b->n, 0);
  std::vector<int32_t> chan_of(G, -1), rank_of(G, 0);
  for (int k = 0; k < 8; ++k) {
    auto &bin = bins[k];
    if (bin.empty()) continue;
    // split per_xcd blocks by largest remainder, at least one each
    long wsum = 0;
    for (int c : bin) wsum += work[c];
    int left = per_xcd - (int)bin.size();
    std::vector<double> rem(bin.size());
    int used = 0;
    for (size_t q = 0; q < bin.size(); ++q) {
      const double share = (double)left * work[bin[q]] / (double)std::max<long>(wsum, 1);
      const int fl = (int)std::floor(share);
      b->group[bin[q]] = 1 + fl;
      used += fl;
      rem[q] = share - fl;
    }
    std::vector<size_t> idx(bin.size());
    std::iota(idx.begin(), idx.end(), 0);
    std::sort(idx.begin(), idx.end(), [&](size_t x, size_t y) { return rem[x] > rem[y]; });
    for (size_t q = 0; q < idx.size() && used < left; ++q, ++used) b->group[bin[idx[q]]] += 1;
    // never more blocks than tiles
    for (int c : bin) b->group[c] = std::min<int32_t>(b->group[c], (int32_t)std::max<long>(work[c], 1));
    // assign the XCD's blocks (ids k, k+8, k+16, ...) to its channels in order
    int slot = 0;
    for (int c : bin)
      for (int r = 0; r < b->group[c]; ++r, ++slot) {
        const int blk = k + 8 * slot;
        chan_of[blk] = c;
        rank_of[blk] = r;
      }
  }
  // trailing unused blocks: compact the grid to the highest used block
  int last = -1;
  for (int blk = 0; blk < G; ++blk)
    if (chan_of[blk] >= 0) last = blk;
  // blocks without a channel inside the grid join channel 0's group as idle
  // members is not allowed (they would alter barrier counts); instead they are
  // given a channel with rank beyond its tiles: they still count in barriers
  for (int blk = 0; blk <= last; ++blk)
    if (chan_of[blk] < 0) {
      const int k = blk & 7;
      const int c = bins[k].empty() ? 0 : bins[k][0];
      chan_of[blk] = c;
      rank_of[blk] = b->group[c];
      b->group[c] += 1;
    }
  b->grid_persistent = last + 1;
  chan_of.resize(b->grid_persistent);
  rank_of.resize(b->grid_persistent);
  HIP_TRY(hipMalloc(&b->d_chan_of, sizeof(int32_t) * chan_of.size()));
  HIP_TRY(hipMalloc(&b->d_rank_of, sizeof(int32_t) * rank_of.size()));
  HIP_TRY(hipMalloc(&b->d_group, sizeof(int32_t) * b->n));
  HIP_TRY(hipMemcpy(b->d_chan_of, chan_of.data(), sizeof(int32_t) * chan_of.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(b->d_rank_of, rank_of.data(), sizeof(int32_t) * rank_of.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(b->d_group, b->group.data(), sizeof(int32_t) * b->n, hipMemcpyHostToDevice));
  return LB_OK;
}

template <int D, typename S, typename R>
void launch_step(lb_batch *b) {
  const Args<S, R> *args = reinterpret_cast<const Args<S, R> *>(b->d_args);
  if constexpr (D == 2) {
    hipLaunchKernelGGL((k_phase_batch<2, S, R, 1>), dim3(b->n_phase), dim3(64, 4), 0, b->stream, args,
                       b->d_ctl, b->d_phase);
    if (b->cfg_by == 8)
      hipLaunchKernelGGL((k_main_batch<2, S, R, 8, 1, H2>), dim3(b->n_main), dim3(64, 8), 0, b->stream,
                         args, b->d_ctl, b->d_main);
    else if (b->cfg_by == 16)
      hipLaunchKernelGGL((k_main_batch<2, S, R, 16, 1, H2>), dim3(b->n_main), dim3(64, 16), 0, b->stream,
                         args, b->d_ctl, b->d_main);
    else
      hipLaunchKernelGGL((k_main_batch<2, S, R, BY2, TZ2, H2>), dim3(b->n_main), dim3(64, BY2), 0,
                         b->stream, args, b->d_ctl, b->d_main);
  } else {
    hipLaunchKernelGGL((k_phase_batch<3, S, R, TZP3>), dim3(b->n_phase), dim3(64, 4), 0, b->stream,
                       args, b->d_ctl, b->d_phase);
    hipLaunchKernelGGL((k_main_batch<3, S, R, BY3, TZ3, H3>), dim3(b->n_main), dim3(64, BY3), 0,
                       b->stream, args, b->d_ctl, b->d_main);
  }
  hipLaunchKernelGGL(k_batch_end, dim3(b->n), dim3(256), 0, b->stream, b->d_ctl);
}

void launch_step_any(lb_batch *b) {
  const bool d2 = b->D == 2;
  switch (b->store) {
    case LB_STORE_FP32: d2 ? launch_step<2, float, double>(b) : launch_step<3, float, double>(b); break;
    case LB_STORE_FP16_DEV: d2 ? launch_step<2, __half, float>(b) : launch_step<3, __half, float>(b); break;
    case LB_STORE_BF16_DEV:
      d2 ? launch_step<2, __hip_bfloat16, float>(b) : launch_step<3, __hip_bfloat16, float>(b);
      break;
    default: d2 ? launch_step<2, float, float>(b) : launch_step<3, float, float>(b); break;
  }
}

// Records LB_GRAPH_CHUNK steps of the launch mode into a graph (once).
int ensure_launch_graph(lb_batch *b) {
  if (b->launch_graph || !b->graph_ok) return LB_OK;
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    b->graph_ok = 0;
    return LB_OK;
  }
  for (int k = 0; k < LB_GRAPH_CHUNK; ++k) launch_step_any(b);
  hipError_t e = hipStreamEndCapture(b->stream, &g);
  if (e == hipSuccess) e = hipGraphInstantiate(&b->launch_graph, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    b->launch_graph = nullptr;
    b->graph_ok = 0;
  }
  return LB_OK;
}

// Graph of the persistent mode: reset of the channel barrier counters and the
// error flag (fill kernels), then the cooperative persistent kernel node.
int ensure_pers_graph(lb_batch *b, int64_t nsteps) {
  if (!b->graph_ok) return LB_OK;
  if (b->pers_graph && b->pers_graph_steps == nsteps) return LB_OK;
  if (b->pers_graph) {
    (void)hipGraphExecDestroy(b->pers_graph);
    b->pers_graph = nullptr;
  }
  hipGraph_t g = nullptr;
  hipError_t e = hipGraphCreate(&g, 0);
  hipGraphNode_t n_reset = nullptr, n_err = nullptr, n_run = nullptr;
  int nbar = b->n;
  uint32_t zero = 0;
  int one = 1;
  (void)one;
  if (e == hipSuccess) {
    void *a[] = {&b->d_bar, &nbar, &zero};
    hipKernelNodeParams kp{};
    kp.func = reinterpret_cast<void *>(&k_fill_u32);
    kp.gridDim = dim3((b->n + 255) / 256);
    kp.blockDim = dim3(256);
    kp.kernelParams = a;
    e = hipGraphAddKernelNode(&n_reset, g, nullptr, 0, &kp);
  }
  int n1 = 1;
  uint32_t *errp = reinterpret_cast<uint32_t *>(b->d_err);
  if (e == hipSuccess) {
    void *a[] = {&errp, &n1, &zero};
    hipKernelNodeParams kp{};
    kp.func = reinterpret_cast<void *>(&k_fill_u32);
    kp.gridDim = dim3(1);
    kp.blockDim = dim3(256);
    kp.kernelParams = a;
    e = hipGraphAddKernelNode(&n_err, g, &n_reset, 1, &kp);
  }
  int ns = (int)nsteps;
  if (e == hipSuccess) {
    void *a[] = {&b->d_args, &b->d_ctl, &b->d_chan_of, &b->d_rank_of, &b->d_group, &b->d_bar, &b->d_err, &ns};
    hipKernelNodeParams kp{};
    kp.func = const_cast<void *>(persistent_kernel(b));
    kp.gridDim = dim3(b->grid_persistent);
    kp.blockDim = dim3(64, 4);
    kp.kernelParams = a;
    e = hipGraphAddKernelNode(&n_run, g, &n_err, 1, &kp);
  }
  if (e == hipSuccess) {
    hipKernelNodeAttrValue v{};
    v.cooperative = 1;
    e = hipGraphKernelNodeSetAttribute(n_run, hipKernelNodeAttributeCooperative, &v);
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&b->pers_graph, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    b->pers_graph = nullptr;
    b->graph_ok = 0;
  } else {
    b->pers_graph_steps = nsteps;
  }
  return LB_OK;
}

int upload_ctl(lb_batch *b, int mode) {
  for (int c = 0; c < b->n; ++c) {
    lb_handle *h = b->h[c];
    ChanCtl &k = b->ctl[c];
    k.t = h->t;
    k.parity = h->cur;
    k.n_main = mode == LB_BATCH_LAUNCH ? main_count_by(b, h->p, b->cfg_by) : main_count(b, h->p);
  }
  HIP_TRY(hipMemcpyAsync(b->d_ctl, b->ctl.data(), sizeof(ChanCtl) * b->n, hipMemcpyHostToDevice, b->stream));
  return LB_OK;
}

int download_ctl(lb_batch *b) {
  HIP_TRY(hipMemcpyAsync(b->ctl.data(), b->d_ctl, sizeof(ChanCtl) * b->n, hipMemcpyDeviceToHost, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  for (int c = 0; c < b->n; ++c) {
    b->h[c]->t = b->ctl[c].t;
    b->h[c]->cur = b->ctl[c].parity;
  }
  return LB_OK;
}

int apply_config(lb_batch *b, int mode, int order, int by) {
  if (b->D == 3) by = 0;
  if (by != 0 && by != 4 && by != 8 && by != 16) return fail(LB_EINVAL, "main-tile height must be 4, 8 or 16");
  if (mode != LB_BATCH_LAUNCH && mode != LB_BATCH_PERSISTENT) return fail(LB_EINVAL, "unknown mode");
  if (order != 0 && order != 1) return fail(LB_EINVAL, "unknown tile order");
  if (by == 4) by = 0;
  if (b->d_main && order == b->cfg_order && by == b->cfg_by) {
    b->cfg_mode = mode;
    return LB_OK;
  }
  auto tp = tile_table(b, true, order, 0), tm = tile_table(b, false, order, by);
  if (b->d_phase) (void)hipFree(b->d_phase);
  if (b->d_main) (void)hipFree(b->d_main);
  b->d_phase = b->d_main = nullptr;
  HIP_TRY(hipMalloc(&b->d_phase, sizeof(TileRef) * tp.size()));
  HIP_TRY(hipMalloc(&b->d_main, sizeof(TileRef) * tm.size()));
  HIP_TRY(hipMemcpy(b->d_phase, tp.data(), sizeof(TileRef) * tp.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(b->d_main, tm.data(), sizeof(TileRef) * tm.size(), hipMemcpyHostToDevice));
  b->n_phase = (int)tp.size();
  b->n_main = (int)tm.size();
  b->cfg_mode = mode;
  b->cfg_order = order;
  b->cfg_by = by;
  if (b->launch_graph) {  // recorded with the previous tables
    (void)hipGraphExecDestroy(b->launch_graph);
    b->launch_graph = nullptr;
  }
  return LB_OK;
}

}  // namespace

extern "C" {

int lb_batch_create(const lb_params *p, int32_t n, void *hip_stream, lb_batch **out) {
  if (!out || !p || n < 1) return fail(LB_EINVAL, "bad batch arguments");
  *out = nullptr;
  for (int c = 0; c < n; ++c) {
    int rc = validate(&p[c]);
    if (rc) return rc;
    if (p[c].lattice != p[0].lattice || p[c].storage != p[0].storage)
      return fail(LB_EINVAL, "all channels of a batch share lattice and storage");
    if (p[c].obs_every != p[0].obs_every) return fail(LB_EINVAL, "all channels share obs_every");
    if (p[c].nci_mode != 0)
      return fail(LB_EINVAL, "channel %d: batches run the integer NCI probe only (nci_mode 0)", c);
  }
  lb_batch *b = new (std::nothrow) lb_batch();
  if (!b) return fail(LB_ENOMEM, "host allocation failed");
  b->n = n;
  b->D = p[0].lattice == LB_D2Q9 ? 2 : 3;
  b->store = p[0].storage;
  b->stream = (hipStream_t)hip_stream;
  int rc = LB_OK;
  if (!b->stream) {  // graphs cannot be captured on the NULL stream
    hipError_t e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
    if (e != hipSuccess) rc = fail(LB_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
    else b->own_stream = 1;
  }
  b->h.assign(n, nullptr);
  for (int c = 0; c < n && !rc; ++c) rc = lb_create(&p[c], (void *)b->stream, &b->h[c]);
  if (!rc) {
    switch (b->store) {
      case LB_STORE_FP32: rc = build_tables_t<float, double>(b); break;
      case LB_STORE_FP16_DEV: rc = build_tables_t<__half, float>(b); break;
      case LB_STORE_BF16_DEV: rc = build_tables_t<__hip_bfloat16, float>(b); break;
      default: rc = build_tables_t<float, float>(b); break;
    }
  }
  if (!rc) {
    b->ctl.resize(n);
    for (int c = 0; c < n; ++c) {
      lb_handle *h = b->h[c];
      ChanCtl k{};
      k.obs = h->obs;
      k.partials = h->partials;
      k.n_main = main_count(b, h->p);
      k.n_phase = phase_count(b, h->p);
      k.active = 1;
      k.retire = h->p.conv_window > 0;
      k.t = 0;
      k.inv_nx = 1.0 / h->p.nx;
      k.W = h->p.conv_window;
      k.m = h->p.conv_m;
      k.eps = h->p.conv_eps;
      k.mass_tol = h->p.mass_tol;
      k.obs_every = h->p.obs_every;
      k.parity = 0;
      b->ctl[c] = k;
    }
    hipError_t e = hipMalloc(&b->d_ctl, sizeof(ChanCtl) * n);
    if (e != hipSuccess) rc = fail(LB_ENOMEM, "hipMalloc: %s", hipGetErrorString(e));
  }
  if (!rc) rc = apply_config(b, LB_BATCH_LAUNCH, 0, 0);
  if (!rc) {
    hipError_t e = hipMalloc(&b->d_bar, sizeof(uint32_t) * n);
    if (e == hipSuccess) e = hipMalloc(&b->d_err, sizeof(int32_t));
    if (e == hipSuccess) e = hipMemset(b->d_err, 0, sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&b->d_flags, sizeof(int32_t) * n);
    if (e == hipSuccess) e = hipMemset(b->d_flags, 0, sizeof(int32_t) * n);
    b->flags.assign(n, 0);
    if (e != hipSuccess) rc = fail(LB_EDEVICE, "batch tables: %s", hipGetErrorString(e));
  }
  if (!rc) rc = build_groups(b);
  if (rc) {
    lb_batch_destroy(b);
    return rc;
  }
  *out = b;
  return LB_OK;
}

void lb_batch_destroy(lb_batch *b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  else (void)hipDeviceSynchronize();
  if (b->launch_graph) (void)hipGraphExecDestroy(b->launch_graph);
  if (b->pers_graph) (void)hipGraphExecDestroy(b->pers_graph);
  (void)hipFree(b->d_args);
  (void)hipFree(b->d_ctl);
  (void)hipFree(b->d_phase);
  (void)hipFree(b->d_main);
  (void)hipFree(b->d_chan_of);
  (void)hipFree(b->d_rank_of);
  (void)hipFree(b->d_group);
  (void)hipFree(b->d_bar);
  (void)hipFree(b->d_err);
  (void)hipFree(b->d_flags);
  for (lb_handle *h : b->h) lb_destroy(h);
  if (b->own_stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

int lb_batch_init_fields(lb_batch *b, int32_t c, const double *rho1, const double *rho2, const double *u) {
  if (!b || c < 0 || c >= b->n) return fail(LB_EINVAL, "bad channel");
  int rc = lb_init_fields(b->h[c], rho1, rho2, u);
  if (rc) return rc;
  b->ctl[c].active = 1;
  b->ctl[c].t = 0;
  return LB_OK;
}

int lb_batch_step(lb_batch *b, int64_t n, int32_t mode) {
  if (!b || n < 0) return fail(LB_EINVAL, "bad arguments");
  if (mode == LB_BATCH_AUTO) mode = b->cfg_mode;
  if (mode != LB_BATCH_LAUNCH && mode != LB_BATCH_PERSISTENT) return fail(LB_EINVAL, "unknown mode");
  for (lb_handle *h : b->h)
    if (!h->initialised) return fail(LB_ESTATE, "every channel must be initialised");
  if (n == 0) return LB_OK;
  // The first step after initialisation reads the explicit initial state; it
  // runs as one plain step per channel and counts as the first of the n steps.
  int n_explicit = 0;
  for (lb_handle *h : b->h) n_explicit += h->explicit_src;
  if (n_explicit != 0 && n_explicit != b->n)
    return fail(LB_ESTATE, "channels must be (re)initialised together");
  int64_t steps = n;
  if (n_explicit) {
    for (int c = 0; c < b->n; ++c) {
      int rc = lb_step(b->h[c], 1);
      if (rc) return rc;
    }
    steps -= 1;
  }
  int rc = upload_ctl(b, mode);
  if (rc) return rc;
  if (steps == 0) {
  } else if (mode == LB_BATCH_LAUNCH) {
    rc = ensure_launch_graph(b);
    if (rc) return rc;
    int64_t done = 0;
    if (b->launch_graph)
      for (; done + LB_GRAPH_CHUNK <= steps; done += LB_GRAPH_CHUNK)
        HIP_TRY(hipGraphLaunch(b->launch_graph, b->stream));
    for (; done < steps; ++done) launch_step_any(b);
    HIP_TRY(hipGetLastError());
  } else {
    if (steps > INT32_MAX) return fail(LB_EINVAL, "too many steps for one persistent launch");
    rc = ensure_pers_graph(b, steps);
    if (rc) return rc;
    if (b->pers_graph) {
      HIP_TRY(hipGraphLaunch(b->pers_graph, b->stream));
    } else {
      int nbar = b->n;
      hipLaunchKernelGGL(k_fill_u32, dim3((nbar + 255) / 256), dim3(256), 0, b->stream, b->d_bar, nbar, 0u);
      hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, b->stream, reinterpret_cast<uint32_t *>(b->d_err), 1, 0u);
      int ns = (int)steps;
      void *a[] = {&b->d_args, &b->d_ctl, &b->d_chan_of, &b->d_rank_of, &b->d_group, &b->d_bar, &b->d_err, &ns};
      HIP_TRY(hipLaunchCooperativeKernel(persistent_kernel(b), dim3(b->grid_persistent), dim3(64, 4), a, 0,
                                         b->stream));
    }
  }
  hipLaunchKernelGGL(k_gather_flags, dim3((b->n + 255) / 256), dim3(256), 0, b->stream, b->d_ctl, b->n,
                     b->d_flags);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(b->flags.data(), b->d_flags, sizeof(int32_t) * b->n, hipMemcpyDeviceToHost,
                         b->stream));
  rc = download_ctl(b);
  if (rc) return rc;
  if (mode == LB_BATCH_PERSISTENT && steps > 0) {
    int32_t err = 0;
    HIP_TRY(hipMemcpy(&err, b->d_err, sizeof err, hipMemcpyDeviceToHost));
    if (err) return fail(LB_EDEVICE, "persistent launch: a channel barrier timed out");
  }
  int bad = 0, first = -1;
  for (int c = 0; c < b->n; ++c)
    if (b->flags[c]) {
      if (first < 0) first = c;
      ++bad;
    }
  if (bad)
    return fail(LB_ENUMERIC, "%d channel(s) flagged a NaN/Inf or mass drift (first: channel %d, flags %d)", bad,
                first, b->flags[first]);
  return LB_OK;
}

int lb_batch_flags(lb_batch *b, int32_t *flags) {
  if (!b || !flags) return fail(LB_EINVAL, "NULL argument");
  for (int c = 0; c < b->n; ++c) flags[c] = b->flags[c];
  return LB_OK;
}

int lb_batch_observables(lb_batch *b, int32_t c, lb_obs *out) {
  if (!b || c < 0 || c >= b->n) return fail(LB_EINVAL, "bad channel");
  return lb_observables(b->h[c], out);
}

int lb_batch_get_fields(lb_batch *b, int32_t c, double *rho1, double *rho2, double *u) {
  if (!b || c < 0 || c >= b->n) return fail(LB_EINVAL, "bad channel");
  return lb_get_fields(b->h[c], rho1, rho2, u);
}

int lb_batch_info(lb_batch *b, int32_t c, int64_t *steps, int32_t *active, int32_t *blocks) {
  if (!b || c < 0 || c >= b->n) return fail(LB_EINVAL, "bad channel");
  if (steps) *steps = b->h[c]->t;
  if (active) *active = b->ctl[c].active;
  if (blocks) *blocks = b->group.empty() ? 0 : b->group[c];
  return LB_OK;
}

int lb_batch_graphs(lb_batch *b) { return b ? b->graph_ok : -1; }

int lb_batch_set_config(lb_batch *b, int32_t mode, int32_t tile_order, int32_t main_by) {
  if (!b) return fail(LB_EINVAL, "NULL batch");
  return apply_config(b, mode, tile_order, main_by);
}

int lb_batch_get_config(lb_batch *b, int32_t *mode, int32_t *tile_order, int32_t *main_by) {
  if (!b) return fail(LB_EINVAL, "NULL batch");
  if (mode) *mode = b->cfg_mode;
  if (tile_order) *tile_order = b->cfg_order;
  if (main_by) *main_by = b->cfg_by == 0 ? (b->D == 2 ? BY2 : BY3) : b->cfg_by;
  return LB_OK;
}

int lb_batch_tune(lb_batch *b, int32_t trial_steps, double *best_ms_per_step) {
  if (!b || trial_steps < 1) return fail(LB_EINVAL, "bad arguments");
  struct Cand { int mode, order, by; };
  std::vector<Cand> cands;
  const std::vector<int> bys = b->D == 2 ? std::vector<int>{4, 8, 16} : std::vector<int>{4};
  for (int order = 0; order < 2; ++order)
    for (int by : bys) cands.push_back({LB_BATCH_LAUNCH, order, by});
  cands.push_back({LB_BATCH_PERSISTENT, 0, 4});
  double best = 1e300;
  Cand win = cands[0];
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  int rc = LB_OK;
  for (const Cand &c : cands) {
    // a channel that goes non-finite does not stop the timing (the flag
    // stays set and the next lb_batch_step reports it)
    rc = apply_config(b, c.mode, c.order, c.by);
    if (!rc) rc = lb_batch_step(b, 2, c.mode);  // warm-up (also records the graph)
    if (rc == LB_ENUMERIC) rc = LB_OK;
    if (rc) break;
    HIP_TRY(hipEventRecord(e0, b->stream));
    rc = lb_batch_step(b, trial_steps, c.mode);
    if (rc == LB_ENUMERIC) rc = LB_OK;
    if (rc) break;
    HIP_TRY(hipEventRecord(e1, b->stream));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    const double per = ms / trial_steps;
    if (per < best) {
      best = per;
      win = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  if (best_ms_per_step) *best_ms_per_step = best;
  return apply_config(b, win.mode, win.order, win.by);
}

}  // extern "C"
