// ws_net.hip -- U-Net of the learned warm start (C ABI in include/wsnet.h).
//
// Architecture (levels L, base channels C0, C_l = C0 << l, image H x W):
//   encoder level l: conv3x3+ReLU (in -> C_l), conv3x3+ReLU (C_l -> C_l),
//                    2x2 max pool to level l+1 (l < L-1)
//   decoder level l (l = L-2 .. 0): 2x2 stride-2 transposed conv (C_{l+1} -> C_l),
//                    concat [up | encoder output of level l], conv3x3+ReLU
//                    (2 C_l -> C_l), conv3x3+ReLU (C_l -> C_l)
//   head: 1x1 conv (C0 -> cout), no activation; loss: mean squared error.
// Input channels are padded to 8 and head outputs to 8 (padding weights zero).
//
// Flat FP32 parameter order (weights then bias of each layer):
//   for l = 0..L-1:  e1[l].W [C_l][3][3][cin_l], e1[l].b [C_l],
//                    e2[l].W [C_l][3][3][C_l],   e2[l].b [C_l]      (cin_0 = 8, cin_l = C_{l-1})
//   for l = L-2..0:  up[l].W [4][C_l][C_{l+1}] (4 = 2 dy + dx), up[l].b [C_l],
//                    d1[l].W [C_l][3][3][2 C_l], d1[l].b [C_l],
//                    d2[l].W [C_l][3][3][C_l],   d2[l].b [C_l]
//   head.W [8][C0], head.b [8]
#include "wsnet.h"
#include "ws_direct.hpp"

#include <hip/hip_runtime.h>
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

using namespace wsk;

namespace {

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

#define HTRY(expr)                                                                         \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(WS_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

struct Conv {
  int KS, Cin, Cout;
  bool relu;
  int64_t w_off, b_off;  // into the flat parameter vector
  bf16 *Wt = nullptr, *WtT = nullptr;
  int64_t nw() const { return (int64_t)Cout * KS * KS * Cin; }
};

struct Up {
  int Cin, Cout;
  int64_t w_off, b_off;
  bf16 *Wt = nullptr, *WtT = nullptr;
  int64_t nw() const { return 4LL * Cout * Cin; }
};

template <typename T>
struct Buf {
  T *p = nullptr;
  int cs = 0;  // channel stride
};

}  // namespace

struct ws_net {
  ws_config cfg;
  int L, C0;
  hipStream_t stream;
  int64_t np = 0;
  float *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr;
  int64_t adam_t = 0;
  std::vector<Conv> e1, e2, d1, d2;
  std::vector<Up> up;
  Conv head;
  // activations (BF16) and gradients (FP32), per level
  Buf<bf16> xin;                 // packed input, 8 channels
  std::vector<Buf<bf16>> pool;   // pool output feeding level l (l >= 1)
  std::vector<Buf<uint8_t>> parg;  // its argmax codes, when the forward fused the pooling
  std::vector<char> pool_fused;    // per level: the last forward wrote parg
  std::vector<Buf<bf16>> mid_e, cat, mid_d, dec;
  Buf<bf16> bott;                // encoder output of the last level
  Buf<float> y;                  // head output, 8 channels
  std::vector<Buf<bf16>> dpool, dmid_e, dcat, dmid_d, ddec;  // activation gradients (BF16)
  Buf<bf16> dbott, dy;
  // split partials of every weight gradient of a backward pass, each layer
  // in its own range, summed by one k_wreduce launch per WJ_MAX layers at
  // the end of the pass
  float *scratch = nullptr;
  size_t scratch_floats = 0, scratch_used = 0;
  std::vector<WJob> jobs;
  // weight gradients run on a second stream (default priority), each after
  // an event on the network's stream that marks its output gradient final,
  // beside the data gradients; joined before the split sums
  hipStream_t side = nullptr;
  std::vector<hipEvent_t> evs;  // fork events, reused every pass
  hipEvent_t ev_join = nullptr;
  size_t ev_next = 0;
  bool on_side = false, side_pending = false;
  bool head_lds_set = false;  // the training head's dynamic LDS limit raised
  double *loss_part = nullptr, *loss = nullptr;
  int n_loss_blocks = 0;
  std::vector<void *> allocs;
  int64_t bytes = 0;
};

namespace {

int chans(const ws_net *n, int l) { return n->C0 << l; }
int imgH(const ws_net *n, int l) { return n->cfg.H >> l; }
int imgW(const ws_net *n, int l) { return n->cfg.W >> l; }

template <typename T>
int dalloc(ws_net *n, T **p, size_t count) {
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void **)p, count * sizeof(T));
  if (e != hipSuccess) return fail(WS_ENOMEM, "hipMalloc(%zu): %s", count * sizeof(T), hipGetErrorString(e));
  n->allocs.push_back((void *)*p);
  n->bytes += (int64_t)(count * sizeof(T));
  HTRY(hipMemsetAsync(*p, 0, count * sizeof(T), n->stream));
  return WS_OK;
}

template <typename T>
int buf(ws_net *n, Buf<T> &b, int l, int cs) {
  b.cs = cs;
  return dalloc(n, &b.p, (size_t)n->cfg.max_batch * imgH(n, l) * imgW(n, l) * cs);
}

Conv make_conv(int64_t &off, int KS, int Cin, int Cout, bool relu) {
  Conv c;
  c.KS = KS;
  c.Cin = Cin;
  c.Cout = Cout;
  c.relu = relu;
  c.w_off = off;
  off += c.nw();
  c.b_off = off;
  off += Cout;
  return c;
}

Up make_up(int64_t &off, int Cin, int Cout) {
  Up u;
  u.Cin = Cin;
  u.Cout = Cout;
  u.w_off = off;
  off += u.nw();
  u.b_off = off;
  off += Cout;
  return u;
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

// BF16 weight copies of every layer from the FP32 master weights, one launch
int refresh_weights(ws_net *n) {
  WTable t{};
  int blk = 0;
  auto add = [&](const float *W, bf16 *Wt, bf16 *WtT, int Cout, int Cin, int KS, int up, int64_t nw) {
    if (t.n == MAX_WLAYERS) return;  // not reached: 6 levels make 28 layers
    t.l[t.n] = WLayer{W, Wt, WtT, Cout, Cin, KS, up, blk};
    ++t.n;
    blk += (int)blocks(nw);
  };
  auto conv = [&](Conv &c) { add(n->params + c.w_off, c.Wt, c.WtT, c.Cout, c.Cin, c.KS, 0, c.nw()); };
  for (auto &c : n->e1) conv(c);
  for (auto &c : n->e2) conv(c);
  for (auto &c : n->d1) conv(c);
  for (auto &c : n->d2) conv(c);
  conv(n->head);
  for (auto &u : n->up) add(n->params + u.w_off, u.Wt, u.WtT, u.Cout, u.Cin, 2, 1, u.nw());
  hipLaunchKernelGGL(k_refresh_weights, dim3((unsigned)blk), dim3(256), 0, n->stream, t);
  HTRY(hipGetLastError());
  return WS_OK;
}

// Block tile of a GEMM: BN from the output width (32 / 64 / 128), BM = 128
// unless the tile count would leave the chip idle or the problem needs rows
// grouped by a divisor (the up-sampling parity).
struct Tile {
  int bm, bn;
};

Tile pick_tile(int M, int N, int row_group) {
  Tile t{128, N <= 32 ? 32 : (N <= 64 ? 64 : 128)};
  auto tiles = [&](const Tile &x) { return (int64_t)((M + x.bm - 1) / x.bm) * ((N + x.bn - 1) / x.bn); };
  if ((row_group && row_group % 128) || tiles(t) < 1024) t.bm = 64;
  if (t.bn == 128 && tiles(t) < 512) t.bn = 64;
  return t;
}

// Tile of a split weight-gradient GEMM (small M, wide N; splits fill the chip).
Tile pick_tile_split(int M, int N) { return Tile{M <= 64 ? 64 : 128, N <= 32 ? 32 : (N <= 64 ? 64 : 128)}; }

// Tiles that run 64-deep K steps (two MFMA slices per LDS stage, twice the
// work per global-load wait): measured faster only for the 3x3 data gradient
// at 128 x 32 (105 -> 87 us at level 0) and the 3x3 forward at 64 x 128
// (44 -> 38 us); elsewhere the larger LDS stage costs more occupancy than it
// saves.  Split-K problems keep 32 (their chunks are multiples of 32).
template <class P>
struct DeepK {
  static constexpr int bm = 0, bn = 0;
};
template <>
struct DeepK<ConvBwdData<3>> {
  static constexpr int bm = 128, bn = 32;
};
template <bool RELU, bool F32>
struct DeepK<ConvFwd<3, RELU, F32>> {
  static constexpr int bm = 64, bn = 128;
};

template <class Prob, int BMt, int BNt>
void launch(ws_net *n, const Prob &p, int M, int N, int splits) {
  constexpr int KB = (BMt == DeepK<Prob>::bm && BNt == DeepK<Prob>::bn) ? 64 : BK;
  dim3 grid((M + BMt - 1) / BMt, (N + BNt - 1) / BNt, splits);
  hipLaunchKernelGGL((k_gemm<Prob, BMt, BNt, KB>), grid, dim3(256), 0, n->on_side ? n->side : n->stream, p);
}

template <class Prob>
void gemm(ws_net *n, const Prob &p, int M, int N, int splits, Tile t) {
  if (t.bm == 128) {
    if (t.bn == 32) launch<Prob, 128, 32>(n, p, M, N, splits);
    else if (t.bn == 64) launch<Prob, 128, 64>(n, p, M, N, splits);
    else launch<Prob, 128, 128>(n, p, M, N, splits);
  } else {
    if (t.bn == 32) launch<Prob, 64, 32>(n, p, M, N, splits);
    else if (t.bn == 64) launch<Prob, 64, 64>(n, p, M, N, splits);
    else launch<Prob, 64, 128>(n, p, M, N, splits);
  }
}

// split count and chunk (pixels per split, a multiple of the K step) for a
// weight-gradient GEMM over P pixels: about 1024 blocks in all
void split_plan(int P, int M, int N, int &splits, int &chunk) {
  const Tile t = pick_tile_split(M, N);
  const int tiles = ((M + t.bm - 1) / t.bm) * ((N + t.bn - 1) / t.bn);
  int s = std::max(1, 1024 / std::max(tiles, 1));
  s = std::min(s, std::max(1, P / (4 * BK)));
  // the partials are written once and read back once: at most 8M floats
  // (32 MB) of them unless that leaves fewer than 4 splits
  s = std::min(s, std::max(4, (int)((8 << 20) / ((int64_t)M * N))));
  chunk = ((P + s - 1) / s + BK - 1) / BK * BK;
  splits = (P + chunk - 1) / chunk;
}

// Direct 3x3 kernels (ws_direct.hpp) serve a level whose image is a whole
// number of 8 x 32 tiles and whose channel counts are multiples of 32 (the
// staged operand may also be the 8-channel network input); other shapes, and
// every layer under conv_algo = 1, use the implicit GEMM.
bool direct_ok(const ws_net *n, const Img &g, int Kc, int Nc, bool c8_ok) {
  return n->cfg.conv_algo == 0 && g.W % DT_W == 0 && g.H % DT_H == 0 && Nc % 32 == 0 &&
         (Kc % 32 == 0 || (c8_ok && Kc == 8));
}

// Input channels per direct weight-gradient block (16 HW, 2 HW waves): 16
// for the padded network input, 32 at 32 channels, else 64 (the
// output-gradient tile is staged once per block, so wider blocks read it
// fewer times).
int direct_whw(int Cin) { return Cin == 8 ? 1 : (Cin % 64 == 0 ? 4 : 2); }

// Split plan of a direct weight gradient, each block summing a run of
// tiles: 192 blocks of 4 or 8 waves, 512 of the 2-wave blocks of the padded
// input.  Alone on the GPU, 256 (one per CU: registers and LDS hold one
// 8-wave block per CU) measured best (1.45 ms per training step, against
// 1.51 with 192 / 384 / 768 blocks at hw 4 / 2 / 1 and 1.53 with a second
// round); since the weight gradients run beside the data gradients, 192
// leaves them room (1.152 ms with 256, 1.144 with 128, 1.130 with 192).
void direct_wplan(int ntiles, int Cin, int Cout, int &splits, int &tps) {
  const int hw = direct_whw(Cin);
  const int combos = std::max(1, Cin / (16 * hw)) * (Cout / 32);
  const int want = std::max(1, (hw == 1 ? 512 : 192) / combos);
  tps = std::max(1, (ntiles + want - 1) / want);
  splits = (ntiles + tps - 1) / tps;
}

// A block computes 32 NW output channels with 4 NW waves (NW N groups share
// each staged input tile, which is then read once per 32 NW channels, not
// once per 32): NW = 2 where the output channels allow (four groups would
// leave 128 registers per lane and spill), else 1.  Each block
// runs enough tiles to leave about 512 blocks, so that one tile's loads
// overlap the previous tile's MFMAs.
template <bool BWD, bool C8, int NW>
void launch_dconv_nw(ws_net *n, DConv p) {
  const int nb = p.Nc / (32 * NW);
  const int want = std::max(1, 512 / (nb * NW));
  p.tpb = std::max(1, (p.T.n + want - 1) / want);
  dim3 grid((unsigned)((p.T.n + p.tpb - 1) / p.tpb), (unsigned)nb);
  // the weights of one or two 32-channel slices are staged once per block
  // (one slice: forward 24.9 -> 20.1 us at level 0, data gradient 1.308 ->
  // 1.301 ms per training step; two: 1.256 -> 1.243 ms); more slices reload
  // each item's
  if (C8 || p.Kc == 32)
    hipLaunchKernelGGL((k_dconv<BWD, C8, NW, 1>), grid, dim3(256 * NW), 0, n->stream, p);
  else if (p.Kc == 64)
    hipLaunchKernelGGL((k_dconv<BWD, C8, NW, 2>), grid, dim3(256 * NW), 0, n->stream, p);
  else hipLaunchKernelGGL((k_dconv<BWD, C8, NW, 0>), grid, dim3(256 * NW), 0, n->stream, p);
}

template <bool BWD, bool C8>
void launch_dconv(ws_net *n, const DConv &p) {
  if (p.Nc % 64 == 0) launch_dconv_nw<BWD, C8, 2>(n, p);
  else launch_dconv_nw<BWD, C8, 1>(n, p);
}

template <int KS, bool RELU, bool F32>
int conv_fwd_t(ws_net *n, const Conv &c, Img g, View<const bf16> in, View<bf16> out, View<float> outf) {
  ConvFwd<KS, RELU, F32> p;
  p.g = g;
  p.in = in;
  p.Cin = c.Cin;
  p.Cout = c.Cout;
  p.Wt = c.Wt;
  p.bias = n->params + c.b_off;
  p.out = out;
  p.outf = outf;
  p.dCin = Div::make(c.Cin);
  gemm(n, p, g.B * g.H * g.W, c.Cout, 1, pick_tile(g.B * g.H * g.W, c.Cout, 0));
  return WS_OK;
}

// pool.p set: also writes the output's 2x2 max pooling there when the direct
// kernel runs (*pooled = true), else leaves it to the caller.
int conv_fwd(ws_net *n, const Conv &c, Img g, View<const bf16> in, View<bf16> out,
             View<bf16> pool = View<bf16>{nullptr, 0, 0}, bool *pooled = nullptr, uint8_t *parg = nullptr) {
  if (pooled) *pooled = false;
  if (c.KS == 3 && c.relu && direct_ok(n, g, c.Cin, c.Cout, true)) {
    DConv p{};
    p.g = g;
    p.T = DTiles::make(g.B, g.H, g.W);
    p.x = in;
    p.Kc = c.Cin;
    p.Nc = c.Cout;
    p.Wk = c.Wt;
    p.bias = n->params + c.b_off;
    p.y = out;
    p.pool = pool;
    p.parg = parg;
    if (pooled) *pooled = pool.p != nullptr;
    if (c.Cin == 8) launch_dconv<false, true>(n, p);
    else launch_dconv<false, false>(n, p);
    return WS_OK;
  }
  return c.relu ? conv_fwd_t<3, true, false>(n, c, g, in, out, View<float>{nullptr, 0, 0})
                : conv_fwd_t<3, false, false>(n, c, g, in, out, View<float>{nullptr, 0, 0});
}

// GEMM shape of a conv weight gradient: Cout x (K+1), or transposed when Cout
// is narrow (the wide im2col dimension then fills the 128-row tiles).
struct WShape {
  bool tr;
  int M, N;
};
WShape wshape(int Cout, int Kw1) { return Cout < 64 ? WShape{true, Kw1, Cout} : WShape{false, Cout, Kw1}; }

// The next range of split partials, splits x M (Kw + 1) floats (a multiple
// of 4), or nullptr when the scratch sized at creation cannot hold it.
float *take_partials(ws_net *n, int splits, int M, int Kw) {
  const size_t count = (size_t)splits * M * (Kw + 1);
  if (n->scratch_used + count > n->scratch_floats) return nullptr;
  float *p = n->scratch + n->scratch_used;
  n->scratch_used += count;
  return p;
}

// side_mark records the network's stream's progress; weight-gradient
// launches between side_begin(that mark) and side_end go to the side stream,
// after everything queued before the mark.  Out of events: no side stream.
hipEvent_t side_mark(ws_net *n) {
  if (n->ev_next >= n->evs.size()) return nullptr;
  hipEvent_t e = n->evs[n->ev_next++];
  return hipEventRecord(e, n->stream) == hipSuccess ? e : nullptr;
}
int side_begin(ws_net *n, hipEvent_t mark) {
  if (!mark) return WS_OK;
  HTRY(hipStreamWaitEvent(n->side, mark, 0));
  n->on_side = n->side_pending = true;
  return WS_OK;
}
void side_end(ws_net *n) { n->on_side = false; }
// The network's stream waits for every weight gradient.
int side_join(ws_net *n) {
  if (n->side_pending) {
    HTRY(hipEventRecord(n->ev_join, n->side));
    HTRY(hipStreamWaitEvent(n->stream, n->ev_join, 0));
  }
  n->side_pending = false;
  n->ev_next = 0;
  return WS_OK;
}

// Queues the sum of partials [splits][M][Kw+1] into dW [M][Kw] and the bias
// column into db: row m's bias when Cb = M, else db[c] = sum over rows
// m = c (mod Cb).
void queue_split_reduce(ws_net *n, const float *partial, int splits, int M, int Kw, float *dW, float *db, int Cb) {
  WJob j{};
  j.partial = partial;
  j.dW = dW;
  j.db = db;
  j.splits = splits;
  j.E = M * (Kw + 1);
  j.Kw = Kw;
  j.Cb = Cb;
  n->jobs.push_back(j);
}

// Launches the queued sums, WJ_MAX layers per launch, and frees the scratch.
// (on the side stream when `side`: after the weight gradients queued there;
// the partials stay reserved until the pass ends)
void flush_split_reduce(ws_net *n, bool side = false) {
  for (size_t i = 0; i < n->jobs.size(); i += WJ_MAX) {
    WJobs J{};
    int blk = 0;
    for (size_t k = i; k < n->jobs.size() && k < i + WJ_MAX; ++k) {
      WJob j = n->jobs[k];
      j.blk0 = blk;
      j.gsh = 0;
      while (j.gsh < 4 && (16 << j.gsh) < j.splits) ++j.gsh;  // at most 16 splits per group, or 16 groups
      j.nbw = (j.E / 4 + (64 * WR_G >> j.gsh) - 1) / (64 * WR_G >> j.gsh);
      const int rows = j.E / (j.Kw + 1);
      blk += j.nbw + (j.Cb < rows ? (j.Cb + WR_G - 1) / WR_G : 0);
      J.j[J.n++] = j;
    }
    hipLaunchKernelGGL(k_wreduce, dim3((unsigned)blk), dim3(64 * WR_G), 0, side ? n->side : n->stream, J);
  }
  n->jobs.clear();
  if (!side) n->scratch_used = 0;
}

template <int KS, bool TR>
void conv_bwd_weight(ws_net *n, const Conv &c, Img g, View<const bf16> in, View<const bf16> dout, int chunk,
                     int splits, const WShape &ws, float *partial) {
  ConvBwdWeight<KS, TR> pw;
  pw.g = g;
  pw.dout = dout;
  pw.in = in;
  pw.Cin = c.Cin;
  pw.Cout = c.Cout;
  pw.dCin = Div::make(c.Cin);
  pw.chunk = chunk;
  pw.partial = partial;
  gemm(n, pw, ws.M, ws.N, splits, pick_tile_split(ws.M, ws.N));
}

// Of a conv layer, from its output gradient dout (stored masked by the
// layer's ReLU): parts & DGRAD, the data gradient (if din.p), stored masked
// by dmask > 0 (the output of the layer that produced the input) on channels
// >= mc0, no mask when dmask.p is null; parts & WGRAD, the weight and bias
// gradients (on the side stream between side_begin and side_end).
constexpr int DGRAD = 1, WGRAD = 2;
template <int KS, bool RELU>
int conv_bwd_t(ws_net *n, const Conv &c, Img g, View<const bf16> in, View<const bf16> dout, View<bf16> din,
               View<const bf16> dmask, int mc0, int parts = DGRAD | WGRAD) {
  const int P = g.B * g.H * g.W;
  const int Kw = KS * KS * c.Cin;
  const bool wdirect = KS == 3 && RELU && direct_ok(n, g, c.Cin, c.Cout, true);
  const bool ddirect = din.p && KS == 3 && RELU && direct_ok(n, g, c.Cout, c.Cin, false);
  if (din.p && (parts & DGRAD)) {
    if (ddirect) {
      DConv pd{};
      pd.g = g;
      pd.T = DTiles::make(g.B, g.H, g.W);
      pd.dx = dout;
      pd.Kc = c.Cout;
      pd.Nc = c.Cin;
      pd.Wk = c.WtT;
      pd.dy = din;
      pd.dmask = dmask;
      pd.mc0 = mc0;
      launch_dconv<true, false>(n, pd);
    } else {
      ConvBwdData<KS> pd;
      pd.g = g;
      pd.dout = dout;
      pd.Cin = c.Cin;
      pd.Cout = c.Cout;
      pd.WtT = c.WtT;
      pd.din = din;
      pd.mask = dmask;
      pd.mc0 = mc0;
      pd.dCout = Div::make(c.Cout);
      gemm(n, pd, P, c.Cin, 1, pick_tile(P, c.Cin, 0));
    }
  }
  if (!(parts & WGRAD)) return WS_OK;
  const hipStream_t wst = n->on_side ? n->side : n->stream;
  if (wdirect) {
    DWGrad pw{};
    pw.g = g;
    pw.T = DTiles::make(g.B, g.H, g.W);
    pw.dout = dout;
    pw.in = in;
    pw.Cin = c.Cin;
    pw.Cout = c.Cout;
    int splits;
    direct_wplan(pw.T.n, c.Cin, c.Cout, splits, pw.tps);
    pw.partial = take_partials(n, splits, c.Cout, Kw);
    if (!pw.partial) return fail(WS_EINVAL, "split scratch too small");
    const int hw = direct_whw(c.Cin);
    const dim3 grid((unsigned)splits, (unsigned)(c.Cout / 32), (unsigned)std::max(1, c.Cin / (16 * hw)));
    if (hw == 1) hipLaunchKernelGGL((k_dwgrad<true, 1>), grid, dim3(128), 0, wst, pw);
    else if (hw == 2) hipLaunchKernelGGL((k_dwgrad<false, 2>), grid, dim3(256), 0, wst, pw);
    else hipLaunchKernelGGL((k_dwgrad<false, 4>), grid, dim3(512), 0, wst, pw);
    queue_split_reduce(n, pw.partial, splits, c.Cout, Kw, n->grads + c.w_off, n->grads + c.b_off, c.Cout);
  } else {
    const WShape ws = wshape(c.Cout, Kw + 1);
    int splits, chunk;
    split_plan(P, ws.M, ws.N, splits, chunk);
    float *part = take_partials(n, splits, c.Cout, Kw);
    if (!part) return fail(WS_EINVAL, "split scratch too small");
    if (ws.tr) conv_bwd_weight<KS, true>(n, c, g, in, dout, chunk, splits, ws, part);
    else conv_bwd_weight<KS, false>(n, c, g, in, dout, chunk, splits, ws, part);
    queue_split_reduce(n, part, splits, c.Cout, Kw, n->grads + c.w_off, n->grads + c.b_off, c.Cout);
  }
  return WS_OK;
}

// The direct up-sampling forward serves input rows that are whole 32-pixel
// segments with Cout of 32, 64 or 128; the implicit GEMM covers the rest,
// both up-sampling gradients, and conv_algo = 1.
bool up_direct_fwd(const ws_net *n, const Img &gin, const Up &u) {
  return n->cfg.conv_algo == 0 && gin.W % 32 == 0 && (u.Cout == 32 || u.Cout == 64 || u.Cout == 128) &&
         u.Cin % 32 == 0;
}

int up_fwd(ws_net *n, const Up &u, Img gin, View<const bf16> in, View<bf16> out) {
  if (up_direct_fwd(n, gin, u)) {
    DUp p{};
    p.g = gin;
    p.segs = gin.W / 32;
    p.Cin = u.Cin;
    p.Cout = u.Cout;
    p.in = in;
    p.Wt = u.Wt;
    p.bias = n->params + u.b_off;
    p.out = out;
    const dim3 grid((unsigned)(gin.B * gin.H * p.segs));
    if (u.Cout == 32) hipLaunchKernelGGL(k_upfwd<2>, grid, dim3(256), 0, n->stream, p);
    else if (u.Cout == 64) hipLaunchKernelGGL(k_upfwd<4>, grid, dim3(256), 0, n->stream, p);
    else hipLaunchKernelGGL(k_upfwd<8>, grid, dim3(256), 0, n->stream, p);
    return WS_OK;
  }
  UpFwd p;
  p.g = gin;
  p.in = in;
  p.Cin = u.Cin;
  p.Cout = u.Cout;
  p.Wt = u.Wt;
  p.bias = n->params + u.b_off;
  p.out = out;
  const int Pin = gin.B * gin.H * gin.W;
  p.dPin = Div::make(Pin);
  gemm(n, p, 4 * Pin, u.Cout, 1, pick_tile(4 * Pin, u.Cout, Pin));
  return WS_OK;
}

// Direct up-sampling weight gradient: input rows of whole 32-pixel segments,
// Cout and Cin multiples of 32.  Split plan: about 4096 waves in all.
bool up_direct_wgrad(const ws_net *n, const Img &gin, const Up &u) {
  return n->cfg.conv_algo == 0 && gin.W % 32 == 0 && u.Cout % 32 == 0 && u.Cin % 32 == 0;
}
void up_wplan(const Img &gin, const Up &u, int &hw, int &splits, int &ipb) {
  hw = u.Cin % 64 == 0 ? 4 : 2;
  const int items = (gin.B * gin.H * (gin.W / 32) + 3) / 4;
  const int combos = 4 * (u.Cout / 32) * (u.Cin / (16 * hw));
  const int want = std::max(1, 4096 / (2 * hw) / combos);  // 2048, 8192, 16384 waves measured slower
  ipb = std::max(1, (items + want - 1) / want);
  splits = (items + ipb - 1) / ipb;
}

int up_bwd(ws_net *n, const Up &u, Img gin, View<const bf16> in, View<const bf16> dout, View<bf16> din,
           int parts = DGRAD | WGRAD) {
  const int P = gin.B * gin.H * gin.W;
  const hipStream_t wst = n->on_side ? n->side : n->stream;
  if (!(parts & WGRAD)) {
  } else if (up_direct_wgrad(n, gin, u)) {
    DUpW pw{};
    pw.g = gin;
    pw.segs = gin.W / 32;
    pw.nseg = gin.B * gin.H * pw.segs;
    pw.dout = dout;
    pw.in = in;
    pw.Cin = u.Cin;
    pw.Cout = u.Cout;
    int hw, splits;
    up_wplan(gin, u, hw, splits, pw.ipb);
    pw.partial = take_partials(n, splits, 4 * u.Cout, u.Cin);
    if (!pw.partial) return fail(WS_EINVAL, "split scratch too small");
    const dim3 grid((unsigned)splits, (unsigned)(4 * u.Cout / 32), (unsigned)(u.Cin / (16 * hw)));
    if (hw == 4) hipLaunchKernelGGL(k_upwgrad<4>, grid, dim3(512), 0, wst, pw);
    else hipLaunchKernelGGL(k_upwgrad<2>, grid, dim3(256), 0, wst, pw);
    queue_split_reduce(n, pw.partial, splits, 4 * u.Cout, u.Cin, n->grads + u.w_off, n->grads + u.b_off, u.Cout);
  } else {
    int splits, chunk;
    split_plan(P, 4 * u.Cout, u.Cin + 1, splits, chunk);
    UpBwdWeight pw;
    pw.g = gin;
    pw.dout = dout;
    pw.in = in;
    pw.Cin = u.Cin;
    pw.Cout = u.Cout;
    pw.chunk = chunk;
    pw.partial = take_partials(n, splits, 4 * u.Cout, u.Cin);
    if (!pw.partial) return fail(WS_EINVAL, "split scratch too small");
    pw.dCout = Div::make(u.Cout);
    gemm(n, pw, 4 * u.Cout, u.Cin + 1, splits, pick_tile_split(4 * u.Cout, u.Cin + 1));
    queue_split_reduce(n, pw.partial, splits, 4 * u.Cout, u.Cin, n->grads + u.w_off, n->grads + u.b_off, u.Cout);
  }
  if (!(parts & DGRAD)) return WS_OK;
  UpBwdData pd;
  pd.g = gin;
  pd.dout = dout;
  pd.Cin = u.Cin;
  pd.Cout = u.Cout;
  pd.WtT = u.WtT;
  pd.din = din;
  pd.mask = in;  // the up-sampling input is a ReLU output: its gradient is stored masked
  pd.dCout = Div::make(u.Cout);
  gemm(n, pd, P, u.Cin, 1, pick_tile(P, u.Cin, 0));
  return WS_OK;
}

template <typename T>
View<const T> cv(const Buf<T> &b, int coff = 0) { return View<const T>{b.p, b.cs, coff}; }
template <typename T>
View<T> mv(Buf<T> &b, int coff = 0) { return View<T>{b.p, b.cs, coff}; }

// The fused training head (k_head) serves conv_algo 0 with at most 256 head
// input channels; else the head, loss and head gradients are separate kernels.
bool head_fused(const ws_net *n) { return n->cfg.conv_algo == 0 && n->C0 <= 256; }
int head_nt(int C0) {
  int nt = 1;
  while (16 * nt < C0) nt *= 2;
  return nt;
}
// Runs of 256 pixels over at most 1024 blocks (4 waves per SIMD; 256 and 512
// blocks measured 45 and 33 us against 30 at 3x128x256, batch 16; 2048
// slowed the split sum of the 2048 partials).
void head_plan(int P, int &grid, int &rpb) {
  const int runs = (P + 255) / 256;
  grid = std::min(1024, runs);
  rpb = (runs + grid - 1) / grid;
  grid = (runs + rpb - 1) / rpb;
}

// head = false: stops before the head (the training head computes it)
int forward(ws_net *n, const float *x, int B, bool head = true) {
  const int L = n->L;
  const int P0 = B * n->cfg.H * n->cfg.W;
  hipLaunchKernelGGL(k_pack_input, dim3(blocks(P0)), dim3(256), 0, n->stream, x, P0, n->cfg.cin, n->xin.p);
  for (int l = 0; l < L; ++l) {
    Img g = Img::make(B, imgH(n, l), imgW(n, l));
    const int C = chans(n, l);
    View<const bf16> in = l == 0 ? cv(n->xin) : cv(n->pool[l]);
    int rc = conv_fwd(n, n->e1[l], g, in, mv(n->mid_e[l]));
    if (rc) return rc;
    View<bf16> eout = l < L - 1 ? mv(n->cat[l], C) : mv(n->bott);
    bool pooled = false;
    rc = conv_fwd(n, n->e2[l], g, cv(n->mid_e[l]), eout, l < L - 1 ? mv(n->pool[l + 1]) : View<bf16>{nullptr, 0, 0},
                  &pooled, l < L - 1 ? n->parg[l + 1].p : nullptr);
    if (rc) return rc;
    if (l < L - 1) n->pool_fused[l + 1] = pooled;
    if (l < L - 1 && !pooled) {
      const int64_t cnt = (int64_t)B * (g.H / 2) * (g.W / 2) * (C / 8);  // 8 channels per thread
      hipLaunchKernelGGL(k_pool_fwd, dim3(blocks(cnt)), dim3(256), 0, n->stream, g,
                         View<const bf16>{eout.p, eout.cs, eout.coff}, C, mv(n->pool[l + 1]));
    }
  }
  for (int l = L - 2; l >= 0; --l) {
    Img gl = Img::make(B, imgH(n, l), imgW(n, l)), gu = Img::make(B, imgH(n, l + 1), imgW(n, l + 1));
    View<const bf16> uin = l == L - 2 ? cv(n->bott) : cv(n->dec[l + 1]);
    int rc = up_fwd(n, n->up[l], gu, uin, mv(n->cat[l], 0));
    if (rc) return rc;
    rc = conv_fwd(n, n->d1[l], gl, cv(n->cat[l]), mv(n->mid_d[l]));
    if (rc) return rc;
    rc = conv_fwd(n, n->d2[l], gl, cv(n->mid_d[l]), mv(n->dec[l]));
    if (rc) return rc;
  }
  if (head) {
    Img g0 = Img::make(B, n->cfg.H, n->cfg.W);
    int rc = conv_fwd_t<1, false, true>(n, n->head, g0, cv(n->dec[0]), View<bf16>{nullptr, 0, 0}, mv(n->y));
    if (rc) return rc;
  }
  HTRY(hipGetLastError());
  return WS_OK;
}

// Loss (into n->loss) and all gradients, after forward(n, x, B, !head_fused(n)).
int backward(ws_net *n, const float *target, int B) {
  const int L = n->L;
  if (int e = side_join(n)) return e;  // a pass that ended early may have left work on the side stream
  n->jobs.clear();
  n->scratch_used = 0;
  Img g0 = Img::make(B, n->cfg.H, n->cfg.W);
  const int P = B * n->cfg.H * n->cfg.W;
  int rc = WS_OK, nlb;
  if (head_fused(n)) {
    DHead h{};
    h.P = P;
    h.C0 = n->C0;
    h.cout = n->cfg.cout;
    h.act = cv(n->dec[0]);
    h.W = n->head.Wt;
    h.bias = n->params + n->head.b_off;
    h.t = target;
    h.Pc = (float)((double)P * n->cfg.cout);
    h.dact = mv(n->ddec[0]);
    h.loss = n->loss_part;
    int grid;
    head_plan(P, grid, h.rpb);
    h.partial = take_partials(n, grid, 8, n->C0);
    if (!h.partial) return fail(WS_EINVAL, "split scratch too small");
    const int nt = head_nt(n->C0);
    const size_t lds = head_lds_bytes(n->C0, nt);
    switch (nt) {
#define WS_HEAD(NT)                                                                                   \
  case NT:                                                                                            \
    if (lds > 65536 && !n->head_lds_set) { /* once: more than the default dynamic LDS */             \
      HTRY(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_head<NT>),                           \
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));                \
      n->head_lds_set = true;                                                                         \
    }                                                                                                 \
    hipLaunchKernelGGL(k_head<NT>, dim3(grid), dim3(256), lds, n->stream, h);                         \
    break;
      WS_HEAD(1) WS_HEAD(2) WS_HEAD(4) WS_HEAD(8) WS_HEAD(16)
#undef WS_HEAD
      default: return fail(WS_EINVAL, "head input channels beyond 256");
    }
    queue_split_reduce(n, h.partial, grid, 8, n->C0, n->grads + n->head.w_off, n->grads + n->head.b_off, 8);
    nlb = grid;
  } else {
    nlb = (int)blocks(P);
    hipLaunchKernelGGL(k_mse, dim3(nlb), dim3(256), 0, n->stream, n->y.p, target, P, n->cfg.cout, n->dy.p,
                       n->loss_part);
    rc = conv_bwd_t<1, false>(n, n->head, g0, cv(n->dec[0]), cv(n->dy), mv(n->ddec[0]), cv(n->dec[0]), 0);
    if (rc) return rc;
  }
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1024), 0, n->stream, n->loss_part, nlb,
                     1.0 / ((double)P * n->cfg.cout), n->loss);
  // Each level's data gradients run on the network's stream; once they have
  // made the level's output gradients final, one fork runs its weight
  // gradients on the side stream (one event per level, not per layer: each
  // costs the network's stream about 6 us; 1.146 -> 1.121 ms per step).
  const View<const bf16> none{nullptr, 0, 0};
  for (int l = 0; l <= L - 2; ++l) {
    Img gl = Img::make(B, imgH(n, l), imgW(n, l)), gu = Img::make(B, imgH(n, l + 1), imgW(n, l + 1));
    rc = conv_bwd_t<3, true>(n, n->d2[l], gl, cv(n->mid_d[l]), cv(n->ddec[l]), mv(n->dmid_d[l]), cv(n->mid_d[l]), 0,
                             DGRAD);
    if (rc) return rc;
    // the concatenation [up-sampled | skip]: only the skip part is a ReLU output
    rc = conv_bwd_t<3, true>(n, n->d1[l], gl, cv(n->cat[l]), cv(n->dmid_d[l]), mv(n->dcat[l]), cv(n->cat[l]),
                             n->up[l].Cout, DGRAD);
    if (rc) return rc;
    View<const bf16> uin = l == L - 2 ? cv(n->bott) : cv(n->dec[l + 1]);
    View<bf16> dup = l == L - 2 ? mv(n->dbott) : mv(n->ddec[l + 1]);
    if ((rc = side_begin(n, side_mark(n)))) return rc;
    rc = conv_bwd_t<3, true>(n, n->d2[l], gl, cv(n->mid_d[l]), cv(n->ddec[l]), View<bf16>{nullptr, 0, 0}, none, 0,
                             WGRAD);
    if (!rc) rc = conv_bwd_t<3, true>(n, n->d1[l], gl, cv(n->cat[l]), cv(n->dmid_d[l]), View<bf16>{nullptr, 0, 0},
                                      none, 0, WGRAD);
    if (!rc) rc = up_bwd(n, n->up[l], gu, uin, cv(n->dcat[l], 0), dup, WGRAD);
    side_end(n);
    if (rc) return rc;
    rc = up_bwd(n, n->up[l], gu, uin, cv(n->dcat[l], 0), dup, DGRAD);
    if (rc) return rc;
  }
  // the head's and decoder's sums, on the side stream after their weight
  // gradients, beside the encoder's gradients
  if (n->side_pending) flush_split_reduce(n, true);
  for (int l = L - 1; l >= 0; --l) {
    Img g = Img::make(B, imgH(n, l), imgW(n, l));
    const int C = chans(n, l);
    View<const bf16> deout = l < L - 1 ? cv(n->dcat[l], C) : cv(n->dbott);
    rc = conv_bwd_t<3, true>(n, n->e2[l], g, cv(n->mid_e[l]), deout, mv(n->dmid_e[l]), cv(n->mid_e[l]), 0, DGRAD);
    if (rc) return rc;
    View<const bf16> in = l == 0 ? cv(n->xin) : cv(n->pool[l]);
    View<bf16> din = l == 0 ? View<bf16>{nullptr, 0, 0} : mv(n->dpool[l]);
    // level 0's weight gradients end the pass: on the network's stream
    if (l > 0 && (rc = side_begin(n, side_mark(n)))) return rc;
    rc = conv_bwd_t<3, true>(n, n->e2[l], g, cv(n->mid_e[l]), deout, View<bf16>{nullptr, 0, 0}, none, 0, WGRAD);
    if (!rc) rc = conv_bwd_t<3, true>(n, n->e1[l], g, in, cv(n->dmid_e[l]), View<bf16>{nullptr, 0, 0}, none, 0, WGRAD);
    side_end(n);
    if (rc) return rc;
    // the pooled input is no ReLU output: the pooling backward applies the mask
    rc = conv_bwd_t<3, true>(n, n->e1[l], g, in, cv(n->dmid_e[l]), din, View<const bf16>{nullptr, 0, 0}, 0, DGRAD);
    if (rc) return rc;
    if (l > 0) {  // route the pooled gradient into the level l-1 encoder output
      Img gp = Img::make(B, imgH(n, l - 1), imgW(n, l - 1));
      const int Cp = chans(n, l - 1);
      const int64_t cnt = (int64_t)B * g.H * g.W * Cp;
      if (n->pool_fused[l])
        hipLaunchKernelGGL(k_pool_bwd_arg, dim3(blocks(cnt)), dim3(256), 0, n->stream, gp,
                           (const uint8_t *)n->parg[l].p, Cp, cv(n->dpool[l]), mv(n->dcat[l - 1], Cp));
      else
        hipLaunchKernelGGL(k_pool_bwd, dim3(blocks(cnt)), dim3(256), 0, n->stream, gp, cv(n->cat[l - 1], Cp), Cp,
                           cv(n->dpool[l]), mv(n->dcat[l - 1], Cp));
    }
  }
  rc = side_join(n);
  if (rc) return rc;
  flush_split_reduce(n);
  HTRY(hipGetLastError());
  return WS_OK;
}

int check_batch(const ws_net *n, int B) {
  if (B < 1 || B > n->cfg.max_batch) return fail(WS_EINVAL, "batch %d outside 1..%d", B, n->cfg.max_batch);
  return WS_OK;
}

}  // namespace

extern "C" {

int ws_create(const ws_config *c, void *hip_stream, ws_net **out) {
  if (!c || !out) return fail(WS_EINVAL, "NULL argument");
  *out = nullptr;
  if (c->levels < 2 || c->levels > 6) return fail(WS_EINVAL, "levels must be 2..6");
  if (c->base < 8 || c->base % 8) return fail(WS_EINVAL, "base channels must be a multiple of 8");
  if (c->cin < 1 || c->cin > 8 || c->cout < 1 || c->cout > 8) return fail(WS_EINVAL, "cin, cout must be 1..8");
  if (c->max_batch < 1) return fail(WS_EINVAL, "max_batch must be >= 1");
  if (c->conv_algo < 0 || c->conv_algo > 1) return fail(WS_EINVAL, "conv_algo must be 0 or 1");
  const int div = 1 << (c->levels - 1);
  if (c->H % div || c->W % div) return fail(WS_EINVAL, "H and W must be divisible by 2^(levels-1)");
  // the up-sampling GEMM keeps one output parity per 64-row tile
  const int64_t Plow = (int64_t)(c->H / div) * (c->W / div);
  if (Plow % 64) return fail(WS_EINVAL, "lowest level must hold a multiple of 64 pixels");
  // element indices of the largest activation buffer ([up | skip] at level 0) are 32-bit
  if ((int64_t)c->max_batch * c->H * c->W * std::max(2 * c->base, 8) >= (1LL << 31))
    return fail(WS_EINVAL, "max_batch * H * W * 2 * base must stay below 2^31");
  ws_net *n = new (std::nothrow) ws_net();
  if (!n) return fail(WS_ENOMEM, "host allocation failed");
  n->cfg = *c;
  n->L = c->levels;
  n->C0 = c->base;
  n->stream = (hipStream_t)hip_stream;
  {
    bool ok = hipStreamCreateWithFlags(&n->side, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&n->ev_join, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; ok && i < 64; ++i) {
      hipEvent_t e;
      ok = hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
      if (ok) n->evs.push_back(e);
    }
    if (!ok) {
      ws_destroy(n);
      return fail(WS_EDEVICE, "stream or event creation failed");
    }
  }
  const int L = n->L;
  int64_t off = 0;
  for (int l = 0; l < L; ++l) {
    const int C = chans(n, l), Cin = l == 0 ? 8 : chans(n, l - 1);
    n->e1.push_back(make_conv(off, 3, Cin, C, true));
    n->e2.push_back(make_conv(off, 3, C, C, true));
  }
  n->up.resize(L - 1);
  n->d1.resize(L - 1);
  n->d2.resize(L - 1);
  for (int l = L - 2; l >= 0; --l) {
    const int C = chans(n, l);
    n->up[l] = make_up(off, chans(n, l + 1), C);
    n->d1[l] = make_conv(off, 3, 2 * C, C, true);
    n->d2[l] = make_conv(off, 3, C, C, true);
  }
  n->head = make_conv(off, 1, n->C0, 8, false);
  n->np = off;
  int rc = WS_OK;
  rc = rc ? rc : dalloc(n, &n->params, n->np);
  rc = rc ? rc : dalloc(n, &n->grads, n->np);
  rc = rc ? rc : dalloc(n, &n->m, n->np);
  rc = rc ? rc : dalloc(n, &n->v, n->np);
  auto wcopies = [&](bf16 *&Wt, bf16 *&WtT, int64_t nw) {
    if (!rc) rc = dalloc(n, &Wt, nw);
    if (!rc) rc = dalloc(n, &WtT, nw);
  };
  for (auto &x : n->e1) wcopies(x.Wt, x.WtT, x.nw());
  for (auto &x : n->e2) wcopies(x.Wt, x.WtT, x.nw());
  for (auto &x : n->d1) wcopies(x.Wt, x.WtT, x.nw());
  for (auto &x : n->d2) wcopies(x.Wt, x.WtT, x.nw());
  for (auto &x : n->up) wcopies(x.Wt, x.WtT, x.nw());
  wcopies(n->head.Wt, n->head.WtT, n->head.nw());
  // activations and gradients
  n->pool.resize(L);
  n->parg.resize(L);
  n->pool_fused.assign(L, 0);
  n->dpool.resize(L);
  n->mid_e.resize(L);
  n->dmid_e.resize(L);
  n->cat.resize(L);
  n->dcat.resize(L);
  n->mid_d.resize(L);
  n->dmid_d.resize(L);
  n->dec.resize(L);
  n->ddec.resize(L);
  if (!rc) rc = buf(n, n->xin, 0, 8);
  for (int l = 0; l < L && !rc; ++l) {
    const int C = chans(n, l);
    if (l > 0) {
      rc = buf(n, n->pool[l], l, chans(n, l - 1));
      if (!rc) rc = buf(n, n->parg[l], l, chans(n, l - 1));
      if (!rc) rc = buf(n, n->dpool[l], l, chans(n, l - 1));
    }
    if (!rc) rc = buf(n, n->mid_e[l], l, C);
    if (!rc) rc = buf(n, n->dmid_e[l], l, C);
    if (l < L - 1) {
      if (!rc) rc = buf(n, n->cat[l], l, 2 * C);
      if (!rc) rc = buf(n, n->dcat[l], l, 2 * C);
      if (!rc) rc = buf(n, n->mid_d[l], l, C);
      if (!rc) rc = buf(n, n->dmid_d[l], l, C);
      if (!rc) rc = buf(n, n->dec[l], l, C);
      if (!rc) rc = buf(n, n->ddec[l], l, C);
    }
  }
  if (!rc) rc = buf(n, n->bott, L - 1, chans(n, L - 1));
  if (!rc) rc = buf(n, n->dbott, L - 1, chans(n, L - 1));
  if (!rc) rc = buf(n, n->y, 0, 8);
  if (!rc) rc = buf(n, n->dy, 0, 8);
  // split partials of all weight gradients of one backward pass (each layer
  // keeps its own range until the pass ends); per layer the larger of the
  // implicit-GEMM and the direct plan, the most over batch sizes
  size_t worst = 0;
  for (int B = 1; B <= c->max_batch; ++B) {  // splits depend on the batch
    size_t total = 0;
    auto gemm_need = [&](int l, int M, int N) {
      int splits, chunk;
      split_plan(B * imgH(n, l) * imgW(n, l), M, N, splits, chunk);
      return (size_t)splits * M * N;
    };
    auto conv = [&](int lv, const Conv &cv) {
      const WShape w = wshape(cv.Cout, cv.KS * cv.KS * cv.Cin + 1);
      size_t need = gemm_need(lv, w.M, w.N);
      const Img g = Img::make(B, imgH(n, lv), imgW(n, lv));
      if (cv.KS == 3 && cv.relu && direct_ok(n, g, cv.Cin, cv.Cout, true)) {
        int splits, tps;
        direct_wplan(DTiles::make(B, g.H, g.W).n, cv.Cin, cv.Cout, splits, tps);
        need = std::max(need, (size_t)splits * cv.Cout * (cv.KS * cv.KS * cv.Cin + 1));
      }
      total += need;
    };
    for (int l = 0; l < L; ++l) {
      conv(l, n->e1[l]);
      conv(l, n->e2[l]);
      if (l < L - 1) {
        conv(l, n->d1[l]);
        conv(l, n->d2[l]);
        const Up &u = n->up[l];
        size_t need = gemm_need(l + 1, 4 * u.Cout, u.Cin + 1);  // over the input (coarser) pixels
        const Img gu = Img::make(B, imgH(n, l + 1), imgW(n, l + 1));
        if (up_direct_wgrad(n, gu, u)) {
          int hw, splits, ipb;
          up_wplan(gu, u, hw, splits, ipb);
          need = std::max(need, (size_t)splits * 4 * u.Cout * (u.Cin + 1));
        }
        total += need;
      }
    }
    conv(0, n->head);
    {
      int grid, rpb;
      head_plan(B * c->H * c->W, grid, rpb);
      total += (size_t)grid * 8 * (n->C0 + 1);  // the training head's partials
    }
    worst = std::max(worst, total);
  }
  n->scratch_floats = worst;
  if (!rc) rc = dalloc(n, &n->scratch, worst);
  n->n_loss_blocks = (int)blocks((int64_t)c->max_batch * c->H * c->W);  // k_mse: a pixel per thread
  if (!rc) rc = dalloc(n, &n->loss_part, n->n_loss_blocks);
  if (!rc) rc = dalloc(n, &n->loss, 1);
  if (!rc) {
    hipError_t e = hipStreamSynchronize(n->stream);
    if (e != hipSuccess) rc = fail(WS_EDEVICE, "hipStreamSynchronize: %s", hipGetErrorString(e));
  }
  if (rc) {
    ws_destroy(n);
    return rc;
  }
  *out = n;
  return WS_OK;
}

void ws_destroy(ws_net *n) {
  if (!n) return;
  if (n->stream) (void)hipStreamSynchronize(n->stream);
  else (void)hipDeviceSynchronize();
  if (n->side) {
    (void)hipStreamSynchronize(n->side);
    (void)hipStreamDestroy(n->side);
  }
  for (hipEvent_t e : n->evs) (void)hipEventDestroy(e);
  if (n->ev_join) (void)hipEventDestroy(n->ev_join);
  for (void *p : n->allocs) (void)hipFree(p);
  delete n;
}

int64_t ws_num_params(const ws_net *n) { return n ? n->np : -1; }
int64_t ws_device_bytes(const ws_net *n) { return n ? n->bytes : -1; }

int ws_set_params(ws_net *n, const float *host, int64_t count) {
  if (!n || !host) return fail(WS_EINVAL, "NULL argument");
  if (count != n->np) return fail(WS_EINVAL, "expected %lld parameters", (long long)n->np);
  HTRY(hipMemcpyAsync(n->params, host, sizeof(float) * count, hipMemcpyHostToDevice, n->stream));
  HTRY(hipMemsetAsync(n->m, 0, sizeof(float) * count, n->stream));
  HTRY(hipMemsetAsync(n->v, 0, sizeof(float) * count, n->stream));
  n->adam_t = 0;
  int rc = refresh_weights(n);
  if (rc) return rc;
  HTRY(hipStreamSynchronize(n->stream));
  return WS_OK;
}

int ws_get_params(ws_net *n, float *host, int64_t count) {
  if (!n || !host || count != n->np) return fail(WS_EINVAL, "bad arguments");
  HTRY(hipMemcpyAsync(host, n->params, sizeof(float) * count, hipMemcpyDeviceToHost, n->stream));
  HTRY(hipStreamSynchronize(n->stream));
  return WS_OK;
}

int ws_get_grads(ws_net *n, float *host, int64_t count) {
  if (!n || !host || count != n->np) return fail(WS_EINVAL, "bad arguments");
  HTRY(hipMemcpyAsync(host, n->grads, sizeof(float) * count, hipMemcpyDeviceToHost, n->stream));
  HTRY(hipStreamSynchronize(n->stream));
  return WS_OK;
}

int ws_forward(ws_net *n, const float *x, int32_t batch, float *y) {
  if (!n || !x || !y) return fail(WS_EINVAL, "NULL argument");
  int rc = check_batch(n, batch);
  if (rc) return rc;
  rc = forward(n, x, batch);
  if (rc) return rc;
  const int P = batch * n->cfg.H * n->cfg.W;
  hipLaunchKernelGGL(k_unpack_output, dim3(blocks((int64_t)P * n->cfg.cout)), dim3(256), 0, n->stream, n->y.p, 8, P,
                     n->cfg.cout, y);
  HTRY(hipGetLastError());
  return WS_OK;
}

int ws_backward(ws_net *n, const float *x, const float *target, int32_t batch, double *loss) {
  if (!n || !x || !target) return fail(WS_EINVAL, "NULL argument");
  int rc = check_batch(n, batch);
  if (rc) return rc;
  rc = forward(n, x, batch, !head_fused(n));
  if (rc) return rc;
  rc = backward(n, target, batch);
  if (rc) return rc;
  if (loss) {
    HTRY(hipMemcpyAsync(loss, n->loss, sizeof(double), hipMemcpyDeviceToHost, n->stream));
    HTRY(hipStreamSynchronize(n->stream));
  }
  return WS_OK;
}

int ws_adam(ws_net *n, float lr, float beta1, float beta2, float eps, float weight_decay) {
  if (!n) return fail(WS_EINVAL, "NULL network");
  n->adam_t += 1;
  const float c1 = 1.f - powf(beta1, (float)n->adam_t), c2 = 1.f - powf(beta2, (float)n->adam_t);
  hipLaunchKernelGGL(k_adam, dim3(blocks(n->np)), dim3(256), 0, n->stream, n->params, n->grads, n->m, n->v, n->np, lr,
                     beta1, beta2, eps, c1, c2, weight_decay);
  HTRY(hipGetLastError());
  return refresh_weights(n);
}

int ws_train_step(ws_net *n, const float *x, const float *target, int32_t batch, float lr, double *loss) {
  int rc = ws_backward(n, x, target, batch, loss);
  if (rc) return rc;
  return ws_adam(n, lr, 0.9f, 0.999f, 1e-8f, 0.f);
}

int ws_flops(const ws_net *n, int32_t batch, double *fwd, double *bwd) {
  if (!n) return fail(WS_EINVAL, "NULL network");
  double f = 0;
  for (int l = 0; l < n->L; ++l) {
    const double P = (double)batch * imgH(n, l) * imgW(n, l);
    auto conv = [&](const Conv &c) { f += 2.0 * P * c.Cout * c.KS * c.KS * c.Cin; };
    conv(n->e1[l]);
    conv(n->e2[l]);
    if (l < n->L - 1) {
      conv(n->d1[l]);
      conv(n->d2[l]);
      f += 2.0 * P * n->up[l].Cout * n->up[l].Cin;  // each output pixel: Cin MACs per channel
    }
  }
  f += 2.0 * batch * n->cfg.H * n->cfg.W * 8 * n->C0;
  if (fwd) *fwd = f;
  if (bwd) *bwd = 2.0 * f;
  return WS_OK;
}

int ws_malloc(int64_t bytes, void **p) {
  if (!p || bytes < 0) return fail(WS_EINVAL, "bad arguments");
  hipError_t e = hipMalloc(p, bytes ? bytes : 1);
  if (e != hipSuccess) return fail(WS_ENOMEM, "hipMalloc: %s", hipGetErrorString(e));
  return WS_OK;
}

int ws_free(void *p) {
  HTRY(hipFree(p));
  return WS_OK;
}

int ws_memcpy(void *dst, const void *src, int64_t bytes, int32_t kind) {
  if (bytes < 0) return fail(WS_EINVAL, "negative size");
  if (kind < 0 || kind > 2) return fail(WS_EINVAL, "copy kind must be 0, 1 or 2");
  const hipMemcpyKind k = kind == 0 ? hipMemcpyHostToDevice : kind == 1 ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
  HTRY(hipDeviceSynchronize());  // after work queued on any stream
  HTRY(hipMemcpy(dst, src, bytes, k));
  return WS_OK;
}

int ws_sync(void) {
  HTRY(hipDeviceSynchronize());
  return WS_OK;
}

const char *ws_last_error(void) { return g_err.c_str(); }

}  // extern "C"
