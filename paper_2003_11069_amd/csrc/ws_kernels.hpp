// ws_kernels.hpp -- HIP kernels (gfx950) of the learned warm start: a U-Net
// (3x3 convolutions + ReLU, 2x2 max pooling, 2x2 stride-2 transposed
// convolutions, skip concatenation, 1x1 head) trained with MSE and Adam.
//
// All convolutions are implicit GEMMs on v_mfma_f32_16x16x32_bf16 (BF16
// operands, FP32 accumulation).  Lane layout of that instruction (verified on
// the device): lane l holds A[l%16][8(l/16)..+7], B[8(l/16)..+7][l%16] and
// receives D[4(l/16)+r][l%16], r = 0..3.
//
// Layout: activations NHWC BF16 with an explicit channel stride and offset
// (a decoder input is one buffer holding [up-sampled | skip] channels),
// gradients NHWC FP32, weights BF16 copies of FP32 master parameters.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wsk {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f4;
typedef __bf16 bf16;

constexpr int BM = 64, BN = 64, BK = 32;  // block tile (M x N), K step
constexpr int LDK = BK + 8;               // LDS row stride (bf16), 80 bytes

__device__ __forceinline__ bf16x8 zero8() {
  bf16x8 z;
  for (int j = 0; j < 8; ++j) z[j] = (bf16)0.f;
  return z;
}

// NHWC tensor view: element (pixel p, channel c) at p*cs + coff + c.
template <typename T>
struct View {
  T *p;
  int cs, coff;
};

struct Img {
  int B, H, W;
  __device__ __forceinline__ int P() const { return B * H * W; }
};

// ---------------------------------------------------------------------------
// GEMM engine: C[M,N] = sum_k A[m,k] B[k,n].  The problem fills the LDS tiles
// As[64][LDK] (row m, k contiguous) and Bs[64][LDK] (column n, k contiguous)
// for the tile (m0, n0, k0) and consumes the accumulators in store().  K may
// be split over gridDim.z (problem decides the range of each split).
template <class P>
__global__ __launch_bounds__(256) void k_gemm(P prob) {
  __shared__ __attribute__((aligned(16))) bf16 As[BM][LDK];
  __shared__ __attribute__((aligned(16))) bf16 Bs[BN][LDK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  int kbeg, kend;
  prob.krange(blockIdx.z, kbeg, kend);
  f4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    prob.fill_a(As, m0, k0, kend, tid);
    prob.fill_b(Bs, n0, k0, kend, tid);
    __syncthreads();
    const int r = lane & 15, kq = 8 * (lane >> 4);
    bf16x8 a[2], b[2];
    for (int i = 0; i < 2; ++i) a[i] = *reinterpret_cast<const bf16x8 *>(&As[wm + 16 * i + r][kq]);
    for (int j = 0; j < 2; ++j) b[j] = *reinterpret_cast<const bf16x8 *>(&Bs[wn + 16 * j + r][kq]);
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + q;
        const int n = n0 + wn + 16 * j + (lane & 15);
        prob.store(m, n, acc[i][j][q], blockIdx.z);
      }
}

// Default tile fill: each of 256 threads writes 8 consecutive k of one row,
// obtained from row8(row, k) (zero beyond the matrix).
template <bool IS_A, class P>
__device__ __forceinline__ void fill_rows(const P &p, bf16 (*S)[LDK], int r0, int k0, int kend, int tid) {
  const int row = tid >> 2, kq = (tid & 3) * 8;
  const int k = k0 + kq;
  bf16x8 v = zero8();
  if (k < kend) {
    if constexpr (IS_A) v = p.a8(r0 + row, k);
    else v = p.b8(r0 + row, k);
  }
  *reinterpret_cast<bf16x8 *>(&S[row][kq]) = v;
}

// ---------------------------------------------------------------------------
// KSxKS convolution, stride 1, zero padding KS/2, forward:
//   out[p, co] = act( sum_{ky,kx,ci} W[co][(ky*KS+kx)*Cin + ci] in[p + (ky-r, kx-r), ci] + b[co] )
// M = pixels, N = Cout, K = KS*KS*Cin (Cin multiple of 8).
template <int KS, bool RELU, bool OUT_F32>
struct ConvFwd {
  Img g;
  View<const bf16> in;
  int Cin, Cout;
  const bf16 *Wt;   // [Cout][K]
  const float *bias;
  View<bf16> out;      // BF16 output (OUT_F32 = false)
  View<float> outf;    // FP32 output (OUT_F32 = true)
  __device__ __forceinline__ int K() const { return KS * KS * Cin; }
  __device__ __forceinline__ void krange(int, int &b, int &e) const { b = 0; e = K(); }
  __device__ __forceinline__ bf16x8 a8(int m, int k) const {
    if (m >= g.P()) return zero8();
    const int tap = k / Cin, ci = k - tap * Cin;
    const int x = m % g.W, t = m / g.W, y = t % g.H, b = t / g.H;
    const int yy = y + tap / KS - KS / 2, xx = x + tap % KS - KS / 2;
    if (yy < 0 || yy >= g.H || xx < 0 || xx >= g.W) return zero8();
    const int q = (b * g.H + yy) * g.W + xx;
    return *reinterpret_cast<const bf16x8 *>(in.p + (size_t)q * in.cs + in.coff + ci);
  }
  __device__ __forceinline__ bf16x8 b8(int n, int k) const {
    if (n >= Cout) return zero8();
    return *reinterpret_cast<const bf16x8 *>(Wt + (size_t)n * K() + k);
  }
  __device__ __forceinline__ void fill_a(bf16 (*S)[LDK], int m0, int k0, int ke, int tid) const {
    fill_rows<true>(*this, S, m0, k0, ke, tid);
  }
  __device__ __forceinline__ void fill_b(bf16 (*S)[LDK], int n0, int k0, int ke, int tid) const {
    fill_rows<false>(*this, S, n0, k0, ke, tid);
  }
  __device__ __forceinline__ void store(int m, int n, float v, int) const {
    if (m >= g.P() || n >= Cout) return;
    v += bias[n];
    if (RELU) v = v > 0.f ? v : 0.f;
    if (OUT_F32) outf.p[(size_t)m * outf.cs + outf.coff + n] = v;
    else out.p[(size_t)m * out.cs + out.coff + n] = (bf16)v;
  }
};

// Gradient operand of a layer output: dOut (FP32) times the ReLU mask of the
// forward output (act > 0), rounded to BF16 for the MFMA.
template <bool RELU>
__device__ __forceinline__ bf16x8 grad8(const View<const float> &d, const View<const bf16> &act, int q, int c) {
  const float *s = d.p + (size_t)q * d.cs + d.coff + c;
  bf16x8 v;
  if (RELU) {
    const bf16x8 a = *reinterpret_cast<const bf16x8 *>(act.p + (size_t)q * act.cs + act.coff + c);
    for (int j = 0; j < 8; ++j) v[j] = (bf16)((float)a[j] > 0.f ? s[j] : 0.f);
  } else {
    for (int j = 0; j < 8; ++j) v[j] = (bf16)s[j];
  }
  return v;
}

// Backward-data of ConvFwd: dIn[p, ci] = sum_{ky,kx,co} WtT[ci][(ky*KS+kx)*Cout + co]
//   dPre[p + (ky-r, kx-r), co],  WtT = weights flipped in (ky,kx) and transposed.
// M = pixels, N = Cin, K = KS*KS*Cout (Cout multiple of 8).  Writes or adds FP32.
template <int KS, bool RELU>
struct ConvBwdData {
  Img g;
  View<const float> dout;
  View<const bf16> act;  // forward output (ReLU mask)
  int Cin, Cout;
  const bf16 *WtT;  // [Cin][K]
  View<float> din;
  int accumulate;
  __device__ __forceinline__ int K() const { return KS * KS * Cout; }
  __device__ __forceinline__ void krange(int, int &b, int &e) const { b = 0; e = K(); }
  __device__ __forceinline__ bf16x8 a8(int m, int k) const {
    if (m >= g.P()) return zero8();
    const int tap = k / Cout, co = k - tap * Cout;
    const int x = m % g.W, t = m / g.W, y = t % g.H, b = t / g.H;
    const int yy = y + tap / KS - KS / 2, xx = x + tap % KS - KS / 2;
    if (yy < 0 || yy >= g.H || xx < 0 || xx >= g.W) return zero8();
    return grad8<RELU>(dout, act, (b * g.H + yy) * g.W + xx, co);
  }
  __device__ __forceinline__ bf16x8 b8(int n, int k) const {
    if (n >= Cin) return zero8();
    return *reinterpret_cast<const bf16x8 *>(WtT + (size_t)n * K() + k);
  }
  __device__ __forceinline__ void fill_a(bf16 (*S)[LDK], int m0, int k0, int ke, int tid) const {
    fill_rows<true>(*this, S, m0, k0, ke, tid);
  }
  __device__ __forceinline__ void fill_b(bf16 (*S)[LDK], int n0, int k0, int ke, int tid) const {
    fill_rows<false>(*this, S, n0, k0, ke, tid);
  }
  __device__ __forceinline__ void store(int m, int n, float v, int) const {
    if (m >= g.P() || n >= Cin) return;
    float *d = din.p + (size_t)m * din.cs + din.coff + n;
    *d = accumulate ? *d + v : v;
  }
};

// Backward-weight of ConvFwd, split over pixels:
//   dW[co][k] = sum_p dPre[p, co] im2col(in)[p, k],  db[co] = sum_p dPre[p, co]
// (the bias is column k = K of a ones column).  M = Cout, N = K + 1, reduction
// over pixels; split z writes partial[z][m][n] (FP32), summed in fixed order by
// k_split_reduce.  Tiles are filled transposed through LDS: each thread loads
// 8 consecutive channels of one pixel.
template <int KS, bool RELU>
struct ConvBwdWeight {
  Img g;
  View<const float> dout;
  View<const bf16> act;
  View<const bf16> in;
  int Cin, Cout;
  int chunk;          // pixels per split (multiple of BK)
  float *partial;     // [splits][Cout][K+1]
  __device__ __forceinline__ int Kw() const { return KS * KS * Cin; }
  __device__ __forceinline__ void krange(int z, int &b, int &e) const {
    b = z * chunk;
    e = min(g.P(), b + chunk);
  }
  __device__ __forceinline__ void fill_a(bf16 (*S)[LDK], int m0, int k0, int ke, int tid) const {
    const int pl = tid >> 3, cl = (tid & 7) * 8;  // 32 pixels x 64 channels
    const int p = k0 + pl, co = m0 + cl;
    bf16x8 v = (p < ke && co < Cout) ? grad8<RELU>(dout, act, p, co) : zero8();
    for (int j = 0; j < 8; ++j) S[cl + j][pl] = v[j];
  }
  __device__ __forceinline__ void fill_b(bf16 (*S)[LDK], int n0, int k0, int ke, int tid) const {
    const int pl = tid >> 3, nl = (tid & 7) * 8;
    const int p = k0 + pl, n = n0 + nl;
    bf16x8 v = zero8();
    if (p < ke) {
      if (n < Kw()) {
        const int tap = n / Cin, ci = n - tap * Cin;
        const int x = p % g.W, t = p / g.W, y = t % g.H, b = t / g.H;
        const int yy = y + tap / KS - KS / 2, xx = x + tap % KS - KS / 2;
        if (yy >= 0 && yy < g.H && xx >= 0 && xx < g.W)
          v = *reinterpret_cast<const bf16x8 *>(in.p + (size_t)((b * g.H + yy) * g.W + xx) * in.cs + in.coff + ci);
      } else if (n == Kw()) {
        v[0] = (bf16)1.f;
      }
    }
    for (int j = 0; j < 8; ++j) S[nl + j][pl] = v[j];
  }
  __device__ __forceinline__ void store(int m, int n, float v, int z) const {
    if (m >= Cout || n > Kw()) return;
    partial[((size_t)z * Cout + m) * (Kw() + 1) + n] = v;
  }
};

// ---------------------------------------------------------------------------
// 2x2 stride-2 transposed convolution (up-sampling), forward:
//   out[(b, 2y+dy, 2x+dx), co] = sum_ci W[d][co][ci] in[(b,y,x), ci] + b[co], d = 2dy+dx.
// Rows are ordered parity-major, m = d*Pin + p, so a 64-row tile has one
// parity (Pin is a multiple of 64).  M = 4 Pin, N = Cout, K = Cin.
struct UpFwd {
  Img g;  // input image
  View<const bf16> in;
  int Cin, Cout;
  const bf16 *Wt;  // [4][Cout][Cin]
  const float *bias;
  View<bf16> out;  // output image (2H x 2W)
  __device__ __forceinline__ void krange(int, int &b, int &e) const { b = 0; e = Cin; }
  __device__ __forceinline__ bf16x8 a8(int m, int k) const {
    const int Pin = g.P();
    if (m >= 4 * Pin) return zero8();
    const int p = m % Pin;
    return *reinterpret_cast<const bf16x8 *>(in.p + (size_t)p * in.cs + in.coff + k);
  }
  __device__ __forceinline__ void fill_a(bf16 (*S)[LDK], int m0, int k0, int ke, int tid) const {
    fill_rows<true>(*this, S, m0, k0, ke, tid);
  }
  __device__ __forceinline__ void fill_b(bf16 (*S)[LDK], int n0, int k0, int ke, int tid) const {
    const int row = tid >> 2, kq = (tid & 3) * 8;
    const int d = (blockIdx.x * BM) / g.P();
    const int n = n0 + row, k = k0 + kq;
    bf16x8 v = (n < Cout && k < ke) ? *reinterpret_cast<const bf16x8 *>(Wt + ((size_t)d * Cout + n) * Cin + k)
                                    : zero8();
    *reinterpret_cast<bf16x8 *>(&S[row][kq]) = v;
  }
  __device__ __forceinline__ void store(int m, int n, float v, int) const {
    const int Pin = g.P();
    if (m >= 4 * Pin || n >= Cout) return;
    const int d = m / Pin, p = m % Pin;
    const int x = p % g.W, t = p / g.W, y = t % g.H, b = t / g.H;
    const int Y = 2 * y + (d >> 1), X = 2 * x + (d & 1);
    const size_t q = ((size_t)b * 2 * g.H + Y) * 2 * g.W + X;
    out.p[q * out.cs + out.coff + n] = (bf16)(v + bias[n]);
  }
};

// Backward-data of UpFwd: dIn[p, ci] = sum_{d,co} WT[ci][d*Cout + co] dOut[up(p,d), co].
// M = Pin, N = Cin, K = 4 Cout.  No activation on the up-sampling output.
struct UpBwdData {
  Img g;
  View<const float> dout;  // output-image gradient
  int Cin, Cout;
  const bf16 *WtT;  // [Cin][4][Cout]
  View<float> din;
  __device__ __forceinline__ void krange(int, int &b, int &e) const { b = 0; e = 4 * Cout; }
  __device__ __forceinline__ bf16x8 a8(int m, int k) const {
    if (m >= g.P()) return zero8();
    const int d = k / Cout, co = k - d * Cout;
    const int x = m % g.W, t = m / g.W, y = t % g.H, b = t / g.H;
    const int q = (b * 2 * g.H + 2 * y + (d >> 1)) * 2 * g.W + 2 * x + (d & 1);
    const float *s = dout.p + (size_t)q * dout.cs + dout.coff + co;
    bf16x8 v;
    for (int j = 0; j < 8; ++j) v[j] = (bf16)s[j];
    return v;
  }
  __device__ __forceinline__ bf16x8 b8(int n, int k) const {
    if (n >= Cin) return zero8();
    return *reinterpret_cast<const bf16x8 *>(WtT + (size_t)n * 4 * Cout + k);
  }
  __device__ __forceinline__ void fill_a(bf16 (*S)[LDK], int m0, int k0, int ke, int tid) const {
    fill_rows<true>(*this, S, m0, k0, ke, tid);
  }
  __device__ __forceinline__ void fill_b(bf16 (*S)[LDK], int n0, int k0, int ke, int tid) const {
    fill_rows<false>(*this, S, n0, k0, ke, tid);
  }
  __device__ __forceinline__ void store(int m, int n, float v, int) const {
    if (m >= g.P() || n >= Cin) return;
    din.p[(size_t)m * din.cs + din.coff + n] = v;
  }
};

// Backward-weight of UpFwd: dW[d][co][ci] = sum_p dOut[up(p,d), co] in[p, ci],
// db[co] = sum over all output pixels of dOut[., co] (ones column at ci = Cin).
// M = 4 Cout (m = d*Cout + co), N = Cin + 1, reduction over input pixels, split.
struct UpBwdWeight {
  Img g;
  View<const float> dout;
  View<const bf16> in;
  int Cin, Cout;
  int chunk;
  float *partial;  // [splits][4*Cout][Cin+1]
  __device__ __forceinline__ void krange(int z, int &b, int &e) const {
    b = z * chunk;
    e = min(g.P(), b + chunk);
  }
  __device__ __forceinline__ void fill_a(bf16 (*S)[LDK], int m0, int k0, int ke, int tid) const {
    const int pl = tid >> 3, ml = (tid & 7) * 8;
    const int p = k0 + pl, m = m0 + ml;
    bf16x8 v = zero8();
    if (p < ke && m < 4 * Cout) {
      const int d = m / Cout, co = m - d * Cout;
      const int x = p % g.W, t = p / g.W, y = t % g.H, b = t / g.H;
      const int q = (b * 2 * g.H + 2 * y + (d >> 1)) * 2 * g.W + 2 * x + (d & 1);
      const float *s = dout.p + (size_t)q * dout.cs + dout.coff + co;
      for (int j = 0; j < 8; ++j) v[j] = (bf16)s[j];
    }
    for (int j = 0; j < 8; ++j) S[ml + j][pl] = v[j];
  }
  __device__ __forceinline__ void fill_b(bf16 (*S)[LDK], int n0, int k0, int ke, int tid) const {
    const int pl = tid >> 3, nl = (tid & 7) * 8;
    const int p = k0 + pl, n = n0 + nl;
    bf16x8 v = zero8();
    if (p < ke) {
      if (n < Cin) v = *reinterpret_cast<const bf16x8 *>(in.p + (size_t)p * in.cs + in.coff + n);
      else if (n == Cin) v[0] = (bf16)1.f;
    }
    for (int j = 0; j < 8; ++j) S[nl + j][pl] = v[j];
  }
  __device__ __forceinline__ void store(int m, int n, float v, int z) const {
    if (m >= 4 * Cout || n > Cin) return;
    partial[((size_t)z * 4 * Cout + m) * (Cin + 1) + n] = v;
  }
};

// Sums split partials [splits][M][Kw+1] in fixed order into dW[m][k] (k < Kw)
// and, for the ones column, db[m mod Cb] (accumulated over the rows sharing it).
static __global__ __launch_bounds__(256) void k_split_reduce(const float *partial, int splits, int M, int Kw,
                                                      float *dW, float *db, int Cb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int Nw = Kw + 1;
  if (i >= M * Kw && i >= Cb) return;
  if (i < M * Kw) {
    const int m = i / Kw, k = i - m * Kw;
    float s = 0.f;
    for (int z = 0; z < splits; ++z) s += partial[((size_t)z * M + m) * Nw + k];
    dW[i] = s;
  }
  if (i < Cb) {  // bias of output channel i: rows m with m mod Cb == i
    float s = 0.f;
    for (int m = i; m < M; m += Cb)
      for (int z = 0; z < splits; ++z) s += partial[((size_t)z * M + m) * Nw + Kw];
    db[i] = s;
  }
}

// ---------------------------------------------------------------------------
// 2x2 max pooling (stride 2): forward on BF16, backward routes the gradient to
// the first maximum in the order (0,0), (0,1), (1,0), (1,1) and adds it to the
// input gradient.
static __global__ __launch_bounds__(256) void k_pool_fwd(Img g, View<const bf16> in, int C, View<bf16> out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;  // output element
  const int Ho = g.H / 2, Wo = g.W / 2;
  if (i >= g.B * Ho * Wo * C) return;
  const int c = i % C, t = i / C, x = t % Wo, t2 = t / Wo, y = t2 % Ho, b = t2 / Ho;
  float best = -INFINITY;
  for (int d = 0; d < 4; ++d) {
    const size_t q = ((size_t)b * g.H + 2 * y + (d >> 1)) * g.W + 2 * x + (d & 1);
    const float v = (float)in.p[q * in.cs + in.coff + c];
    if (v > best) best = v;
  }
  out.p[(size_t)t * out.cs + out.coff + c] = (bf16)best;
}

static __global__ __launch_bounds__(256) void k_pool_bwd(Img g, View<const bf16> in, int C, View<const float> dout,
                                                  View<float> din) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int Ho = g.H / 2, Wo = g.W / 2;
  if (i >= g.B * Ho * Wo * C) return;
  const int c = i % C, t = i / C, x = t % Wo, t2 = t / Wo, y = t2 % Ho, b = t2 / Ho;
  float best = -INFINITY;
  int arg = 0;
  for (int d = 0; d < 4; ++d) {
    const size_t q = ((size_t)b * g.H + 2 * y + (d >> 1)) * g.W + 2 * x + (d & 1);
    const float v = (float)in.p[q * in.cs + in.coff + c];
    if (v > best) { best = v; arg = d; }
  }
  const size_t q = ((size_t)b * g.H + 2 * y + (arg >> 1)) * g.W + 2 * x + (arg & 1);
  din.p[q * din.cs + din.coff + c] += dout.p[(size_t)t * dout.cs + dout.coff + c];
}

// Network input: FP32 NHWC [P][cin] -> BF16 [P][8] (channels padded with zeros).
static __global__ __launch_bounds__(256) void k_pack_input(const float *x, int P, int cin, bf16 *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P * 8) return;
  const int p = i / 8, c = i % 8;
  out[i] = (bf16)(c < cin ? x[(size_t)p * cin + c] : 0.f);
}

// MSE over the first `cout` channels of the head output (stride cs): per-block
// partial sums (fixed order) and dY = 2 (y - t) / (P cout), zero padding.
static __global__ __launch_bounds__(256) void k_mse(const float *y, int cs, const float *t, int P, int cout,
                                             float *dy, double *partial) {
  __shared__ double sh[256];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double e = 0.0;
  if (i < P * cs) {
    const int p = i / cs, c = i % cs;
    float g = 0.f;
    if (c < cout) {
      const float d = y[i] - t[(size_t)p * cout + c];
      e = (double)d * d;
      g = 2.f * d / (float)((double)P * cout);
    }
    dy[i] = g;
  }
  sh[threadIdx.x] = e;
  __syncthreads();
  for (int s = 128; s >= 1; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

static __global__ __launch_bounds__(256) void k_sum_partials(const double *partial, int n, double scale, double *out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) s += partial[k];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0] * scale;
}

// Adam (bias-corrected) on FP32 master parameters.
static __global__ __launch_bounds__(256) void k_adam(float *w, const float *g, float *m, float *v, int64_t n, float lr,
                                              float b1, float b2, float eps, float c1, float c2, float wd) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i] + wd * w[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// BF16 weight copies of a KSxKS convolution: Wt[co][k] = W[co][k] and the
// flipped transpose WtT[ci][(ky*KS+kx)*Cout + co] = W[co][((KS-1-ky)*KS+KS-1-kx)*Cin + ci].
static __global__ __launch_bounds__(256) void k_conv_weights(const float *W, int Cout, int Cin, int KS, bf16 *Wt,
                                                      bf16 *WtT) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int K = KS * KS * Cin;
  if (i >= Cout * K) return;
  const int co = i / K, k = i - co * K, tap = k / Cin, ci = k - tap * Cin;
  const int ky = tap / KS, kx = tap % KS;
  const bf16 v = (bf16)W[i];
  Wt[i] = v;
  const int ftap = (KS - 1 - ky) * KS + (KS - 1 - kx);
  if (WtT) WtT[(size_t)ci * KS * KS * Cout + ftap * Cout + co] = v;
}

// BF16 copies of an up-sampling weight W[d][co][ci]: Wt = W, WtT[ci][d*Cout + co].
static __global__ __launch_bounds__(256) void k_up_weights(const float *W, int Cout, int Cin, bf16 *Wt, bf16 *WtT) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 4 * Cout * Cin) return;
  const int ci = i % Cin, t = i / Cin, co = t % Cout, d = t / Cout;
  const bf16 v = (bf16)W[i];
  Wt[i] = v;
  WtT[(size_t)ci * 4 * Cout + d * Cout + co] = v;
}

static __global__ __launch_bounds__(256) void k_fill_f32(float *p, int64_t n, float v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Head output (stride cs, first cout channels) -> FP32 NHWC [P][cout].
static __global__ __launch_bounds__(256) void k_unpack_output(const float *y, int cs, int P, int cout, float *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P * cout) return;
  out[i] = y[(size_t)(i / cout) * cs + i % cout];
}

}  // namespace wsk
