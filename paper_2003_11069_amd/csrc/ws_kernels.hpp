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
// gradients of activations NHWC BF16 (every consumer takes them as a BF16
// MFMA operand; only the pooling backward adds two of them), weights BF16
// copies of FP32 master parameters, weight gradients FP32.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

namespace wsk {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f4;
typedef __bf16 bf16;

constexpr int BK = 32;       // K step of the GEMM engine
constexpr int LDK = BK + 8;  // LDS row stride (bf16), 80 bytes

__device__ __forceinline__ bf16x8 zero8() {
  bf16x8 z;
  for (int j = 0; j < 8; ++j) z[j] = (bf16)0.f;
  return z;
}

// Exact unsigned division n / d for n < 2^31 by multiply and shift
// (Granlund & Montgomery, PLDI 1994): m = ceil(2^(31+l) / d), l = ceil(log2 d),
// q = (n m) >> (31 + l).  Built on the host.
struct Div {
  uint32_t d, m, s;
  static Div make(uint32_t d) {
    int l = 0;
    while ((1ull << l) < d) ++l;
    Div r;
    r.d = d;
    r.m = (uint32_t)(((1ull << (31 + l)) + d - 1) / d);
    r.s = 31u + (uint32_t)l;
    return r;
  }
  __device__ __forceinline__ uint32_t q(uint32_t n) const { return (uint32_t)(((uint64_t)n * m) >> s); }
};

// NHWC tensor view: element (pixel p, channel c) at p*cs + coff + c.
template <typename T>
struct View {
  T *p;
  int cs, coff;
};

// Image batch geometry with the divisions used to split a pixel index.
struct Img {
  int B, H, W;
  Div dH, dW;
  static Img make(int B, int H, int W) { return Img{B, H, W, Div::make(H), Div::make(W)}; }
  __device__ __forceinline__ int P() const { return B * H * W; }
  __device__ __forceinline__ void split(int m, int &b, int &y, int &x) const {
    const uint32_t t = dW.q((uint32_t)m);
    x = m - (int)t * W;
    b = (int)dH.q(t);
    y = (int)t - b * H;
  }
};

// ---------------------------------------------------------------------------
// GEMM engine: C[M,N] = sum_k A[m,k] B[k,n] on v_mfma_f32_16x16x32_bf16.
// Block tile BM x BN (BM in {64,128}, BN in {32,64,128}), 4 waves in 2 x 2,
// each (BM/2) x (BN/2) of 16 x 16 MFMA tiles; K in steps of KB (32 or 64,
// one or two MFMA slices) through two
// LDS buffers, the next step's global loads issued before the current step's
// MFMAs (one barrier per step).  The problem supplies 8-element operand
// chunks -- ROW: 8 consecutive k of one row; COL: 8 consecutive rows at one
// k, gathered for COLV = 2 consecutive k and stored transposed into LDS as
// 4-byte rows (two k per thread keep every thread gathering) -- and consumes
// the accumulators in store().  K may be split over
// gridDim.z (the problem decides each split's range).
enum { ROW = 0, COL = 1 };
constexpr int COLV = 2;  // consecutive k per COL chunk

template <int LAYOUT, int R, int KB = BK>
struct ChunkMap {
  static constexpr int N = LAYOUT == ROW ? R * KB / 8 : R * KB / (8 * COLV);  // chunks per tile
  static constexpr int V = LAYOUT == ROW ? 1 : COLV;                          // bf16x8 per chunk
  __device__ __forceinline__ static void at(int q, int &row, int &k) {
    if (LAYOUT == ROW) {
      row = q / (KB / 8);
      k = (q % (KB / 8)) * 8;
    } else {
      row = (q % (R / 8)) * 8;
      k = (q / (R / 8)) * COLV;
    }
  }
};

// Stores one chunk (V vectors starting at v) into an LDS tile.
template <int LAYOUT, int LD = LDK>
__device__ __forceinline__ void put_chunk(bf16 (*S)[LD], int row, int k, const bf16x8 *v) {
  if (LAYOUT == ROW) {
    *reinterpret_cast<bf16x8 *>(&S[row][k]) = v[0];
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      typedef __attribute__((ext_vector_type(COLV))) __bf16 bfv;
      bfv w;
#pragma unroll
      for (int t = 0; t < COLV; ++t) w[t] = v[t][j];
      *reinterpret_cast<bfv *>(&S[row + j][k]) = w;
    }
  }
}

// Problems with BF16 outputs in rows of 8 channels supply keep8(m, n) (the
// output mask of such a row) and store8(m, n, v, keep): the engine stages the
// block's results through LDS and stores 16-byte rows, all of a thread's
// masks read before its first store (a store might alias them).
template <class P, class = void>
struct HasRows : std::false_type {};
template <class P>
struct HasRows<P, decltype((void)&P::store8)> : std::true_type {};

template <class P, int BM_, int BN_, int KB = BK>
__global__ __launch_bounds__(256) void k_gemm(P prob) {
  constexpr int WM = BM_ / 2, WN = BN_ / 2, TM = WM / 16, TN = WN / 16;
  constexpr int LD = KB + 8;  // LDS row stride (bf16)
  using MA = ChunkMap<P::A_LAYOUT, BM_, KB>;
  using MB = ChunkMap<P::B_LAYOUT, BN_, KB>;
  constexpr int CA = (MA::N + 255) / 256, CB = (MB::N + 255) / 256;
  __shared__ __attribute__((aligned(16))) bf16 smem[2 * (BM_ + BN_) * LD];
  auto As = reinterpret_cast<bf16 (*)[BM_][LD]>(smem);
  auto Bs = reinterpret_cast<bf16 (*)[BN_][LD]>(smem + 2 * BM_ * LD);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.x * BM_, n0 = blockIdx.y * BN_;
  const int wm = (wave >> 1) * WM, wn = (wave & 1) * WN;
  int kbeg, kend;
  prob.krange(blockIdx.z, kbeg, kend);
  f4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  constexpr int VA = MA::V, VB = MB::V;
  bf16x8 ra[CA * VA], rb[CB * VB];
  auto load = [&](int k0) {
#pragma unroll
    for (int c = 0; c < CA; ++c) {
      const int q = tid + 256 * c;
      int row, k;
      MA::at(q, row, k);
      if (q < MA::N) {
#pragma unroll
        for (int t = 0; t < VA; ++t) ra[c * VA + t] = prob.a(m0 + row, k0 + k + t, kend, m0);
      }
    }
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      const int q = tid + 256 * c;
      int row, k;
      MB::at(q, row, k);
      if (q < MB::N) {
#pragma unroll
        for (int t = 0; t < VB; ++t) rb[c * VB + t] = prob.b(n0 + row, k0 + k + t, kend, m0);
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int c = 0; c < CA; ++c) {
      const int q = tid + 256 * c;
      int row, k;
      MA::at(q, row, k);
      if (q < MA::N) put_chunk<P::A_LAYOUT, LD>(As[buf], row, k, &ra[c * VA]);
    }
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      const int q = tid + 256 * c;
      int row, k;
      MB::at(q, row, k);
      if (q < MB::N) put_chunk<P::B_LAYOUT, LD>(Bs[buf], row, k, &rb[c * VB]);
    }
  };
  if (kbeg < kend) {
    load(kbeg);
    store(0);
  }
  __syncthreads();
  int buf = 0;
  const int r = lane & 15, kq = 8 * (lane >> 4);
  for (int k0 = kbeg; k0 < kend; k0 += KB) {
    const bool more = k0 + KB < kend;
    if (more) load(k0 + KB);
#pragma unroll
    for (int ks = 0; ks < KB; ks += 32) {  // 32-deep MFMA slices of the LDS stage
      bf16x8 a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) a[i] = *reinterpret_cast<const bf16x8 *>(&As[buf][wm + 16 * i + r][ks + kq]);
#pragma unroll
      for (int j = 0; j < TN; ++j) b[j] = *reinterpret_cast<const bf16x8 *>(&Bs[buf][wn + 16 * j + r][ks + kq]);
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  if constexpr (HasRows<P>::value) {
    constexpr int OPB = BN_ + 8, R8 = BN_ / 8, NCH = BM_ * R8 / 256;  // 16-byte rows per thread
    static_assert(BM_ * OPB <= 2 * (BM_ + BN_) * LD, "output tile exceeds the staging LDS");
    bf16 *O = smem;
    __syncthreads();  // the last K step's reads are done
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          O[(wm + 16 * i + 4 * (lane >> 4) + q) * OPB + wn + 16 * j + (lane & 15)] = (bf16)acc[i][j][q];
    __syncthreads();
    bf16x8 kp[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      const int e = tid + 256 * c, r = e / R8, c8 = (e - r * R8) * 8;
      kp[c] = prob.keep8(m0 + r, n0 + c8);
    }
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      const int e = tid + 256 * c, r = e / R8, c8 = (e - r * R8) * 8;
      prob.store8(m0 + r, n0 + c8, *reinterpret_cast<const bf16x8 *>(&O[r * OPB + c8]), kp[c]);
    }
  } else {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + q;
          const int n = n0 + wn + 16 * j + (lane & 15);
          prob.store(m, n, acc[i][j][q], blockIdx.z);
        }
  }
}

// ---------------------------------------------------------------------------
// KSxKS convolution, stride 1, zero padding KS/2, forward:
//   out[p, co] = act( sum_{ky,kx,ci} W[co][(ky*KS+kx)*Cin + ci] in[p + (ky-r, kx-r), ci] + b[co] )
// M = pixels, N = Cout, K = KS*KS*Cin (Cin multiple of 8).
template <int KS, bool RELU, bool OUT_F32>
struct ConvFwd {
  static constexpr int A_LAYOUT = ROW, B_LAYOUT = ROW;
  Img g;
  View<const bf16> in;
  int Cin, Cout;
  Div dCin;
  const bf16 *Wt;   // [Cout][K]
  const float *bias;
  View<bf16> out;      // BF16 output (OUT_F32 = false)
  View<float> outf;    // FP32 output (OUT_F32 = true)
  __device__ __forceinline__ int K() const { return KS * KS * Cin; }
  __device__ __forceinline__ void krange(int, int &b, int &e) const { b = 0; e = K(); }
  __device__ __forceinline__ bf16x8 a(int m, int k, int kend, int) const {
    if (m >= g.P() || k >= kend) return zero8();
    const int tap = (int)dCin.q((uint32_t)k), ci = k - tap * Cin;
    int b, y, x;
    g.split(m, b, y, x);
    const int yy = y + tap / KS - KS / 2, xx = x + tap % KS - KS / 2;
    if (yy < 0 || yy >= g.H || xx < 0 || xx >= g.W) return zero8();
    const int q = (b * g.H + yy) * g.W + xx;
    return *reinterpret_cast<const bf16x8 *>(in.p + (size_t)q * in.cs + in.coff + ci);
  }
  __device__ __forceinline__ bf16x8 b(int n, int k, int kend, int) const {
    if (n >= Cout || k >= kend) return zero8();
    return *reinterpret_cast<const bf16x8 *>(Wt + (size_t)n * K() + k);
  }
  __device__ __forceinline__ void store(int m, int n, float v, int) const {
    if (m >= g.P() || n >= Cout) return;
    v += bias[n];
    if (RELU) v = v > 0.f ? v : 0.f;
    if (OUT_F32) outf.p[(size_t)m * outf.cs + outf.coff + n] = v;
    else out.p[(size_t)m * out.cs + out.coff + n] = (bf16)v;
  }
};

// Eight channels of pixel q of a BF16 tensor.
__device__ __forceinline__ bf16x8 ld8(const View<const bf16> &d, int q, int c) {
  return *reinterpret_cast<const bf16x8 *>(d.p + (size_t)q * d.cs + d.coff + c);
}

// The gradient of a ReLU layer's output is stored as zero where the layer's
// output (mask) is not positive, for channels c >= mc0 (channels below mc0 of
// a concatenated buffer are not a ReLU output); no mask when mask.p is null.
// Every activation gradient is stored this way, so the consumers (data and
// weight gradients of that layer) read it as their operand directly.
// row_mask: the mask of output row (pixel m, channels n .. n + 7), the
// producer's output there, or ones where none applies (mc0 is a multiple of 8,
// so a row is either wholly below it or not).
__device__ __forceinline__ bf16x8 row_mask(const View<const bf16> &mask, int mc0, int P, int C, int m, int n) {
  if (mask.p && n >= mc0 && m < P && n < C) return ld8(mask, m, n);
  bf16x8 o;
#pragma unroll
  for (int j = 0; j < 8; ++j) o[j] = (bf16)1.f;
  return o;
}
__device__ __forceinline__ void store_masked(const View<bf16> &d, int m, int n, bf16x8 v, bf16x8 k) {
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = (float)k[j] > 0.f ? v[j] : (bf16)0.f;
  *reinterpret_cast<bf16x8 *>(d.p + (size_t)m * d.cs + d.coff + n) = v;
}

// Backward-data of ConvFwd: dIn[p, ci] = sum_{ky,kx,co} WtT[ci][(ky*KS+kx)*Cout + co]
//   dPre[p + (ky-r, kx-r), co],  WtT = weights flipped in (ky,kx) and transposed,
// dPre the layer's output gradient, already masked by its ReLU.  M = pixels,
// N = Cin, K = KS*KS*Cout (Cout multiple of 8).  Writes BF16, masked by the
// ReLU of the layer that produced the input (row_mask).
template <int KS>
struct ConvBwdData {
  static constexpr int A_LAYOUT = ROW, B_LAYOUT = ROW;
  Img g;
  View<const bf16> dout;
  int Cin, Cout;
  Div dCout;
  const bf16 *WtT;  // [Cin][K]
  View<bf16> din;
  View<const bf16> mask;  // output mask (the input's producer), channels >= mc0
  int mc0;
  __device__ __forceinline__ int K() const { return KS * KS * Cout; }
  __device__ __forceinline__ void krange(int, int &b, int &e) const { b = 0; e = K(); }
  __device__ __forceinline__ bf16x8 a(int m, int k, int kend, int) const {
    if (m >= g.P() || k >= kend) return zero8();
    const int tap = (int)dCout.q((uint32_t)k), co = k - tap * Cout;
    int b, y, x;
    g.split(m, b, y, x);
    const int yy = y + tap / KS - KS / 2, xx = x + tap % KS - KS / 2;
    if (yy < 0 || yy >= g.H || xx < 0 || xx >= g.W) return zero8();
    return ld8(dout, (b * g.H + yy) * g.W + xx, co);
  }
  __device__ __forceinline__ bf16x8 b(int n, int k, int kend, int) const {
    if (n >= Cin || k >= kend) return zero8();
    return *reinterpret_cast<const bf16x8 *>(WtT + (size_t)n * K() + k);
  }
  __device__ __forceinline__ void store(int m, int n, float v, int) const {
    if (m >= g.P() || n >= Cin) return;
    din.p[(size_t)m * din.cs + din.coff + n] = (bf16)v;
  }
  __device__ __forceinline__ bf16x8 keep8(int m, int n) const { return row_mask(mask, mc0, g.P(), Cin, m, n); }
  __device__ __forceinline__ void store8(int m, int n, bf16x8 v, bf16x8 k) const {
    if (m < g.P() && n < Cin) store_masked(din, m, n, v, k);
  }
};

// Backward-weight of ConvFwd, split over pixels:
//   dW[co][k] = sum_p dPre[p, co] im2col(in)[p, k],  db[co] = sum_p dPre[p, co]
// (the bias is column k = K of a ones column).  Reduction over pixels; split z
// writes partial[z][co][k] (FP32), summed in fixed order by k_wreduce.
// Both operands are COL chunks (8 channels of one pixel).  TR = false: M =
// Cout, N = K + 1; TR = true (narrow Cout): M = K + 1, N = Cout.
template <int KS, bool TR = false>
struct ConvBwdWeight {
  static constexpr int A_LAYOUT = COL, B_LAYOUT = COL;
  Img g;
  View<const bf16> dout;  // output gradient, masked by the layer's ReLU
  View<const bf16> in;
  int Cin, Cout;
  Div dCin;
  int chunk;          // pixels per split (multiple of BK)
  float *partial;     // [splits][Cout][K+1]
  __device__ __forceinline__ int Kw() const { return KS * KS * Cin; }
  __device__ __forceinline__ void krange(int z, int &b, int &e) const {
    b = z * chunk;
    e = min(g.P(), b + chunk);
  }
  __device__ __forceinline__ bf16x8 dpre(int co, int p, int kend) const {
    return (p < kend && co < Cout) ? ld8(dout, p, co) : zero8();
  }
  __device__ __forceinline__ bf16x8 col(int n, int p, int kend) const {
    bf16x8 v = zero8();
    if (p >= kend) return v;
    if (n < Kw()) {
      const int tap = (int)dCin.q((uint32_t)n), ci = n - tap * Cin;
      int b, y, x;
      g.split(p, b, y, x);
      const int yy = y + tap / KS - KS / 2, xx = x + tap % KS - KS / 2;
      if (yy >= 0 && yy < g.H && xx >= 0 && xx < g.W)
        v = *reinterpret_cast<const bf16x8 *>(in.p + (size_t)((b * g.H + yy) * g.W + xx) * in.cs + in.coff + ci);
    } else if (n == Kw()) {
      v[0] = (bf16)1.f;
    }
    return v;
  }
  __device__ __forceinline__ bf16x8 a(int m, int p, int kend, int) const { return TR ? col(m, p, kend) : dpre(m, p, kend); }
  __device__ __forceinline__ bf16x8 b(int n, int p, int kend, int) const { return TR ? dpre(n, p, kend) : col(n, p, kend); }
  __device__ __forceinline__ void store(int m, int n, float v, int z) const {
    const int co = TR ? n : m, k = TR ? m : n;
    if (co >= Cout || k > Kw()) return;
    partial[((size_t)z * Cout + co) * (Kw() + 1) + k] = v;
  }
};

// ---------------------------------------------------------------------------
// 2x2 stride-2 transposed convolution (up-sampling), forward:
//   out[(b, 2y+dy, 2x+dx), co] = sum_ci W[d][co][ci] in[(b,y,x), ci] + b[co], d = 2dy+dx.
// Rows are ordered parity-major, m = d*Pin + p, so a block tile has one
// parity (Pin is a multiple of the tile height).  M = 4 Pin, N = Cout, K = Cin.
struct UpFwd {
  static constexpr int A_LAYOUT = ROW, B_LAYOUT = ROW;
  Img g;  // input image
  View<const bf16> in;
  int Cin, Cout;
  Div dPin;
  const bf16 *Wt;  // [4][Cout][Cin]
  const float *bias;
  View<bf16> out;  // output image (2H x 2W)
  __device__ __forceinline__ void krange(int, int &b, int &e) const { b = 0; e = Cin; }
  __device__ __forceinline__ bf16x8 a(int m, int k, int kend, int) const {
    const int Pin = g.P();
    if (m >= 4 * Pin || k >= kend) return zero8();
    const int p = m - (int)dPin.q((uint32_t)m) * Pin;
    return *reinterpret_cast<const bf16x8 *>(in.p + (size_t)p * in.cs + in.coff + k);
  }
  __device__ __forceinline__ bf16x8 b(int n, int k, int kend, int m0) const {
    if (n >= Cout || k >= kend) return zero8();
    const int d = (int)dPin.q((uint32_t)m0);
    return *reinterpret_cast<const bf16x8 *>(Wt + ((size_t)d * Cout + n) * Cin + k);
  }
  __device__ __forceinline__ void store(int m, int n, float v, int) const {
    const int Pin = g.P();
    if (m >= 4 * Pin || n >= Cout) return;
    const int d = (int)dPin.q((uint32_t)m), p = m - d * Pin;
    int b, y, x;
    g.split(p, b, y, x);
    const int Y = 2 * y + (d >> 1), X = 2 * x + (d & 1);
    const size_t q = ((size_t)b * 2 * g.H + Y) * 2 * g.W + X;
    out.p[q * out.cs + out.coff + n] = (bf16)(v + bias[n]);
  }
};

// Output-pixel index of input pixel p under up-sampling parity d.
__device__ __forceinline__ int up_pixel(const Img &g, int p, int d) {
  int b, y, x;
  g.split(p, b, y, x);
  return (b * 2 * g.H + 2 * y + (d >> 1)) * 2 * g.W + 2 * x + (d & 1);
}

// Backward-data of UpFwd: dIn[p, ci] = sum_{d,co} WtT[ci][d*Cout + co] dOut[up(p,d), co].
// M = Pin, N = Cin, K = 4 Cout.  No activation on the up-sampling output.
struct UpBwdData {
  static constexpr int A_LAYOUT = ROW, B_LAYOUT = ROW;
  Img g;
  View<const bf16> dout;  // output-image gradient
  int Cin, Cout;
  Div dCout;
  const bf16 *WtT;  // [Cin][4][Cout]
  View<bf16> din;
  View<const bf16> mask;  // the input's producer's output (ReLU mask)
  __device__ __forceinline__ void krange(int, int &b, int &e) const { b = 0; e = 4 * Cout; }
  __device__ __forceinline__ bf16x8 a(int m, int k, int kend, int) const {
    if (m >= g.P() || k >= kend) return zero8();
    const int d = (int)dCout.q((uint32_t)k), co = k - d * Cout;
    return *reinterpret_cast<const bf16x8 *>(dout.p + (size_t)up_pixel(g, m, d) * dout.cs + dout.coff + co);
  }
  __device__ __forceinline__ bf16x8 b(int n, int k, int kend, int) const {
    if (n >= Cin || k >= kend) return zero8();
    return *reinterpret_cast<const bf16x8 *>(WtT + (size_t)n * 4 * Cout + k);
  }
  __device__ __forceinline__ void store(int m, int n, float v, int) const {
    if (m >= g.P() || n >= Cin) return;
    din.p[(size_t)m * din.cs + din.coff + n] = (bf16)v;
  }
  __device__ __forceinline__ bf16x8 keep8(int m, int n) const { return row_mask(mask, 0, g.P(), Cin, m, n); }
  __device__ __forceinline__ void store8(int m, int n, bf16x8 v, bf16x8 k) const {
    if (m < g.P() && n < Cin) store_masked(din, m, n, v, k);
  }
};

// Backward-weight of UpFwd: dW[d][co][ci] = sum_p dOut[up(p,d), co] in[p, ci],
// db[co] = sum over all output pixels of dOut[., co] (ones column at ci = Cin).
// M = 4 Cout (m = d*Cout + co), N = Cin + 1, reduction over input pixels, split.
struct UpBwdWeight {
  static constexpr int A_LAYOUT = COL, B_LAYOUT = COL;
  Img g;
  View<const bf16> dout;
  View<const bf16> in;
  int Cin, Cout;
  Div dCout;
  int chunk;
  float *partial;  // [splits][4*Cout][Cin+1]
  __device__ __forceinline__ void krange(int z, int &b, int &e) const {
    b = z * chunk;
    e = min(g.P(), b + chunk);
  }
  __device__ __forceinline__ bf16x8 a(int m, int p, int kend, int) const {
    if (p >= kend || m >= 4 * Cout) return zero8();
    const int d = (int)dCout.q((uint32_t)m), co = m - d * Cout;
    return *reinterpret_cast<const bf16x8 *>(dout.p + (size_t)up_pixel(g, p, d) * dout.cs + dout.coff + co);
  }
  __device__ __forceinline__ bf16x8 b(int n, int p, int kend, int) const {
    bf16x8 v = zero8();
    if (p >= kend) return v;
    if (n < Cin) v = *reinterpret_cast<const bf16x8 *>(in.p + (size_t)p * in.cs + in.coff + n);
    else if (n == Cin) v[0] = (bf16)1.f;
    return v;
  }
  __device__ __forceinline__ void store(int m, int n, float v, int z) const {
    if (m >= 4 * Cout || n > Cin) return;
    partial[((size_t)z * 4 * Cout + m) * (Cin + 1) + n] = v;
  }
};

// ---------------------------------------------------------------------------
// 2x2 max pooling (stride 2): forward on BF16, backward routes the gradient to
// the first maximum in the order (0,0), (0,1), (1,0), (1,1) and adds it to the
// input gradient where that maximum is positive (the pooled input is a ReLU
// output, and its stored gradient is masked).  The forward handles one pooled pixel and 8 channels (C is
// a multiple of 8) per thread, with 16-byte vectors.
__device__ __forceinline__ void pool_split(const Img &g, int i, int C8, int &c, int &t, int &b, int &y, int &x) {
  const int Ho = g.H / 2, Wo = g.W / 2;
  c = (i % C8) * 8;
  t = i / C8;  // pooled pixel
  x = t % Wo;
  const int t2 = t / Wo;
  y = t2 % Ho;
  b = t2 / Ho;
}
__device__ __forceinline__ size_t pool_src(const Img &g, int b, int y, int x, int d) {
  return ((size_t)b * g.H + 2 * y + (d >> 1)) * g.W + 2 * x + (d & 1);
}

static __global__ __launch_bounds__(256) void k_pool_fwd(Img g, View<const bf16> in, int C, View<bf16> out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;  // (pooled pixel, 8-channel chunk)
  const int C8 = C / 8;
  if (i >= g.B * (g.H / 2) * (g.W / 2) * C8) return;
  int c, t, b, y, x;
  pool_split(g, i, C8, c, t, b, y, x);
  bf16x8 v[4];
#pragma unroll
  for (int d = 0; d < 4; ++d)
    v[d] = *reinterpret_cast<const bf16x8 *>(in.p + pool_src(g, b, y, x, d) * in.cs + in.coff + c);
  bf16x8 r;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    float best = -INFINITY;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const float f = (float)v[d][j];
      if (f > best) best = f;
    }
    r[j] = (bf16)best;
  }
  *reinterpret_cast<bf16x8 *>(out.p + (size_t)t * out.cs + out.coff + c) = r;
}

// Backward: a thread per pooled element (consecutive threads take consecutive
// channels, so the read-modify-write of the maximum's element is coalesced;
// 8-channel vectors measured slower here).  Used after an implicit-GEMM
// forward; after the direct forward, k_pool_bwd_arg reads the window
// positions that forward recorded instead of the four activations.
static __global__ __launch_bounds__(256) void k_pool_bwd(Img g, View<const bf16> in, int C, View<const bf16> dout,
                                                  View<bf16> din) {
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
  if (!(best > 0.f)) return;
  const size_t q = ((size_t)b * g.H + 2 * y + (arg >> 1)) * g.W + 2 * x + (arg & 1);
  bf16 &d = din.p[q * din.cs + din.coff + c];
  d = (bf16)((float)d + (float)dout.p[(size_t)t * dout.cs + dout.coff + c]);
}

// Backward from the window positions the fused forward recorded (255: the
// maximum was not positive, nothing to add): a thread per pooled element,
// as k_pool_bwd, without reading the activations.
static __global__ __launch_bounds__(256) void k_pool_bwd_arg(Img g, const uint8_t *arg, int C, View<const bf16> dout,
                                                      View<bf16> din) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int Ho = g.H / 2, Wo = g.W / 2;
  if (i >= g.B * Ho * Wo * C) return;
  const int d = arg[i];
  if (d > 3) return;
  const int c = i % C, t = i / C, x = t % Wo, t2 = t / Wo, y = t2 % Ho, b = t2 / Ho;
  const size_t q = ((size_t)b * g.H + 2 * y + (d >> 1)) * g.W + 2 * x + (d & 1);
  bf16 &v = din.p[q * din.cs + din.coff + c];
  v = (bf16)((float)v + (float)dout.p[(size_t)t * dout.cs + dout.coff + c]);
}

// Network input: FP32 NHWC [P][cin] -> BF16 [P][8] (channels padded with
// zeros), a pixel per thread.
static __global__ __launch_bounds__(256) void k_pack_input(const float *x, int P, int cin, bf16 *out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  bf16x8 v;
#pragma unroll
  for (int c = 0; c < 8; ++c) v[c] = (bf16)(c < cin ? x[(size_t)p * cin + c] : 0.f);
  *reinterpret_cast<bf16x8 *>(out + (size_t)p * 8) = v;
}

// MSE over the first `cout` channels of the head output (8 channels per
// pixel), a pixel per thread: per-block partial sums (the pixel's channels in
// order, then a fixed tree) and dY = 2 (y - t) / (P cout) stored as BF16, zero padding.
static __global__ __launch_bounds__(256) void k_mse(const float *y, const float *t, int P, int cout, bf16 *dy,
                                             double *partial) {
  __shared__ double sh[256];
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  double e = 0.0;
  if (p < P) {
    const float4 *ys = reinterpret_cast<const float4 *>(y + (size_t)p * 8);
    const float4 y0 = ys[0], y1 = ys[1];
    const float yv[8] = {y0.x, y0.y, y0.z, y0.w, y1.x, y1.y, y1.z, y1.w};
    float gv[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      gv[c] = 0.f;
      if (c < cout) {
        const float d = yv[c] - t[(size_t)p * cout + c];
        e += (double)d * d;
        gv[c] = 2.f * d / (float)((double)P * cout);
      }
    }
    bf16x8 gb;
#pragma unroll
    for (int c = 0; c < 8; ++c) gb[c] = (bf16)gv[c];
    *reinterpret_cast<bf16x8 *>(dy + (size_t)p * 8) = gb;
  }
  sh[threadIdx.x] = e;
  __syncthreads();
  for (int s = 128; s >= 1; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

// One block of 1024 threads: thread t adds partials t, t + 1024, ... in four
// interleaved sums (loads in flight together), then a fixed tree.
static __global__ __launch_bounds__(1024) void k_sum_partials(const double *partial, int n, double scale, double *out) {
  __shared__ double sh[1024];
  const int t = threadIdx.x;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int k = t;
  for (; k + 3 * 1024 < n; k += 4 * 1024) {
    a0 += partial[k];
    a1 += partial[k + 1024];
    a2 += partial[k + 2 * 1024];
    a3 += partial[k + 3 * 1024];
  }
  for (; k < n; k += 1024) a0 += partial[k];
  sh[t] = (a0 + a1) + (a2 + a3);
  __syncthreads();
  for (int w = 512; w >= 1; w >>= 1) {
    if (t < w) sh[t] += sh[t + w];
    __syncthreads();
  }
  if (t == 0) *out = sh[0] * scale;
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

// All layers' BF16 weight copies in one launch (the table travels in the
// kernel argument; layer l owns the blocks from blk0).  A KSxKS convolution
// W[co][k]: Wt = W and the flipped transpose
// WtT[ci][(ky*KS+kx)*Cout + co] = W[co][((KS-1-ky)*KS+KS-1-kx)*Cin + ci];
// an up-sampling W[d][co][ci] (up = 1): Wt = W, WtT[ci][d*Cout + co].
struct WLayer {
  const float *W;
  bf16 *Wt, *WtT;
  int Cout, Cin, KS, up, blk0;
};
constexpr int MAX_WLAYERS = 32;
struct WTable {
  WLayer l[MAX_WLAYERS];
  int n;
};
static __global__ __launch_bounds__(256) void k_refresh_weights(WTable t) {
  int li = 0;
  while (li + 1 < t.n && (int)blockIdx.x >= t.l[li + 1].blk0) ++li;  // block-uniform
  const WLayer &L = t.l[li];
  const int i = ((int)blockIdx.x - L.blk0) * 256 + threadIdx.x;
  if (L.up) {
    if (i >= 4 * L.Cout * L.Cin) return;
    const int ci = i % L.Cin, q = i / L.Cin, co = q % L.Cout, d = q / L.Cout;
    const bf16 v = (bf16)L.W[i];
    L.Wt[i] = v;
    L.WtT[(size_t)ci * 4 * L.Cout + d * L.Cout + co] = v;
  } else {
    const int K = L.KS * L.KS * L.Cin;
    if (i >= L.Cout * K) return;
    const int co = i / K, k = i - co * K, tap = k / L.Cin, ci = k - tap * L.Cin;
    const int ky = tap / L.KS, kx = tap % L.KS;
    const bf16 v = (bf16)L.W[i];
    L.Wt[i] = v;
    const int ftap = (L.KS - 1 - ky) * L.KS + (L.KS - 1 - kx);
    if (L.WtT) L.WtT[(size_t)ci * L.KS * L.KS * L.Cout + ftap * L.Cout + co] = v;
  }
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
