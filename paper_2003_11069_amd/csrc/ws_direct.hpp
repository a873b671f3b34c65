// ws_direct.hpp -- direct kernels of the warm-start U-Net on
// v_mfma_f32_16x16x32_bf16: 3x3 convolutions (stride 1, zero padding 1) of
// images whose width is a multiple of 32 and height a multiple of 8, and the
// up-sampling forward and weight gradient of rows of whole 32-pixel segments.
//
// A convolution block works through a run of 8 x 32 pixel tiles of one
// image.  It stages each tile and its one-pixel halo in LDS once per
// 32-channel slice and reads all nine taps from there (the implicit GEMM of
// ws_kernels.hpp gathers every tap from global memory, and converts a
// backward operand once per tap).
//
//   k_dconv      forward (BF16 input; bias, ReLU, BF16 output, optionally
//                also its 2x2 max pooling) and
//                backward-data (the layer's output gradient, stored already
//                masked by its ReLU; BF16 output, masked by the ReLU of the
//                input's producer).  The staged operand
//                has Kc channels (a multiple of 32, or the 8 of the padded
//                network input), the output Nc (a multiple of 32).  Weights
//                [Nc][9][Kc]: the forward W, or for backward-data its
//                flipped transpose.
//   k_dwgrad     weight and bias gradient.  Both operands are staged
//                transposed (pixels contiguous, the reduction dimension of
//                the MFMA); the input window of taps kx = 1, 2 is the staged
//                row shifted by one or two pixels in registers.  A block sums
//                a run of tiles and writes partial sums [split][Cout][9 Cin + 1]
//                (bias last).
//   k_wreduce    sums weight-gradient partials over splits in a fixed order,
//                the partials of several layers in one launch.
//   k_upfwd      2x2 stride-2 transposed convolution, forward;
//   k_upwgrad    its weight and bias gradient, staged transposed like
//                k_dwgrad, partial sums [split][4 Cout][Cin + 1].
//   k_head       the 1x1 head, the loss and the head's gradients, for
//                training, in one pass.
//
// Lane layout of the MFMA (as in ws_kernels.hpp): lane l holds
// A[l%16][8(l/16)..+7] and B[8(l/16)..+7][l%16] and receives
// D[4(l/16)+r][l%16], r = 0..3.
#pragma once
#include "ws_kernels.hpp"

namespace wsk {

constexpr int DT_H = 8, DT_W = 32;           // pixel tile of a block
constexpr int DH = DT_H + 2, DW = DT_W + 2;  // with the halo
constexpr int DP = 40;                       // LDS pitch (bf16) of one pixel's 32-channel slice: 80 B

// Tiles of a batch of images: tile t = (b, row band, column band), column band fastest.
struct DTiles {
  int tx, ty, n;
  static DTiles make(int B, int H, int W) { return DTiles{W / DT_W, H / DT_H, B * (H / DT_H) * (W / DT_W)}; }
  __device__ __forceinline__ void at(int t, int &b, int &y0, int &x0) const {
    const int xi = t % tx;
    t /= tx;
    const int yi = t % ty;
    b = t / ty;
    y0 = yi * DT_H;
    x0 = xi * DT_W;
  }
};

// Workgroups are dealt round-robin to the eight XCDs; give each XCD a run of
// consecutive tiles so that neighbouring tiles' halos meet in the same L2.
__device__ __forceinline__ int xcd_tile(int bid, int n) { return n % 8 ? bid : (bid % 8) * (n / 8) + bid / 8; }

typedef __attribute__((ext_vector_type(4))) uint32_t u32x4;

__device__ __forceinline__ uint32_t pack_bf16(bf16 lo, bf16 hi) {
  return (uint32_t)__builtin_bit_cast(uint16_t, lo) | ((uint32_t)__builtin_bit_cast(uint16_t, hi) << 16);
}

// ---------------------------------------------------------------------------
struct DConv {
  Img g;
  DTiles T;
  int tpb;               // tiles per block (block b runs tiles b tpb ..)
  View<const bf16> x;    // forward: input activations (Kc channels)
  View<const bf16> dx;   // backward-data: output gradient of the layer (Kc
                         // channels), already masked by the layer's ReLU
  int Kc, Nc;
  const bf16 *Wk;        // [Nc][9][Kc]
  const float *bias;     // forward
  View<bf16> y;          // forward output (Nc channels)
  View<bf16> pool;       // forward: when set, also its 2x2 max pooling (Nc channels)
  uint8_t *parg;         // with pool: per pooled element the window position of
                         // its first maximum (0..3), or 255 where that maximum
                         // is not positive, [pooled pixel][Nc]
  View<bf16> dy;         // backward-data output (stored, not added)
  View<const bf16> dmask;  // backward-data: output of the input's producer; dy
  int mc0;                 // is zeroed where it is not positive, channels >= mc0
};

// Block: a run of tpb tiles x 32 NW output channels (blockIdx.y), 4 NW
// waves.  Wave w computes rows 2 (w % 4), 2 (w % 4) + 1 of a tile (four
// 16-pixel M tiles) for output channels 32 (w / 4) .. + 31 (two N tiles);
// several N groups in one block share each staged input tile.  The block
// walks (tile, 32-channel slice) items; the global loads of item i + 1 are
// issued before the MFMAs of item i and land in registers, all of an item's
// loads together, so memory latency overlaps the MFMAs.
// SW = 1, 2: the weights of all (at most SW) 32-channel slices are staged
// once per block; SW = 0: each item stages its slice's weights.
template <bool BWD, bool C8, int NW, int SW>
__global__ __launch_bounds__(256 * NW, 2) void k_dconv(DConv P) {
  constexpr int NT = 2, BN = 32 * NW, NTH = 256 * NW;
  constexpr int XP = C8 ? 8 : DP;  // the padded input has one 8-channel chunk per pixel
  constexpr int NWS = C8 ? 3 : 9;  // weight stages per slice: 4-tap groups, or taps
  constexpr int CPP = C8 ? 1 : 4;  // 8-channel chunks per staged pixel
  constexpr int XN = DH * DW * CPP, XIT = (XN + NTH - 1) / NTH;
  constexpr int WN = NWS * BN * 4, WIT = (WN + NTH - 1) / NTH;
  constexpr int OP = 32 + 8;  // pixel pitch of the output staged through Xs
  constexpr int XS = DH * DW * XP > 4 * NW * 64 * OP ? DH * DW * XP : 4 * NW * 64 * OP;
  __shared__ __attribute__((aligned(16))) bf16 Xs[XS];
  constexpr int WSL = NWS * BN * DP;  // one slice's weights (bf16)
  __shared__ __attribute__((aligned(16))) bf16 Ws[WSL * (SW > 0 ? SW : 1)];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, l16 = lane & 15, g = lane >> 4;
  const int rg = wave & 3, ng = wave >> 2;  // row pair, N group
  const int n0 = blockIdx.y * BN, nw0 = n0 + 32 * ng, H = P.g.H, W = P.g.W;
  const int slices = (C8 || SW == 1) ? 1 : P.Kc / 32;
  const int blk = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  const int t0 = blk * P.tpb, t1 = min(P.T.n, t0 + P.tpb);
  const int items = (t1 - t0) * slices;
  f4 acc[4][NT];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  // staging registers (BF16; a backward item's loads are all issued before
  // the first is converted, so they are in flight together)
  bf16x8 xa[XIT], wr[WIT];
  float bias[NT];
#pragma unroll
  for (int j = 0; j < NT; ++j) bias[j] = BWD ? 0.f : P.bias[nw0 + 16 * j + l16];
  // per-thread staging geometry, fixed for every tile: each item's pixel
  // offset from the tile's first pixel (its halo row and column are
  // recomputed where needed, which costs fewer registers)
  int rel[XIT];
#pragma unroll
  for (int it = 0; it < XIT; ++it) {
    const int pix = (tid + NTH * it) / CPP, rr = pix / DW;
    rel[it] = (rr - 1) * W + (pix - rr * DW) - 1;
  }
  auto wload = [&](int s) {
#pragma unroll
    for (int it = 0; it < WIT; ++it) {
      const int q = tid + NTH * it;
      const int gq = q & 3, n = (q >> 2) % BN, w = (q >> 2) / BN;
      wr[it] = zero8();
      if (q < WN) {
        if (C8) {  // k = 8 gq + ci of stage w is tap 4 w + gq
          const int tap = 4 * w + gq;
          if (tap < 9) wr[it] = *reinterpret_cast<const bf16x8 *>(P.Wk + ((size_t)(n0 + n) * 9 + tap) * 8);
        } else {
          wr[it] = *reinterpret_cast<const bf16x8 *>(P.Wk + ((size_t)(n0 + n) * 9 + w) * P.Kc + s * 32 + 8 * gq);
        }
      }
    }
  };
  auto wstore = [&](int sd) {
#pragma unroll
    for (int it = 0; it < WIT; ++it) {
      const int q = tid + NTH * it;
      if (q < WN) {
        const int gq = q & 3, n = (q >> 2) % BN, w = (q >> 2) / BN;
        *reinterpret_cast<bf16x8 *>(&Ws[sd * WSL + (w * BN + n) * DP + 8 * gq]) = wr[it];
      }
    }
  };
  const View<const bf16> &X = BWD ? P.dx : P.x;  // the staged operand
  auto gload = [&](int item) {
    const int t = t0 + item / slices, s = item % slices;
    int b, y0, x0;
    P.T.at(t, b, y0, x0);
    const int64_t tb = (int64_t)(b * H + y0) * W + x0;  // the tile's first pixel
    const bf16 *xb = X.p + tb * X.cs + X.coff + s * 32;
#pragma unroll
    for (int it = 0; it < XIT; ++it) {
      const int q = tid + NTH * it;
      const int pix = q / CPP, ch = (q - pix * CPP) * 8, rr = pix / DW;
      const int yy = y0 + rr - 1, xx = x0 + pix - rr * DW - 1;
      const bool in = q < XN && yy >= 0 && yy < H && xx >= 0 && xx < W;
      xa[it] = in ? *reinterpret_cast<const bf16x8 *>(xb + rel[it] * X.cs + ch) : zero8();
    }
    if (!SW) wload(s);
  };
  // backward-data: the output mask of the tile's 16-byte output rows (four per
  // lane, as the epilogue stores them), loaded before the next item's staging
  // so that waiting for it does not wait for the prefetch
  bf16x8 mk[BWD ? 4 : 1];
  auto mload = [&](int item) {
    int b, y0, x0;
    P.T.at(t0 + item / slices, b, y0, x0);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int e = lane + 64 * k, px = e / 4, c8 = (e - px * 4) * 8;
      const int row = 2 * rg + px / 32, col = px % 32, c = n0 + 32 * ng + c8;
      const size_t p = (size_t)(b * H + y0 + row) * W + x0 + col;
      if (c >= P.mc0) {
        mk[k] = *reinterpret_cast<const bf16x8 *>(P.dmask.p + p * P.dmask.cs + P.dmask.coff + c);
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) mk[k][j] = (bf16)1.f;  // not a ReLU output: kept
      }
    }
  };
  auto lstore = [&](int item) {
#pragma unroll
    for (int it = 0; it < XIT; ++it) {
      const int q = tid + NTH * it;
      if (q < XN) {
        const int pix = q / CPP, ch = (q - pix * CPP) * 8;
        *reinterpret_cast<bf16x8 *>(&Xs[pix * XP + ch]) = xa[it];
      }
    }
    if (!SW) wstore(0);
  };
  if (SW && items > 0) {  // every slice's weights, staged once
    for (int sl = 0; sl < slices; ++sl) {
      wload(sl);
      wstore(sl);
    }
  }
  if (items > 0) gload(0);
  for (int item = 0; item < items; ++item) {
    if (item) __syncthreads();  // the previous item's reads are done
    lstore(item);
    __syncthreads();
    if (BWD && P.dmask.p && item % slices == slices - 1) mload(item);
    if (item + 1 < items) gload(item + 1);
    const bf16 *Wsl = Ws + (SW ? (item % slices) * WSL : 0);
#pragma unroll
    for (int w = 0; w < NWS; ++w) {
      int ky, kx;
      bool ok = true;
      if (C8) {
        const int tap = 4 * w + g;
        ok = tap < 9;
        ky = tap / 3;
        kx = tap - 3 * ky;
      } else {
        ky = w / 3;
        kx = w - 3 * ky;
      }
      bf16x8 bw[NT];
#pragma unroll
      for (int j = 0; j < NT; ++j)
        bw[j] = *reinterpret_cast<const bf16x8 *>(&Wsl[(w * BN + 32 * ng + 16 * j + l16) * DP + 8 * g]);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = 2 * rg + (i >> 1), col = 16 * (i & 1) + l16;
        bf16x8 a;
        if (C8) a = ok ? *reinterpret_cast<const bf16x8 *>(&Xs[((row + ky) * DW + col + kx) * 8]) : zero8();
        else a = *reinterpret_cast<const bf16x8 *>(&Xs[((row + ky) * DW + col + kx) * DP + 8 * g]);
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw[j], acc[i][j], 0, 0, 0);
      }
    }
    if (item % slices != slices - 1) continue;
    // the tile's last slice: bias and ReLU (forward), then each wave's 64
    // pixels x 32 channels through its own part of Xs (pixel pitch OP) as
    // 16-byte rows, masked (backward-data) and stored; no global loads here
    // (they would wait for the prefetch)
    int b, y0, x0;
    P.T.at(t0 + item / slices, b, y0, x0);
    __syncthreads();  // every wave is done reading Xs for this item
    bf16 *O = Xs + wave * 64 * OP;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < NT; ++j) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float r = acc[i][j][q] + bias[j];
          O[(32 * (i >> 1) + 16 * (i & 1) + 4 * g + q) * OP + 16 * j + l16] = (bf16)(BWD ? r : r > 0.f ? r : 0.f);
        }
        acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      }
    __syncthreads();
    const View<bf16> &Y = BWD ? P.dy : P.y;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int e = lane + 64 * k, px = e / 4, c8 = (e - px * 4) * 8;
      const int row = 2 * rg + px / 32, col = px % 32;
      const size_t p = (size_t)(b * H + y0 + row) * W + x0 + col;
      bf16x8 v = *reinterpret_cast<const bf16x8 *>(&O[px * OP + c8]);
      if (BWD && P.dmask.p) {
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = (float)mk[k][j] > 0.f ? v[j] : (bf16)0.f;
      }
      *reinterpret_cast<bf16x8 *>(Y.p + p * Y.cs + Y.coff + n0 + 32 * ng + c8) = v;
    }
    if (!BWD && P.pool.p) {
      // the wave's two rows are one row of 2x2 windows (y0 and the row pair
      // are even): lane = (pooled pixel of 16, 8-channel chunk)
      const int px = lane >> 2, c8 = (lane & 3) * 8;
      bf16x8 m = *reinterpret_cast<const bf16x8 *>(&O[(2 * px) * OP + c8]);
      uint32_t arg[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
      for (int d = 1; d < 4; ++d) {
        const bf16x8 o = *reinterpret_cast<const bf16x8 *>(&O[(32 * (d >> 1) + 2 * px + (d & 1)) * OP + c8]);
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if ((float)o[j] > (float)m[j]) {
            m[j] = o[j];
            arg[j] = d;
          }
      }
      const size_t q = ((size_t)b * (H / 2) + (y0 / 2 + rg)) * (W / 2) + x0 / 2 + px;
      *reinterpret_cast<bf16x8 *>(P.pool.p + q * P.pool.cs + P.pool.coff + n0 + 32 * ng + c8) = m;
      uint32_t lo = 0, hi = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        lo |= ((float)m[j] > 0.f ? arg[j] : 255u) << (8 * j);
        hi |= ((float)m[j + 4] > 0.f ? arg[j + 4] : 255u) << (8 * j);
      }
      *reinterpret_cast<uint2 *>(P.parg + q * P.Nc + n0 + 32 * ng + c8) = make_uint2(lo, hi);
    }
  }
}

// ---------------------------------------------------------------------------
struct DWGrad {
  Img g;
  DTiles T;
  int tps;                 // tiles per split (split z sums tiles z tps ..)
  View<const bf16> dout;   // output gradient of the layer (Cout channels),
                           // already masked by the layer's ReLU
  View<const bf16> in;     // the layer's input (Cin channels)
  int Cin, Cout;
  float *partial;          // [splits][Cout][9 Cin + 1]
};

constexpr int WA_P = DT_H * DT_W + 8;  // co pitch (bf16) of the transposed output gradient: 528 B
constexpr int WB_R = 40;               // row pitch of the transposed input (34 columns used)
constexpr int WB_P = DH * WB_R + 8;    // ci pitch: 816 B
// Each group of 8 channels starts a further WA_O / WB_O bf16 on: eight rows
// of either pitch span a whole number of bank rows, so without it the
// staging writes of the 4 (8) channel groups in one instruction all hit the
// same banks.  Measured per training step: weight gradients 411 us without
// the offsets, 371 with 32 / 16, 360 with 16 / 8 (8 / 8, 24 / 8 and 16 / 24
// within 4 us of it, 64 / 32 slower).
constexpr int WA_O = 16, WB_O = 8;
__device__ __forceinline__ int wa_row(int co) { return co * WA_P + (co >> 3) * WA_O; }
__device__ __forceinline__ int wb_row(int ci) { return ci * WB_P + (ci >> 3) * WB_O; }

// Block (split, 32 output channels, 16 HW input channels; HW = 1 for the
// padded network input, whose channels 8..15 are staged as zeros), 2 HW
// waves.  Wave w: output channels 16 (w & 1), input channels 16 (w >> 1), all
// nine taps; K = the 32 pixels of one tile row.  The output-gradient tile is
// staged once for all 16 HW input channels.
template <bool C8, int HW>
__global__ __launch_bounds__(128 * HW, 2) void k_dwgrad(DWGrad P) {
  constexpr int CI = 16 * HW, NTH = 128 * HW;
  __shared__ __attribute__((aligned(16))) bf16 As[32 * WA_P + 4 * WA_O];        // dPre^T [co][r][c]
  __shared__ __attribute__((aligned(16))) bf16 Bs[CI * WB_P + CI / 8 * WB_O];   // in^T [ci][rr][cc], pixel (y0+rr-1, x0+cc-1)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, l16 = lane & 15, g = lane >> 4;
  const int mt = wave & 1, h = wave >> 1;
  const int co0 = blockIdx.y * 32, ci0 = blockIdx.z * CI;
  const int H = P.g.H, W = P.g.W;
  f4 acc[9], accb = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k = 0; k < 9; ++k) acc[k] = f4{0.f, 0.f, 0.f, 0.f};
  bf16x8 ones;
#pragma unroll
  for (int j = 0; j < 8; ++j) ones[j] = (bf16)1.f;
  const int z = blockIdx.x;
  const int tb = z * P.tps, te = min(P.T.n, tb + P.tps);
  // staging registers of one tile: output gradient and input, two pixels x
  // 8 channels per item
  constexpr int AN = DT_H * DT_W / 2 * 4, AIT = AN / NTH;
  constexpr int NCH = CI / 8, BN_ = DH * (DW / 2) * NCH, BIT = (BN_ + NTH - 1) / NTH;
  bf16x8 ga[AIT][2], ib[BIT][2];
  auto gload = [&](int t) {
    int b, y0, x0;
    P.T.at(t, b, y0, x0);
#pragma unroll
    for (int it = 0; it < AIT; ++it) {
      const int q = tid + NTH * it;
      const int cq = q & 3, pp = q >> 2, r = pp >> 4, c = 2 * (pp & 15);
      const int p = (b * H + y0 + r) * W + x0 + c;
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const size_t o = (size_t)(p + e);
        ga[it][e] = *reinterpret_cast<const bf16x8 *>(P.dout.p + o * P.dout.cs + P.dout.coff + co0 + 8 * cq);
      }
    }
#pragma unroll
    for (int it = 0; it < BIT; ++it) {
      const int q = tid + NTH * it;
      const int cq = q % NCH, pp = q / NCH, rr = pp / (DW / 2), cc = 2 * (pp - rr * (DW / 2));
      const int yy = y0 + rr - 1, xa = x0 + cc - 1;
      ib[it][0] = ib[it][1] = zero8();
      if (q < BN_ && (!C8 || cq == 0) && yy >= 0 && yy < H) {
        const bf16 *rowp = P.in.p + (size_t)(b * H + yy) * W * P.in.cs + P.in.coff + ci0 + 8 * cq;
        if (xa >= 0) ib[it][0] = *reinterpret_cast<const bf16x8 *>(rowp + (size_t)xa * P.in.cs);
        if (xa + 1 < W) ib[it][1] = *reinterpret_cast<const bf16x8 *>(rowp + (size_t)(xa + 1) * P.in.cs);
      }
    }
  };
  auto lstore = [&]() {
#pragma unroll
    for (int it = 0; it < AIT; ++it) {
      const int q = tid + NTH * it;
      const int cq = q & 3, pp = q >> 2, r = pp >> 4, c = 2 * (pp & 15);
#pragma unroll
      for (int j = 0; j < 8; ++j)
        *reinterpret_cast<uint32_t *>(&As[wa_row(8 * cq + j) + r * DT_W + c]) = pack_bf16(ga[it][0][j], ga[it][1][j]);
    }
#pragma unroll
    for (int it = 0; it < BIT; ++it) {
      const int q = tid + NTH * it;
      if (q < BN_) {
        const int cq = q % NCH, pp = q / NCH, rr = pp / (DW / 2), cc = 2 * (pp - rr * (DW / 2));
#pragma unroll
        for (int j = 0; j < 8; ++j)
          *reinterpret_cast<uint32_t *>(&Bs[wb_row(8 * cq + j) + rr * WB_R + cc]) = pack_bf16(ib[it][0][j], ib[it][1][j]);
      }
    }
  };
  if (tb < te) gload(tb);
  for (int t = tb; t < te; ++t) {
    __syncthreads();  // the previous tile's reads are done
    lstore();
    __syncthreads();
    if (t + 1 < te) gload(t + 1);
    {
      // each staged input row rr is read once and serves the output rows
      // r = rr - ky, ky = 0..2 (tap row ky); the three column shifts kx come
      // from one 16-byte read and the next 4 bytes
      bf16x8 a[DT_H];
#pragma unroll
      for (int rr = 0; rr < DH; ++rr) {
        if (rr < DT_H) {
          a[rr] = *reinterpret_cast<const bf16x8 *>(&As[wa_row(16 * mt + l16) + rr * DT_W + 8 * g]);
          if (h == 0) accb = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[rr], ones, accb, 0, 0, 0);
        }
        const bf16 *src = &Bs[wb_row(16 * h + l16) + rr * WB_R + 8 * g];
        const u32x4 lo = *reinterpret_cast<const u32x4 *>(src);
        const uint32_t hi = *reinterpret_cast<const uint32_t *>(src + 8);
        u32x4 s1, s2;  // windows starting one and two pixels further right
        s1[0] = __builtin_amdgcn_alignbyte(lo[1], lo[0], 2);
        s1[1] = __builtin_amdgcn_alignbyte(lo[2], lo[1], 2);
        s1[2] = __builtin_amdgcn_alignbyte(lo[3], lo[2], 2);
        s1[3] = __builtin_amdgcn_alignbyte(hi, lo[3], 2);
        s2[0] = lo[1];
        s2[1] = lo[2];
        s2[2] = lo[3];
        s2[3] = hi;
#pragma unroll
        for (int ky = 0; ky < 3; ++ky) {
          const int r = rr - ky;
          if (r < 0 || r >= DT_H) continue;
          acc[3 * ky + 0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[r], __builtin_bit_cast(bf16x8, lo), acc[3 * ky + 0], 0, 0, 0);
          acc[3 * ky + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[r], __builtin_bit_cast(bf16x8, s1), acc[3 * ky + 1], 0, 0, 0);
          acc[3 * ky + 2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[r], __builtin_bit_cast(bf16x8, s2), acc[3 * ky + 2], 0, 0, 0);
        }
      }
    }
  }
  const int Kw = 9 * P.Cin;
  const int ci = ci0 + 16 * h + l16;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int co = co0 + 16 * mt + 4 * g + q;
    float *row = P.partial + ((size_t)z * P.Cout + co) * (Kw + 1);
    if (ci < P.Cin) {
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) row[tap * P.Cin + ci] = acc[tap][q];
    }
    if (h == 0 && blockIdx.z == 0 && l16 == 0) row[Kw] = accb[q];
  }
}

// Weight and bias gradient of the up-sampling, for input rows of whole
// 32-pixel segments:  dW[d][co][ci] = sum_p dOut[up(p,d), co] in[p, ci] over
// input pixels p, db[co] = sum over d and p of dOut[up(p,d), co].  A block
// (split, 32 output channels of one parity d, 16 HW input channels; 2 HW
// waves) sums a run of items of 128 input pixels (four segments), both
// operands staged transposed (pixels contiguous, the MFMA's reduction
// dimension) as in k_dwgrad, the next item's loads issued before the current
// MFMAs.  Partials [split][4 Cout][Cin + 1]: row d Cout + co, the last column
// the row's bias sum (k_wreduce adds those of the four parities).
struct DUpW {
  Img g;                   // input image
  int segs, nseg;          // 32-pixel segments per row, in all
  int ipb;                 // items (4 segments) per split
  View<const bf16> dout;   // gradient of the output image (Cout channels)
  View<const bf16> in;     // input (Cin channels)
  int Cin, Cout;
  float *partial;
};
constexpr int UW_K = 128, UW_P = UW_K + 8;  // input pixels per item; LDS pitch (bf16)
// channel groups of 8 offset as in k_dwgrad (the pitch times 8 spans whole bank rows)
__device__ __forceinline__ int uwa_row(int co) { return co * UW_P + (co >> 3) * 32; }
__device__ __forceinline__ int uwb_row(int ci) { return ci * UW_P + (ci >> 3) * 16; }

template <int HW>
__global__ __launch_bounds__(128 * HW, 2) void k_upwgrad(DUpW P) {
  constexpr int CI = 16 * HW, NTH = 128 * HW;
  constexpr int AN = UW_K / 2 * 4, AIT = (AN + NTH - 1) / NTH;  // pixel pairs x 8-channel chunks
  constexpr int BNI = UW_K / 2 * (CI / 8), BIT = (BNI + NTH - 1) / NTH;
  __shared__ __attribute__((aligned(16))) bf16 As[32 * UW_P + 4 * 32];       // dOut^T [co][px]
  __shared__ __attribute__((aligned(16))) bf16 Bs[CI * UW_P + CI / 8 * 16];  // in^T [ci][px]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, l16 = lane & 15, g = lane >> 4;
  const int mt = wave & 1, h = wave >> 1;
  const int cot = P.Cout / 32, d = blockIdx.y / cot, co0 = (blockIdx.y % cot) * 32, ci0 = blockIdx.z * CI;
  const int H = P.g.H, W = P.g.W, z = blockIdx.x;
  const int items_total = (P.nseg + 3) / 4;
  const int i0 = z * P.ipb, i1 = min(items_total, i0 + P.ipb);
  f4 acc = f4{0.f, 0.f, 0.f, 0.f}, accb = acc;
  bf16x8 ones;
#pragma unroll
  for (int j = 0; j < 8; ++j) ones[j] = (bf16)1.f;
  bf16x8 ga[AIT][2], ib[BIT][2];
  // input pixel k (0..127) of item it: its segment, row and column; -1 if past the last segment
  auto pixel = [&](int it, int k, int &row, int &x) {
    const int sg = it * 4 + k / 32;
    if (sg >= P.nseg) return false;
    row = sg / P.segs;
    x = (sg - row * P.segs) * 32 + k % 32;
    return true;
  };
  auto gload = [&](int it) {
#pragma unroll
    for (int a = 0; a < AIT; ++a) {
      const int q = tid + NTH * a;
      const int cq = q & 3, k = 2 * (q >> 2);
      int row, x;
      ga[a][0] = ga[a][1] = zero8();
      if (q < AN && pixel(it, k, row, x)) {
        const int y = row % H, b = row / H;
        const size_t Yr = ((size_t)b * 2 * H + 2 * y + (d >> 1)) * 2 * W + (d & 1);
#pragma unroll
        for (int e = 0; e < 2; ++e)
          ga[a][e] = *reinterpret_cast<const bf16x8 *>(P.dout.p + (Yr + 2 * (x + e)) * P.dout.cs + P.dout.coff + co0 +
                                                       8 * cq);
      }
    }
#pragma unroll
    for (int a = 0; a < BIT; ++a) {
      const int q = tid + NTH * a;
      const int cq = q % (CI / 8), k = 2 * (q / (CI / 8));
      int row, x;
      ib[a][0] = ib[a][1] = zero8();
      if (q < BNI && pixel(it, k, row, x)) {
        const bf16 *s = P.in.p + ((size_t)row * W + x) * P.in.cs + P.in.coff + ci0 + 8 * cq;
        ib[a][0] = *reinterpret_cast<const bf16x8 *>(s);
        ib[a][1] = *reinterpret_cast<const bf16x8 *>(s + P.in.cs);
      }
    }
  };
  auto lstore = [&]() {
#pragma unroll
    for (int a = 0; a < AIT; ++a) {
      const int q = tid + NTH * a;
      if (q < AN) {
        const int cq = q & 3, k = 2 * (q >> 2);
#pragma unroll
        for (int j = 0; j < 8; ++j)
          *reinterpret_cast<uint32_t *>(&As[uwa_row(8 * cq + j) + k]) = pack_bf16(ga[a][0][j], ga[a][1][j]);
      }
    }
#pragma unroll
    for (int a = 0; a < BIT; ++a) {
      const int q = tid + NTH * a;
      if (q < BNI) {
        const int cq = q % (CI / 8), k = 2 * (q / (CI / 8));
#pragma unroll
        for (int j = 0; j < 8; ++j)
          *reinterpret_cast<uint32_t *>(&Bs[uwb_row(8 * cq + j) + k]) = pack_bf16(ib[a][0][j], ib[a][1][j]);
      }
    }
  };
  if (i0 < i1) gload(i0);
  for (int it = i0; it < i1; ++it) {
    __syncthreads();  // the previous item's reads are done
    lstore();
    __syncthreads();
    if (it + 1 < i1) gload(it + 1);
#pragma unroll
    for (int ks = 0; ks < UW_K / 32; ++ks) {
      const bf16x8 av = *reinterpret_cast<const bf16x8 *>(&As[uwa_row(16 * mt + l16) + 32 * ks + 8 * g]);
      const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(&Bs[uwb_row(16 * h + l16) + 32 * ks + 8 * g]);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
      if (h == 0) accb = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, ones, accb, 0, 0, 0);
    }
  }
  const int ci = ci0 + 16 * h + l16;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int m = d * P.Cout + co0 + 16 * mt + 4 * g + q;
    float *row = P.partial + ((size_t)z * 4 * P.Cout + m) * (P.Cin + 1);
    if (ci < P.Cin) row[ci] = acc[q];
    if (h == 0 && blockIdx.z == 0 && l16 == 0) row[P.Cin] = accb[q];
  }
}

// Fixed-order sums of split partials, several weight gradients per launch.
// Job j: partials [splits][E] (E = rows (Kw + 1), a multiple of 4; column Kw
// of each row is that row's bias sum) into dW [rows][Kw] and db.  Cb = rows:
// db[m] is row m's bias.  Cb < rows (the up-sampling, rows d Cout + co): db[c]
// sums the bias columns of rows c, c + Cb, ...
// A weight block has 16 waves; a job with G split groups (G = 2^gsh, about
// splits / 16, at most 16) gives each lane a float4 of partials and each run
// of G waves 256 consecutive elements: group g adds splits g, g + G, ... in
// four interleaved partial sums, then the groups combine by a fixed tree (so
// a lane adds at most 16 loads but for the 512 splits of the padded input's
// layer, whatever the split count).  A bias block of a
// Cb < rows job gives one bias to each of its 16 waves: lane l adds the terms
// l, l + 64, ... of (split, row) in split-major order, then a fixed shuffle
// tree, lane 0's sum being the result.
constexpr int WR_G = 16, WJ_MAX = 24;
struct WJob {
  const float *partial;
  float *dW, *db;
  int splits, E, Kw, Cb;
  int blk0, nbw;  // first block; weight blocks (then ceil(Cb / 16) bias blocks if Cb < rows)
  int gsh;        // log2 of the split groups
};
struct WJobs {
  int n;
  WJob j[WJ_MAX];
};

static __global__ __launch_bounds__(64 * WR_G) void k_wreduce(WJobs J) {
  __shared__ float4 sh[WR_G][64];
  int jj = 0;
  while (jj + 1 < J.n && (int)blockIdx.x >= J.j[jj + 1].blk0) ++jj;
  const WJob &jb = J.j[jj];
  const int blk = (int)blockIdx.x - jb.blk0;
  const int lane = threadIdx.x & 63, gr = threadIdx.x >> 6;
  const int rows = jb.E / (jb.Kw + 1);
  if (blk >= jb.nbw) {  // bias block
    const int c = (blk - jb.nbw) * WR_G + gr, R = rows / jb.Cb, T = jb.splits * R;
    if (c >= jb.Cb) return;
    float s = 0.f;
    for (int t = lane; t < T; t += 64) {
      const int z = t / R, k = t - z * R;
      s += jb.partial[(size_t)z * jb.E + (size_t)(c + k * jb.Cb) * (jb.Kw + 1) + jb.Kw];
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) jb.db[c] = s;
    return;
  }
  const int G = 1 << jb.gsh, g = gr & (G - 1);
  const int e4 = (blk * (WR_G >> jb.gsh) + (gr >> jb.gsh)) * 64 + lane, E4 = jb.E / 4, splits = jb.splits;
  float4 a0 = {0.f, 0.f, 0.f, 0.f}, a1 = a0, a2 = a0, a3 = a0;
  if (e4 < E4) {
    const float4 *p = reinterpret_cast<const float4 *>(jb.partial) + e4;
    const size_t st = (size_t)E4;
    int z = g;
    for (; z + 3 * G < splits; z += 4 * G) {
      const float4 v0 = p[z * st], v1 = p[(z + G) * st], v2 = p[(z + 2 * G) * st], v3 = p[(z + 3 * G) * st];
      a0.x += v0.x; a0.y += v0.y; a0.z += v0.z; a0.w += v0.w;
      a1.x += v1.x; a1.y += v1.y; a1.z += v1.z; a1.w += v1.w;
      a2.x += v2.x; a2.y += v2.y; a2.z += v2.z; a2.w += v2.w;
      a3.x += v3.x; a3.y += v3.y; a3.z += v3.z; a3.w += v3.w;
    }
    for (; z < splits; z += G) {
      const float4 v = p[z * st];
      a0.x += v.x; a0.y += v.y; a0.z += v.z; a0.w += v.w;
    }
  }
  float4 s;
  s.x = (a0.x + a1.x) + (a2.x + a3.x);
  s.y = (a0.y + a1.y) + (a2.y + a3.y);
  s.z = (a0.z + a1.z) + (a2.z + a3.z);
  s.w = (a0.w + a1.w) + (a2.w + a3.w);
  sh[gr][lane] = s;
  __syncthreads();
  for (int w = G / 2; w >= 1; w >>= 1) {
    if (g < w) {
      float4 &d = sh[gr][lane];
      const float4 o = sh[gr + w][lane];
      d.x += o.x; d.y += o.y; d.z += o.z; d.w += o.w;
    }
    __syncthreads();
  }
  if (g == 0 && e4 < E4) {
    const float4 v = sh[gr][lane];
    const float vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int e = 4 * e4 + k, m = e / (jb.Kw + 1), c = e - m * (jb.Kw + 1);
      if (c < jb.Kw) jb.dW[(size_t)m * jb.Kw + c] = vv[k];
      else if (jb.Cb == rows) jb.db[m] = vv[k];
    }
  }
}

// ---------------------------------------------------------------------------
// 2x2 stride-2 transposed convolution (up-sampling), forward, for an input
// image whose width is a multiple of 32, without the implicit GEMM's
// scattered 2-byte stores.  A block owns a 32-pixel segment of one input
// row; wave d (parity dy = d >> 1, dx = d & 1) computes
//   out[(2y+dy, 2x+dx), co] = b[co] + sum_ci W[d][co][ci] in[(y,x), ci]
// for the segment's 32 pixels and all Cout channels and writes them as
// 16-byte rows through LDS.  (A direct data gradient, with each wave loading
// its operand itself, measured slower than the implicit GEMM, which
// stages it once per block: 18.5 -> 41 us at level 0; it is not used.)
struct DUp {
  Img g;                  // input image
  int segs;               // 32-pixel segments per input row
  int Cin, Cout;
  View<const bf16> in;    // input (Cin channels)
  const bf16 *Wt;         // [4][Cout][Cin]
  const float *bias;
  View<bf16> out;         // output image, 2H x 2W (Cout channels)
};

template <int NT>  // NT = Cout / 16
__global__ __launch_bounds__(256) void k_upfwd(DUp P) {
  constexpr int OPU = 16 * NT + 8;  // LDS pixel pitch of the staged output (bf16)
  __shared__ __attribute__((aligned(16))) bf16 Os[4][32 * OPU];
  const int lane = threadIdx.x & 63, d = threadIdx.x >> 6, l16 = lane & 15, g = lane >> 4;
  const int H = P.g.H, W = P.g.W;
  const int seg = blockIdx.x, x0 = (seg % P.segs) * 32, row = seg / P.segs;  // row = b H + y
  const int y = row % H, b = row / H;
  f4 acc[2][NT];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  const bf16 *ip = P.in.p + ((size_t)row * W + x0) * P.in.cs + P.in.coff;
  for (int k0 = 0; k0 < P.Cin; k0 += 32) {
    bf16x8 a[2], bw[NT];
#pragma unroll
    for (int i = 0; i < 2; ++i)
      a[i] = *reinterpret_cast<const bf16x8 *>(ip + (size_t)(16 * i + l16) * P.in.cs + k0 + 8 * g);
#pragma unroll
    for (int j = 0; j < NT; ++j)
      bw[j] = *reinterpret_cast<const bf16x8 *>(P.Wt + ((size_t)d * P.Cout + 16 * j + l16) * P.Cin + k0 + 8 * g);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < NT; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], bw[j], acc[i][j], 0, 0, 0);
  }
  bf16 *O = Os[d];
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    const float bj = P.bias[16 * j + l16];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q) O[(16 * i + 4 * g + q) * OPU + 16 * j + l16] = (bf16)(acc[i][j][q] + bj);
  }
  __syncthreads();
  const int Y = 2 * y + (d >> 1), dx = d & 1;
  constexpr int CH = 2 * NT;  // 16-byte chunks per output pixel
  for (int e = lane; e < 32 * CH; e += 64) {
    const int px = e / CH, c8 = (e - px * CH) * 8;
    const size_t q = ((size_t)b * 2 * H + Y) * 2 * W + 2 * (x0 + px) + dx;
    *reinterpret_cast<bf16x8 *>(P.out.p + q * P.out.cs + P.out.coff + c8) =
        *reinterpret_cast<const bf16x8 *>(&O[px * OPU + c8]);
  }
}

// ---------------------------------------------------------------------------
// Training head: the 1x1 head (C0 -> 8 channels, the first cout real), the
// loss and the head's backward in one pass over the last decoder output:
//   y[p][o]    = b[o] + sum_c W[o][c] act[p][c]             (FP32, o < cout)
//   loss       = sum over p and o < cout of (y - t)^2         (FP64)
//   dy[p][o]   = BF16(2 (y - t) / (P cout)), 0 for o >= cout
//   dact[p][c] = BF16(sum_o W[o][c] dy[p][o]) where act[p][c] > 0, else 0
//                (act is a ReLU output; its gradient is stored masked)
//   dW[o][c]   = sum_p dy[p][o] act[p][c],  db[o] = sum_p dy[p][o]
// The products are those of the implicit-GEMM head (BF16 weights and
// activations, FP32 sums); only the summation order differs.  A block takes
// runs of 256 pixels, a pixel per thread for y, the loss, dy and dact; dW and
// db go through the MFMA: the run's dy^T (16 rows, 8..15 zero) and act^T
// (channels padded to 16 NT) are staged in LDS, pixels contiguous, and wave w
// adds K steps 2w and 2w + 1 of every run.  At the end the four waves' sums
// are added in order; the block writes partials [block][8][C0 + 1] (bias
// last) and the FP64 loss sum of its pixels.
struct DHead {
  int P, C0, cout, rpb;    // pixels, head input channels, real outputs, runs per block
  View<const bf16> act;    // last decoder output (C0 channels)
  const bf16 *W;           // [8][C0]
  const float *bias;       // [8]
  const float *t;          // target [P][cout]
  float Pc;                // P cout
  View<bf16> dact;         // gradient of act
  float *partial;          // [blocks][8][C0 + 1]
  double *loss;            // [blocks]
};
constexpr int HD_P = 256 + 8;  // LDS pitch (bf16) of a staged row of 256 pixels

inline size_t head_lds_bytes(int C0, int NT) { return (size_t)8 * C0 * 4 + (size_t)16 * HD_P * 2 + (size_t)16 * NT * HD_P * 2; }

template <int NT>
__global__ __launch_bounds__(256) void k_head(DHead P) {
  extern __shared__ __attribute__((aligned(16))) unsigned char hsm[];
  __shared__ double lsh[256];
  const int C0 = P.C0, C8 = C0 / 8, NP = 16 * NT + 1;
  float *Wf = reinterpret_cast<float *>(hsm);         // [8][C0]
  bf16 *dyT = reinterpret_cast<bf16 *>(Wf + 8 * C0);  // [16][HD_P]
  bf16 *acT = dyT + 16 * HD_P;                        // [16 NT][HD_P]
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, l16 = lane & 15, g = lane >> 4;
  for (int i = tid; i < 8 * C0; i += 256) Wf[i] = (float)P.W[i];
  for (int i = tid; i < 8 * HD_P; i += 256) dyT[8 * HD_P + i] = (bf16)0.f;
  for (int i = tid; i < (16 * NT - C0) * HD_P; i += 256) acT[C0 * HD_P + i] = (bf16)0.f;
  float bias[8];
#pragma unroll
  for (int o = 0; o < 8; ++o) bias[o] = P.bias[o];
  f4 acc[NT], accb = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) acc[nt] = f4{0.f, 0.f, 0.f, 0.f};
  bf16x8 ones;
#pragma unroll
  for (int j = 0; j < 8; ++j) ones[j] = (bf16)1.f;
  double esum = 0.0;
  const int nruns = (P.P + 255) / 256, r0 = blockIdx.x * P.rpb, r1 = min(nruns, r0 + P.rpb);
  __syncthreads();
  for (int r = r0; r < r1; ++r) {
    const int p = r * 256 + tid;
    const bool live = p < P.P;
    float y[8];
#pragma unroll
    for (int o = 0; o < 8; ++o) y[o] = bias[o];
    const bf16 *ap = P.act.p + (size_t)p * P.act.cs + P.act.coff;
    constexpr bool KEEP = NT <= 4;  // the pixel's activations stay in registers for the mask
    bf16x8 av[KEEP ? 2 * NT : 1];
#pragma unroll
    for (int k = 0; k < (KEEP ? 2 * NT : C8); ++k) {
      if (k >= C8) break;
      const bf16x8 v = live ? *reinterpret_cast<const bf16x8 *>(ap + 8 * k) : zero8();
      if constexpr (KEEP) av[k] = v;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const float a = (float)v[j];
#pragma unroll
        for (int o = 0; o < 8; ++o) y[o] += Wf[o * C0 + 8 * k + j] * a;
        acT[(8 * k + j) * HD_P + tid] = v[j];
      }
    }
    float dy[8];
#pragma unroll
    for (int o = 0; o < 8; ++o) {
      dy[o] = 0.f;
      if (live && o < P.cout) {
        const float d = y[o] - P.t[(size_t)p * P.cout + o];
        esum += (double)d * d;
        dy[o] = (float)(bf16)(2.f * d / P.Pc);
      }
      dyT[o * HD_P + tid] = (bf16)dy[o];
    }
    if (live) {
      bf16 *dp = P.dact.p + (size_t)p * P.dact.cs + P.dact.coff;
#pragma unroll
      for (int k = 0; k < (KEEP ? 2 * NT : C8); ++k) {
        if (k >= C8) break;
        const bf16x8 a = KEEP ? av[k] : *reinterpret_cast<const bf16x8 *>(ap + 8 * k);  // the ReLU mask
        bf16x8 v;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          float s = 0.f;
#pragma unroll
          for (int o = 0; o < 8; ++o) s += Wf[o * C0 + 8 * k + j] * dy[o];
          v[j] = (float)a[j] > 0.f ? (bf16)s : (bf16)0.f;
        }
        *reinterpret_cast<bf16x8 *>(dp + 8 * k) = v;
      }
    }
    __syncthreads();
#pragma unroll
    for (int ks = 2 * w; ks < 2 * w + 2; ++ks) {
      const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&dyT[l16 * HD_P + 32 * ks + 8 * g]);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const bf16x8 b = *reinterpret_cast<const bf16x8 *>(&acT[(16 * nt + l16) * HD_P + 32 * ks + 8 * g]);
        acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[nt], 0, 0, 0);
      }
      accb = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, ones, accb, 0, 0, 0);
    }
    __syncthreads();
  }
  // the four waves' sums, rows o = 4 g + q < 8, in the staging area
  float *red = reinterpret_cast<float *>(acT);  // [4][8][16 NT + 1]
  if (g < 2) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int o = 4 * g + q;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) red[(w * 8 + o) * NP + 16 * nt + l16] = acc[nt][q];
      if (l16 == 0) red[(w * 8 + o) * NP + 16 * NT] = accb[q];
    }
  }
  lsh[tid] = esum;
  __syncthreads();
  for (int i = tid; i < 8 * (C0 + 1); i += 256) {
    const int o = i / (C0 + 1), c = i - o * (C0 + 1), cc = c == C0 ? 16 * NT : c;
    float s = 0.f;
#pragma unroll
    for (int v = 0; v < 4; ++v) s += red[(v * 8 + o) * NP + cc];
    P.partial[(size_t)blockIdx.x * 8 * (C0 + 1) + i] = s;
  }
  for (int s = 128; s >= 1; s >>= 1) {
    if (tid < s) lsh[tid] += lsh[tid + s];
    __syncthreads();
  }
  if (tid == 0) P.loss[blockIdx.x] = lsh[0];
}

}  // namespace wsk
