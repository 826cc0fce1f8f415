// Learned IDA denoiser on gfx950: an 8-layer 3x3 convolutional network with
// 64 channels (layer 1: 2 -> 64, layers 2..7: 64 -> 64, layer 8: 64 -> 1),
// bias and ReLU after layers 1..7, zero padding, residual output
//   D(v) = v - 255 f([v / 255, min(sigma, 255) / 255]).
// Weights and activations are bfloat16, sums are float32.  The stand-in for
// the paper's DnCNN (Section VI-4), which has 17 layers with batch
// normalisation; its trained weights are not available.
//
// Parameter blob (float32, caller-owned), layer after layer: weights
// [C_out][3][3][C_in] then bias [C_out]; tap = 3 dy + dx for the offsets
// (dy - 1, dx - 1).  Activations are NHWC: pixel p of an image holds its 64
// channels contiguously; an image's pixels use the plan's decoded-image
// numbering (out_off + y W' + x).
#pragma once

#include "common.hpp"

namespace abcs {

namespace cnn {
constexpr int kCh = 64;
constexpr int kLayers = 8;
// Parameter offsets in the float32 blob.
constexpr int kW1 = 0, kB1 = kW1 + 64 * 9 * 2;                 // 1152
constexpr int kMid0 = kB1 + 64;                                // 1216
constexpr int kMidW = 64 * 9 * 64, kMidStride = kMidW + 64;    // 36864, 36928
constexpr int kW8 = kMid0 + 6 * kMidStride;                    // 222784
constexpr int kB8 = kW8 + 9 * 64;                              // 223360
constexpr int kParams = kB8 + 1;                               // 223361
constexpr int kTileH = 8, kTileW = 16;                         // pixels per conv tile
constexpr int kPxStride = 72;                                  // bf16 per staged pixel (64 + pad)
}  // namespace cnn

struct CnnTile {
  int32_t img, y0, x0, pad_;
};

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

// float32 -> bfloat16, round to nearest even (v_cvt_pk_bf16_f32; NaN stays NaN).
__device__ __forceinline__ unsigned short f2bf(float f) { return __builtin_bit_cast(unsigned short, (__bf16)f); }
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float((uint32_t)h << 16); }
// Two float32 -> two bfloat16 (round to nearest even) in one register, a in
// the low half: one paired conversion, the same bits as f2bf of each.
__device__ __forceinline__ uint32_t pack_bf2(float a, float b) {
  typedef float f32x2v __attribute__((ext_vector_type(2)));
  typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2v){a, b}, bf16x2v));
}

// float32 blob -> bfloat16 copies: mid-layer weights in blob order
// ([C_out][tap][C_in]) and, when wt is not null, their transposes with flipped
// taps ([C_in][8 - tap][C_out]) for the input-gradient convolution; layers 1
// and 8 as bfloat16-rounded float32.
__global__ __launch_bounds__(256) void k_cnn_prep(const float* __restrict__ blob, unsigned short* __restrict__ wmid,
                                                 unsigned short* __restrict__ wt, float* __restrict__ w1r,
                                                 float* __restrict__ w8r) {
  using namespace cnn;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < 6 * kMidW) {
    const int l = i / kMidW, e = i - l * kMidW;
    const float w = blob[kMid0 + l * kMidStride + e];
    const unsigned short h = f2bf(w);
    wmid[i] = h;
    if (wt) {
      const int co = e / (9 * 64), tap = (e / 64) % 9, ci = e % 64;
      wt[l * kMidW + (ci * 9 + (8 - tap)) * 64 + co] = h;
    }
  }
  if (i < 64 * 9 * 2) w1r[i] = bf2f(f2bf(blob[kW1 + i]));
  if (i < 9 * 64) w8r[i] = bf2f(f2bf(blob[kW8 + i]));
}

// Layers 2..7 (64 -> 64) on bfloat16 MFMA (v_mfma_f32_16x16x32_bf16).  A
// workgroup computes an 8 x 16-pixel tile: the input tile and its one-pixel
// halo are staged in LDS (zero outside the image), each wavefront keeps the
// weights of 32 output channels in VGPRs (the A operand: 16 channels x 32
// K-values per MFMA, K = tap x input channel) and multiplies them with 16
// pixels x 32 K-values read from LDS (the B operand) for 4 rows of the tile.
// MODE 0: out = bf16(ReLU(sum + bias)).
// MODE 1 (input gradient): weights are the transposed, tap-flipped copy,
//         out = bf16(sum) where mask > 0 (the ReLU of the layer below), else 0.
// MODE 2: out = bf16(sum) (the pre-normalisation values of DnCNN's layers).
//
// Inference (MODE 0) can take the network's first and last layers in:
// kCnnInFirst: the layer's input is layer 1's output, computed while the
//   tile is staged from the network input v (4 bytes per pixel) instead of
//   read as 64 channels (128 bytes per pixel): for the tile and its halo,
//   sum over the 9 taps of w1[c][tap][0] v(q) / 255 + w1[c][tap][1] sigma',
//   on bfloat16 MFMA with every float32 operand split into two bfloat16
//   halves (v / 255 and sigma' = min(sigma, 255) / 255 as hi + lo, weights
//   exact in bfloat16), K = 36 of two 16x16x32 products, then
//   bf16(ReLU(sum + b1)), zero outside the image.
// kCnnOutTaps: instead of its 64 channels a (bfloat16, as stored), the layer
//   writes for each pixel q the nine partial sums t_tap(q) = sum_c w8[tap][c]
//   a_c(q) of the last layer (one 16x16x32 product per row: taps as A rows,
//   a wave's 32 channels as K; the two halves of the channels added in
//   float32), 36 bytes per pixel in nine planes of the plan's pixels, and
//   k_cnn_taps_out adds them up: out(p) = v(p) - 255 (b8 + sum_tap
//   t_tap(p + offset_tap)).
// kCnnKeep (training): kCnnInFirst also writes layer 1's output of the tile
//   to fz.keep, kCnnOutTaps also writes the layer's own output to `out`, so
//   that the backward pass has every activation; the arithmetic is that of
//   inference, so a training step's forward output equals abcs_denoise's.
// kCnnInFirst also serves MODE 2 (DnCNN's training forward).
constexpr int kCnnInFirst = 1, kCnnOutTaps = 2, kCnnKeep = 4;

// Layer 1 for the staged tile of a middle layer (kCnnInFirst): the tile's
// (kTileH + 2) x (kTileW + 2) pixels, taken 16 at a time in raster order
// (wave w takes groups w, w + 4, w + 8), get their 64 channels in `tile`
// (which has room for the last group's 12 spare pixels, so that every lane
// stores).  win holds, over the tile with a two-pixel halo, the four
// bfloat16 K slots of one tap: v / 255 as hi and lo, and sigma' as hi and lo
// where the pixel lies in the image (all zero outside it); w1s the A
// operands (channel c, K slot 4 tap + part); sb1 the bias (16-byte aligned).
// Selections are masks, not branches.
__device__ __forceinline__ void stage_first_layer(const CnnTile& tl, const ImgDev& im, const uint2* win,
                                                  const unsigned short* w1s, const float* sb1, unsigned short* tile,
                                                  int wave, int g, int n) {
  using namespace cnn;
  constexpr int TH = kTileH + 2, TW = kTileW + 2, VW = kTileW + 4;
  constexpr int NPX = TH * TW, NGRP = (NPX + 15) / 16;
  static_assert(NGRP == 3 * kWavesPerGroup, "three pixel groups per wave");
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int t = 16 * (wave + kWavesPerGroup * i) + n;
    const bool valid = t < NPX;
    const int tc = valid ? t : 0;
    const int ty = tc / TW, tx = tc - ty * TW;
    // B operands: K slots 32 kc + 8 g .. + 7 are taps 8 kc + 2 g and 8 kc + 2 g + 1
    uint4 bw[2];
#pragma unroll
    for (int kc = 0; kc < 2; ++kc) {
      uint2 h2[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int tap = 8 * kc + 2 * g + h;
        const bool use = valid && tap < 9;
        const int tp = use ? tap : 0;
        const int dy = tp / 3, dx = tp - 3 * (tp / 3);
        const uint32_t m = use ? 0xffffffffu : 0u;
        const uint2 w = win[(ty + dy) * VW + tx + dx];
        h2[h] = make_uint2(w.x & m, w.y & m);
      }
      bw[kc] = make_uint4(h2[0].x, h2[0].y, h2[1].x, h2[1].y);
    }
    const int cy = tl.y0 + ty - 1, cx = tl.x0 + tx - 1;
    const bool inside = valid && (unsigned)cy < (unsigned)im.Hc && (unsigned)cx < (unsigned)im.Wc;
    const uint32_t keep = inside ? 0xffffffffu : 0u;
    f32x4 acc[4];
#pragma unroll
    for (int cg = 0; cg < 4; ++cg) {
      acc[cg] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kc = 0; kc < 2; ++kc) {
        const bf16x8 a = *(const bf16x8*)(w1s + (16 * cg + n) * 64 + 32 * kc + 8 * g);
        acc[cg] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(bf16x8, bw[kc]), acc[cg], 0, 0, 0);
      }
    }
#pragma unroll
    for (int cg = 0; cg < 4; ++cg) {
      // acc[cg][q]: channel 16 cg + 4 g + q of pixel t
      const int c0 = 16 * cg + 4 * g;
      const float4 bb = *(const float4*)(sb1 + c0);
      uint2 pk;
      pk.x = pack_bf2(fmaxf(acc[cg][0] + bb.x, 0.f), fmaxf(acc[cg][1] + bb.y, 0.f)) & keep;
      pk.y = pack_bf2(fmaxf(acc[cg][2] + bb.z, 0.f), fmaxf(acc[cg][3] + bb.w, 0.f)) & keep;
      *(uint2*)(tile + t * kPxStride + c0) = pk;
    }
  }
}

// out(p) = v(p) - 255 (b8 + sum over taps of t_tap(p + offset_tap)), the
// planes t_tap written by the last middle layer (kCnnOutTaps), zero outside
// the image, taps in order.  Two 8 x 16-pixel tiles per workgroup, one
// pixel per thread.
__global__ __launch_bounds__(256) void k_cnn_taps_out(const ImgDev* __restrict__ imgs,
                                                     const CnnTile* __restrict__ tiles, int ntiles, int64_t pixels,
                                                     const float* __restrict__ taps, const float* __restrict__ v,
                                                     const float* __restrict__ b8p, float* __restrict__ out) {
  using namespace cnn;
  const int ti = 2 * blockIdx.x + (threadIdx.x >> 7);
  if (ti >= ntiles) return;
  const CnnTile tl = tiles[ti];
  const ImgDev im = imgs[tl.img];
  const int y = tl.y0 + ((threadIdx.x & 127) >> 4), x = tl.x0 + (threadIdx.x & 15);
  const float* tp = taps + im.out_off;
  float sum = 0.f;
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) {
    const int yy = y + tap / 3 - 1, xx = x + tap % 3 - 1;
    if ((unsigned)yy < (unsigned)im.Hc && (unsigned)xx < (unsigned)im.Wc)
      sum += tp[tap * pixels + (int64_t)yy * im.Wc + xx];
  }
  const int64_t p = im.out_off + (int64_t)y * im.Wc + x;
  out[p] = v[p] - 255.f * (b8p[0] + sum);
}

struct CnnFuse {
  const float* v;        // kCnnInFirst: the network input (plan pixels)
  const float* sigma;    //   per image
  const float* w1r;      //   layer 1 weights, bfloat16-rounded float32
  const float* b1;       //   layer 1 bias
  const float* w8r;      // kCnnOutTaps: layer 8 weights, bfloat16-rounded float32
  float* taps;           //   nine planes of `plane` floats
  int64_t plane;
  unsigned short* keep;  // kCnnInFirst | kCnnKeep: layer 1's output
};

template <int MODE, int FUSE = 0>
__global__ __launch_bounds__(256, 2) void k_cnn_mid(const ImgDev* __restrict__ imgs, const CnnTile* __restrict__ tiles,
                                                int ntiles, const unsigned short* __restrict__ in,
                                                const unsigned short* __restrict__ w, const float* __restrict__ bias,
                                                const unsigned short* __restrict__ mask,
                                                unsigned short* __restrict__ out, CnnFuse fz) {
  using namespace cnn;
  constexpr bool FIRST = (FUSE & kCnnInFirst) != 0, TAPS = (FUSE & kCnnOutTaps) != 0;
  constexpr bool KEEP = (FUSE & kCnnKeep) != 0;
  static_assert(MODE == 0 || (MODE == 2 && !TAPS) || FUSE == 0, "forward layers only");
  constexpr int TH = kTileH + 2, TW = kTileW + 2;
  // (kCnnInFirst: room for the 12 spare pixels of layer 1's last group)
  __shared__ __attribute__((aligned(16))) unsigned short tile[(TH * TW + (FIRST ? 12 : 0)) * kPxStride];
  // the tile's outputs, so that each pixel's 64 channels leave in one
  // 128-byte line (two waves hold its two halves)
  constexpr bool ACT_OUT = !TAPS || KEEP;
  __shared__ __attribute__((aligned(16))) unsigned short obuf[ACT_OUT ? kTileH * kTileW * kPxStride : 1];
  // kCnnOutTaps: the two channel halves' partial sums, [half][row][tap][pixel]
  __shared__ float tpart[TAPS ? 2 * kTileH * 9 * kTileW : 1];
  const int wave = wave_in_group();
  const int lane = threadIdx.x & 63, g = lane >> 4, n = lane & 15;
  const int cbase = (wave & 1) * 32;   // output channels of this wave
  const int rbase = (wave >> 1) * 4;   // tile rows of this wave
  // kCnnInFirst: layer 1's B operand slots over the tile and a two-pixel
  // halo, and its A operands: channel c, K slot 4 tap + part (part 0, 1:
  // weight of v, 2, 3: weight of sigma'), slots 36..63 zero
  constexpr int VH = kTileH + 4, VW = kTileW + 4;
  __shared__ uint2 win[FIRST ? VH * VW : 1];
  __shared__ __attribute__((aligned(16))) unsigned short w1s[FIRST ? kCh * 64 : 1];
  __shared__ __attribute__((aligned(16))) float sb1[FIRST ? kCh : 1];
  if constexpr (FIRST) {
    for (int t = threadIdx.x; t < kCh * 64; t += 256) {
      const int c = t >> 6, k = t & 63, tap = k >> 2, part = k & 3;
      w1s[t] = k < 36 ? f2bf(fz.w1r[c * 18 + 2 * tap + (part >> 1)]) : (unsigned short)0;
    }
    if (threadIdx.x < kCh) sb1[threadIdx.x] = fz.b1[threadIdx.x];
  }
  // kCnnOutTaps: A operand of the last layer, row n = tap (n < 9), K slot
  // 8 g + j = channel cbase + 4 g + j (j < 4) or cbase + 16 + 4 g + j - 4
  bf16x8 w8a;
  if constexpr (TAPS) {
    u16x8 t8;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int c = cbase + (j < 4 ? 4 * g + j : 16 + 4 * g + j - 4);
      t8[j] = n < 9 ? f2bf(fz.w8r[n * kCh + c]) : (unsigned short)0;
    }
    w8a = __builtin_bit_cast(bf16x8, t8);
  }
  // A operands, loaded once per workgroup: weights of output channel
  // cbase + 16 cg + n, K slice (tap, 32 kc + 8 g .. + 8).
  bf16x8 wa[2][9][2];
#pragma unroll
  for (int cg = 0; cg < 2; ++cg)
#pragma unroll
    for (int tap = 0; tap < 9; ++tap)
#pragma unroll
      for (int kc = 0; kc < 2; ++kc)
        wa[cg][tap][kc] = *(const bf16x8*)(w + ((cbase + 16 * cg + n) * 9 + tap) * kCh + 32 * kc + 8 * g);
  __shared__ __attribute__((aligned(16))) float sbias[kCh];
  if (threadIdx.x < kCh) sbias[threadIdx.x] = MODE == 0 ? bias[threadIdx.x] : 0.f;

  // The input tile (with its one-pixel halo, zero outside the image) of the
  // next tile is loaded into registers while the current one is computed
  // (kCnnInFirst: v over the tile with a two-pixel halo, one value a thread).
  constexpr int NST = FIRST ? 1 : (TH * TW * 8 + 255) / 256;
  static_assert(!FIRST || VH * VW <= 256, "one v value per thread");
  u16x8 pre[NST];
  float vpre = 0.f, spre = 0.f;
  auto fetch = [&](int tj) {
    const CnnTile tn = tiles[tj];
    const ImgDev imn = imgs[tn.img];
    if constexpr (FIRST) {
      const __amdgpu_buffer_rsrc_t rv = make_rsrc(fz.v + imn.out_off, imn.Hc * imn.Wc * 4);
      const int t = threadIdx.x;
      const int ty = t / VW, tx = t - ty * VW;
      const int y = tn.y0 + ty - 2, x = tn.x0 + tx - 2;
      const bool ok = t < VH * VW && (unsigned)y < (unsigned)imn.Hc && (unsigned)x < (unsigned)imn.Wc;
      vpre = __uint_as_float(
          __builtin_amdgcn_raw_buffer_load_b32(rv, ok ? (uint32_t)((y * imn.Wc + x) * 4) : 0xffffffffu, 0, 0));
      spre = fz.sigma[tn.img];
    } else {
      // the image's activations; offsets outside it read as zero
      const __amdgpu_buffer_rsrc_t ra = make_rsrc(in + imn.out_off * kCh, imn.Hc * imn.Wc * kCh * 2);
#pragma unroll
      for (int sidx = 0; sidx < NST; ++sidx) {
        const int t = threadIdx.x + 256 * sidx;
        const int px = t >> 3, part = t & 7;
        const int ty = px / TW, tx = px - ty * TW;
        const int y = tn.y0 + ty - 1, x = tn.x0 + tx - 1;
        const bool ok = t < TH * TW * 8 && (unsigned)y < (unsigned)imn.Hc && (unsigned)x < (unsigned)imn.Wc;
        const uint32_t off = ok ? (uint32_t)(((y * imn.Wc + x) * kCh + part * 8) * 2) : 0xffffffffu;
        pre[sidx] = __builtin_bit_cast(u16x8, __builtin_amdgcn_raw_buffer_load_b128(ra, off, 0, 0));
      }
    }
  };
  if ((int)blockIdx.x < ntiles) fetch(blockIdx.x);
  for (int ti = blockIdx.x; ti < ntiles; ti += gridDim.x) {
    const CnnTile tl = tiles[ti];
    const ImgDev im = imgs[tl.img];
    __syncthreads();  // previous tile fully consumed
    if constexpr (FIRST) {
      if (threadIdx.x < VH * VW) {
        // the K slots of this window pixel: v / 255 (zero outside the image:
        // the load above reads zero there) and sigma' where inside
        const int ty = threadIdx.x / VW, tx = threadIdx.x - ty * VW;
        const int y = tl.y0 + ty - 2, x = tl.x0 + tx - 2;
        const bool in_img = (unsigned)y < (unsigned)im.Hc && (unsigned)x < (unsigned)im.Wc;
        const float sg = fminf(spre, 255.f) * (1.f / 255.f);
        const unsigned short sh = f2bf(sg), sl = f2bf(sg - bf2f(sh));
        const float xv = vpre * (1.f / 255.f);
        const unsigned short vh = f2bf(xv), vl = f2bf(xv - bf2f(vh));
        win[threadIdx.x] = make_uint2((uint32_t)vh | ((uint32_t)vl << 16),
                                      in_img ? ((uint32_t)sh | ((uint32_t)sl << 16)) : 0u);
      }
      __syncthreads();
      if (ti + (int)gridDim.x < ntiles) fetch(ti + gridDim.x);
      stage_first_layer(tl, im, win, w1s, sb1, tile, wave, g, n);
      __syncthreads();
      if constexpr (KEEP) {
        // layer 1's output over the tile (without its halo), whole lines
        for (int t = threadIdx.x; t < kTileH * kTileW * 8; t += 256) {
          const int px = t >> 3, part = t & 7, py = px / kTileW, pxx = px - py * kTileW;
          *(u16x8*)(fz.keep + (im.out_off + (int64_t)(tl.y0 + py) * im.Wc + tl.x0 + pxx) * kCh + part * 8) =
              *(const u16x8*)(tile + ((py + 1) * TW + pxx + 1) * kPxStride + part * 8);
        }
      }
    } else {
#pragma unroll
      for (int sidx = 0; sidx < NST; ++sidx) {
        const int t = threadIdx.x + 256 * sidx;
        if (t < TH * TW * 8) *(u16x8*)(tile + (t >> 3) * kPxStride + (t & 7) * 8) = pre[sidx];
      }
      __syncthreads();
      if (ti + (int)gridDim.x < ntiles) fetch(ti + gridDim.x);
    }
    // The wave's four rows at once (8 independent accumulators): each input
    // row's operand is read from LDS once and feeds every output row it
    // borders (tap row dy = input row - output row), so a tile takes 36 LDS
    // reads per wave rather than 72.  Each accumulator still sums its taps
    // and K halves in tap order.
    {
      constexpr int R = 4;
      f32x4 acc[R][2];
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int cg = 0; cg < 2; ++cg) acc[r][cg] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ir = 0; ir < R + 2; ++ir) {
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
#pragma unroll
          for (int kc = 0; kc < 2; ++kc) {
            const bf16x8 b = *(const bf16x8*)(tile + ((rbase + ir) * TW + (n + dx)) * kPxStride + 8 * g + 32 * kc);
#pragma unroll
            for (int r = 0; r < R; ++r) {
              const int dy = ir - r;
              if (dy < 0 || dy > 2) continue;
#pragma unroll
              for (int cg = 0; cg < 2; ++cg)
                acc[r][cg] =
                    __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[cg][3 * dy + dx][kc], b, acc[r][cg], 0, 0, 0);
            }
          }
        }
      }
      constexpr int r2 = 0;
      // acc[r][cg][q] = output channel cbase + 16 cg + 4 g + q of pixel (row r, col n)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int y = tl.y0 + rbase + r2 + r, x = tl.x0 + n;
        const int64_t pix = im.out_off + (int64_t)y * im.Wc + x;  // (the mask's pixel, MODE 1)
        u16x8 ob;  // kCnnOutTaps: the pixel's 8 outputs of this lane, in the K order of w8a
#pragma unroll
        for (int cg = 0; cg < 2; ++cg) {
          const int c0 = cbase + 16 * cg + 4 * g;
          uint2 pk;  // the four outputs as bfloat16, channel c0 in the low half of x
          if (MODE == 0) {
            const float4 bb = *(const float4*)(sbias + c0);
            pk.x = pack_bf2(fmaxf(acc[r][cg][0] + bb.x, 0.f), fmaxf(acc[r][cg][1] + bb.y, 0.f));
            pk.y = pack_bf2(fmaxf(acc[r][cg][2] + bb.z, 0.f), fmaxf(acc[r][cg][3] + bb.w, 0.f));
          } else if (MODE == 2) {
            pk.x = pack_bf2(acc[r][cg][0], acc[r][cg][1]);
            pk.y = pack_bf2(acc[r][cg][2], acc[r][cg][3]);
          } else {
            const uint2 mk = *(const uint2*)(mask + pix * kCh + c0);
            const unsigned short m4[4] = {(unsigned short)(mk.x & 0xffff), (unsigned short)(mk.x >> 16),
                                          (unsigned short)(mk.y & 0xffff), (unsigned short)(mk.y >> 16)};
            unsigned short o[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) o[q] = bf2f(m4[q]) > 0.f ? f2bf(acc[r][cg][q]) : (unsigned short)0;
            pk.x = (uint32_t)o[0] | ((uint32_t)o[1] << 16);
            pk.y = (uint32_t)o[2] | ((uint32_t)o[3] << 16);
          }
          if constexpr (TAPS) {
            ob[cg * 4 + 0] = (unsigned short)(pk.x & 0xffff);
            ob[cg * 4 + 1] = (unsigned short)(pk.x >> 16);
            ob[cg * 4 + 2] = (unsigned short)(pk.y & 0xffff);
            ob[cg * 4 + 3] = (unsigned short)(pk.y >> 16);
          }
          if constexpr (ACT_OUT) *(uint2*)(obuf + ((rbase + r2 + r) * kTileW + n) * kPxStride + c0) = pk;
        }
        if constexpr (TAPS) {
          // the wave's 32 channels of pixel (row, n) against the nine taps'
          // weights: lane (g, n) receives taps 4 g + q of pixel n
          const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
          const f32x4 tp = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w8a, __builtin_bit_cast(bf16x8, ob), zero, 0, 0, 0);
          float* part = tpart + (((wave & 1) * kTileH + rbase + r2 + r) * 9) * kTileW;
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (4 * g + q < 9) part[(4 * g + q) * kTileW + n] = tp[q];
        }
      }
    }
    __syncthreads();  // every wave's outputs are in obuf / tpart
    if constexpr (TAPS) {
      for (int t = threadIdx.x; t < 9 * kTileH * kTileW; t += 256) {
        const int tap = t / (kTileH * kTileW), px = t - tap * (kTileH * kTileW);
        const int py = px / kTileW, pxx = px - py * kTileW;
        const int i0 = (py * 9 + tap) * kTileW + pxx;
        const float sum = tpart[i0] + tpart[i0 + kTileH * 9 * kTileW];
        fz.taps[tap * fz.plane + im.out_off + (int64_t)(tl.y0 + py) * im.Wc + tl.x0 + pxx] = sum;
      }
    }
    if constexpr (ACT_OUT) {
      for (int t = threadIdx.x; t < kTileH * kTileW * 8; t += 256) {
        const int px = t >> 3, part = t & 7;
        const int y = tl.y0 + px / kTileW, x = tl.x0 + px % kTileW;
        *(u16x8*)(out + (im.out_off + (int64_t)y * im.Wc + x) * kCh + part * 8) =
            *(const u16x8*)(obuf + px * kPxStride + part * 8);
      }
    }
  }
}

// Layer 8 (64 -> 1) and the residual, out = v - 255 (b8 + sum w8 a7), on
// bfloat16 MFMA.  A workgroup loops over 8 x 16-pixel tiles, each staged with
// its halo in LDS as in k_cnn_mid.  The A operand holds the 32 weights of
// (tap, K chunk) in row 0 only (lanes n = 0, read from LDS), so row 0 of the
// product is the layer's output for 16 pixels; wave w computes rows 2w, 2w+1.
__global__ __launch_bounds__(256) void k_cnn_last(const ImgDev* __restrict__ imgs, const CnnTile* __restrict__ tiles,
                                                 int ntiles, const float* __restrict__ v,
                                                 const unsigned short* __restrict__ act,
                                                 const float* __restrict__ w8r, const float* __restrict__ b8p,
                                                 float* __restrict__ out) {
  using namespace cnn;
  constexpr int TH = kTileH + 2, TW = kTileW + 2;
  __shared__ __attribute__((aligned(16))) unsigned short tile[TH * TW * kPxStride];
  __shared__ __attribute__((aligned(16))) unsigned short w8s[9 * kCh];
  for (int t = threadIdx.x; t < 9 * kCh; t += 256) w8s[t] = f2bf(w8r[t]);
  const int wave = wave_in_group();
  const int lane = threadIdx.x & 63, g = lane >> 4, n = lane & 15;
  const float b8 = b8p[0];
  // The next tile's activations (with the one-pixel halo, zero outside the
  // image) are loaded into registers while the current tile is computed.
  constexpr int NST = (TH * TW * 8 + 255) / 256;
  u16x8 pre[NST];
  auto fetch = [&](int tj) {
    const CnnTile tn = tiles[tj];
    const ImgDev imn = imgs[tn.img];
    const __amdgpu_buffer_rsrc_t ra = make_rsrc(act + imn.out_off * kCh, imn.Hc * imn.Wc * kCh * 2);
#pragma unroll
    for (int sidx = 0; sidx < NST; ++sidx) {
      const int t = threadIdx.x + 256 * sidx;
      const int px = t >> 3, part = t & 7;
      const int ty = px / TW, tx = px - ty * TW;
      const int y = tn.y0 + ty - 1, x = tn.x0 + tx - 1;
      const bool ok = t < TH * TW * 8 && (unsigned)y < (unsigned)imn.Hc && (unsigned)x < (unsigned)imn.Wc;
      const uint32_t off = ok ? (uint32_t)(((y * imn.Wc + x) * kCh + part * 8) * 2) : 0xffffffffu;
      pre[sidx] = __builtin_bit_cast(u16x8, __builtin_amdgcn_raw_buffer_load_b128(ra, off, 0, 0));
    }
  };
  if ((int)blockIdx.x < ntiles) fetch(blockIdx.x);
  for (int ti = blockIdx.x; ti < ntiles; ti += gridDim.x) {
    const CnnTile tl = tiles[ti];
    const ImgDev im = imgs[tl.img];
    __syncthreads();  // previous tile consumed (and w8s written)
#pragma unroll
    for (int sidx = 0; sidx < NST; ++sidx) {
      const int t = threadIdx.x + 256 * sidx;
      if (t < TH * TW * 8) *(u16x8*)(tile + (t >> 3) * kPxStride + (t & 7) * 8) = pre[sidx];
    }
    __syncthreads();
    if (ti + (int)gridDim.x < ntiles) fetch(ti + gridDim.x);
    f32x4 acc[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) acc[r] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int dy = tap / 3, dx = tap % 3;
#pragma unroll
      for (int kc = 0; kc < 2; ++kc) {
        const u16x8 wz = {0, 0, 0, 0, 0, 0, 0, 0};
        const u16x8 wv = *(const u16x8*)(w8s + tap * kCh + 32 * kc + 8 * g);
        const bf16x8 wa = __builtin_bit_cast(bf16x8, n == 0 ? wv : wz);
#pragma unroll
        for (int r = 0; r < 2; ++r) {
          const bf16x8 b =
              *(const bf16x8*)(tile + ((2 * wave + r + dy) * TW + (n + dx)) * kPxStride + 8 * g + 32 * kc);
          acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa, b, acc[r], 0, 0, 0);
        }
      }
    }
    if (g == 0) {
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const int64_t p = im.out_off + (int64_t)(tl.y0 + 2 * wave + r) * im.Wc + tl.x0 + n;
        out[p] = v[p] - 255.f * (b8 + acc[r][0]);
      }
    }
  }
}

// Fallback gate of the learned denoisers (int32[1 + n], zero on entry):
// gate[1 + i] = 1 for an image whose network output holds a non-finite
// value, gate[0] = 1 when any image is flagged.
__global__ __launch_bounds__(256) void k_cnn_check(const int32_t* __restrict__ pix_img, int64_t pixels,
                                                  const float* __restrict__ out, int32_t* __restrict__ gate) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= pixels) return;
  if (!__builtin_isfinite(out[p])) {
    atomicOr(&gate[1 + pix_img[p >> kPixChunkShift]], 1);
    atomicOr(&gate[0], 1);
  }
}

// Flags every image whose noise level lies outside the range the network
// accepts, range[0] <= sigma <= range[1] (a NaN sigma is outside).
__global__ void k_cnn_sigma_gate(const float* __restrict__ sigma, int n, const float* __restrict__ range,
                                 int32_t* __restrict__ gate) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float sg = sigma[i];
  if (!(sg >= range[0] && sg <= range[1])) {
    atomicOr(&gate[1 + i], 1);
    atomicOr(&gate[0], 1);
  }
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int n, int32_t v) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// Training: loss, gradients, Adam.  The loss is the mean over the batch's
// pixels of ((D(v) - target) / 255)^2; df = dL/df = -2 (D(v) - target) / (255 n)
// since D(v) = v - 255 f.
// ---------------------------------------------------------------------------

// df and one partial loss sum per 256-pixel block (fixed order).
__global__ __launch_bounds__(256) void k_cnn_loss(const float* __restrict__ out, const float* __restrict__ target,
                                                 int64_t pixels, float* __restrict__ df,
                                                 double* __restrict__ loss_part) {
  __shared__ double sh[256];
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double l = 0.0;
  if (p < pixels) {
    const float d = (out[p] - target[p]) * (1.f / 255.f);
    df[p] = -2.f * d / (float)pixels;
    l = (double)d * (double)d;
  }
  sh[threadIdx.x] = l;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss_part[blockIdx.x] = sh[0];
}

// Sum `n` float64 partials in order into out[0] (single thread; n is small).
// loss = sum of the n partials / pixels; one workgroup of 256 threads: thread
// t sums partials t, t + 256, ..., then a fixed tree (deterministic).
__global__ __launch_bounds__(256) void k_sum_loss(const double* __restrict__ part, int64_t n, int64_t pixels,
                                                  float* __restrict__ loss) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += part[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = (float)(sh[0] / (double)pixels);
}

// Layer-8 input gradient: dz7[q][c] = [a7[q][c] > 0] sum_tap w8[tap][c] df[q - off(tap)].
__global__ __launch_bounds__(256) void k_cnn_last_bwd(const ImgDev* __restrict__ imgs,
                                                     const int32_t* __restrict__ pix_img, int64_t pixels,
                                                     const float* __restrict__ df,
                                                     const unsigned short* __restrict__ a7,
                                                     const float* __restrict__ w8r, unsigned short* __restrict__ dz7) {
  using namespace cnn;
  __shared__ float sw[9 * 64];
  for (int t = threadIdx.x; t < 9 * 64; t += 256) sw[t] = w8r[t];
  __syncthreads();
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= pixels) return;
  const ImgDev im = imgs[pix_img[q >> kPixChunkShift]];
  const int64_t lq = q - im.out_off;
  const int y = (int)(lq / im.Wc), x = (int)(lq - (int64_t)y * im.Wc);
  float d[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    // output pixel p = q - off(tap) read input q through tap
    const int yy = y - (t / 3 - 1), xx = x - (t % 3 - 1);
    d[t] = (yy >= 0 && yy < im.Hc && xx >= 0 && xx < im.Wc) ? df[im.out_off + (int64_t)yy * im.Wc + xx] : 0.f;
  }
  const u16x8* a = (const u16x8*)(a7 + q * kCh);
  u16x8* o = (u16x8*)(dz7 + q * kCh);
#pragma unroll
  for (int part = 0; part < 8; ++part) {
    const u16x8 av = a[part];
    u16x8 ov;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int c = part * 8 + k;
      float g = 0.f;
#pragma unroll
      for (int t = 0; t < 9; ++t) g = fmaf(sw[t * 64 + c], d[t], g);
      ov[k] = bf2f(av[k]) > 0.f ? f2bf(g) : (unsigned short)0;
    }
    o[part] = ov;
  }
}

// Weight and bias gradients of layer 8 (64 -> 1):
//   dW8[tap][c] = sum_p df[p] a7[p + off(tap)][c],  db8 = sum_p df[p].
// Workgroups loop over 8 x 16-pixel tiles; thread t owns channel c = t % 64
// and every fourth pixel of a tile (t / 64 = 0..3), keeping 9 + 1 sums; the
// four pixel phases are added in a fixed order at the end and the
// workgroup's partial sums go to part[wg][577] (tap * 64 + c, then db8).
__global__ __launch_bounds__(256) void k_cnn_last_wgrad(const ImgDev* __restrict__ imgs,
                                                       const CnnTile* __restrict__ tiles, int ntiles,
                                                       const float* __restrict__ df,
                                                       const unsigned short* __restrict__ a7,
                                                       float* __restrict__ part) {
  using namespace cnn;
  __shared__ float sh[4][9 * 64 + 1];
  const int c = threadIdx.x & 63, pq = threadIdx.x >> 6;
  float acc[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  float bacc = 0.f;
  for (int ti = blockIdx.x; ti < ntiles; ti += gridDim.x) {
    const CnnTile tl = tiles[ti];
    const ImgDev im = imgs[tl.img];
    for (int px = pq; px < kTileH * kTileW; px += 4) {
      const int y = tl.y0 + px / kTileW, x = tl.x0 + px % kTileW;
      const float dv = df[im.out_off + (int64_t)y * im.Wc + x];
      bacc += dv;
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) {
        const int yy = y + tap / 3 - 1, xx = x + tap % 3 - 1;
        if (yy >= 0 && yy < im.Hc && xx >= 0 && xx < im.Wc)
          acc[tap] = fmaf(dv, bf2f(a7[(im.out_off + (int64_t)yy * im.Wc + xx) * kCh + c]), acc[tap]);
      }
    }
  }
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) sh[pq][tap * 64 + c] = acc[tap];
  if (c == 0) sh[pq][576] = bacc;
  __syncthreads();
  for (int o = threadIdx.x; o < 577; o += 256)
    part[(int64_t)blockIdx.x * 577 + o] = ((sh[0][o] + sh[1][o]) + sh[2][o]) + sh[3][o];
}

// Weight and bias gradients of layer 1 (2 -> 64) from dz1 and the network
// input [v / 255, min(sigma, 255) / 255] (zero outside the image):
// 64 x 9 x 2 weights (co * 18 + tap * 2 + c) + 64 biases = 1216 outputs.
// Same scheme as k_cnn_last_wgrad: thread t owns output channel co = t % 64
// and every fourth pixel of each tile, with 18 + 1 sums.
__global__ __launch_bounds__(256) void k_cnn_first_wgrad(const ImgDev* __restrict__ imgs,
                                                        const CnnTile* __restrict__ tiles, int ntiles,
                                                        const float* __restrict__ v, const float* __restrict__ sigma,
                                                        const unsigned short* __restrict__ dz1,
                                                        float* __restrict__ part) {
  using namespace cnn;
  __shared__ float sh[4][1216];
  const int co = threadIdx.x & 63, pq = threadIdx.x >> 6;
  float acc[18];
#pragma unroll
  for (int k = 0; k < 18; ++k) acc[k] = 0.f;
  float bacc = 0.f;
  for (int ti = blockIdx.x; ti < ntiles; ti += gridDim.x) {
    const CnnTile tl = tiles[ti];
    const ImgDev im = imgs[tl.img];
    const float s = fminf(sigma[tl.img], 255.f) * (1.f / 255.f);
    for (int px = pq; px < kTileH * kTileW; px += 4) {
      const int y = tl.y0 + px / kTileW, x = tl.x0 + px % kTileW;
      const int64_t p = im.out_off + (int64_t)y * im.Wc + x;
      const float gz = bf2f(dz1[p * kCh + co]);
      bacc += gz;
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) {
        const int yy = y + tap / 3 - 1, xx = x + tap % 3 - 1;
        if (yy >= 0 && yy < im.Hc && xx >= 0 && xx < im.Wc) {
          acc[2 * tap] = fmaf(gz, v[im.out_off + (int64_t)yy * im.Wc + xx] * (1.f / 255.f), acc[2 * tap]);
          acc[2 * tap + 1] = fmaf(gz, s, acc[2 * tap + 1]);
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < 18; ++k) sh[pq][co * 18 + k] = acc[k];
  sh[pq][1152 + co] = bacc;
  __syncthreads();
  for (int o = threadIdx.x; o < 1216; o += 256)
    part[(int64_t)blockIdx.x * 1216 + o] = ((sh[0][o] + sh[1][o]) + sh[2][o]) + sh[3][o];
}

// Weight and bias gradients of a 64 -> 64 layer on bfloat16 MFMA:
//   dW[co][tap][ci] = sum_p dz[p][co] a[p + off(tap)][ci],  db[co] = sum_p dz[p][co]
// as a GEMM with K = pixels.  A workgroup walks 8 x 16-pixel tiles; each tile
// is staged transposed in LDS (dz as [co][pixel], a with its halo as three
// column-shifted copies [dx][ci][row][col]) so that both operands are 8
// consecutive pixels per lane.  Wave w owns input channels 16 w .. 16 w + 15
// for all 9 taps and all 64 output channels (36 accumulators).  Partial sums
// of the workgroup go to part[wg][36928] in blob order (weights, then bias).
__global__ __launch_bounds__(256) void k_cnn_mid_wgrad(const ImgDev* __restrict__ imgs,
                                                      const CnnTile* __restrict__ tiles, int ntiles,
                                                      const unsigned short* __restrict__ dz,
                                                      const unsigned short* __restrict__ a,
                                                      float* __restrict__ part) {
  using namespace cnn;
  constexpr int NPX = kTileH * kTileW;  // 128
  __shared__ __attribute__((aligned(16))) unsigned short dzT[64 * NPX];
  __shared__ __attribute__((aligned(16))) unsigned short aT[3 * 64 * (kTileH + 2) * kTileW];
  const int wave = wave_in_group();
  const int lane = threadIdx.x & 63, g = lane >> 4, n = lane & 15;
  f32x4 acc[4][9];
#pragma unroll
  for (int cg = 0; cg < 4; ++cg)
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) acc[cg][tap] = (f32x4){0.f, 0.f, 0.f, 0.f};
  float bacc = 0.f;  // threads 4c: bias gradient of channel c
  for (int ti = blockIdx.x; ti < ntiles; ti += gridDim.x) {
    const CnnTile tl = tiles[ti];
    const ImgDev im = imgs[tl.img];
    __syncthreads();
    // dz tile -> dzT[co][row * 16 + col].  Item t is pixel t % NPX, channels
    // 8 (t / NPX) .. + 7: the lanes of a wavefront take consecutive pixels of
    // one channel group, so that their transposed 16-bit writes land in
    // different LDS banks.
    for (int t = threadIdx.x; t < NPX * 8; t += 256) {
      const int px = t % NPX, part8 = t / NPX;
      const int y = tl.y0 + px / kTileW, x = tl.x0 + px % kTileW;
      const u16x8 val = *(const u16x8*)(dz + (im.out_off + (int64_t)y * im.Wc + x) * kCh + part8 * 8);
#pragma unroll
      for (int k = 0; k < 8; ++k) dzT[(part8 * 8 + k) * NPX + px] = val[k];
    }
    // a tile with halo -> aT[dx][ci][row][col] = a[y0 - 1 + row][x0 - 1 + dx + col][ci]
    // (item t: halo pixel t % 180, channels 8 (t / 180) .. + 7, as above)
    constexpr int NHALO = (kTileH + 2) * (kTileW + 2);
    for (int t = threadIdx.x; t < NHALO * 8; t += 256) {
      const int px = t % NHALO, part8 = t / NHALO;
      const int row = px / (kTileW + 2), col = px % (kTileW + 2);
      const int y = tl.y0 - 1 + row, x = tl.x0 - 1 + col;
      u16x8 val = {0, 0, 0, 0, 0, 0, 0, 0};
      if (y >= 0 && y < im.Hc && x >= 0 && x < im.Wc)
        val = *(const u16x8*)(a + (im.out_off + (int64_t)y * im.Wc + x) * kCh + part8 * 8);
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const int c = col - dx;
        if (c >= 0 && c < kTileW) {
#pragma unroll
          for (int k = 0; k < 8; ++k)
            aT[((dx * 64 + part8 * 8 + k) * (kTileH + 2) + row) * kTileW + c] = val[k];
        }
      }
    }
    __syncthreads();
    {
      // bias gradient: thread t sums channel t / 4 over pixels 32 (t % 4) ..
      // + 31, starting at a channel-dependent rotation so that the lanes of a
      // wavefront read different banks; lanes t .. t + 3 then combine.
      const int c = threadIdx.x >> 2, q = threadIdx.x & 3;
      float s4 = 0.f;
#pragma unroll 8
      for (int i = 0; i < 32; ++i) s4 += bf2f(dzT[c * NPX + 32 * q + ((i + 2 * c) & 31)]);
      s4 += __shfl_xor(s4, 1, 64);
      s4 += __shfl_xor(s4, 2, 64);
      bacc += s4;  // lanes with q == 0 keep the channel's sum
    }
    // K = 128 pixels in 4 chunks of 32 (2 rows x 16 cols); lane group g
    // covers row 2 kc + g / 2, columns 8 (g % 2) .. + 8.
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
      const int row = 2 * kc + (g >> 1), col = 8 * (g & 1);
      bf16x8 av[4];
#pragma unroll
      for (int cg = 0; cg < 4; ++cg) av[cg] = *(const bf16x8*)(dzT + (16 * cg + n) * NPX + row * kTileW + col);
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) {
        const int dy = tap / 3, dx = tap % 3;
        const bf16x8 bv =
            *(const bf16x8*)(aT + ((dx * 64 + 16 * wave + n) * (kTileH + 2) + row + dy) * kTileW + col);
#pragma unroll
        for (int cg = 0; cg < 4; ++cg)
          acc[cg][tap] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[cg], bv, acc[cg][tap], 0, 0, 0);
      }
    }
  }
  // acc[cg][tap][r] = dW[co = 16 cg + 4 g + r][tap][ci = 16 wave + n]
  float* out = part + (int64_t)blockIdx.x * kMidStride;
#pragma unroll
  for (int cg = 0; cg < 4; ++cg)
#pragma unroll
    for (int tap = 0; tap < 9; ++tap)
#pragma unroll
      for (int r = 0; r < 4; ++r) out[((16 * cg + 4 * g + r) * 9 + tap) * 64 + 16 * wave + n] = acc[cg][tap][r];
  if ((threadIdx.x & 3) == 0) out[kMidW + (threadIdx.x >> 2)] = bacc;
}

// out[i] = sum over w < nparts of part[w * stride + i] (fixed order).
__global__ __launch_bounds__(256) void k_sum_parts(const float* __restrict__ part, int nparts, int64_t stride,
                                                  int64_t len, float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= len) return;
  float s = 0.f;
#pragma unroll 8
  for (int w = 0; w < nparts; ++w) s += part[(int64_t)w * stride + i];
  out[i] = s;
}

// The same sum for few outputs and many partials: one workgroup per output,
// thread t adds partials t, t + 256, ..., then a fixed tree.
__global__ __launch_bounds__(256) void k_sum_parts_wide(const float* __restrict__ part, int nparts, int64_t stride,
                                                       float* __restrict__ out) {
  __shared__ float sh[256];
  const int64_t i = blockIdx.x;
  float s = 0.f;
  for (int w = threadIdx.x; w < nparts; w += 256) s += part[(int64_t)w * stride + i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i] = sh[0];
}

// Adam with bias correction: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
// p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                                             const float* __restrict__ grad, int64_t n, float lr, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float g = grad[i];
  const float mi = 0.9f * m[i] + 0.1f * g;
  const float vi = 0.999f * v[i] + 0.001f * g * g;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

}  // namespace abcs
