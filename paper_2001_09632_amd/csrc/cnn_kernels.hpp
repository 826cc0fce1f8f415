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

__device__ __forceinline__ unsigned short f2bf(float f) {
  // round to nearest even
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);  // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float((uint32_t)h << 16); }

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

// Layer 1 (2 -> 64): thread per pixel, output bfloat16 NHWC.
__global__ __launch_bounds__(256) void k_cnn_first(const ImgDev* __restrict__ imgs, int n_imgs,
                                                  const int32_t* __restrict__ pix_img, int64_t pixels,
                                                  const float* __restrict__ v, const float* __restrict__ sigma,
                                                  const float* __restrict__ w1r, const float* __restrict__ blob,
                                                  unsigned short* __restrict__ act) {
  using namespace cnn;
  __shared__ float sw[64 * 18];
  __shared__ float sb[64];
  for (int t = threadIdx.x; t < 64 * 18; t += 256) sw[t] = w1r[t];
  if (threadIdx.x < 64) sb[threadIdx.x] = blob[kB1 + threadIdx.x];
  __syncthreads();
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= pixels) return;
  const ImgDev im = imgs[pix_img[p >> 8]];
  const int64_t lp = p - im.out_off;
  const int y = (int)(lp / im.Wc), x = (int)(lp - (int64_t)y * im.Wc);
  const float s = fminf(sigma[pix_img[p >> 8]], 255.f) * (1.f / 255.f);
  float in0[9], in1[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    const int yy = y + t / 3 - 1, xx = x + t % 3 - 1;
    const bool ok = yy >= 0 && yy < im.Hc && xx >= 0 && xx < im.Wc;
    in0[t] = ok ? v[im.out_off + (int64_t)yy * im.Wc + xx] * (1.f / 255.f) : 0.f;
    in1[t] = ok ? s : 0.f;
  }
  u16x8* dst = (u16x8*)(act + p * kCh);
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    u16x8 o;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int co = q * 8 + k;
      float a = sb[co];
#pragma unroll
      for (int t = 0; t < 9; ++t) a = fmaf(sw[co * 18 + t * 2], in0[t], fmaf(sw[co * 18 + t * 2 + 1], in1[t], a));
      o[k] = f2bf(fmaxf(a, 0.f));
    }
    dst[q] = o;
  }
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
template <int MODE>
__global__ __launch_bounds__(256) void k_cnn_mid(const ImgDev* __restrict__ imgs, const CnnTile* __restrict__ tiles,
                                                int ntiles, const unsigned short* __restrict__ in,
                                                const unsigned short* __restrict__ w, const float* __restrict__ bias,
                                                const unsigned short* __restrict__ mask,
                                                unsigned short* __restrict__ out) {
  using namespace cnn;
  constexpr int TH = kTileH + 2, TW = kTileW + 2;
  __shared__ __attribute__((aligned(16))) unsigned short tile[TH * TW * kPxStride];
  const int wave = wave_in_group();
  const int lane = threadIdx.x & 63, g = lane >> 4, n = lane & 15;
  const int cbase = (wave & 1) * 32;   // output channels of this wave
  const int rbase = (wave >> 1) * 4;   // tile rows of this wave
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
  float bs[2][4];
#pragma unroll
  for (int cg = 0; cg < 2; ++cg)
#pragma unroll
    for (int q = 0; q < 4; ++q) bs[cg][q] = MODE == 0 ? bias[cbase + 16 * cg + 4 * g + q] : 0.f;

  for (int ti = blockIdx.x; ti < ntiles; ti += gridDim.x) {
    const CnnTile tl = tiles[ti];
    const ImgDev im = imgs[tl.img];
    __syncthreads();  // previous tile fully consumed
    // stage the input tile with halo: 16 bytes (8 channels) per thread and pass
    for (int t = threadIdx.x; t < TH * TW * 8; t += 256) {
      const int px = t >> 3, part = t & 7;
      const int ty = px / TW, tx = px - ty * TW;
      const int y = tl.y0 + ty - 1, x = tl.x0 + tx - 1;
      u16x8 val = {0, 0, 0, 0, 0, 0, 0, 0};
      if (y >= 0 && y < im.Hc && x >= 0 && x < im.Wc)
        val = *(const u16x8*)(in + (im.out_off + (int64_t)y * im.Wc + x) * kCh + part * 8);
      *(u16x8*)(tile + px * kPxStride + part * 8) = val;
    }
    __syncthreads();
    // Two rows at a time: 4 independent accumulators per wave.
#pragma unroll 1
    for (int r2 = 0; r2 < 4; r2 += 2) {
      f32x4 acc[2][2];
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int cg = 0; cg < 2; ++cg) acc[r][cg] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) {
        const int dy = tap / 3, dx = tap % 3;
#pragma unroll
        for (int kc = 0; kc < 2; ++kc) {
#pragma unroll
          for (int r = 0; r < 2; ++r) {
            const bf16x8 b =
                *(const bf16x8*)(tile + ((rbase + r2 + r + dy) * TW + (n + dx)) * kPxStride + 8 * g + 32 * kc);
#pragma unroll
            for (int cg = 0; cg < 2; ++cg)
              acc[r][cg] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[cg][tap][kc], b, acc[r][cg], 0, 0, 0);
          }
        }
      }
      // acc[r][cg][q] = output channel cbase + 16 cg + 4 g + q of pixel (row r2 + r, col n)
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const int y = tl.y0 + rbase + r2 + r, x = tl.x0 + n;
        const int64_t pix = im.out_off + (int64_t)y * im.Wc + x;
#pragma unroll
        for (int cg = 0; cg < 2; ++cg) {
          const int c0 = cbase + 16 * cg + 4 * g;
          unsigned short o[4];
          if (MODE == 0) {
#pragma unroll
            for (int q = 0; q < 4; ++q) o[q] = f2bf(fmaxf(acc[r][cg][q] + bs[cg][q], 0.f));
          } else {
            const uint2 mk = *(const uint2*)(mask + pix * kCh + c0);
            const unsigned short m4[4] = {(unsigned short)(mk.x & 0xffff), (unsigned short)(mk.x >> 16),
                                          (unsigned short)(mk.y & 0xffff), (unsigned short)(mk.y >> 16)};
#pragma unroll
            for (int q = 0; q < 4; ++q) o[q] = bf2f(m4[q]) > 0.f ? f2bf(acc[r][cg][q]) : (unsigned short)0;
          }
          uint2 pk;
          pk.x = (uint32_t)o[0] | ((uint32_t)o[1] << 16);
          pk.y = (uint32_t)o[2] | ((uint32_t)o[3] << 16);
          *(uint2*)(out + pix * kCh + c0) = pk;
        }
      }
    }
  }
}

// Layer 8 (64 -> 1) and the residual: out = v - 255 (b8 + sum w8 a7).
// Thread per pixel.
__global__ __launch_bounds__(256) void k_cnn_last(const ImgDev* __restrict__ imgs, const int32_t* __restrict__ pix_img,
                                                 int64_t pixels, const float* __restrict__ v,
                                                 const unsigned short* __restrict__ act,
                                                 const float* __restrict__ w8r, const float* __restrict__ blob,
                                                 float* __restrict__ out) {
  using namespace cnn;
  __shared__ float sw[9 * 64];
  for (int t = threadIdx.x; t < 9 * 64; t += 256) sw[t] = w8r[t];
  __syncthreads();
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= pixels) return;
  const ImgDev im = imgs[pix_img[p >> 8]];
  const int64_t lp = p - im.out_off;
  const int y = (int)(lp / im.Wc), x = (int)(lp - (int64_t)y * im.Wc);
  float f = blob[kB8];
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    const int yy = y + t / 3 - 1, xx = x + t % 3 - 1;
    if (yy < 0 || yy >= im.Hc || xx < 0 || xx >= im.Wc) continue;
    const u16x8* a = (const u16x8*)(act + (im.out_off + (int64_t)yy * im.Wc + xx) * kCh);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const u16x8 h = a[q];
#pragma unroll
      for (int k = 0; k < 8; ++k) f = fmaf(sw[t * 64 + q * 8 + k], bf2f(h[k]), f);
    }
  }
  out[p] = v[p] - 255.f * f;
}

}  // namespace abcs
