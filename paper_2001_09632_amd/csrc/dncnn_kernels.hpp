// DnCNN-17 with batch normalisation (Section VI-4: layer 1 conv + ReLU,
// layers 2..16 conv + batch normalisation + ReLU, layer 17 conv), built from
// the learned denoiser's convolution kernels plus the normalisation kernels
// below.  Same input (v / 255 and the sigma map) and residual output as the
// 8-layer network.
//
// Parameter blob (float32): W1 [64][3][3][2], b1 [64]; for each of the 15
// middle layers W [64][3][3][64], gamma [64], beta [64]; W17 [1][3][3][64],
// b17.  Running statistics (after the blob when used as a denoiser): for each
// middle layer mean [64] then variance [64].
//
// Training normalises with the batch mean and biased batch variance (eps
// 1e-5, sums in float64 over all pixels of the batch) and moves the running
// statistics by 0.1 towards them; inference folds the running statistics into
// the middle convolutions: W' = W s, b' = beta - mean s, s = gamma /
// sqrt(var + eps) per output channel.
#pragma once

#include "common.hpp"
#include "cnn_kernels.hpp"

namespace abcs {

namespace dn {
constexpr int kCh = 64;
constexpr int kMid = 15;
constexpr int kW1 = 0, kB1 = 1152, kMid0 = 1216;
constexpr int kMidW = 64 * 9 * 64;                    // 36864
constexpr int kMidStride = kMidW + 128;               // W, gamma, beta
constexpr int kW17 = kMid0 + kMid * kMidStride;       // 556096
constexpr int kB17 = kW17 + 9 * 64;                   // 556672
constexpr int kParams = kB17 + 1;                     // 556673
constexpr int kRunning = kMid * 128;                  // 1920
constexpr float kEps = 1e-5f;
constexpr float kMomentum = 0.1f;
}  // namespace dn

// bfloat16 middle weights in blob order ([C_out][tap][C_in]) and, when wt is
// not null, their tap-flipped transposes; with `running`, the weights are
// scaled by s = gamma / sqrt(var + eps) per output channel and bias[l][c] =
// beta - mean s (inference); layers 1 and 17 as bfloat16-rounded float32.
__global__ __launch_bounds__(256) void k_dn_prep(const float* __restrict__ blob, const float* __restrict__ running,
                                                unsigned short* __restrict__ wmid, unsigned short* __restrict__ wt,
                                                float* __restrict__ bias, float* __restrict__ w1r,
                                                float* __restrict__ w17r) {
  using namespace dn;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < (int64_t)kMid * kMidW) {
    const int l = (int)(i / kMidW), e = (int)(i - (int64_t)l * kMidW);
    const int co = e / (9 * 64), tap = (e / 64) % 9, ci = e % 64;
    const float* m = blob + kMid0 + (int64_t)l * kMidStride;
    float w = m[e];
    if (running) {
      const float* r = running + l * 128;
      w *= m[kMidW + co] / sqrtf(r[64 + co] + kEps);
    }
    const unsigned short h = f2bf(w);
    wmid[i] = h;
    if (wt) wt[(int64_t)l * kMidW + (ci * 9 + (8 - tap)) * 64 + co] = h;
  }
  if (running && i < kMid * 64) {
    const int l = (int)(i / 64), c = (int)(i % 64);
    const float* m = blob + kMid0 + (int64_t)l * kMidStride;
    const float* r = running + l * 128;
    const float sc = m[kMidW + c] / sqrtf(r[64 + c] + kEps);
    bias[i] = m[kMidW + 64 + c] - r[c] * sc;
  }
  if (i < 64 * 9 * 2) w1r[i] = bf2f(f2bf(blob[kW1 + i]));
  if (i < 9 * 64) w17r[i] = bf2f(f2bf(blob[kW17 + i]));
}

// Per-channel sums over a pixel range of x [pixels][64] (bfloat16):
// part[wg][c] = sum x, part[wg][64 + c] = sum x^2 (float64).  With `zst`
// (channel mean and 1 / sqrt(var + eps) at [c], [64 + c]) and gy, the sums are
// instead of gy and gy * (x - mean) rstd: the two reductions of the
// normalisation's backward pass.  Thread t handles channel t % 64 of every
// fourth pixel.
__global__ __launch_bounds__(256) void k_bn_sums(const unsigned short* __restrict__ x,
                                                const unsigned short* __restrict__ gy,
                                                const float* __restrict__ zst, int64_t pixels, int64_t chunk,
                                                double* __restrict__ part) {
  __shared__ double sh[2][256];
  const int c = threadIdx.x & 63, r = threadIdx.x >> 6;
  const int64_t p0 = (int64_t)blockIdx.x * chunk, p1 = min(pixels, p0 + chunk);
  double s1 = 0.0, s2 = 0.0;
  if (gy == nullptr) {
    for (int64_t p = p0 + r; p < p1; p += 4) {
      const double v = bf2f(x[p * 64 + c]);
      s1 += v;
      s2 += v * v;
    }
  } else {
    const float mu = zst[c], rs = zst[64 + c];
    for (int64_t p = p0 + r; p < p1; p += 4) {
      const double g = bf2f(gy[p * 64 + c]);
      const double zh = (double)((bf2f(x[p * 64 + c]) - mu) * rs);
      s1 += g;
      s2 += g * zh;
    }
  }
  sh[0][threadIdx.x] = s1;
  sh[1][threadIdx.x] = s2;
  __syncthreads();
  if (r == 0) {
    part[(int64_t)blockIdx.x * 128 + c] = sh[0][c] + sh[0][c + 64] + sh[0][c + 128] + sh[0][c + 192];
    part[(int64_t)blockIdx.x * 128 + 64 + c] = sh[1][c] + sh[1][c + 64] + sh[1][c + 128] + sh[1][c + 192];
  }
}

// out[i] = sum over w < nparts of part[w * 128 + i], i < 128, in a fixed
// order: one workgroup per output, thread t adds partials t, t + 256, ...,
// then a fixed tree.
__global__ __launch_bounds__(256) void k_bn_reduce(const double* __restrict__ part, int nparts,
                                                  double* __restrict__ out) {
  __shared__ double sh[256];
  const int i = blockIdx.x;
  double s = 0.0;
  for (int w = threadIdx.x; w < nparts; w += 256) s += part[(int64_t)w * 128 + i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i] = sh[0];
}

// Training-mode normalisation: mean and biased variance from the sums, then
// act = bf16(ReLU(gamma (z - mean) rstd + beta)); the mean and rstd go to zst
// for the backward pass and (block 0) the running statistics move by the
// momentum.  8 channels per thread.
__global__ __launch_bounds__(256) void k_bn_apply(const unsigned short* __restrict__ z,
                                                 const double* __restrict__ sums, const float* __restrict__ gamma,
                                                 const float* __restrict__ beta, int64_t pixels,
                                                 float* __restrict__ zst, float* __restrict__ running,
                                                 unsigned short* __restrict__ act) {
  __shared__ float smu[64], srs[64], sg[64], sb[64];
  if (threadIdx.x < 64) {
    const int c = threadIdx.x;
    const double mu = sums[c] / (double)pixels;
    double var = sums[64 + c] / (double)pixels - mu * mu;
    var = var > 0.0 ? var : 0.0;
    smu[c] = (float)mu;
    srs[c] = (float)(1.0 / sqrt(var + (double)dn::kEps));
    sg[c] = gamma[c];
    sb[c] = beta[c];
    if (blockIdx.x == 0) {
      zst[c] = (float)mu;
      zst[64 + c] = srs[c];
      if (running) {
        running[c] = (1.f - dn::kMomentum) * running[c] + dn::kMomentum * (float)mu;
        running[64 + c] = (1.f - dn::kMomentum) * running[64 + c] + dn::kMomentum * (float)var;
      }
    }
  }
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;  // group of 8 channels
  if (i >= pixels * 8) return;
  const int c0 = (int)(i & 7) * 8;
  const u16x8 zv = *(const u16x8*)(z + i * 8);
  u16x8 o;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int c = c0 + k;
    const float y = sg[c] * ((bf2f(zv[k]) - smu[c]) * srs[c]) + sb[c];
    o[k] = f2bf(fmaxf(y, 0.f));
  }
  *(u16x8*)(act + i * 8) = o;
}

// Backward through the normalisation: with S1 = sum gy, S2 = sum gy zhat,
//   gz = gamma rstd (gy - S1 / P - zhat S2 / P),
// and (block 0) dgamma = S2, dbeta = S1 into the gradient blob.
__global__ __launch_bounds__(256) void k_bn_backward(const unsigned short* __restrict__ gy,
                                                    const unsigned short* __restrict__ z,
                                                    const float* __restrict__ zst, const double* __restrict__ sums,
                                                    const float* __restrict__ gamma, int64_t pixels,
                                                    float* __restrict__ dgamma, unsigned short* __restrict__ gz) {
  __shared__ float smu[64], srs[64], sg[64], sm1[64], sm2[64];
  if (threadIdx.x < 64) {
    const int c = threadIdx.x;
    smu[c] = zst[c];
    srs[c] = zst[64 + c];
    sg[c] = gamma[c];
    sm1[c] = (float)(sums[c] / (double)pixels);
    sm2[c] = (float)(sums[64 + c] / (double)pixels);
    if (blockIdx.x == 0) {
      dgamma[c] = (float)sums[64 + c];
      dgamma[64 + c] = (float)sums[c];
    }
  }
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= pixels * 8) return;
  const int c0 = (int)(i & 7) * 8;
  const u16x8 gv = *(const u16x8*)(gy + i * 8);
  const u16x8 zv = *(const u16x8*)(z + i * 8);
  u16x8 o;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int c = c0 + k;
    const float zh = (bf2f(zv[k]) - smu[c]) * srs[c];
    o[k] = f2bf(sg[c] * srs[c] * (bf2f(gv[k]) - sm1[c] - zh * sm2[c]));
  }
  *(u16x8*)(gz + i * 8) = o;
}

}  // namespace abcs
