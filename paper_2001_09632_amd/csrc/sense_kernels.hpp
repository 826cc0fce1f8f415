// Phase-2 sensing (zigzag prefix of each block's 2D DCT) and the masked
// inverse 2D-DCT decoder, one wavefront per tile of 16x16 blocks.
#pragma once

#include "common.hpp"
#include "transform16.hpp"

namespace abcs {

// Clamp a block's coefficient range to its image's part of y, so that a
// corrupt k or offset can never make a kernel touch memory outside y.
__device__ __forceinline__ int guard_count(const ImgDev& im, int kk, int64_t off) {
  const int64_t lo = im.meas_off, hi = im.meas_off + im.n_meas;
  if (off < lo || off > hi || kk <= 0) return 0;
  const int64_t room = hi - off;
  const int64_t c = kk < room ? kk : room;
  return c < 256 ? (int)c : 256;
}

// Per-wave staging buffer: one block of coefficients in zigzag order.
struct WaveLds {
  float c[256];
};

// y[off_i + z] = C_i[zigzag[z]] for z < k_i.  The transform output is written
// to LDS at its zigzag rank and copied to y with unit-stride stores.
__global__ __launch_bounds__(kGroupThreads) void k_sense16(const ImgDev* __restrict__ imgs,
                                                          const Tile* __restrict__ tiles, int ntiles,
                                                          const uint8_t* __restrict__ px,
                                                          const int32_t* __restrict__ k_all,
                                                          const int64_t* __restrict__ off_all,
                                                          float* __restrict__ y) {
  __shared__ WaveLds lds[kWavesPerGroup];
  const int wave = blockIdx.x * kWavesPerGroup + (threadIdx.x >> 6);
  if (wave >= ntiles) return;
  const int lane = threadIdx.x & 63;
  float* buf = lds[threadIdx.x >> 6].c;
  const Tile tl = tiles[wave];
  const ImgDev im = imgs[tl.img];
  Lane16 L;
  lane16_init(L);

  // Lane b < count holds block b's k and offset.
  int32_t my_k = 0;
  int64_t my_off = 0;
  if (lane < tl.count) {
    my_k = k_all[im.blk_off + tl.first + lane];
    my_off = off_all[im.blk_off + tl.first + lane];
  }
  uint32_t pw[kTileBlocks];
#pragma unroll
  for (int b = 0; b < kTileBlocks; ++b) {
    if (b < tl.count) {
      const int blk = tl.first + b;
      const int by = blk / im.nbx, bx = blk - by * im.nbx;
      pw[b] = *(const uint32_t*)(px + im.px_off + (int64_t)(by * 16 + L.n) * im.pitch + bx * 16 + 4 * L.g);
    }
  }
#pragma unroll
  for (int b = 0; b < kTileBlocks; ++b) {
    if (b < tl.count) {
      const int64_t off = __shfl(my_off, b, 64);
      const int kk = guard_count(im, __shfl(my_k, b, 64), off);
      float a[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) a[c] = (float)((pw[b] >> (8 * c)) & 0xffu);
      const f32x4 C = dct16_fwd(a, L);
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (L.zr[r] < kk) buf[L.zr[r]] = C[r];
      wave_lds_sync();
      for (int z = lane; z < kk; z += 64) y[off + z] = buf[z];
      wave_lds_sync();
    }
  }
}

// out = D^T C D per block with C zero beyond the block's k_i zigzag entries.
__global__ __launch_bounds__(kGroupThreads) void k_reconstruct16(const ImgDev* __restrict__ imgs,
                                                                const Tile* __restrict__ tiles, int ntiles,
                                                                const float* __restrict__ y,
                                                                const int32_t* __restrict__ k_all,
                                                                const int64_t* __restrict__ off_all,
                                                                float* __restrict__ out) {
  __shared__ WaveLds lds[kWavesPerGroup];
  const int wave = blockIdx.x * kWavesPerGroup + (threadIdx.x >> 6);
  if (wave >= ntiles) return;
  const int lane = threadIdx.x & 63;
  float* buf = lds[threadIdx.x >> 6].c;
  const Tile tl = tiles[wave];
  const ImgDev im = imgs[tl.img];
  Lane16 L;
  lane16_init(L);

  int32_t my_k = 0;
  int64_t my_off = 0;
  if (lane < tl.count) {
    my_k = k_all[im.blk_off + tl.first + lane];
    my_off = off_all[im.blk_off + tl.first + lane];
  }
  // Coefficients of the next block, loaded one block ahead.
  float nxt[4];
  auto load_block = [&](int b, float v[4]) {
    const int64_t off = __shfl(my_off, b, 64);
    const int kk = guard_count(im, __shfl(my_k, b, 64), off);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int z = lane + 64 * q;
      v[q] = (z < kk) ? y[off + z] : 0.f;
    }
  };
  load_block(0, nxt);
  for (int b = 0; b < tl.count; ++b) {
    float cur[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) cur[q] = nxt[q];
    if (b + 1 < tl.count) load_block(b + 1, nxt);
    const int kk = guard_count(im, __shfl(my_k, b, 64), __shfl(my_off, b, 64));
#pragma unroll
    for (int q = 0; q < 4; ++q) buf[lane + 64 * q] = cur[q];
    wave_lds_sync();
    float e[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) e[c] = (L.zr[c] < kk) ? buf[L.zr[c]] : 0.f;
    wave_lds_sync();
    const f32x4 X = idct16_inv(e, L);
    const int blk = tl.first + b;
    const int by = blk / im.nbx, bx = blk - by * im.nbx;
    float4* dst = (float4*)(out + im.out_off + (int64_t)(by * 16 + L.n) * im.Wc + bx * 16 + 4 * L.g);
    *dst = make_float4(X[0], X[1], X[2], X[3]);
  }
}

}  // namespace abcs
