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

// y[off_i + z] = C_i[zigzag[z]] for z < k_i.  Each lane stores its four
// coefficients at their zigzag rank through a buffer resource that spans
// exactly the block's k_i entries of y, so coefficients beyond the budget are
// dropped by the range check.  The tile loop is straight-line code: slots past
// the end of a tile get empty resources.
__global__ __launch_bounds__(kGroupThreads) void k_sense16(const ImgDev* __restrict__ imgs,
                                                          const Tile* __restrict__ tiles, int ntiles,
                                                          const uint8_t* __restrict__ px,
                                                          const int32_t* __restrict__ k_all,
                                                          const int64_t* __restrict__ off_all,
                                                          float* __restrict__ y) {
  const int wave = blockIdx.x * kWavesPerGroup + wave_in_group();
  if (wave >= ntiles) return;
  const Tile tl = tiles[wave];
  const ImgDev im = imgs[tl.img];
  Lane16 L;
  lane16_init(L);
  int zoff[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) zoff[r] = 4 * L.zr[r];

  uint32_t pw[kTileBlocks];
#pragma unroll
  for (int b = 0; b < kTileBlocks; ++b) {
    const bool valid = b < tl.count;
    pw[b] = load_block_px(im, px, tl.first + (valid ? b : 0), valid, L);
  }
  const int32_t* kt = k_all + im.blk_off + tl.first;
  const int64_t* ot = off_all + im.blk_off + tl.first;
#pragma unroll
  for (int b = 0; b < kTileBlocks; ++b) {
    const bool valid = b < tl.count;
    const int bi = valid ? b : 0;
    const int64_t off = ot[bi];
    const int kk = valid ? guard_count(im, kt[bi], off) : 0;
    float a[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) a[c] = (float)((pw[b] >> (8 * c)) & 0xffu);
    const f32x4 C = dct16_fwd(a, L);
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(y + off, 4 * kk);
#pragma unroll
    for (int r = 0; r < 4; ++r)
      __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(C[r]), rs, zoff[r], 0, 0);
  }
}

// out = D^T C D per block with C zero beyond the block's k_i zigzag entries.
// Each lane gathers the four coefficients it feeds to the transform straight
// from y through a buffer resource spanning the block's k_i entries; ranks
// beyond k_i read as 0, which is the zero fill.  Gathers for block b + kAhead
// are issued while block b is transformed.  Straight-line code: slots past the
// end of a tile get empty resources.
constexpr int kAhead = 4;

__global__ __launch_bounds__(kGroupThreads) void k_reconstruct16(const ImgDev* __restrict__ imgs,
                                                                const Tile* __restrict__ tiles, int ntiles,
                                                                const float* __restrict__ y,
                                                                const int32_t* __restrict__ k_all,
                                                                const int64_t* __restrict__ off_all,
                                                                float* __restrict__ out) {
  const int wave = blockIdx.x * kWavesPerGroup + wave_in_group();
  if (wave >= ntiles) return;
  const Tile tl = tiles[wave];
  const ImgDev im = imgs[tl.img];
  Lane16 L;
  lane16_init(L);
  int zoff[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) zoff[c] = 4 * L.zr[c];
  const int32_t* kt = k_all + im.blk_off + tl.first;
  const int64_t* ot = off_all + im.blk_off + tl.first;
  const int out_lane = (L.n * im.Wc + 4 * L.g) * 4;   // byte offset of the lane's row segment

  float e[kTileBlocks][4];
#pragma unroll
  for (int s = 0; s < kTileBlocks + kAhead; ++s) {
    if (s < kTileBlocks) {
      const bool valid = s < tl.count;
      const int si = valid ? s : 0;
      const int64_t off = ot[si];
      const int kk = valid ? guard_count(im, kt[si], off) : 0;
      const __amdgpu_buffer_rsrc_t rs = make_rsrc(y + off, 4 * kk);
#pragma unroll
      for (int c = 0; c < 4; ++c)
        e[s][c] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, zoff[c], 0, 0));
    }
    const int b = s - kAhead;
    if (b >= 0) {
      const bool valid = b < tl.count;
      const f32x4 X = idct16_inv(e[b], L);
      const int blk = tl.first + (valid ? b : 0);
      const int by = blk / im.nbx, bx = blk - by * im.nbx;
      const __amdgpu_buffer_rsrc_t ro =
          make_rsrc(out + im.out_off + (int64_t)(by * 16) * im.Wc + bx * 16, valid ? 4 * (15 * im.Wc + 16) : 0);
      __builtin_amdgcn_raw_buffer_store_b128(
          __builtin_bit_cast(__attribute__((ext_vector_type(4))) unsigned int, X), ro, out_lane, 0, 0);
    }
  }
}

}  // namespace abcs
