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

// Per-wave LDS staging of one block's coefficients in zigzag order.
struct WaveLds {
  float c[256];
};

// y[off_i + z] = C_i[zigzag[z]] for z < k_i.  The transform output goes to
// LDS at its zigzag rank and leaves with unit-stride stores of the block's k_i
// coefficients (slot z of store q is lane + 64 q); slots at or beyond k_i get
// an out-of-range offset and are dropped.  Blocks are taken in pairs, so that
// the matrix cores always have two independent product chains of the wave to
// work on.
template <int P, int XF = kXfDCT>
__global__ __launch_bounds__(kGroupThreads) void k_sense16(const ImgDev* __restrict__ imgs,
                                                          const Tile* __restrict__ tiles, int ntiles, int split,
                                                          const uint8_t* __restrict__ px,
                                                          const int32_t* __restrict__ k_all,
                                                          const int64_t* __restrict__ off_all,
                                                          float* __restrict__ y) {
  __shared__ WaveLds lds[kWavesPerGroup][2];
  __shared__ PxStage stage[kWavesPerGroup];
  const int wave = blockIdx.x * kWavesPerGroup + wave_in_group();
  if (wave >= (ntiles << split)) return;
  const Tile tl = split_tile(tiles, wave, split, 16);
  if (tl.count == 0) return;
  const ImgDev im = imgs[tl.img];
  Lane16 L;
  lane16_init<XF>(L);
  Lane16P<P> H;
  if (P != kPrecFP32) lane16p_init(H, L);
  TileIO io;
  tile_io_init(io, im, tl, px, y, k_all, off_all, L);
  float* buf[2] = {lds[wave_in_group()][0].c, lds[wave_in_group()][1].c};
  uint32_t* st = stage[wave_in_group()].w;
  const int lane = threadIdx.x & 63;
  stage_tile_px(io, im.pitch, tl.count, st);
  wave_lds_sync();
#pragma unroll
  for (int b0 = 0; b0 < kTileBlocks; b0 += 2) {
    if (b0 >= tl.count) break;  // a short tile (image edge, launch split) ends early
    f32x4 C[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint32_t pw = staged_px(st, b0 + h, L);
      float a[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) a[c] = (float)((pw >> (8 * c)) & 0xffu);
      C[h] = P == kPrecFP32 ? dct16_fwd(a, L) : dct16_fwd_p<P>(a, H);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int r = 0; r < 4; ++r) buf[h][L.zr[r]] = C[h][r];
    wave_lds_sync();
    float yv[2][4];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int q = 0; q < 4; ++q) yv[h][q] = buf[h][lane + 64 * q];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int kk = __builtin_amdgcn_readlane(io.k, b0 + h);
      const uint32_t rel4 = 4u * (uint32_t)__builtin_amdgcn_readlane(io.rel_lo, b0 + h);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (64 * q < kk) {
          const int z = lane + 64 * q;
          const uint32_t voff = z < kk ? rel4 + 4u * (uint32_t)z : 0xffffffffu;
          __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(yv[h][q]), io.y, voff, 0, 0);
        }
      }
    }
    wave_lds_sync();
  }
}

// out = D^T C D per block with C zero beyond the block's k_i zigzag entries.
// Lane l loads coefficients 4l .. 4l+3 of a block with one 16-byte load
// (lanes wholly past k_i get an out-of-range offset and read nothing; the
// slots past k_i in the last partial quad are zeroed in registers), the block
// goes to LDS in zigzag order and is gathered from there in the transform's
// operand layout.  All loads of a tile are issued before any store.  Blocks
// are stored in pairs: lanes n < 8 of each 16-lane row hold rows of block b
// and lanes n >= 8 rows of block b + 1 (a DPP row rotation), so every store
// writes 8 rows x 128 bytes.  The decoded image is not read again by this
// kernel, so the stores are non-temporal (streamed past the caches).
__device__ __forceinline__ float row_ror8(float v) {
  return __uint_as_float(__builtin_amdgcn_update_dpp(0u, __float_as_uint(v), 0x128, 0xf, 0xf, false));
}

// Cache policy bits of a buffer store: non-temporal.
constexpr int kStoreNT = 2;

template <int P, int XF = kXfDCT>
__global__ __launch_bounds__(kGroupThreads) void k_reconstruct16(const ImgDev* __restrict__ imgs,
                                                                const Tile* __restrict__ tiles, int ntiles, int split,
                                                                const float* __restrict__ y,
                                                                const int32_t* __restrict__ k_all,
                                                                const int64_t* __restrict__ off_all,
                                                                float* __restrict__ out) {
  typedef __attribute__((ext_vector_type(4))) unsigned int u32x4;
  __shared__ WaveLds lds[kWavesPerGroup][2];
  const int wave = blockIdx.x * kWavesPerGroup + wave_in_group();
  if (wave >= (ntiles << split)) return;
  const Tile tl = split_tile(tiles, wave, split, 16);
  if (tl.count == 0) return;
  const ImgDev im = imgs[tl.img];
  Lane16 L;
  lane16_init<XF>(L);
  Lane16P<P> H;
  if (P != kPrecFP32) lane16p_init(H, L);
  Lane16T T;
  if (P == kPrecFP32) lane16t_init<XF>(T, L);
  TileIO io;
  tile_io_init(io, im, tl, nullptr, y, k_all, off_all, L);
  const int lane = threadIdx.x & 63;
  u32x4 v[kTileBlocks];
#pragma unroll
  for (int b = 0; b < kTileBlocks; ++b) {
    const int kk = __builtin_amdgcn_readlane(io.k, b);  // 0 past the tile's end
    const uint32_t rel4 = 4u * (uint32_t)__builtin_amdgcn_readlane(io.rel_lo, b);
    const uint32_t voff = 4 * lane < kk ? rel4 + 16u * (uint32_t)lane : 0xffffffffu;
    v[b] = __builtin_amdgcn_raw_buffer_load_b128(io.y, voff, 0, 0);
  }
  const __amdgpu_buffer_rsrc_t ro = make_rsrc(out + tl.out_base, 4 * (15 * im.Wc + 16 * tl.count));
  const bool lo = L.n < 8;
  const int row = lo ? L.n : L.n - 8;
  const uint32_t o1 = 4u * (uint32_t)(row * im.Wc + (lo ? 0 : 16) + 4 * L.g);
  const uint32_t o2 = o1 + 4u * 8u * (uint32_t)im.Wc;
  float* buf0 = lds[wave_in_group()][0].c;
  float* buf1 = lds[wave_in_group()][1].c;
#pragma unroll
  for (int b = 0; b < kTileBlocks; b += 2) {
    if (b >= tl.count) break;
    // coefficients of this lane's quad that lie past the block's k
    const int kA = __builtin_amdgcn_readlane(io.k, b);
    const int kB = __builtin_amdgcn_readlane(io.k, b + 1);
    const int ka = kA - 4 * lane;
    const int kb = kB - 4 * lane;
    u32x4 va = v[b], vb = v[b + 1];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      va[j] = j < ka ? va[j] : 0u;
      vb[j] = j < kb ? vb[j] : 0u;
    }
    *(u32x4*)&buf0[4 * lane] = va;
    *(u32x4*)&buf1[4 * lane] = vb;
    wave_lds_sync();
    float e0[4], e1[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      e0[c] = buf0[P == kPrecFP32 ? T.zp[c] : L.zr[c]];
      e1[c] = buf1[P == kPrecFP32 ? T.zp[c] : L.zr[c]];
    }
    wave_lds_sync();
    f32x4 A, Bv;
    if (P == kPrecFP32) {
      idct16_inv_trunc2(e0, e1, T, idct16_steps(kA > kB ? kA : kB), A, Bv);
    } else {
      A = idct16_inv_p<P>(e0, H);
      Bv = idct16_inv_p<P>(e1, H);
    }
    f32x4 S1, S2;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float ra = row_ror8(A[r]);
      const float rb = row_ror8(Bv[r]);
      S1[r] = lo ? A[r] : rb;
      S2[r] = lo ? ra : Bv[r];
    }
    // Slots past the tile's end get out-of-range offsets (the resource's
    // linear extent alone would let them reach the next pixel row).
    const bool keep = lo ? (b < tl.count) : (b + 1 < tl.count);
    const uint32_t v1 = keep ? o1 + 64u * b : 0xffffffffu;
    const uint32_t v2 = keep ? o2 + 64u * b : 0xffffffffu;
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, S1), ro, v1, 0, kStoreNT);
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, S2), ro, v2, 0, kStoreNT);
  }
}

// Sensing and the local decoder in one pass (float32): every block's forward
// transform, its first k_i zigzag coefficients written to y as k_sense16
// does, and the masked inverse of the same coefficients written to out as
// k_reconstruct16 does.  The forward transform leaves its output in the
// truncated inverse's input layout (dct16_fwd_s), so the decoder reads the
// coefficients from registers (masked past k_i by zigzag rank); only y goes
// through LDS, to leave in unit-stride runs.  Both transforms compute the
// same bits as k_sense16<kPrecFP32> and k_reconstruct16<kPrecFP32>.  The
// forward products of the next pair of blocks are issued before the current
// pair's stores and inverse, so that the matrix cores have work while the
// wave waits on LDS and memory.
// LDS of one workgroup of k_encode16: per wave two coefficient buffers and the
// tile's pixels.
struct EncodeLds {
  WaveLds coef[kWavesPerGroup][2];
  PxStage stage[kWavesPerGroup];
};

// One wave's tile (see k_encode16).  FULL: the tile holds kTileBlocks
// blocks, so the loop runs straight through (a separate instantiation: the
// early exit a shorter tile needs costs the full one about 4 %).
template <int XF, bool FULL = false>
__device__ __forceinline__ void encode16_tile(const ImgDev& im, const Tile& tl, const uint8_t* __restrict__ px,
                                              const int32_t* __restrict__ k_all,
                                              const int64_t* __restrict__ off_all, float* __restrict__ y,
                                              float* __restrict__ out, EncodeLds& el) {
  typedef __attribute__((ext_vector_type(4))) unsigned int u32x4;
  WaveLds (*lds)[2] = el.coef;
  PxStage* stage = el.stage;
  Lane16 L;
  lane16_init<XF>(L);
  Lane16T T;
  lane16t_init<XF>(T, L);
  Lane16S S;
  lane16s_init<XF>(S, L);
  TileIO io;
  tile_io_init(io, im, tl, px, y, k_all, off_all, L);
  float* buf[2] = {lds[wave_in_group()][0].c, lds[wave_in_group()][1].c};
  uint32_t* st = stage[wave_in_group()].w;
  const int lane = threadIdx.x & 63;
  const __amdgpu_buffer_rsrc_t ro = make_rsrc(out + tl.out_base, 4 * (15 * im.Wc + 16 * tl.count));
  const bool lo = L.n < 8;
  const int row = lo ? L.n : L.n - 8;
  const uint32_t o1 = 4u * (uint32_t)(row * im.Wc + (lo ? 0 : 16) + 4 * L.g);
  const uint32_t o2 = o1 + 4u * 8u * (uint32_t)im.Wc;
  stage_tile_px(io, im.pitch, tl.count, st);
  wave_lds_sync();
  auto forward = [&](int b) {
    const uint32_t pw = staged_px(st, b, L);
    float a[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) a[c] = (float)((pw >> (8 * c)) & 0xffu);
    return dct16_fwd_s(a, S);
  };
  f32x4 C[2] = {forward(0), forward(1)};
#pragma unroll
  for (int b0 = 0; b0 < kTileBlocks; b0 += 2) {
    if (!FULL && b0 >= tl.count) break;  // a short tile (image edge, launch split) ends early
    f32x4 Cn[2] = {C[0], C[1]};
    if (b0 + 2 < kTileBlocks && (FULL || b0 + 2 < tl.count)) {
      Cn[0] = forward(b0 + 2);
      Cn[1] = forward(b0 + 3);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int r = 0; r < 4; ++r) buf[h][T.zp[r]] = C[h][r];
    wave_lds_sync();
    // all of the pair's LDS reads first, one wait, then the stores
    float yv[2][4];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int q = 0; q < 4; ++q) yv[h][q] = buf[h][lane + 64 * q];
    int kk[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      kk[h] = __builtin_amdgcn_readlane(io.k, b0 + h);
      const uint32_t rel4 = 4u * (uint32_t)__builtin_amdgcn_readlane(io.rel_lo, b0 + h);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (64 * q < kk[h]) {
          const int z = lane + 64 * q;
          const uint32_t voff = z < kk[h] ? rel4 + 4u * (uint32_t)z : 0xffffffffu;
          __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(yv[h][q]), io.y, voff, 0, 0);
        }
      }
    }
    wave_lds_sync();
    float e[2][4];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int r = 0; r < 4; ++r) e[h][r] = T.zp[r] < kk[h] ? C[h][r] : 0.f;
    f32x4 A, Bv;
    idct16_inv_trunc2(e[0], e[1], T, idct16_steps(kk[0] > kk[1] ? kk[0] : kk[1]), A, Bv);
    f32x4 S1, S2;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float ra = row_ror8(A[r]);
      const float rb = row_ror8(Bv[r]);
      S1[r] = lo ? A[r] : rb;
      S2[r] = lo ? ra : Bv[r];
    }
    const bool keep = lo ? (b0 < tl.count) : (b0 + 1 < tl.count);
    const uint32_t v1 = keep ? o1 + 64u * b0 : 0xffffffffu;
    const uint32_t v2 = keep ? o2 + 64u * b0 : 0xffffffffu;
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, S1), ro, v1, 0, kStoreNT);
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, S2), ro, v2, 0, kStoreNT);
    C[0] = Cn[0];
    C[1] = Cn[1];
  }
}

template <int XF = kXfDCT>
__global__ __launch_bounds__(kGroupThreads) void k_encode16(const ImgDev* __restrict__ imgs,
                                                           const Tile* __restrict__ tiles, int ntiles, int split,
                                                           const uint8_t* __restrict__ px,
                                                           const int32_t* __restrict__ k_all,
                                                           const int64_t* __restrict__ off_all,
                                                           float* __restrict__ y, float* __restrict__ out) {
  __shared__ EncodeLds el;
  const int wave = blockIdx.x * kWavesPerGroup + wave_in_group();
  if (wave >= (ntiles << split)) return;
  const Tile tl = split_tile(tiles, wave, split, 16);
  if (tl.count == 0) return;
  if (tl.count == kTileBlocks)
    encode16_tile<XF, true>(imgs[tl.img], tl, px, k_all, off_all, y, out, el);
  else
    encode16_tile<XF, false>(imgs[tl.img], tl, px, k_all, off_all, y, out, el);
}

}  // namespace abcs
