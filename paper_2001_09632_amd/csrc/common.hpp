// Internal definitions shared by the host side and the kernels of libabcs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace abcs {

// Blocks handled by one wavefront in the block-parallel kernels.  Tiles never
// cross an image boundary, so a wave reads one image descriptor per tile.
constexpr int kTileBlocks = 16;
constexpr int kWavesPerGroup = 4;
constexpr int kGroupThreads = 64 * kWavesPerGroup;

// Per-pixel kernels find a pixel's image from a table with one entry per
// 64 decoded pixels (every image holds a multiple of 64 pixels: B >= 8).
constexpr int kPixChunkShift = 6;

enum Mode : int32_t { kModeZZ = 0, kModeBBV = 1, kModeDD = 2 };

// Per-image parameters, derived on the host from the descriptor (eqs 16-21,
// Table 1, Alg 2 step 2) and read by every kernel.
struct ImgDev {
  int64_t px_off;    // byte offset of pixel (0,0)
  int64_t blk_off;   // first block in batch arrays
  int64_t meas_off;  // first coefficient in y
  int64_t out_off;   // first decoded pixel
  int64_t pool;      // P: coefficients apportioned by weight
  int64_t n_meas;    // coefficients of this image in y
  int32_t pitch;     // bytes per pixel row
  int32_t Hc, Wc;    // cropped size
  int32_t nbx, nby, nB;
  int32_t B;
  int32_t mode;      // effective budget rule (BBV with n_S = 0 runs as ZZ)
  int32_t kz;        // floor(B^2 C_R)
  int32_t L, X0, nS; // BBV sampling stride, first offset, samples per side
  int32_t m1;        // DD phase-1 coefficients
  int32_t T;         // DD threshold
  int32_t cap;       // per-block cap of the apportioned part
  int32_t ap_slot;   // histogram apportionment: slot of the image's tables for the
                     // multi-workgroup last pass (images of more than 8192 blocks), else -1
};

// Up to kTileBlocks horizontally adjacent blocks of one block row of one
// image.  Offsets of the tile's first block are precomputed so that a block's
// addresses are the tile's plus a compile-time multiple of 16.
struct Tile {
  int32_t img;     // image index
  int32_t first;   // first block (raster index inside the image)
  int32_t count;   // blocks in this tile (1..kTileBlocks)
  int32_t by;      // block row
  int64_t px_base; // byte offset of the first block's top-left pixel
  int64_t out_base;// float offset of the first block's top-left decoded pixel
};

// Launch split: a launch of the sensing and decoding kernels may give each
// tile to 2^split wavefronts (split 0 .. 2), wave w taking run w % 2^split,
// of kTileBlocks >> split blocks, of tile w >> split.  The run is a tile of
// its own (count 0 when it starts past the tile's end), so the kernels treat
// it as any other tile.  B is the block size (pixels per block column).
constexpr int kMaxSplit = 2;
__device__ __forceinline__ Tile split_tile(const Tile* tiles, int w, int split, int B) {
  Tile t = tiles[w >> split];
  const int per = kTileBlocks >> split;
  const int b0 = (w & ((1 << split) - 1)) * per;
  const int c = t.count - b0;
  t.first += b0;
  t.count = c < 0 ? 0 : (c < per ? c : per);
  t.px_base += (int64_t)b0 * B;
  t.out_base += (int64_t)b0 * B;
  return t;
}

// Index of the calling wavefront inside its workgroup, as a scalar (the
// compiler cannot prove threadIdx.x >> 6 uniform on its own, and everything
// derived from it would otherwise live in vector registers).
__device__ __forceinline__ int wave_in_group() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// Raw buffer resource over `bytes` bytes at `base`: loads beyond the range
// return 0 and stores beyond it are dropped by the hardware range check.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, bytes, 0x00020000);
}

}  // namespace abcs
