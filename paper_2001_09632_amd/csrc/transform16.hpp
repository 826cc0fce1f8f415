// 16 x 16 orthonormal 2D DCT-II and its inverse on one wavefront with the
// gfx950 FP32 matrix cores (v_mfma_f32_16x16x4_f32).
//
// A 16x16x4 MFMA multiplies a 16x4 tile A by a 4x16 tile B.  Lane l = 16g + n
// (g = l / 16, n = l % 16) supplies A[n][g] and B[g][n] and receives
// D[4g + r][n] in accumulator register r.  The four K-slots g of chunk c are
// mapped to the summation indices 4g + c, so that
//   * the pixel operand of a lane is row n, columns 4g .. 4g+3 of the block
//     (one 32-bit load of uint8 pixels, or one float4 load), and
//   * the accumulator of the first product is, register by register, the
//     B operand of the second product: no data moves between lanes.
//
// Forward  C = D X D^T:   T = X D^T  (A = X,   B = D^T), then C = D T.
//   in : a[c] = X[n][4g+c]          out: C[4g+r][n]
// Inverse  X = D^T C D, computed as X^T = D^T (C^T D)^T... i.e.
//   Q = C^T D (A = C^T, B = D), then X^T = D^T Q (A = D^T, B = Q)
//   in : e[c] = C[4g+c][n]          out: X[n][4g+r]
// so a forward output feeds the inverse directly and both pixel-side layouts
// are "row n, columns 4g .. 4g+3".
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace abcs {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Orthonormal DCT-II basis of order 16, D[u*16 + j], float32 and float64
// copies of the host-built float64 table; zigzag rank of coefficient (u, v).
__constant__ float c_D16[256];
__constant__ double c_D16d[256];
__constant__ uint8_t c_zzrank16[256];

struct Lane16 {
  int g, n;
  float dR[4];   // D[n][4g+c]
  float dT[4];   // D[4g+c][n]
  int zr[4];     // zigzag rank of coefficient (4g+c, n)
};

__device__ __forceinline__ void lane16_init(Lane16& L) {
  const int lane = threadIdx.x & 63;
  L.g = lane >> 4;
  L.n = lane & 15;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    L.dR[c] = c_D16[L.n * 16 + 4 * L.g + c];
    L.dT[c] = c_D16[(4 * L.g + c) * 16 + L.n];
    L.zr[c] = c_zzrank16[(4 * L.g + c) * 16 + L.n];
  }
}

__device__ __forceinline__ f32x4 dct16_fwd(const float a[4], const Lane16& L) {
  f32x4 t = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int c = 0; c < 4; ++c) t = __builtin_amdgcn_mfma_f32_16x16x4f32(a[c], L.dR[c], t, 0, 0, 0);
  f32x4 out = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int c = 0; c < 4; ++c) out = __builtin_amdgcn_mfma_f32_16x16x4f32(L.dR[c], t[c], out, 0, 0, 0);
  return out;
}

__device__ __forceinline__ f32x4 idct16_inv(const float e[4], const Lane16& L) {
  f32x4 q = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int c = 0; c < 4; ++c) q = __builtin_amdgcn_mfma_f32_16x16x4f32(e[c], L.dT[c], q, 0, 0, 0);
  f32x4 out = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int c = 0; c < 4; ++c) out = __builtin_amdgcn_mfma_f32_16x16x4f32(L.dT[c], q[c], out, 0, 0, 0);
  return out;
}

// Pixel operand of a lane for block `blk` of an image: row n, columns
// 4g .. 4g+3, read through a resource spanning the block's 16 rows (an empty
// resource, for a slot past the end of a tile, reads 0).
__device__ __forceinline__ uint32_t load_block_px(const ImgDev& im, const uint8_t* px, int blk, bool valid,
                                                  const Lane16& L) {
  const int by = blk / im.nbx, bx = blk - by * im.nbx;
  const uint8_t* base = px + im.px_off + (int64_t)(by * 16) * im.pitch + bx * 16;
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(base, valid ? 15 * im.pitch + 16 : 0);
  return __builtin_amdgcn_raw_buffer_load_b32(rs, L.n * im.pitch + 4 * L.g, 0, 0);
}

// Order the wave's LDS writes before its following LDS reads (and reads before
// later writes).  LDS instructions of one wavefront execute in issue order;
// this stops the compiler from moving accesses across the point.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int wave_sum_i32(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ float wave_sum_f32(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Float64 DCT coefficient (u, v) of a 16x16 uint8 block in the fixed order
// T[r] = sum_j X[r][j] D[v][j] (j ascending), C = sum_r D[u][r] T[r]
// (r ascending), every product and sum rounded on its own.  Used to settle
// DD threshold decisions that the float32 path cannot decide.  `words` is the
// block staged in LDS in the transform's operand layout: word 16g + r holds
// pixels (r, 4g .. 4g+3), one per byte; `D` is the float64 basis.
__device__ __attribute__((noinline)) double dct16_coef_f64(const uint32_t* words, const double* D, int u, int v) {
#pragma clang fp contract(off)
  double c = 0.0;
  for (int r = 0; r < 16; ++r) {
    double t = 0.0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const double x = (double)((words[(j >> 2) * 16 + r] >> (8 * (j & 3))) & 0xffu);
      const double p = x * D[v * 16 + j];
      t = t + p;
    }
    const double q = D[u * 16 + r] * t;
    c = c + q;
  }
  return c;
}

}  // namespace abcs
