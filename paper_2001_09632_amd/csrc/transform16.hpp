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
// Orthonormal sequency-ordered Walsh-Hadamard basis of order 16, W[s*16 + j]
// (entries +-1/4, exact in every format used here).
__constant__ float c_W16[256];
__constant__ double c_W16d[256];

// Transform of a block: the 2D DCT-II or the 2D Walsh-Hadamard transform.
// The 16x16 kernels below take either basis; the transform is C = D X D^T in
// both cases.
constexpr int kXfDCT = 0, kXfWHT = 1;
template <int XF>
struct Basis16 {
  __device__ static const float* D() { return XF == kXfWHT ? c_W16 : c_D16; }
  __device__ static const double* Dd() { return XF == kXfWHT ? c_W16d : c_D16d; }
};

struct Lane16 {
  int g, n;
  float dR[4];   // D[n][4g+c]
  float dT[4];   // D[4g+c][n]
  int zr[4];     // zigzag rank of coefficient (4g+c, n)
};

template <int XF = kXfDCT>
__device__ __forceinline__ void lane16_init(Lane16& L) {
  const int lane = threadIdx.x & 63;
  const float* D = Basis16<XF>::D();
  L.g = lane >> 4;
  L.n = lane & 15;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    L.dR[c] = D[L.n * 16 + 4 * L.g + c];
    L.dT[c] = D[(4 * L.g + c) * 16 + L.n];
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

// Inverse transform of zigzag-truncated blocks, skipping the products whose
// operands are all zero.  The K slots of product c are the frequencies
// 4c .. 4c+3 (instead of c, c+4, c+8, c+12 as in idct16_inv): lane l = 16g + n
// supplies A = C[4c+g][s(n)] with s(n) = 4 (n % 4) + n / 4, so that the
// first product's accumulator register c holds the rows Q[4c+g] of
// Q = C^T D, which are then the K slots of the second product.  A block with
// k coefficients has non-zero entries only on anti-diagonals u + v <= d,
// d the diagonal of zigzag rank k - 1, so both products stop after
// min(4, d / 4 + 1) steps: 1 step for k <= 10, 2 for k <= 36, 3 for k <= 78.
// The skipped steps would add exact zeros, so the result does not depend on
// where the chain stops.
struct Lane16T {
  float dP[4];  // D[4c+g][n]
  int zp[4];    // zigzag rank of coefficient (4c+g, s(n))
};

template <int XF = kXfDCT>
__device__ __forceinline__ void lane16t_init(Lane16T& T, const Lane16& L) {
  const float* D = Basis16<XF>::D();
  const int v = 4 * (L.n & 3) + (L.n >> 2);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    T.dP[c] = D[(4 * c + L.g) * 16 + L.n];
    T.zp[c] = c_zzrank16[(4 * c + L.g) * 16 + v];
  }
}

// Forward transform with its output in the input layout of
// idct16_inv_trunc2: register r of lane l = 16g + n receives C[4r+g][s(n)].
// Both products take the basis rows in the order s: the first as
// B = D[s(n)][4g+c] (so T's columns come out as frequencies s(n)), the second
// as A = D[s(n)][4g+c] (so output row m is frequency s(m), and
// s(4g + r) = 4r + g).  Only the rows and columns of the products move; every
// output is summed over the same K slots in the same order as by dct16_fwd,
// so the values are the same bits.
struct Lane16S {
  float dS[4];  // D[s(n)][4g+c]
};

template <int XF = kXfDCT>
__device__ __forceinline__ void lane16s_init(Lane16S& S, const Lane16& L) {
  const float* D = Basis16<XF>::D();
  const int v = 4 * (L.n & 3) + (L.n >> 2);
#pragma unroll
  for (int c = 0; c < 4; ++c) S.dS[c] = D[v * 16 + 4 * L.g + c];
}

__device__ __forceinline__ f32x4 dct16_fwd_s(const float a[4], const Lane16S& S) {
  f32x4 t = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int c = 0; c < 4; ++c) t = __builtin_amdgcn_mfma_f32_16x16x4f32(a[c], S.dS[c], t, 0, 0, 0);
  f32x4 out = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int c = 0; c < 4; ++c) out = __builtin_amdgcn_mfma_f32_16x16x4f32(S.dS[c], t[c], out, 0, 0, 0);
  return out;
}

// Products per stage for a block whose first k zigzag coefficients may be
// non-zero (diagonals 0-3 hold ranks 0-9, 0-7 ranks 0-35, 0-11 ranks 0-77).
__device__ __forceinline__ int idct16_steps(int k) { return (k > 0) + (k > 10) + (k > 36) + (k > 78); }

// Two blocks' truncated inverses with their product chains interleaved; in:
// e[c] = C[4c+g][s(n)] (zero past each block's k), steps = idct16_steps of
// the larger k (wave-uniform: the smaller block's extra products add exact
// zeros); out X[n][4g+r] as idct16_inv.
__device__ __forceinline__ void idct16_inv_trunc2(const float ea[4], const float eb[4], const Lane16T& T, int steps,
                                                  f32x4& xa, f32x4& xb) {
  f32x4 qa = {0.f, 0.f, 0.f, 0.f}, qb = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if (c < steps) {
      qa = __builtin_amdgcn_mfma_f32_16x16x4f32(ea[c], T.dP[c], qa, 0, 0, 0);
      qb = __builtin_amdgcn_mfma_f32_16x16x4f32(eb[c], T.dP[c], qb, 0, 0, 0);
    }
  }
  xa = {0.f, 0.f, 0.f, 0.f};
  xb = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if (c < steps) {
      xa = __builtin_amdgcn_mfma_f32_16x16x4f32(T.dP[c], qa[c], xa, 0, 0, 0);
      xb = __builtin_amdgcn_mfma_f32_16x16x4f32(T.dP[c], qb[c], xb, 0, 0, 0);
    }
  }
}


// ---------------------------------------------------------------------------
// 16-bit operand modes of the same transforms (v_mfma_f32_16x16x16_f16 /
// _bf16, float32 sums).  Lane l = 16g + n supplies A[n][4g .. 4g+3] and
// B[4g .. 4g+3][n] and receives D[4g+r][n]: the K index is 4g + c, as in the
// float32 chain above, so the operand and output layouts are unchanged.
// Pixels (integers 0..255) are exact in both formats.  The compensated modes
// split every other float32 operand v into hi = round16(v) and
// lo = round16(v - hi) and drop only the lo x lo product: the forward
// transform takes 2 + 3 products, the inverse 3 + 3.  The single-pass modes
// use hi only.
// ---------------------------------------------------------------------------
enum Precision : int { kPrecFP32 = 0, kPrecBF16x3 = 1, kPrecFP16x3 = 2, kPrecBF16 = 3, kPrecFP16 = 4 };

template <int P>
struct Prec16 {
  static constexpr bool kBF = (P == kPrecBF16x3 || P == kPrecBF16);
  static constexpr bool kSplit = (P == kPrecBF16x3 || P == kPrecFP16x3);
};

typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef short s16x4 __attribute__((ext_vector_type(4)));

template <bool BF>
__device__ __forceinline__ unsigned short to16(float x) {
  if (BF) return __builtin_bit_cast(unsigned short, (__bf16)x);
  return __builtin_bit_cast(unsigned short, (_Float16)x);
}
template <bool BF>
__device__ __forceinline__ float from16(unsigned short h) {
  if (BF) return __uint_as_float((uint32_t)h << 16);
  return (float)__builtin_bit_cast(_Float16, h);
}
template <bool BF>
__device__ __forceinline__ f32x4 mfma16(u16x4 a, u16x4 b, f32x4 c) {
  if (BF) return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s16x4, a), __builtin_bit_cast(s16x4, b), c, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(f16x4, a), __builtin_bit_cast(f16x4, b), c, 0, 0, 0);
}

// hi / lo parts of four float32 values
template <bool BF>
__device__ __forceinline__ void split16(const float v[4], u16x4& hi, u16x4& lo) {
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    hi[c] = to16<BF>(v[c]);
    lo[c] = to16<BF>(v[c] - from16<BF>(hi[c]));
  }
}

// Per-lane basis operands: fwd = D[n][4g .. 4g+3], inv = D[4g .. 4g+3][n].
template <int P>
struct Lane16P {
  u16x4 fwd_hi, fwd_lo, inv_hi, inv_lo;
};

template <int P>
__device__ __forceinline__ void lane16p_init(Lane16P<P>& H, const Lane16& L) {
  constexpr bool BF = Prec16<P>::kBF;
  split16<BF>(L.dR, H.fwd_hi, H.fwd_lo);
  split16<BF>(L.dT, H.inv_hi, H.inv_lo);
}

// Forward: in a[c] = X[n][4g+c] (pixel values), out C[4g+r][n].
template <int P>
__device__ __forceinline__ f32x4 dct16_fwd_p(const float a[4], const Lane16P<P>& H) {
  constexpr bool BF = Prec16<P>::kBF;
  u16x4 x;
#pragma unroll
  for (int c = 0; c < 4; ++c) x[c] = to16<BF>(a[c]);
  f32x4 t = {0.f, 0.f, 0.f, 0.f};
  t = mfma16<BF>(x, H.fwd_hi, t);                                // T = X D^T
  if (Prec16<P>::kSplit) t = mfma16<BF>(x, H.fwd_lo, t);
  float tv[4] = {t[0], t[1], t[2], t[3]};
  u16x4 th, tlo;
  split16<BF>(tv, th, tlo);
  f32x4 out = {0.f, 0.f, 0.f, 0.f};
  out = mfma16<BF>(H.fwd_hi, th, out);                           // C = D T
  if (Prec16<P>::kSplit) {
    out = mfma16<BF>(H.fwd_hi, tlo, out);
    out = mfma16<BF>(H.fwd_lo, th, out);
  }
  return out;
}

// Compensated float16 forward transform with the hi and lo halves of each
// product packed into one K = 32 MFMA (v_mfma_f32_16x16x32_f16; lane
// l = 16g + n supplies K slots 8g .. 8g+7, slot c < 4 carrying index 4g + c
// of the hi term and slot 4 + c the same index of the lo term):
//   T = [X | X] [Dhi ; Dlo],   C = [Dhi | Dhi] [Th ; Tl] + [Dlo | 0] [Th ; Tl],
// the same five products as dct16_fwd_p<kPrecFP16x3> in three instructions.
// The two products of C are one accumulation chain of a single opcode: with
// a 16x16x16 instruction accumulating straight onto the 16x16x32 result the
// compiler emitted the pair back to back and the sums came out wrong.
// The operands are assembled from whole 4-wide vectors with shufflevector:
// filling the 8-wide vectors element by element from the bits of a u16x4 was
// also compiled wrongly (every slot got element 0).  Layout as dct16_fwd.
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

struct Lane16K32 {
  f16x8 d_hilo;  // slots: Dhi[n][4g+c], then Dlo[n][4g+c]
  f16x8 d_hihi;  // slots: Dhi[n][4g+c] twice
  f16x8 d_lo0;   // slots: Dlo[n][4g+c], then zero
};

__device__ __forceinline__ void lane16k32_init(Lane16K32& K, const Lane16& L) {
  u16x4 hi, lo;
  split16<false>(L.dR, hi, lo);
  const f16x4 h = __builtin_bit_cast(f16x4, hi), l = __builtin_bit_cast(f16x4, lo);
  const f16x4 z = {0, 0, 0, 0};
  K.d_hilo = __builtin_shufflevector(h, l, 0, 1, 2, 3, 4, 5, 6, 7);
  K.d_hihi = __builtin_shufflevector(h, h, 0, 1, 2, 3, 0, 1, 2, 3);
  K.d_lo0 = __builtin_shufflevector(l, z, 0, 1, 2, 3, 4, 5, 6, 7);
}

__device__ __forceinline__ f32x4 dct16_fwd_f16k32(const float a[4], const Lane16K32& K) {
  u16x4 xh;
#pragma unroll
  for (int c = 0; c < 4; ++c) xh[c] = to16<false>(a[c]);
  const f16x4 x4 = __builtin_bit_cast(f16x4, xh);
  const f16x8 x = __builtin_shufflevector(x4, x4, 0, 1, 2, 3, 0, 1, 2, 3);
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  const f32x4 t = __builtin_amdgcn_mfma_f32_16x16x32_f16(x, K.d_hilo, zero, 0, 0, 0);
  // hi = T rounded to float16, packed two to a register once; lo = T - hi
  // rounded to float16, with hi widened from those packed registers (the
  // values of split16, without converting T to float16 a second time)
  typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  const f16x2 h01 = __builtin_convertvector((f32x2){t[0], t[1]}, f16x2);
  const f16x2 h23 = __builtin_convertvector((f32x2){t[2], t[3]}, f16x2);
  const f32x2 w01 = __builtin_convertvector(h01, f32x2);
  const f32x2 w23 = __builtin_convertvector(h23, f32x2);
  const f16x2 l01 = __builtin_convertvector((f32x2){t[0] - w01[0], t[1] - w01[1]}, f16x2);
  const f16x2 l23 = __builtin_convertvector((f32x2){t[2] - w23[0], t[3] - w23[1]}, f16x2);
  const f16x4 th = __builtin_shufflevector(h01, h23, 0, 1, 2, 3);
  const f16x4 tl = __builtin_shufflevector(l01, l23, 0, 1, 2, 3);
  const f16x8 tt = __builtin_shufflevector(th, tl, 0, 1, 2, 3, 4, 5, 6, 7);
  const f32x4 out = __builtin_amdgcn_mfma_f32_16x16x32_f16(K.d_hihi, tt, zero, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(K.d_lo0, tt, out, 0, 0, 0);
}

// Inverse: in e[c] = C[4g+c][n], out X[n][4g+r].
template <int P>
__device__ __forceinline__ f32x4 idct16_inv_p(const float e[4], const Lane16P<P>& H) {
  constexpr bool BF = Prec16<P>::kBF;
  u16x4 ch, clo;
  split16<BF>(e, ch, clo);
  f32x4 q = {0.f, 0.f, 0.f, 0.f};
  q = mfma16<BF>(ch, H.inv_hi, q);                                // Q = C^T D
  if (Prec16<P>::kSplit) {
    q = mfma16<BF>(clo, H.inv_hi, q);
    q = mfma16<BF>(ch, H.inv_lo, q);
  }
  float qv[4] = {q[0], q[1], q[2], q[3]};
  u16x4 qh, qlo;
  split16<BF>(qv, qh, qlo);
  f32x4 out = {0.f, 0.f, 0.f, 0.f};
  out = mfma16<BF>(H.inv_hi, qh, out);                            // X^T = D^T Q
  if (Prec16<P>::kSplit) {
    out = mfma16<BF>(H.inv_hi, qlo, out);
    out = mfma16<BF>(H.inv_lo, qh, out);
  }
  return out;
}

// Per-tile addressing of the 16x16-block kernels.  Every block of a tile
// reads and writes through resources set up once per tile; a block's own
// addresses differ from the tile's by compile-time multiples of 16 pixels, and
// the hardware range check of each resource keeps every access inside the
// tile's pixels, the image's part of y and the tile's output rows.
struct TileIO {
  __amdgpu_buffer_rsrc_t px;   // uint8 pixels of the tile's 16 rows
  __amdgpu_buffer_rsrc_t y;    // the image's coefficients in y
  int32_t k;                   // lane b < count: k of block b
  int32_t rel_lo;              // lane b < count: offsets[b] - meas_off (low 32 bits)
};

__device__ __forceinline__ void tile_io_init(TileIO& io, const ImgDev& im, const Tile& tl, const uint8_t* px,
                                             const float* y, const int32_t* k_all, const int64_t* off_all,
                                             const Lane16& L) {
  io.px = make_rsrc(px + tl.px_base, px ? 15 * im.pitch + 16 * tl.count : 0);
  io.y = make_rsrc(y + im.meas_off, y ? (int)(4 * im.n_meas) : 0);
  const int lane = threadIdx.x & 63;
  const __amdgpu_buffer_rsrc_t rk = make_rsrc(k_all + im.blk_off + tl.first, 4 * tl.count);
  const __amdgpu_buffer_rsrc_t ro = make_rsrc(off_all + im.blk_off + tl.first, 8 * tl.count);
  io.k = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(rk, 4 * lane, 0, 0);
  io.rel_lo = (int32_t)(__builtin_amdgcn_raw_buffer_load_b32(ro, 8 * lane, 0, 0) - (uint32_t)im.meas_off);
}

// Pixels of a tile staged in LDS.  The tile's 16 pixel rows (16 blocks x 16
// bytes each) are read with row-contiguous 16-byte loads: lane l of load i
// takes row 4i + l / 16, block l % 16, so each load covers four rows of 256
// contiguous bytes (reading the transform's layout directly instead would
// make every load touch 16 rows for 16 bytes each).  Rows are kPxRow bytes
// apart in LDS; the 16-byte pad puts the 64 words that one transform-layout
// read touches (rows n, words g of a block) in 64 different banks.  Blocks past
// the tile's end read as zero.
constexpr int kPxRow = 272;
struct PxStage {
  uint32_t w[16 * kPxRow / 4];
};

__device__ __forceinline__ void stage_tile_px(const TileIO& io, int pitch, int count, uint32_t* st) {
  typedef __attribute__((ext_vector_type(4))) unsigned int u32x4;
  const int lane = threadIdx.x & 63;
  const int bl = lane & 15, rr = lane >> 4;
  const uint32_t past = bl < count ? 0u : 0xffffffffu;
  u32x4 d[4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
    d[i] = __builtin_amdgcn_raw_buffer_load_b128(io.px, (uint32_t)((4 * i + rr) * pitch + 16 * bl) | past, 0, 0);
#pragma unroll
  for (int i = 0; i < 4; ++i) *(u32x4*)&st[((4 * i + rr) * kPxRow + 16 * bl) / 4] = d[i];
}

// Lane's pixel word of block b from the stage: pixels (n, 4g .. 4g+3).
__device__ __forceinline__ uint32_t staged_px(const uint32_t* st, int b, const Lane16& L) {
  return st[(L.n * kPxRow + 16 * b + 4 * L.g) / 4];
}

// Byte offsets in y of the coefficients of zigzag ranks zr[c] of block b, or
// an out-of-range offset for ranks at or beyond the block's k.
__device__ __forceinline__ void tile_y_offsets(const TileIO& io, int b, const Lane16& L, uint32_t voff[4]) {
  const int kk = __builtin_amdgcn_readlane(io.k, b);
  const uint32_t rel4 = 4u * (uint32_t)__builtin_amdgcn_readlane(io.rel_lo, b);
#pragma unroll
  for (int c = 0; c < 4; ++c) voff[c] = (L.zr[c] < kk) ? rel4 + 4u * (uint32_t)L.zr[c] : 0xffffffffu;
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

}  // namespace abcs
