// Block transforms of B = 8 and B = 32 (DCT and the Walsh-Hadamard transform
// of Section IV).  On the vector ALUs: the phase-1 DD statistic (in float64,
// in the fixed order of the definition) and the IDA transform step.  A
// workgroup takes a tile of up to 16 consecutive blocks of a block row;
// wavefront w handles blocks w, w + 4, ... of it.  Each wavefront keeps its
// block in LDS (row pitch B + 1 floats, so that a row and a column are both
// conflict-free) and runs the separable transform as two passes of B-term dot
// products, one output per lane per step.  The basis and the zigzag rank
// table are staged in LDS once per workgroup.  Sensing and the inverse
// transform of both block sizes run on the float32 matrix cores (k_sense32 /
// k_reconstruct32 and k_sense8 / k_reconstruct8 at the end of this file).
#pragma once

#include "common.hpp"
#include "transform16.hpp"
#include "bm3d_kernels.hpp"

namespace abcs {

// Orthonormal DCT-II bases D[u*B + j] of orders 8 (c_D8, shared with BM3D)
// and 32 (float32 copies of the host-built float64 table and the float64
// table itself), and zigzag ranks of coefficient (u, v) at u*B + v with their
// inverse (rank -> u*B + v).
__constant__ double c_D8d[64];
__constant__ float c_D32[1024];
__constant__ double c_D32d[1024];
__constant__ uint16_t c_zzrank8[64];
__constant__ uint16_t c_zzpos8[64];
__constant__ uint16_t c_zzrank32[1024];
__constant__ uint16_t c_zzpos32[1024];
// Orthonormal sequency-ordered Walsh-Hadamard bases W[s*B + j] (float32 and
// float64; the order-16 basis is declared with the 16x16 transforms).
__constant__ float c_W8[64];
__constant__ double c_W8d[64];
__constant__ float c_W32[1024];
__constant__ double c_W32d[1024];


template <int B, int XF>
struct GenTables;
template <>
struct GenTables<8, kXfDCT> {
  __device__ static const float* D() { return c_D8; }
  __device__ static const double* Dd() { return c_D8d; }
  __device__ static const uint16_t* rank() { return c_zzrank8; }
  __device__ static const uint16_t* pos() { return c_zzpos8; }
};
template <>
struct GenTables<32, kXfDCT> {
  __device__ static const float* D() { return c_D32; }
  __device__ static const double* Dd() { return c_D32d; }
  __device__ static const uint16_t* rank() { return c_zzrank32; }
  __device__ static const uint16_t* pos() { return c_zzpos32; }
};
template <>
struct GenTables<8, kXfWHT> {
  __device__ static const float* D() { return c_W8; }
  __device__ static const double* Dd() { return c_W8d; }
  __device__ static const uint16_t* rank() { return c_zzrank8; }
  __device__ static const uint16_t* pos() { return c_zzpos8; }
};
template <>
struct GenTables<32, kXfWHT> {
  __device__ static const float* D() { return c_W32; }
  __device__ static const double* Dd() { return c_W32d; }
  __device__ static const uint16_t* rank() { return c_zzrank32; }
  __device__ static const uint16_t* pos() { return c_zzpos32; }
};

template <int B>
struct GenShared {
  static constexpr int P = B + 1;        // LDS row pitch (elements)
  static constexpr int NN = B * B;       // coefficients per block
  static constexpr int PER = NN / 64;    // outputs per lane per pass (1 or 16)
  float D[B * P];                        // D[u][j] at u P + j
  uint16_t rank[NN];                     // zigzag rank of (u, v) at u B + v
  float a[kWavesPerGroup][B * P];        // per wave: block / first pass
  float b[kWavesPerGroup][B * P];        // per wave: second pass / rank-ordered buffer
};

template <int B, int XF>
__device__ __forceinline__ void gen_load_tables(GenShared<B>& sh) {
  constexpr int P = B + 1;
  for (int t = threadIdx.x; t < B * B; t += kGroupThreads) {
    sh.D[(t / B) * P + t % B] = GenTables<B, XF>::D()[t];
    sh.rank[t] = GenTables<B, XF>::rank()[t];
  }
}

// Pixels of block bb of the tile into X[r][c] (float, pitch B + 1); 4 pixels
// per 32-bit load (rows are 4-byte aligned: pitch and pixel_offset are
// multiples of 4, block columns multiples of 8).
template <int B>
__device__ __forceinline__ void gen_load_pixels(const __amdgpu_buffer_rsrc_t& rp, int pitch, int bb, float* X) {
  constexpr int P = B + 1, WPR = B / 4;
  const int lane = threadIdx.x & 63;
  for (int idx = lane; idx < B * WPR; idx += 64) {
    const int r = idx / WPR, cw = idx - r * WPR;
    const uint32_t w = __builtin_amdgcn_raw_buffer_load_b32(rp, r * pitch + B * bb + 4 * cw, 0, 0);
#pragma unroll
    for (int c = 0; c < 4; ++c) X[r * P + 4 * cw + c] = (float)((w >> (8 * c)) & 0xffu);
  }
}

// Forward 2D DCT: X (in a) -> C[u][v] (in a), using b.  Operands and the
// intermediate are float32, each B-term sum is accumulated in float64 (the
// vector units run float64 fused multiply-adds at the float32 rate), so the
// result is within a few float32 roundings of exact even at B = 32.
template <int B>
__device__ __forceinline__ void gen_fwd(const float* D, float* a, float* b) {
  constexpr int P = B + 1;
  const int lane = threadIdx.x & 63;
  // T[x][v] = sum_j X[x][j] D[v][j]
  for (int idx = lane; idx < B * B; idx += 64) {
    const int x = idx / B, v = idx - x * B;
    double s = 0.0;
#pragma unroll 8
    for (int j = 0; j < B; ++j) s = fma((double)a[x * P + j], (double)D[v * P + j], s);
    b[x * P + v] = (float)s;
  }
  wave_lds_sync();
  // C[u][v] = sum_x D[u][x] T[x][v]
  for (int idx = lane; idx < B * B; idx += 64) {
    const int u = idx / B, v = idx - u * B;
    double s = 0.0;
#pragma unroll 8
    for (int x = 0; x < B; ++x) s = fma((double)D[u * P + x], (double)b[x * P + v], s);
    a[u * P + v] = (float)s;
  }
  wave_lds_sync();
}

// Inverse 2D DCT: C (in a) -> X[x][x'] (in a), using b; sums as in gen_fwd.
template <int B>
__device__ __forceinline__ void gen_inv(const float* D, float* a, float* b) {
  constexpr int P = B + 1;
  const int lane = threadIdx.x & 63;
  // Q[u][x'] = sum_v C[u][v] D[v][x']
  for (int idx = lane; idx < B * B; idx += 64) {
    const int u = idx / B, xp = idx - u * B;
    double s = 0.0;
#pragma unroll 8
    for (int v = 0; v < B; ++v) s = fma((double)a[u * P + v], (double)D[v * P + xp], s);
    b[u * P + xp] = (float)s;
  }
  wave_lds_sync();
  // X[x][x'] = sum_u D[u][x] Q[u][x']
  for (int idx = lane; idx < B * B; idx += 64) {
    const int x = idx / B, xp = idx - x * B;
    double s = 0.0;
#pragma unroll 8
    for (int u = 0; u < B; ++u) s = fma((double)D[u * P + x], (double)b[u * P + xp], s);
    a[x * P + xp] = (float)s;
  }
  wave_lds_sync();
}

// Block bb's coefficient count and its offset relative to the image's part of
// y, clamped to that part (a corrupt k or offset cannot leave it).
__device__ __forceinline__ void gen_block_range(const ImgDev& im, const int32_t* k_all, const int64_t* off_all,
                                                int64_t blk, int nn, int& kk, int64_t& rel) {
  const int64_t n = im.n_meas;
  int k = k_all[blk];
  int64_t r = off_all[blk] - im.meas_off;
  if (r < 0 || r > n || k < 0) k = 0, r = 0;
  if (k > nn) k = nn;
  if (k > n - r) k = (int)(n - r);
  kk = __builtin_amdgcn_readfirstlane(k);
  rel = r;
}

// The transform half of an IDA iteration (as k_ida_step16): z^t = y - A x^t
// + alpha z^{t-1} on the measured coefficients, v = x + A* z^t, and the
// block's sum of (z^t)^2 in float64 (fixed butterfly order) in part[blk].
template <int B, int XF>
__global__ __launch_bounds__(kGroupThreads) void k_gen_ida_step(const ImgDev* __restrict__ imgs,
                                                               const Tile* __restrict__ tiles, int ntiles,
                                                               const float* __restrict__ y,
                                                               const int32_t* __restrict__ k_all,
                                                               const int64_t* __restrict__ off_all,
                                                               const float* x, float* __restrict__ z,
                                                               float* v, double* __restrict__ part, float alpha,
                                                               const float* __restrict__ alpha_img, int first) {
  constexpr int P = B + 1;
  __shared__ GenShared<B> sh;
  if ((int)blockIdx.x >= ntiles) return;
  gen_load_tables<B, XF>(sh);
  __syncthreads();
  const Tile tl = tiles[blockIdx.x];
  const ImgDev im = imgs[tl.img];
  if (alpha_img) alpha = alpha_img[tl.img];
  const int w = wave_in_group(), lane = threadIdx.x & 63;
  float* a = sh.a[w];
  float* b = sh.b[w];
  const float* ym = y + im.meas_off;
  float* zm = z + im.meas_off;
  for (int bb = w; bb < tl.count; bb += kWavesPerGroup) {
    const int64_t base = tl.out_base + B * bb;
    for (int idx = lane; idx < B * B; idx += 64) {
      const int r = idx / B, c = idx - r * B;
      a[r * P + c] = first ? 0.f : x[base + (int64_t)r * im.Wc + c];
    }
    wave_lds_sync();
    gen_fwd<B>(sh.D, a, b);
    for (int idx = lane; idx < B * B; idx += 64) {
      const int u = idx / B, vv = idx - u * B;
      b[sh.rank[idx]] = a[u * P + vv];
    }
    wave_lds_sync();
    int kk;
    int64_t rel;
    const int64_t blk = im.blk_off + tl.first + bb;
    gen_block_range(im, k_all, off_all, blk, B * B, kk, rel);
    double acc = 0.0;
    for (int zi = lane; zi < kk; zi += 64) {
      const float zo = first ? 0.f : zm[rel + zi];
      const float zn = (ym[rel + zi] - b[zi]) + alpha * zo;
      zm[rel + zi] = zn;
      b[zi] = b[zi] + zn;
      acc += (double)zn * (double)zn;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) part[blk] = acc;
    wave_lds_sync();
    for (int idx = lane; idx < B * B; idx += 64) {
      const int u = idx / B, vv = idx - u * B;
      a[u * P + vv] = b[sh.rank[idx]];
    }
    wave_lds_sync();
    gen_inv<B>(sh.D, a, b);
    for (int idx = lane; idx < B * B; idx += 64) {
      const int r = idx / B, c = idx - r * B;
      v[base + (int64_t)r * im.Wc + c] = a[r * P + c];
    }
    wave_lds_sync();
  }
}

// ---------------------------------------------------------------------------
// B = 32 on the float32 matrix cores.  A 32x32 block is a 2x2 arrangement of
// 16x16 sub-blocks, X_ik = rows 16i.., columns 16k.., and likewise D_ab for
// the basis, so the separable transform becomes products of 16x16 tiles on
// v_mfma_f32_16x16x4f32 with the K mapping of the 16x16 kernels (lane
// l = 16g + n; a stage's accumulators are the next stage's B operand):
//   forward  T_ij = sum_k X_ik D_jk^T,        C_ij = sum_k D_ik T_kj
//   inverse  Q_ij = sum_k C_ki^T D_kj,   (X^T)_ij = sum_k D_ki^T Q_kj
// 32 products per stage (64 per block), one wavefront per tile of up to 16
// blocks, taken one after the other.  For the 16-bit modes lane (g, n) keeps
// the basis tiles in both operand layouts: dR[a][b][c] = D[16a + n][16b + 4g
// + c] and dT[a][b][c] = D[16a + 4g + c][16b + n]; float32 uses the truncated
// layout of Lane32T below.
// ---------------------------------------------------------------------------
struct Lane32 {
  int g, n;
  float dR[2][2][4], dT[2][2][4];
};

template <int XF>
__device__ __forceinline__ void lane32_init(Lane32& L) {
  const float* D = GenTables<32, XF>::D();
  const int lane = threadIdx.x & 63;
  L.g = lane >> 4;
  L.n = lane & 15;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        L.dR[a][b][c] = D[(16 * a + L.n) * 32 + 16 * b + 4 * L.g + c];
        L.dT[a][b][c] = D[(16 * a + 4 * L.g + c) * 32 + 16 * b + L.n];
      }
}

// Float32 B = 32 transforms of zigzag-truncated blocks.  As in the 16x16
// truncated inverse, the inverse's products take four consecutive
// frequencies each: the K slots of product (k, c) are coefficient rows (first
// stage) or rows of Q (second stage) 16k + 4c .. 16k + 4c + 3, so a block with
// k_i coefficients, non-zero only on anti-diagonals u + v <= d (d that of
// zigzag rank k_i - 1), needs the first-stage product (k, c) of output tile
// column i only when 16 (k + i) + 4c <= d and the second-stage product (k, c)
// only when 16k + 4c <= d; the skipped ones would add exact zeros.  The
// forward transform leaves its output in that layout by taking the basis rows
// in the order s(n) = 4 (n % 4) + n / 4 within each 16-row half (only rows
// and columns of the products move: every output is summed over the same K
// slots in the same order as without the permutation), and it computes only
// the output tiles that hold a coefficient of zigzag rank below k_i.
//   forward out C[i][j][r] = C(16i + 4r + g, 16j + s(n));
//   inverse in  e[k][i][c] = C(16k + 4c + g, 16i + s(n)),
//           out X[i][j][r] = X[16j + n][16i + 4g + r].
// Lane (g, n) keeps dS[a][b][c] = D[16a + s(n)][16b + 4g + c] and
// dP[a][b][c] = D[16a + 4c + g][16b + n].
struct Lane32T {
  float dS[2][2][4], dP[2][2][4];
};

template <int XF>
__device__ __forceinline__ void lane32t_init(Lane32T& L) {
  const float* D = GenTables<32, XF>::D();
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, n = lane & 15, sn = 4 * (n & 3) + (n >> 2);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        L.dS[a][b][c] = D[(16 * a + sn) * 32 + 16 * b + 4 * g + c];
        L.dP[a][b][c] = D[(16 * a + 4 * c + g) * 32 + 16 * b + n];
      }
}

// Number of coefficients of a 32x32 block on anti-diagonals below t (the
// zigzag rank of the first coefficient on diagonal t).
__host__ __device__ constexpr int zz32_below(int t) {
  return t <= 32 ? t * (t + 1) / 2 : 1024 - (63 - t) * (64 - t) / 2;
}

// Zigzag rank of the coefficient that register [a][b][c] of this lane holds:
// C(16a + 4c + g, 16b + s(n)) in the truncated float32 layout (TRUNC), else
// C(16a + 4g + c, 16b + n) (the 16-bit modes).
template <bool TRUNC>
__device__ __forceinline__ void zz32_ranks(int zr[2][2][4]) {
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, n = lane & 15, sn = 4 * (n & 3) + (n >> 2);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int c = 0; c < 4; ++c)
        zr[a][b][c] = TRUNC ? c_zzrank32[(16 * a + 4 * c + g) * 32 + 16 * b + sn]
                            : c_zzrank32[(16 * a + 4 * g + c) * 32 + 16 * b + n];
}

// x[i][k][c] = X[16i + n][16k + 4g + c]; kk (wave-uniform) = the block's
// k_i.  Output tiles (i, j)
// with 16 (i + j) past the block's last diagonal are left zero.
__device__ __forceinline__ void dct32_fwd_t(const float x[2][2][4], const Lane32T& L, int kk, f32x4 C[2][2]) {
  f32x4 T[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      f32x4 t = {0.f, 0.f, 0.f, 0.f};
      if (kk > zz32_below(16 * j)) {
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
          for (int c = 0; c < 4; ++c) t = __builtin_amdgcn_mfma_f32_16x16x4f32(x[i][k][c], L.dS[j][k][c], t, 0, 0, 0);
      }
      T[i][j] = t;
    }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      f32x4 o = {0.f, 0.f, 0.f, 0.f};
      if (kk > zz32_below(16 * (i + j))) {
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
          for (int c = 0; c < 4; ++c) o = __builtin_amdgcn_mfma_f32_16x16x4f32(L.dS[i][k][c], T[k][j][c], o, 0, 0, 0);
      }
      C[i][j] = o;
    }
}

// e (zero past the block's kk coefficients) -> X[i][j][r] = X[16j + n][16i + 4g + r]
__device__ __forceinline__ void idct32_inv_t(const float e[2][2][4], const Lane32T& L, int kk, f32x4 X[2][2]) {
  f32x4 Q[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      f32x4 q = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int c = 0; c < 4; ++c)
          if (kk > zz32_below(16 * (k + i) + 4 * c))
            q = __builtin_amdgcn_mfma_f32_16x16x4f32(e[k][i][c], L.dP[k][j][c], q, 0, 0, 0);
      Q[i][j] = q;
    }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      f32x4 o = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int c = 0; c < 4; ++c)
          if (kk > zz32_below(16 * k + 4 * c))
            o = __builtin_amdgcn_mfma_f32_16x16x4f32(L.dP[k][i][c], Q[k][j][c], o, 0, 0, 0);
      X[i][j] = o;
    }
}

// The 16-bit modes of the B = 32 products (see the precision modes of the
// 16x16 transforms): one v_mfma_f32_16x16x{16bf16_1k,16f16} takes the four K
// slots 4g .. 4g+3 that four float32 products take, so a lane's operands of a
// 16x16 tile product pack into one 16-bit 4-vector.  The split modes keep hi
// x hi, hi x lo and lo x hi of every stage; pixels are exact in 16 bits.
template <int P>
struct Lane32P {
  u16x4 r_hi[2][2], r_lo[2][2], t_hi[2][2], t_lo[2][2];  // dR and dT, split
};

template <int P>
__device__ __forceinline__ void lane32p_init(Lane32P<P>& H, const Lane32& L) {
  constexpr bool BF = Prec16<P>::kBF;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      split16<BF>(L.dR[a][b], H.r_hi[a][b], H.r_lo[a][b]);
      split16<BF>(L.dT[a][b], H.t_hi[a][b], H.t_lo[a][b]);
    }
}

// x[i][k][c] = X[16i + n][16k + 4g + c] -> C[i][j][r] = C(16i + 4g + r,
// 16j + n), products in precision P
template <int P>
__device__ __forceinline__ void dct32_fwd_p(const float x[2][2][4], const Lane32P<P>& H, f32x4 C[2][2]) {
  constexpr bool BF = Prec16<P>::kBF, SP = Prec16<P>::kSplit;
  u16x4 xs[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int c = 0; c < 4; ++c) xs[i][k][c] = to16<BF>(x[i][k][c]);
  u16x4 th[2][2], tl[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      f32x4 t = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        t = mfma16<BF>(xs[i][k], H.r_hi[j][k], t);  // T = X D^T
        if (SP) t = mfma16<BF>(xs[i][k], H.r_lo[j][k], t);
      }
      const float tv[4] = {t[0], t[1], t[2], t[3]};
      split16<BF>(tv, th[i][j], tl[i][j]);
    }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      f32x4 o = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        o = mfma16<BF>(H.r_hi[i][k], th[k][j], o);  // C = D T
        if (SP) {
          o = mfma16<BF>(H.r_hi[i][k], tl[k][j], o);
          o = mfma16<BF>(H.r_lo[i][k], th[k][j], o);
        }
      }
      C[i][j] = o;
    }
}

// e[k][i][c] = C(16k + 4g + c, 16i + n) -> X[i][j][r] = X[16j + n][16i +
// 4g + r], products in precision P
template <int P>
__device__ __forceinline__ void idct32_inv_p(const float e[2][2][4], const Lane32P<P>& H, f32x4 X[2][2]) {
  constexpr bool BF = Prec16<P>::kBF, SP = Prec16<P>::kSplit;
  u16x4 eh[2][2], el[2][2];
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int i = 0; i < 2; ++i) split16<BF>(e[k][i], eh[k][i], el[k][i]);
  u16x4 qh[2][2], ql[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      f32x4 q = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        q = mfma16<BF>(eh[k][i], H.t_hi[k][j], q);  // Q = C^T D
        if (SP) {
          q = mfma16<BF>(el[k][i], H.t_hi[k][j], q);
          q = mfma16<BF>(eh[k][i], H.t_lo[k][j], q);
        }
      }
      const float qv[4] = {q[0], q[1], q[2], q[3]};
      split16<BF>(qv, qh[i][j], ql[i][j]);
    }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      f32x4 o = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        o = mfma16<BF>(H.t_hi[k][i], qh[k][j], o);  // X^T = D^T Q
        if (SP) {
          o = mfma16<BF>(H.t_hi[k][i], ql[k][j], o);
          o = mfma16<BF>(H.t_lo[k][i], qh[k][j], o);
        }
      }
      X[i][j] = o;
    }
}

struct WaveLds32 {
  float c[1024];
};

// y[off_i + z] = C_i[zigzag[z]] for z < k_i (B = 32): the block's
// coefficients go to LDS at their zigzag rank, then leave in unit-stride
// stores of k_i values (float32: only the output tiles that hold one of them
// are computed).
template <int XF, int P = kPrecFP32>
__global__ __launch_bounds__(kGroupThreads) void k_sense32(const ImgDev* __restrict__ imgs,
                                                          const Tile* __restrict__ tiles, int ntiles, int split,
                                                          const uint8_t* __restrict__ px,
                                                          const int32_t* __restrict__ k_all,
                                                          const int64_t* __restrict__ off_all,
                                                          float* __restrict__ y) {
  __shared__ WaveLds32 lds[kWavesPerGroup];
  const int wave = blockIdx.x * kWavesPerGroup + wave_in_group();
  if (wave >= (ntiles << split)) return;
  const Tile tl = split_tile(tiles, wave, split, 32);
  if (tl.count == 0) return;
  const ImgDev im = imgs[tl.img];
  constexpr bool TR = (P == kPrecFP32);  // float32: truncated transforms
  Lane32T LT;
  Lane32 L;
  Lane32P<P> H;
  if constexpr (TR) {
    lane32t_init<XF>(LT);
  } else {
    lane32_init<XF>(L);
    lane32p_init<P>(H, L);
  }
  const int lane = threadIdx.x & 63, lg = lane >> 4, ln = lane & 15;
  int zr[2][2][4];  // zigzag rank of the coefficient in each output register
  zz32_ranks<TR>(zr);
  const __amdgpu_buffer_rsrc_t rp = make_rsrc(px + tl.px_base, 31 * im.pitch + 32 * tl.count);
  const __amdgpu_buffer_rsrc_t ry = make_rsrc(y + im.meas_off, (int)(4 * im.n_meas));
  const __amdgpu_buffer_rsrc_t rk = make_rsrc(k_all + im.blk_off + tl.first, 4 * tl.count);
  const __amdgpu_buffer_rsrc_t ro = make_rsrc(off_all + im.blk_off + tl.first, 8 * tl.count);
  const int32_t kl = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(rk, 4 * lane, 0, 0);
  const int32_t rl = (int32_t)(__builtin_amdgcn_raw_buffer_load_b32(ro, 8 * lane, 0, 0) - (uint32_t)im.meas_off);
  float* buf = lds[wave_in_group()].c;
  for (int b = 0; b < tl.count; ++b) {
    float x[2][2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const uint32_t w =
            __builtin_amdgcn_raw_buffer_load_b32(rp, (16 * i + ln) * im.pitch + 32 * b + 16 * k + 4 * lg, 0, 0);
#pragma unroll
        for (int c = 0; c < 4; ++c) x[i][k][c] = (float)((w >> (8 * c)) & 0xffu);
      }
    const int kk = __builtin_amdgcn_readlane(kl, b);
    f32x4 C[2][2];
    if constexpr (TR)
      dct32_fwd_t(x, LT, kk, C);
    else
      dct32_fwd_p<P>(x, H, C);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) buf[zr[i][j][r]] = C[i][j][r];
    wave_lds_sync();
    const uint32_t rel4 = 4u * (uint32_t)__builtin_amdgcn_readlane(rl, b);
    for (int q = 0; q < 16 && 64 * q < kk; ++q) {
      const int z = lane + 64 * q;
      const uint32_t voff = z < kk ? rel4 + 4u * (uint32_t)z : 0xffffffffu;
      __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(buf[z]), ry, voff, 0, 0);
    }
    wave_lds_sync();
  }
}

// out = D^T C D per block (B = 32), C zero beyond the block's k_i zigzag
// entries: the block's coefficients are staged in LDS in zigzag order (zero
// past k_i) and gathered in the inverse's operand layout; in float32 the
// inverse skips the products of all-zero operands.
template <int XF, int P = kPrecFP32>
__global__ __launch_bounds__(kGroupThreads) void k_reconstruct32(const ImgDev* __restrict__ imgs,
                                                                const Tile* __restrict__ tiles, int ntiles, int split,
                                                                const float* __restrict__ y,
                                                                const int32_t* __restrict__ k_all,
                                                                const int64_t* __restrict__ off_all,
                                                                float* __restrict__ out) {
  typedef __attribute__((ext_vector_type(4))) unsigned int u32x4;
  __shared__ WaveLds32 lds[kWavesPerGroup];
  const int wave = blockIdx.x * kWavesPerGroup + wave_in_group();
  if (wave >= (ntiles << split)) return;
  const Tile tl = split_tile(tiles, wave, split, 32);
  if (tl.count == 0) return;
  const ImgDev im = imgs[tl.img];
  constexpr bool TR = (P == kPrecFP32);  // float32: truncated transforms
  Lane32T LT;
  Lane32 L;
  Lane32P<P> H;
  if constexpr (TR) {
    lane32t_init<XF>(LT);
  } else {
    lane32_init<XF>(L);
    lane32p_init<P>(H, L);
  }
  const int lane = threadIdx.x & 63, lg = lane >> 4, ln = lane & 15;
  int zr[2][2][4];  // zigzag rank of the coefficient in each operand register
  zz32_ranks<TR>(zr);
  const __amdgpu_buffer_rsrc_t ry = make_rsrc(y + im.meas_off, (int)(4 * im.n_meas));
  const __amdgpu_buffer_rsrc_t rk = make_rsrc(k_all + im.blk_off + tl.first, 4 * tl.count);
  const __amdgpu_buffer_rsrc_t ro = make_rsrc(off_all + im.blk_off + tl.first, 8 * tl.count);
  const __amdgpu_buffer_rsrc_t rout = make_rsrc(out + tl.out_base, 4 * (31 * im.Wc + 32 * tl.count));
  const int32_t kl = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(rk, 4 * lane, 0, 0);
  const int32_t rl = (int32_t)(__builtin_amdgcn_raw_buffer_load_b32(ro, 8 * lane, 0, 0) - (uint32_t)im.meas_off);
  float* buf = lds[wave_in_group()].c;
  for (int b = 0; b < tl.count; ++b) {
    const int kk = __builtin_amdgcn_readlane(kl, b);
    const uint32_t rel4 = 4u * (uint32_t)__builtin_amdgcn_readlane(rl, b);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int z = lane + 64 * q;
      const uint32_t voff = z < kk ? rel4 + 4u * (uint32_t)z : 0xffffffffu;
      buf[z] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(ry, voff, 0, 0));
    }
    wave_lds_sync();
    float e[2][2][4];
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int c = 0; c < 4; ++c) e[k][i][c] = buf[zr[k][i][c]];
    wave_lds_sync();
    f32x4 X[2][2];
    if constexpr (TR)
      idct32_inv_t(e, LT, kk, X);
    else
      idct32_inv_p<P>(e, H, X);
    // X[i][j][r] = pixel (16j + n, 16i + 4g + r)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const uint32_t off = 4u * (uint32_t)((16 * j + ln) * im.Wc + 32 * b + 16 * i + 4 * lg);
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, X[i][j]), rout, off, 0, kStoreNT);
      }
  }
}

// Sensing and the local decoder in one pass (B = 32): the forward
// transform's output layout is the inverse's input layout (the truncated
// float32 layout, or that of the 16-bit modes), so the decoder takes the
// block's coefficients from registers, masked past k_i by zigzag rank; only
// y goes through LDS.  Same bits as k_sense32 followed by k_reconstruct32.
template <int XF, int P = kPrecFP32>
__global__ __launch_bounds__(kGroupThreads) void k_encode32(const ImgDev* __restrict__ imgs,
                                                           const Tile* __restrict__ tiles, int ntiles, int split,
                                                           const uint8_t* __restrict__ px,
                                                           const int32_t* __restrict__ k_all,
                                                           const int64_t* __restrict__ off_all,
                                                           float* __restrict__ y, float* __restrict__ out) {
  typedef __attribute__((ext_vector_type(4))) unsigned int u32x4;
  __shared__ WaveLds32 lds[kWavesPerGroup];
  const int wave = blockIdx.x * kWavesPerGroup + wave_in_group();
  if (wave >= (ntiles << split)) return;
  const Tile tl = split_tile(tiles, wave, split, 32);
  if (tl.count == 0) return;
  const ImgDev im = imgs[tl.img];
  constexpr bool TR = (P == kPrecFP32);  // float32: truncated transforms
  Lane32T LT;
  Lane32 L;
  Lane32P<P> H;
  if constexpr (TR) {
    lane32t_init<XF>(LT);
  } else {
    lane32_init<XF>(L);
    lane32p_init<P>(H, L);
  }
  const int lane = threadIdx.x & 63, lg = lane >> 4, ln = lane & 15;
  int zr[2][2][4];  // zigzag rank of the coefficient in each output register
  zz32_ranks<TR>(zr);
  const __amdgpu_buffer_rsrc_t rp = make_rsrc(px + tl.px_base, 31 * im.pitch + 32 * tl.count);
  const __amdgpu_buffer_rsrc_t ry = make_rsrc(y + im.meas_off, (int)(4 * im.n_meas));
  const __amdgpu_buffer_rsrc_t rk = make_rsrc(k_all + im.blk_off + tl.first, 4 * tl.count);
  const __amdgpu_buffer_rsrc_t ro = make_rsrc(off_all + im.blk_off + tl.first, 8 * tl.count);
  const __amdgpu_buffer_rsrc_t rout = make_rsrc(out + tl.out_base, 4 * (31 * im.Wc + 32 * tl.count));
  const int32_t kl = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(rk, 4 * lane, 0, 0);
  const int32_t rl = (int32_t)(__builtin_amdgcn_raw_buffer_load_b32(ro, 8 * lane, 0, 0) - (uint32_t)im.meas_off);
  float* buf = lds[wave_in_group()].c;
  for (int b = 0; b < tl.count; ++b) {
    float x[2][2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const uint32_t w =
            __builtin_amdgcn_raw_buffer_load_b32(rp, (16 * i + ln) * im.pitch + 32 * b + 16 * k + 4 * lg, 0, 0);
#pragma unroll
        for (int c = 0; c < 4; ++c) x[i][k][c] = (float)((w >> (8 * c)) & 0xffu);
      }
    const int kk = __builtin_amdgcn_readlane(kl, b);
    f32x4 C[2][2];
    if constexpr (TR)
      dct32_fwd_t(x, LT, kk, C);
    else
      dct32_fwd_p<P>(x, H, C);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) buf[zr[i][j][r]] = C[i][j][r];
    wave_lds_sync();
    const uint32_t rel4 = 4u * (uint32_t)__builtin_amdgcn_readlane(rl, b);
    for (int q = 0; q < 16 && 64 * q < kk; ++q) {
      const int z = lane + 64 * q;
      const uint32_t voff = z < kk ? rel4 + 4u * (uint32_t)z : 0xffffffffu;
      __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(buf[z]), ry, voff, 0, 0);
    }
    wave_lds_sync();
    float e[2][2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) e[i][j][r] = zr[i][j][r] < kk ? C[i][j][r] : 0.f;
    f32x4 X[2][2];
    if constexpr (TR)
      idct32_inv_t(e, LT, kk, X);
    else
      idct32_inv_p<P>(e, H, X);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const uint32_t off = 4u * (uint32_t)((16 * j + ln) * im.Wc + 32 * b + 16 * i + 4 * lg);
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, X[i][j]), rout, off, 0, kStoreNT);
      }
  }
}

// ---------------------------------------------------------------------------
// B = 8 on the float32 matrix cores.  Four consecutive blocks b0 .. b0 + 3 of
// a tile are placed as the quadrants of a 16x16 array (block b0 + 2p + q at
// rows 8p .., columns 8q ..) and transformed with the block-diagonal basis
// diag(D8, D8): its zero off-diagonal blocks keep the quadrants apart, so the
// 16x16 transform of the 16x16 kernels (eight v_mfma_f32_16x16x4f32) yields
// the four 8x8 transforms at once.
//   lane (g, n) operand x[c] = X16[n][4g + c]: block b0 + 2 (n / 8) + g / 2,
//     pixel row n % 8, columns 4 (g % 2) + c;
//   forward output C16[4g + r][n]: block b0 + 2 (g / 2) + n / 8, coefficient
//     (4 (g % 2) + r, n % 8);
//   inverse operand e[c] = C16[4g + c][n] (same block and coefficient as the
//   forward output), output X16[n][4g + r] (same block and pixels as x).
// ---------------------------------------------------------------------------
template <int XF>
__device__ __forceinline__ void lane8x4_init(Lane16& L) {
  const float* D = GenTables<8, XF>::D();
  const int lane = threadIdx.x & 63;
  L.g = lane >> 4;
  L.n = lane & 15;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int j = 4 * L.g + c;  // 0..15
    // diag(D8, D8)[u][j] = D8[u % 8][j % 8] when u / 8 == j / 8, else 0
    L.dR[c] = (L.n >> 3) == (j >> 3) ? D[(L.n & 7) * 8 + (j & 7)] : 0.f;
    L.dT[c] = (j >> 3) == (L.n >> 3) ? D[(j & 7) * 8 + (L.n & 7)] : 0.f;
    L.zr[c] = 0;
  }
}

struct WaveLds8 {
  float c[4][64];
};

template <int XF, int P = kPrecFP32>
__global__ __launch_bounds__(kGroupThreads) void k_sense8(const ImgDev* __restrict__ imgs,
                                                         const Tile* __restrict__ tiles, int ntiles, int split,
                                                         const uint8_t* __restrict__ px,
                                                         const int32_t* __restrict__ k_all,
                                                         const int64_t* __restrict__ off_all,
                                                         float* __restrict__ y) {
  __shared__ WaveLds8 lds[kWavesPerGroup];
  const int wave = blockIdx.x * kWavesPerGroup + wave_in_group();
  if (wave >= (ntiles << split)) return;
  const Tile tl = split_tile(tiles, wave, split, 8);
  if (tl.count == 0) return;
  const ImgDev im = imgs[tl.img];
  Lane16 L;
  lane8x4_init<XF>(L);
  Lane16P<P> H;  // the block-diagonal basis split for the 16-bit modes
  if constexpr (P != kPrecFP32) lane16p_init<P>(H, L);
  const int lane = threadIdx.x & 63;
  // operand side: block quadrant and pixel row / column of this lane
  const int xq = 2 * (L.n >> 3) + (L.g >> 1), xrow = L.n & 7, xcol = 4 * (L.g & 1);
  // output side: block quadrant and zigzag rank of coefficient r
  const int oq = 2 * (L.g >> 1) + (L.n >> 3);
  int zr[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) zr[r] = c_zzrank8[(4 * (L.g & 1) + r) * 8 + (L.n & 7)];
  const __amdgpu_buffer_rsrc_t rp = make_rsrc(px + tl.px_base, 7 * im.pitch + 8 * tl.count);
  const __amdgpu_buffer_rsrc_t ry = make_rsrc(y + im.meas_off, (int)(4 * im.n_meas));
  const __amdgpu_buffer_rsrc_t rk = make_rsrc(k_all + im.blk_off + tl.first, 4 * tl.count);
  const __amdgpu_buffer_rsrc_t ro = make_rsrc(off_all + im.blk_off + tl.first, 8 * tl.count);
  const int32_t kl = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(rk, 4 * lane, 0, 0);
  const int32_t rl = (int32_t)(__builtin_amdgcn_raw_buffer_load_b32(ro, 8 * lane, 0, 0) - (uint32_t)im.meas_off);
  WaveLds8& buf = lds[wave_in_group()];
  for (int b0 = 0; b0 < tl.count; b0 += 4) {
    const int bx = b0 + xq;
    const uint32_t w = __builtin_amdgcn_raw_buffer_load_b32(
        rp, bx < tl.count ? (uint32_t)(xrow * im.pitch + 8 * bx + xcol) : 0xffffffffu, 0, 0);
    float a[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) a[c] = (float)((w >> (8 * c)) & 0xffu);
    f32x4 C;
    if constexpr (P == kPrecFP32)
      C = dct16_fwd(a, L);
    else
      C = dct16_fwd_p<P>(a, H);
#pragma unroll
    for (int r = 0; r < 4; ++r) buf.c[oq][zr[r]] = C[r];
    wave_lds_sync();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int b = b0 + q;
      if (b < tl.count) {
        const int kk = __builtin_amdgcn_readlane(kl, b);
        const uint32_t rel4 = 4u * (uint32_t)__builtin_amdgcn_readlane(rl, b);
        const uint32_t voff = lane < kk ? rel4 + 4u * (uint32_t)lane : 0xffffffffu;
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(buf.c[q][lane]), ry, voff, 0, 0);
      }
    }
    wave_lds_sync();
  }
}

template <int XF, int P = kPrecFP32>
__global__ __launch_bounds__(kGroupThreads) void k_reconstruct8(const ImgDev* __restrict__ imgs,
                                                               const Tile* __restrict__ tiles, int ntiles, int split,
                                                               const float* __restrict__ y,
                                                               const int32_t* __restrict__ k_all,
                                                               const int64_t* __restrict__ off_all,
                                                               float* __restrict__ out) {
  typedef __attribute__((ext_vector_type(4))) unsigned int u32x4;
  __shared__ WaveLds8 lds[kWavesPerGroup];
  const int wave = blockIdx.x * kWavesPerGroup + wave_in_group();
  if (wave >= (ntiles << split)) return;
  const Tile tl = split_tile(tiles, wave, split, 8);
  if (tl.count == 0) return;
  const ImgDev im = imgs[tl.img];
  Lane16 L;
  lane8x4_init<XF>(L);
  Lane16P<P> H;  // the block-diagonal basis split for the 16-bit modes
  if constexpr (P != kPrecFP32) lane16p_init<P>(H, L);
  const int lane = threadIdx.x & 63;
  const int xq = 2 * (L.n >> 3) + (L.g >> 1), xrow = L.n & 7, xcol = 4 * (L.g & 1);
  const int oq = 2 * (L.g >> 1) + (L.n >> 3);
  int zr[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) zr[c] = c_zzrank8[(4 * (L.g & 1) + c) * 8 + (L.n & 7)];
  const __amdgpu_buffer_rsrc_t ry = make_rsrc(y + im.meas_off, (int)(4 * im.n_meas));
  const __amdgpu_buffer_rsrc_t rk = make_rsrc(k_all + im.blk_off + tl.first, 4 * tl.count);
  const __amdgpu_buffer_rsrc_t ro = make_rsrc(off_all + im.blk_off + tl.first, 8 * tl.count);
  const __amdgpu_buffer_rsrc_t rout = make_rsrc(out + tl.out_base, 4 * (7 * im.Wc + 8 * tl.count));
  const int32_t kl = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(rk, 4 * lane, 0, 0);
  const int32_t rl = (int32_t)(__builtin_amdgcn_raw_buffer_load_b32(ro, 8 * lane, 0, 0) - (uint32_t)im.meas_off);
  WaveLds8& buf = lds[wave_in_group()];
  for (int b0 = 0; b0 < tl.count; b0 += 4) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int b = b0 + q;
      const int kk = b < tl.count ? __builtin_amdgcn_readlane(kl, b) : 0;
      const uint32_t rel4 = 4u * (uint32_t)__builtin_amdgcn_readlane(rl, b < tl.count ? b : 0);
      const uint32_t voff = lane < kk ? rel4 + 4u * (uint32_t)lane : 0xffffffffu;
      buf.c[q][lane] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(ry, voff, 0, 0));
    }
    wave_lds_sync();
    float e[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) e[c] = buf.c[oq][zr[c]];
    wave_lds_sync();
    f32x4 X;
    if constexpr (P == kPrecFP32)
      X = idct16_inv(e, L);
    else
      X = idct16_inv_p<P>(e, H);
    const int bx = b0 + xq;
    const uint32_t off = bx < tl.count ? 4u * (uint32_t)(xrow * im.Wc + 8 * bx + xcol) : 0xffffffffu;
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, X), rout, off, 0, kStoreNT);
  }
}

// Sensing and the local decoder in one pass (B = 8): the forward output
// C16[4g + r][n] is the inverse's operand layout, so the decoder takes each
// block's coefficients from registers, masked past its k by zigzag rank (a
// lane's block is b0 + 2 (g / 2) + n / 8).  Same bits as k_sense8 followed
// by k_reconstruct8.
template <int XF, int P = kPrecFP32>
__global__ __launch_bounds__(kGroupThreads) void k_encode8(const ImgDev* __restrict__ imgs,
                                                          const Tile* __restrict__ tiles, int ntiles, int split,
                                                          const uint8_t* __restrict__ px,
                                                          const int32_t* __restrict__ k_all,
                                                          const int64_t* __restrict__ off_all,
                                                          float* __restrict__ y, float* __restrict__ out) {
  typedef __attribute__((ext_vector_type(4))) unsigned int u32x4;
  __shared__ WaveLds8 lds[kWavesPerGroup];
  const int wave = blockIdx.x * kWavesPerGroup + wave_in_group();
  if (wave >= (ntiles << split)) return;
  const Tile tl = split_tile(tiles, wave, split, 8);
  if (tl.count == 0) return;
  const ImgDev im = imgs[tl.img];
  Lane16 L;
  lane8x4_init<XF>(L);
  Lane16P<P> H;  // the block-diagonal basis split for the 16-bit modes
  if constexpr (P != kPrecFP32) lane16p_init<P>(H, L);
  const int lane = threadIdx.x & 63;
  // operand side: block quadrant and pixel row / column of this lane
  const int xq = 2 * (L.n >> 3) + (L.g >> 1), xrow = L.n & 7, xcol = 4 * (L.g & 1);
  // output side: block quadrant and zigzag rank of coefficient r
  const int oq = 2 * (L.g >> 1) + (L.n >> 3);
  int zr[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) zr[r] = c_zzrank8[(4 * (L.g & 1) + r) * 8 + (L.n & 7)];
  const __amdgpu_buffer_rsrc_t rp = make_rsrc(px + tl.px_base, 7 * im.pitch + 8 * tl.count);
  const __amdgpu_buffer_rsrc_t ry = make_rsrc(y + im.meas_off, (int)(4 * im.n_meas));
  const __amdgpu_buffer_rsrc_t rk = make_rsrc(k_all + im.blk_off + tl.first, 4 * tl.count);
  const __amdgpu_buffer_rsrc_t ro = make_rsrc(off_all + im.blk_off + tl.first, 8 * tl.count);
  const __amdgpu_buffer_rsrc_t rout = make_rsrc(out + tl.out_base, 4 * (7 * im.Wc + 8 * tl.count));
  const int32_t kl = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(rk, 4 * lane, 0, 0);
  const int32_t rl = (int32_t)(__builtin_amdgcn_raw_buffer_load_b32(ro, 8 * lane, 0, 0) - (uint32_t)im.meas_off);
  WaveLds8& buf = lds[wave_in_group()];
  for (int b0 = 0; b0 < tl.count; b0 += 4) {
    const int bx = b0 + xq;
    const uint32_t w = __builtin_amdgcn_raw_buffer_load_b32(
        rp, bx < tl.count ? (uint32_t)(xrow * im.pitch + 8 * bx + xcol) : 0xffffffffu, 0, 0);
    float a[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) a[c] = (float)((w >> (8 * c)) & 0xffu);
    f32x4 C;
    if constexpr (P == kPrecFP32)
      C = dct16_fwd(a, L);
    else
      C = dct16_fwd_p<P>(a, H);
#pragma unroll
    for (int r = 0; r < 4; ++r) buf.c[oq][zr[r]] = C[r];
    wave_lds_sync();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int b = b0 + q;
      if (b < tl.count) {
        const int kk = __builtin_amdgcn_readlane(kl, b);
        const uint32_t rel4 = 4u * (uint32_t)__builtin_amdgcn_readlane(rl, b);
        const uint32_t voff = lane < kk ? rel4 + 4u * (uint32_t)lane : 0xffffffffu;
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(buf.c[q][lane]), ry, voff, 0, 0);
      }
    }
    wave_lds_sync();
    // k of this lane's output block (0 past the tile's end: kl reads 0 there)
    const int ko = __shfl(kl, (b0 + oq) & 63, 64);
    float e[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) e[c] = zr[c] < ko ? C[c] : 0.f;
    f32x4 X;
    if constexpr (P == kPrecFP32)
      X = idct16_inv(e, L);
    else
      X = idct16_inv_p<P>(e, H);
    const uint32_t off = bx < tl.count ? 4u * (uint32_t)(xrow * im.Wc + 8 * bx + xcol) : 0xffffffffu;
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, X), rout, off, 0, kStoreNT);
  }
}

// ---------------------------------------------------------------------------
// DD statistics n_i of B = 32 and B = 8 blocks, screened on the float32
// matrix cores and exact: the forward transform decides |c| > T for every
// coefficient of zigzag rank below m1 further than the guard from T; the
// others are recomputed in float64 in the definition's order (T[r] = sum_j
// X[r][j] D[v][j], j ascending; c = sum_r D[u][r] T[r], r ascending; every
// product and sum rounded on its own), B lanes per coefficient: lane r forms
// row r's sum from the block's pixels, the group's first lane adds the rows'
// products in order.  Screening errors (u = 2^-24; a float32 sum of n terms
// errs by at most n u times the sum of their magnitudes; |X| <= 255):
//   B = 32 (|D| <= 0.25, sum_j |D[v][j]| <= sqrt(32) < 5.66): stage 1, 32
//     products of magnitude sum <= 1443: 32 u 1443 = 2.8e-3, plus the float32
//     rounding of D (32 * 255 * 0.25 * 2^-24 = 1.2e-4), so |T| <= 1443.1;
//     stage 2, magnitude sum <= 8165: 32 u 8165 = 1.56e-2, the stage-1 error
//     times 5.66 (1.64e-2) and D's rounding on T (32 * 0.25 * 2^-24 * 1443 =
//     6.9e-4): <= 3.3e-2.  Guard 0.1.
//   B = 8 (|D| <= 0.5, sum_j |D[v][j]| <= sqrt(8) < 2.83; the quadrant
//     packing's 16-slot chains add exact zeros for the other blocks): stage
//     1, magnitude sum <= 721.3: 16 u 721.3 = 6.9e-4 plus D's rounding (8 *
//     255 * 0.5 * 2^-24 = 6.1e-5), so |T| <= 722; stage 2, magnitude sum <=
//     2043: 16 u 2043 = 1.95e-3, the stage-1 error times 2.83 (2.1e-3) and
//     D's rounding on T (8 * 0.5 * 2^-24 * 722 = 1.7e-4): <= 4.3e-3.  Guard
//     0.02.
// ---------------------------------------------------------------------------
constexpr float kDDGuard32 = 0.1f, kDDGuard8 = 0.02f;

// Four wavefronts per tile (a quarter of its blocks each: few, long tiles
// would leave most SIMDs idle), one block at a time (the truncated
// transform computes only the output tiles that hold a rank below m1).
constexpr int kDD32Split = 2;

template <int XF>
__global__ __launch_bounds__(kGroupThreads) void k_dd_stats32(const ImgDev* __restrict__ imgs,
                                                             const Tile* __restrict__ tiles, int ntiles,
                                                             const uint8_t* __restrict__ px,
                                                             int32_t* __restrict__ stat) {
#pragma clang fp contract(off)
  const int wave = blockIdx.x * kWavesPerGroup + wave_in_group();
  if (wave >= (ntiles << kDD32Split)) return;
  const Tile tl = split_tile(tiles, wave, kDD32Split, 32);
  if (tl.count == 0) return;
  const ImgDev im = imgs[tl.img];
  Lane32T LT;
  lane32t_init<XF>(LT);
  const double* Dd = GenTables<32, XF>::Dd();
  const int lane = threadIdx.x & 63, lg = lane >> 4, ln = lane & 15;
  int zr[2][2][4];
  zz32_ranks<true>(zr);
  const int m1 = im.m1 < 1024 ? im.m1 : 1024;
  const float t_hi = (float)im.T + kDDGuard32, t_lo = (float)im.T - kDDGuard32;
  uint64_t inm[2][2][4];  // lanes whose coefficient in register [i][j][r] has rank below m1
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) inm[i][j][r] = __ballot(zr[i][j][r] < m1);
  const __amdgpu_buffer_rsrc_t rp = make_rsrc(px + tl.px_base, 31 * im.pitch + 32 * tl.count);
  int32_t my_stat = 0;  // lane b keeps block b's count
  for (int b = 0; b < tl.count; ++b) {
    float x[2][2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const uint32_t w =
            __builtin_amdgcn_raw_buffer_load_b32(rp, (16 * i + ln) * im.pitch + 32 * b + 16 * k + 4 * lg, 0, 0);
#pragma unroll
        for (int c = 0; c < 4; ++c) x[i][k][c] = (float)((w >> (8 * c)) & 0xffu);
      }
    f32x4 C[2][2];
    dct32_fwd_t(x, LT, m1, C);
    int cnt = 0;
    uint64_t und[2][2][4];
    uint64_t any = 0;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float av = fabsf(C[i][j][r]);
          const uint64_t gt = __ballot(av > t_hi);
          const uint64_t ge = __ballot(av >= t_lo);
          cnt += __popcll(gt & inm[i][j][r]);
          und[i][j][r] = ge & ~gt & inm[i][j][r];
          any |= und[i][j][r];
        }
    if (any != 0) {
      // float64 recheck, two coefficients per pass (lanes 32 e .. 32 e + 31)
      const int e = lane >> 5, rr = lane & 31;
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            uint64_t um = und[i][j][r];
            while (um != 0) {
              const int l0 = __builtin_ctzll(um);
              um &= um - 1;
              int l1 = -1;
              if (um != 0) {
                l1 = __builtin_ctzll(um);
                um &= um - 1;
              }
              const int le = e == 0 ? l0 : l1;
              const bool act = le >= 0;
              const int ls = act ? le : 0;
              // register [i][j][r] of lane ls holds C(16i + 4r + g, 16j + s(n))
              const int u = 16 * i + 4 * r + (ls >> 4);
              const int v = 16 * j + 4 * ((ls & 15) & 3) + ((ls & 15) >> 2);
              double t = 0.0;
              if (act) {
#pragma unroll 1
                for (int q = 0; q < 8; ++q) {
                  const uint32_t w = __builtin_amdgcn_raw_buffer_load_b32(rp, rr * im.pitch + 32 * b + 4 * q, 0, 0);
#pragma unroll
                  for (int c = 0; c < 4; ++c) {
                    const double p = (double)((w >> (8 * c)) & 0xffu) * Dd[v * 32 + 4 * q + c];
                    t = t + p;
                  }
                }
              }
              const double pr = Dd[u * 32 + rr] * t;
              double acc = 0.0;
#pragma unroll 1
              for (int k = 0; k < 32; ++k) acc = acc + __shfl(pr, (lane & 32) + k, 64);
              cnt += __popcll(__ballot(act && rr == 0 && fabs(acc) > (double)im.T));
            }
          }
    }
    if (lane == b) my_stat = cnt;
  }
  if (lane < tl.count) stat[im.blk_off + tl.first + lane] = my_stat;
}

// One wavefront per tile, four blocks per transform in the quadrant packing
// of k_sense8.
template <int XF>
__global__ __launch_bounds__(kGroupThreads) void k_dd_stats8(const ImgDev* __restrict__ imgs,
                                                            const Tile* __restrict__ tiles, int ntiles,
                                                            const uint8_t* __restrict__ px,
                                                            int32_t* __restrict__ stat) {
#pragma clang fp contract(off)
  const int wave = blockIdx.x * kWavesPerGroup + wave_in_group();
  if (wave >= ntiles) return;
  const Tile tl = tiles[wave];
  const ImgDev im = imgs[tl.img];
  Lane16 L;
  lane8x4_init<XF>(L);
  const double* Dd = GenTables<8, XF>::Dd();
  const int lane = threadIdx.x & 63;
  // operand side: block quadrant and pixel row / column of this lane
  const int xq = 2 * (L.n >> 3) + (L.g >> 1), xrow = L.n & 7, xcol = 4 * (L.g & 1);
  // output side: block quadrant; register r holds coefficient (4 (g % 2) + r, n % 8)
  const int oq = 2 * (L.g >> 1) + (L.n >> 3);
  const int m1 = im.m1 < 64 ? im.m1 : 64;
  const float t_hi = (float)im.T + kDDGuard8, t_lo = (float)im.T - kDDGuard8;
  uint64_t inm[4], bq[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) inm[r] = __ballot(c_zzrank8[(4 * (L.g & 1) + r) * 8 + (L.n & 7)] < m1);
#pragma unroll
  for (int q = 0; q < 4; ++q) bq[q] = __ballot(oq == q);
  const __amdgpu_buffer_rsrc_t rp = make_rsrc(px + tl.px_base, 7 * im.pitch + 8 * tl.count);
  int32_t my_stat = 0;  // lane b keeps block b's count
  for (int b0 = 0; b0 < tl.count; b0 += 4) {
    const int bx = b0 + xq;
    const uint32_t w = __builtin_amdgcn_raw_buffer_load_b32(
        rp, bx < tl.count ? (uint32_t)(xrow * im.pitch + 8 * bx + xcol) : 0xffffffffu, 0, 0);
    float a[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) a[c] = (float)((w >> (8 * c)) & 0xffu);
    const f32x4 C = dct16_fwd(a, L);
    int cnt[4] = {0, 0, 0, 0};
    uint64_t und[4], any = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float av = fabsf(C[r]);
      const uint64_t gt = __ballot(av > t_hi) & inm[r];
      const uint64_t ge = __ballot(av >= t_lo);
#pragma unroll
      for (int q = 0; q < 4; ++q) cnt[q] += __popcll(gt & bq[q]);
      und[r] = ge & ~gt & inm[r];
      any |= und[r];
    }
    if (any != 0) {
      // float64 recheck, eight coefficients per pass (lanes 8 e .. 8 e + 7)
      const int e = lane >> 3, rr = lane & 7;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        uint64_t um = und[r];
        while (um != 0) {
          int le = -1;  // this lane group's coefficient: the e-th set lane of um
          uint64_t mm = um;
          for (int k = 0; k < 8 && mm != 0; ++k) {
            const int l = __builtin_ctzll(mm);
            mm &= mm - 1;
            if (k == e) le = l;
          }
          um = mm;
          const bool act = le >= 0;
          const int ls = act ? le : 0;
          const int lgs = ls >> 4, lns = ls & 15;
          const int q = 2 * (lgs >> 1) + (lns >> 3);  // block b0 + q
          const int u = 4 * (lgs & 1) + r, v = lns & 7;
          double t = 0.0;
          if (act) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const uint32_t pw = __builtin_amdgcn_raw_buffer_load_b32(rp, rr * im.pitch + 8 * (b0 + q) + 4 * h, 0, 0);
#pragma unroll
              for (int c = 0; c < 4; ++c) {
                const double p = (double)((pw >> (8 * c)) & 0xffu) * Dd[v * 8 + 4 * h + c];
                t = t + p;
              }
            }
          }
          const double pr = Dd[u * 8 + rr] * t;
          double acc = 0.0;
#pragma unroll
          for (int k = 0; k < 8; ++k) acc = acc + __shfl(pr, (lane & 56) + k, 64);
          const bool hit = act && rr == 0 && fabs(acc) > (double)im.T;
#pragma unroll
          for (int qq = 0; qq < 4; ++qq) cnt[qq] += __popcll(__ballot(hit && q == qq));
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (lane == b0 + q) my_stat = cnt[q];
  }
  if (lane < tl.count) stat[im.blk_off + tl.first + lane] = my_stat;
}

}  // namespace abcs
