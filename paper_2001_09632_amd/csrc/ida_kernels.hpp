// IDA post-processing (Section VI): the transform half of one iteration and
// the per-image noise-level estimate.
//
// With A the block-diagonal zigzag-DCT operator (eq 26), alpha = 1/D_F (eq 28)
// and x^0 = 0, z^{-1} = 0, iteration t computes
//   z^t     = y - A x^t + alpha z^{t-1}          (eqs 25, 28)
//   sigma^t = ||z^t||_2 / sqrt(m)                 (eq 15)
//   v^t     = x^t + A* z^t                        (eq 13, before the denoiser)
// and the denoiser then maps v^t to x^{t+1}.  In the DCT domain of a block,
// with C = D x D^T, the measured coefficients become C + z and the others
// stay C, so v = D^T (C + scatter(z)) D: one forward and one inverse
// transform per block.
#pragma once

#include "common.hpp"
#include "transform16.hpp"

namespace abcs {

// One wavefront per tile.  x and v are H' x W' float32 images (row pitch W');
// z (in: z^{t-1}, out: z^t) is laid out like y; part[blk] receives the block's
// sum of (z^t)^2 in float64, summed in a fixed order.  When `first` is set,
// x^0 = 0 and z^{-1} = 0 are used without reading x or z.  v may alias x.
// The weight of z^{t-1} is alpha_img[image] when alpha_img is not null
// (D-AMP's per-image Onsager coefficient), else alpha.
template <int XF = kXfDCT>
__global__ __launch_bounds__(kGroupThreads) void k_ida_step16(const ImgDev* __restrict__ imgs,
                                                             const Tile* __restrict__ tiles, int ntiles,
                                                             const float* __restrict__ y,
                                                             const int32_t* __restrict__ k_all,
                                                             const int64_t* __restrict__ off_all,
                                                             const float* x, float* __restrict__ z,
                                                             float* v, double* __restrict__ part,
                                                             float alpha, const float* __restrict__ alpha_img,
                                                             int first) {
  const int wave = blockIdx.x * kWavesPerGroup + wave_in_group();
  if (wave >= ntiles) return;
  const Tile tl = tiles[wave];
  const ImgDev im = imgs[tl.img];
  if (alpha_img) alpha = alpha_img[tl.img];
  Lane16 L;
  lane16_init<XF>(L);
  TileIO io;
  tile_io_init(io, im, tl, nullptr, y, k_all, off_all, L);
  const __amdgpu_buffer_rsrc_t rz = make_rsrc(z + im.meas_off, (int)(4 * im.n_meas));
  const int lane = threadIdx.x & 63;
  // x and v: the lane's 4 pixels of row n of block b sit at float offset
  // out_base + n W' + 16 b + 4g.
  const int ext = 4 * (15 * im.Wc + 16 * tl.count);
  const __amdgpu_buffer_rsrc_t rx = make_rsrc(x + tl.out_base, first ? 0 : ext);
  const __amdgpu_buffer_rsrc_t rv = make_rsrc(v + tl.out_base, ext);
  const uint32_t px_off = 4u * (uint32_t)(L.n * im.Wc + 4 * L.g);
  typedef __attribute__((ext_vector_type(4))) unsigned int u32x4;
  double my_part = 0.0;  // lane b keeps block b's sum
#pragma unroll 2
  for (int b = 0; b < kTileBlocks; ++b) {
    const bool valid = b < tl.count;
    // Forward transform of x^t (0 on the first iteration: empty resource).
    const u32x4 xw = __builtin_amdgcn_raw_buffer_load_b128(rx, valid ? px_off + 64u * b : 0xffffffffu, 0, 0);
    float a[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) a[c] = __uint_as_float(xw[c]);
    f32x4 C = dct16_fwd(a, L);
    uint32_t voff[4];
    tile_y_offsets(io, b, L, voff);
    float zz = 0.f;
    double acc = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float yv = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(io.y, voff[r], 0, 0));
      const float zo = first ? 0.f : __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rz, voff[r], 0, 0));
      // residual r = y - (A x) plus the damped previous residual
      const float zn = (yv - C[r]) + alpha * zo;
      // out-of-budget ranks have offset ~0 and y = z = 0 there; keep them out
      const bool meas = voff[r] != 0xffffffffu;
      zz = meas ? zn : 0.f;
      __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(zz), rz, voff[r], 0, 0);
      C[r] = C[r] + zz;
      acc += (double)zz * (double)zz;
    }
    // Fixed-order butterfly sum over the wave.
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == b) my_part = acc;
    float e[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) e[c] = C[c];
    const f32x4 X = idct16_inv(e, L);
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, X), rv, valid ? px_off + 64u * b : 0xffffffffu,
                                           0, 0);
  }
  if (lane < tl.count) part[im.blk_off + tl.first + lane] = my_part;
}

// sigma_i = sqrt(sum of the image's block partials / m_i), one workgroup per
// image; partials are added in block order by a fixed tree.  Also appends
// sigma to trace[t * n + i] when trace is not null.  With part_bbv, the BBV
// images' sample residuals (per-block partials) and sample count join the sum
// and m.
__global__ __launch_bounds__(kGroupThreads) void k_ida_sigma(const ImgDev* __restrict__ imgs,
                                                            const double* __restrict__ part,
                                                            float* __restrict__ sigma, float* __restrict__ trace,
                                                            int n_imgs, int t,
                                                            const double* __restrict__ part_bbv) {
  __shared__ double sh[kGroupThreads];
  const ImgDev im = imgs[blockIdx.x];
  const int tid = threadIdx.x;
  const int per = (im.nB + kGroupThreads - 1) / kGroupThreads;
  const int i0 = min(im.nB, tid * per), i1 = min(im.nB, i0 + per);
  // BBV images with sample rows: their residuals and their count join m
  const bool rows = part_bbv != nullptr && im.mode == kModeBBV;
  const int64_t m = im.n_meas + (rows ? 2LL * im.nS * im.nB + (int64_t)im.nS * (im.nbx + im.nby) : 0);
  double s = 0.0;
  for (int i = i0; i < i1; ++i) s += part[im.blk_off + i] + (rows ? part_bbv[im.blk_off + i] : 0.0);
  sh[tid] = s;
  __syncthreads();
  for (int w = kGroupThreads / 2; w > 0; w >>= 1) {
    if (tid < w) sh[tid] += sh[tid + w];
    __syncthreads();
  }
  if (tid == 0) {
    const float sg = m > 0 ? (float)sqrt(sh[0] / (double)m) : 0.f;
    sigma[blockIdx.x] = sg;
    if (trace) trace[(int64_t)t * n_imgs + blockIdx.x] = sg;
  }
}

// ---------------------------------------------------------------------------
// BBV samples as extra measurements (Section V-A): every sample of eq 19 is a
// signed difference d = I[a] - I[b] of two adjacent pixels.  Layout per BBV
// image (at its sample offset): for each block in raster order its n_S
// top-row then its n_S left-column samples; then the n_S bottom-row samples
// of each block of the last block row; then the n_S right-column samples of
// each block of the last block column.  In IDA they are rows (e_a - e_b)/sqrt 2
// of A with measurements d/sqrt 2; every sample's two pixels lie in its own
// block, so one thread per block owns them.
// ---------------------------------------------------------------------------

struct BbvSample {
  int r, c;      // pixel a (row, column in the cropped image)
  int dr, dc;    // b = a - (dr, dc)
  int64_t slot;  // position in the image's sample list
};

// The s-th sample (0 <= s < bbv_block_count) of block (by, bx).
__device__ __forceinline__ int bbv_block_count(const ImgDev& im, int by, int bx) {
  return 2 * im.nS + (by + 1 == im.nby ? im.nS : 0) + (bx + 1 == im.nbx ? im.nS : 0);
}

__device__ __forceinline__ BbvSample bbv_block_sample(const ImgDev& im, int by, int bx, int s) {
  const int B = im.B, nS = im.nS, r0 = by * B, c0 = bx * B;
  const int64_t nB = im.nB, blk = (int64_t)by * im.nbx + bx;
  int part = s / nS;
  const int j = s - part * nS, k = im.X0 + j * im.L;
  if (part == 2 && by + 1 != im.nby) part = 3;  // no bottom edge: the next group is the right edge
  BbvSample q;
  switch (part) {
    case 0:  // top row
      q = BbvSample{r0, c0 + k, 0, 1, blk * 2 * nS + j};
      break;
    case 1:  // left column
      q = BbvSample{r0 + k, c0, 1, 0, blk * 2 * nS + nS + j};
      break;
    case 2:  // bottom edge of the last block row
      q = BbvSample{r0 + B - 1, c0 + k, 0, 1, 2 * nS * nB + (int64_t)bx * nS + j};
      break;
    default:  // right edge of the last block column
      q = BbvSample{r0 + k, c0 + B - 1, 1, 0, 2 * nS * nB + (int64_t)nS * im.nbx + (int64_t)by * nS + j};
      break;
  }
  return q;
}

// Signed samples of every block of the BBV tiles (one thread per block).
__global__ __launch_bounds__(kGroupThreads) void k_bbv_samples(const ImgDev* __restrict__ imgs,
                                                              const Tile* __restrict__ tiles, int ntiles,
                                                              const uint8_t* __restrict__ px,
                                                              const int64_t* __restrict__ bbv_off,
                                                              float* __restrict__ out) {
  const int t = blockIdx.x * kGroupThreads + threadIdx.x;
  const int ti = t / kTileBlocks, b = t % kTileBlocks;
  if (ti >= ntiles) return;
  const Tile tl = tiles[ti];
  if (b >= tl.count) return;
  const ImgDev im = imgs[tl.img];
  const int by = tl.by, bx = tl.first - tl.by * im.nbx + b;
  const uint8_t* base = px + im.px_off;
  float* o = out + bbv_off[tl.img];
  const int n = bbv_block_count(im, by, bx);
  for (int s = 0; s < n; ++s) {
    const BbvSample q = bbv_block_sample(im, by, bx, s);
    const int a = base[(int64_t)q.r * im.pitch + q.c];
    const int bv = base[(int64_t)(q.r - q.dr) * im.pitch + (q.c - q.dc)];
    o[q.slot] = (float)(a - bv);
  }
}

// Before the transform step: zb = (d - (x_a - x_b)) / sqrt 2 + alpha zb_prev
// (x = 0 and zb_prev = 0 at t = 0); pb[blk] = sum of zb^2 in sample order.
__global__ __launch_bounds__(kGroupThreads) void k_ida_bbv_residual(const ImgDev* __restrict__ imgs,
                                                                   const Tile* __restrict__ tiles, int ntiles,
                                                                   const float* __restrict__ d,
                                                                   const int64_t* __restrict__ bbv_off,
                                                                   const float* __restrict__ x,
                                                                   float* __restrict__ zb, double* __restrict__ pb,
                                                                   float alpha, int first) {
  const int t = blockIdx.x * kGroupThreads + threadIdx.x;
  const int ti = t / kTileBlocks, b = t % kTileBlocks;
  if (ti >= ntiles) return;
  const Tile tl = tiles[ti];
  if (b >= tl.count) return;
  const ImgDev im = imgs[tl.img];
  const int by = tl.by, bx = tl.first - tl.by * im.nbx + b;
  const int64_t off = bbv_off[tl.img];
  const float* xi = x + im.out_off;
  const float r2 = 0.70710678118654752f;  // 1 / sqrt 2
  double acc = 0.0;
  const int n = bbv_block_count(im, by, bx);
  for (int s = 0; s < n; ++s) {
    const BbvSample q = bbv_block_sample(im, by, bx, s);
    float ax = 0.f;
    if (!first) ax = (xi[(int64_t)q.r * im.Wc + q.c] - xi[(int64_t)(q.r - q.dr) * im.Wc + (q.c - q.dc)]) * r2;
    const float zo = first ? 0.f : zb[off + q.slot];
    const float zn = (d[off + q.slot] * r2 - ax) + alpha * zo;
    zb[off + q.slot] = zn;
    acc += (double)zn * (double)zn;
  }
  pb[im.blk_off + tl.first + b] = acc;
}

// After the transform step: v += A_bbv* zb (each block's samples in order).
__global__ __launch_bounds__(kGroupThreads) void k_ida_bbv_scatter(const ImgDev* __restrict__ imgs,
                                                                  const Tile* __restrict__ tiles, int ntiles,
                                                                  const int64_t* __restrict__ bbv_off,
                                                                  const float* __restrict__ zb, float* v) {
  const int t = blockIdx.x * kGroupThreads + threadIdx.x;
  const int ti = t / kTileBlocks, b = t % kTileBlocks;
  if (ti >= ntiles) return;
  const Tile tl = tiles[ti];
  if (b >= tl.count) return;
  const ImgDev im = imgs[tl.img];
  const int by = tl.by, bx = tl.first - tl.by * im.nbx + b;
  const int64_t off = bbv_off[tl.img];
  float* vi = v + im.out_off;
  const float r2 = 0.70710678118654752f;
  const int n = bbv_block_count(im, by, bx);
  for (int s = 0; s < n; ++s) {
    const BbvSample q = bbv_block_sample(im, by, bx, s);
    const float h = zb[off + q.slot] * r2;
    vi[(int64_t)q.r * im.Wc + q.c] += h;
    vi[(int64_t)(q.r - q.dr) * im.Wc + (q.c - q.dc)] -= h;
  }
}

// dst[i] = src[i], i < n (a kernel, so that captured graphs hold kernel nodes only).
__global__ __launch_bounds__(256) void k_copy_f32(const float* __restrict__ src, float* __restrict__ dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// D-AMP / DAMP-D (eqs 14, 24, 27): the Onsager coefficient from a Monte-Carlo
// divergence, div D(v) ~ b . (D(v + eps b) - D(v)) / eps (ref [13]).
// ---------------------------------------------------------------------------

// Per 64-pixel chunk (every image holds whole chunks): the chunk's max |v|
// and the chunk's sum of b (xp - x) in float64, in index order.  One thread
// per chunk.
__global__ __launch_bounds__(256) void k_amp_chunks(int64_t chunks, const float* __restrict__ v,
                                                   const float* __restrict__ b, const float* __restrict__ xp,
                                                   const float* __restrict__ x, float* __restrict__ cmax,
                                                   double* __restrict__ csum) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= chunks) return;
  const int64_t p0 = c << kPixChunkShift;
  if (cmax) {
    float m = 0.f;
    for (int i = 0; i < (1 << kPixChunkShift); ++i) m = fmaxf(m, fabsf(v[p0 + i]));
    cmax[c] = m;
  } else {
    double s = 0.0;
    for (int i = 0; i < (1 << kPixChunkShift); ++i)
      s += (double)b[p0 + i] * ((double)xp[p0 + i] - (double)x[p0 + i]);
    csum[c] = s;
  }
}

// eps[i] = max |v| over image i / 1000 (1e-3 when v is 0), from the chunk
// maxima; one workgroup per image.
__global__ __launch_bounds__(kGroupThreads) void k_amp_eps(const ImgDev* __restrict__ imgs,
                                                          const float* __restrict__ cmax, float* __restrict__ eps) {
  __shared__ float sh[kGroupThreads];
  const ImgDev im = imgs[blockIdx.x];
  const int64_t c0 = im.out_off >> kPixChunkShift, nc = ((int64_t)im.Hc * im.Wc) >> kPixChunkShift;
  float m = 0.f;
  for (int64_t i = threadIdx.x; i < nc; i += kGroupThreads) m = fmaxf(m, cmax[c0 + i]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int w = kGroupThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) eps[blockIdx.x] = sh[0] > 0.f ? sh[0] / 1000.f : 1e-3f;
}

// vp = v + eps[image] b
__global__ __launch_bounds__(256) void k_amp_perturb(const int32_t* __restrict__ pix_img, int64_t pixels,
                                                    const float* __restrict__ v, const float* __restrict__ b,
                                                    const float* __restrict__ eps, float* __restrict__ vp) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= pixels) return;
  vp[p] = v[p] + eps[pix_img[p >> kPixChunkShift]] * b[p];
}

// alpha[i] = scale * (sum over image i of b (xp - x)) / (eps[i] m_i): the
// chunk sums of the image added in a fixed order (strided per thread, then a
// tree); also trace[t * n_imgs + i] when trace is not null.  One workgroup per
// image.
__global__ __launch_bounds__(kGroupThreads) void k_amp_alpha(const ImgDev* __restrict__ imgs,
                                                            const double* __restrict__ csum,
                                                            const float* __restrict__ eps, float scale,
                                                            float* __restrict__ alpha, float* __restrict__ trace,
                                                            int n_imgs, int t) {
  __shared__ double sh[kGroupThreads];
  const ImgDev im = imgs[blockIdx.x];
  const int64_t c0 = im.out_off >> kPixChunkShift, nc = ((int64_t)im.Hc * im.Wc) >> kPixChunkShift;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < nc; i += kGroupThreads) s += csum[c0 + i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = kGroupThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const float a = im.n_meas > 0 ? (float)((double)scale * (sh[0] / (double)eps[blockIdx.x]) / (double)im.n_meas) : 0.f;
    alpha[blockIdx.x] = a;
    if (trace) trace[(int64_t)t * n_imgs + blockIdx.x] = a;
  }
}

__global__ void k_fill_f32(float* __restrict__ p, int64_t n, float v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace abcs
