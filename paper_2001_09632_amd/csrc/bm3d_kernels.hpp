// Plain BM3D denoiser (Dabov et al., ref [22] of the paper) for IDA, gfx950.
//
// Profile (the paper fixes none of it): 8x8 patches, references every 3
// pixels plus the last position of each axis, 39x39 search window clipped to
// the image, patch distance ||P - Q||^2 / 64, grouping threshold 2500 / 400
// and at most 16 / 32 members (cut to a power of two; reference first, then
// increasing distance, ties to the lower raster index), 3D transform = 8x8
// DCT-II of each patch then the Haar transform along the group; stage 1 hard
// thresholding at 2.7 sigma with weight 1 / (sigma^2 max(N_har, 1)), stage 2
// Wiener shrinkage B^2 / (B^2 + sigma^2) with weight
// 1 / (sigma^2 max(||W||^2, 2^-16)); aggregation with an 8x8 Kaiser window
// (beta = 2).  sigma <= 0 returns the input.
//
// Gating (the learned denoisers' fallback): every kernel takes `gate`, null or
// int32[1 + n_imgs] with gate[0] != 0 when any image is to be denoised and
// gate[1 + i] != 0 for each such image; a non-null gate makes the kernels skip
// every other image (its output is left alone) and return at once when
// gate[0] is 0, so an unused fallback costs only the launches.
//
// Aggregation is exact and order-independent: weights are scaled by sigma^2
// (which cancels in num / den) and every contribution is rounded to a 64-bit
// fixed-point integer (2^-24 units) before an integer atomic add, so results
// are bit-identical from run to run.
#pragma once

#include "common.hpp"

namespace abcs {

namespace bm3d {
constexpr int kN1 = 8;
constexpr int kStep = 3;
constexpr int kHalfWin = 19;
constexpr int kN2Ht = 16;
constexpr int kN2Wie = 32;
constexpr float kTauHt = 2500.f;
constexpr float kTauWie = 400.f;
constexpr float kLambda = 2.7f;
constexpr float kWFloor = 1.0f / 65536.f;
constexpr double kFix = 16777216.0;  // 2^24
constexpr int kRefTile = 16;          // references per tile side
// LDS window of a 16x16 reference tile: 15 * 3 + 2 * 19 + 8 = 91 rows/cols.
constexpr int kWin = (kRefTile - 1) * kStep + 2 * kHalfWin + kN1;
}  // namespace bm3d

// Per-image reference grid and buffers.
struct RefTile {
  int32_t img;
  int32_t i0, j0;     // first reference row / column index of the tile
  int32_t ni, nj;     // references in the tile (<= 16 each)
  int32_t pad_;
  int64_t ref_base;   // global index of reference (i0, j0): refs are numbered
                      // per image in raster order of (i, j)
};

__constant__ float c_D8[64];      // orthonormal 8x8 DCT-II, D[u*8 + j]
__constant__ float c_kaiser8[64]; // 2D Kaiser window, K[r*8 + c]

__device__ __forceinline__ int bm3d_ref_pos(int i, int len) {
  const int p = i * bm3d::kStep;
  return p < len - bm3d::kN1 ? p : len - bm3d::kN1;
}

__device__ __forceinline__ int bm3d_nref(int len) {
  const int span = len - bm3d::kN1;
  return span / bm3d::kStep + 1 + (span % bm3d::kStep != 0 ? 1 : 0);
}

// ---------------------------------------------------------------------------
// Block matching.  One thread per reference; the tile's search area is staged
// in LDS (zero outside the image).  For each candidate row offset the thread
// streams each of the 8 patch rows' 46-pixel search segment once and adds its
// squared differences to the 39 candidate columns' sums, so every LDS value
// serves up to 8 candidates.  Candidates are then offered in raster order of
// their position and enter the sorted list only if strictly closer than the
// current last entry, so equal distances keep the lower raster index first.
// groups[ref * (N2 + 1)] = member count (power of two), then member positions
// (row * W' + col) in group order.
// ---------------------------------------------------------------------------
template <int N2>
__device__ __forceinline__ void bm3d_match_tile(int tix, const ImgDev* __restrict__ imgs,
                                                const RefTile* __restrict__ tiles, const float* __restrict__ src,
                                                const float* __restrict__ sigma, float tau,
                                                const int32_t* __restrict__ gate, int32_t* __restrict__ groups) {
  using namespace bm3d;
  constexpr int kSpan = 2 * kHalfWin + 1;    // 39 candidate offsets per axis
  constexpr int kSeg = kSpan + kN1 - 1;      // 46 pixels per search row
  __shared__ float win[kWin * kWin];
  const RefTile tl = tiles[tix];
  if (gate && gate[1 + tl.img] == 0) return;
  const ImgDev im = imgs[tl.img];
  if (!(sigma[tl.img] > 0.f)) return;
  const int H = im.Hc, W = im.Wc;
  const float* img = src + im.out_off;
  // Unclipped window of the tile: row/col wy0 + r of LDS is image row
  // wy0 + r (zero when outside the image).
  const int wy0 = bm3d_ref_pos(tl.i0, H) - kHalfWin;
  const int wx0 = bm3d_ref_pos(tl.j0, W) - kHalfWin;
  for (int t = threadIdx.x; t < kWin * kWin; t += 256) {
    const int r = t / kWin, c = t - r * kWin;
    const int y = wy0 + r, x = wx0 + c;
    win[t] = (y >= 0 && y < H && x >= 0 && x < W) ? img[(int64_t)y * W + x] : 0.f;
  }
  __syncthreads();
  const int ti = threadIdx.x / kRefTile, tj = threadIdx.x % kRefTile;
  if (ti >= tl.ni || tj >= tl.nj) return;
  const int ry = bm3d_ref_pos(tl.i0 + ti, H), rx = bm3d_ref_pos(tl.j0 + tj, W);
  const float* refp = win + (ry - wy0) * kWin + (rx - wx0);  // reference patch, read row by row
  float bd[N2];
  int bi[N2];
  bd[0] = -1.f;  // the reference itself leads the group
  bi[0] = ry * W + rx;
#pragma unroll
  for (int s = 1; s < N2; ++s) {
    bd[s] = 3.0e38f;
    bi[s] = -1;
  }
  const int qy0 = max(0, ry - kHalfWin), qy1 = min(H - kN1, ry + kHalfWin);
  const int qx0 = max(0, rx - kHalfWin), qx1 = min(W - kN1, rx + kHalfWin);
  for (int qy = qy0; qy <= qy1; ++qy) {
    float acc[kSpan];
#pragma unroll
    for (int q = 0; q < kSpan; ++q) acc[q] = 0.f;
    const float* rowp = win + (qy - wy0) * kWin + (rx - kHalfWin - wx0);
#pragma unroll 1
    for (int r = 0; r < kN1; ++r) {
      const float* seg = rowp + r * kWin;
      float rr[kN1];
#pragma unroll
      for (int c = 0; c < kN1; ++c) rr[c] = refp[r * kWin + c];
#pragma unroll
      for (int j = 0; j < kSeg; ++j) {
        const float pj = seg[j];
#pragma unroll
        for (int c = 0; c < kN1; ++c) {
          const int q = j - c;  // candidate column offset using pixel j at patch column c
          if (q >= 0 && q < kSpan) {
            const float dlt = rr[c] - pj;
            acc[q] = fmaf(dlt, dlt, acc[q]);
          }
        }
      }
    }
#pragma unroll
    for (int q = 0; q < kSpan; ++q) {
      const int qx = rx - kHalfWin + q;
      const float d = acc[q] * (1.0f / 64.f);
      if (qx >= qx0 && qx <= qx1 && d <= tau && d < bd[N2 - 1] && !(qy == ry && qx == rx)) {
        const int idx = qy * W + qx;
        // insert keeping (d, raster index) order; earlier equal d stay first
#pragma unroll
        for (int s = N2 - 1; s >= 1; --s) {
          const bool shift = d < bd[s - 1];
          const bool here = !shift && d < bd[s];
          bd[s] = shift ? bd[s - 1] : (here ? d : bd[s]);
          bi[s] = shift ? bi[s - 1] : (here ? idx : bi[s]);
        }
      }
    }
  }
  int cnt = 0;
#pragma unroll
  for (int s = 0; s < N2; ++s) cnt += bi[s] >= 0 ? 1 : 0;
  int n = 1;
  while (n * 2 <= cnt) n *= 2;
  int32_t* g = groups + (tl.ref_base + (int64_t)ti * bm3d_nref(W) + tj) * (N2 + 1);
  g[0] = n;
#pragma unroll
  for (int s = 0; s < N2; ++s)
    if (s < n) g[1 + s] = bi[s];
}

// Workgroups loop over the tiles (a gated launch uses a capped grid, so that
// an unused fallback costs little more than the launch).
template <int N2>
__global__ __launch_bounds__(256) void k_bm3d_match(const ImgDev* __restrict__ imgs, const RefTile* __restrict__ tiles,
                                                   int ntiles, const float* __restrict__ src,
                                                   const float* __restrict__ sigma, float tau,
                                                   const int32_t* __restrict__ gate, int32_t* __restrict__ groups) {
  if (gate && gate[0] == 0) return;
  for (int tix = blockIdx.x; tix < ntiles; tix += gridDim.x) {
    if (tix != (int)blockIdx.x) __syncthreads();  // the previous tile's LDS reads are done
    bm3d_match_tile<N2>(tix, imgs, tiles, src, sigma, tau, gate, groups);
  }
}

// ---------------------------------------------------------------------------
// Collaborative filtering of the groups of an 8x8-reference tile, one
// wavefront per reference at a time; lane (r, c) = (lane / 8, lane % 8) owns
// pixel (r, c) of every member patch and, in the spectrum, coefficient
// (u, v) = (r, c) of every member.  Contributions are summed in LDS over the
// tile's window (every member lies within 19 pixels of its reference) and the
// window is added to the image's accumulators once.
// ---------------------------------------------------------------------------
constexpr int kFiltTile = 8;
constexpr int kFiltWin = (kFiltTile - 1) * bm3d::kStep + 2 * bm3d::kHalfWin + bm3d::kN1;  // 67

struct Dct8Lane {
  float f1[8], f2[8], i1[8], i2[8];
};

__device__ __forceinline__ void dct8_lane_init(Dct8Lane& d, int r, int c) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    d.f1[j] = c_D8[c * 8 + j];   // D[v = c][j]
    d.f2[j] = c_D8[r * 8 + j];   // D[u = r][i]
    d.i1[j] = c_D8[j * 8 + c];   // D[v][j = c]
    d.i2[j] = c_D8[j * 8 + r];   // D[u][i = r]
  }
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 8x8 DCT (or its inverse) of one patch held one value per lane, through LDS.
//  forward: T[r][v] = sum_j X[r][j] D[v][j];  C[u][v] = sum_i D[u][i] T[i][v]
//  inverse: T[u][j] = sum_v C[u][v] D[v][j];  X[i][j] = sum_u D[u][i] T[u][j]
__device__ __forceinline__ float dct8_lane(float x, float* sh, int r, int c, const Dct8Lane& d, bool inverse) {
  const int lane = threadIdx.x & 63;
  sh[lane] = x;
  wave_sync_lds();
  float t = 0.f;
#pragma unroll
  for (int j = 0; j < 8; ++j) t = fmaf(sh[r * 8 + j], inverse ? d.i1[j] : d.f1[j], t);
  wave_sync_lds();
  sh[lane] = t;
  wave_sync_lds();
  float o = 0.f;
#pragma unroll
  for (int i = 0; i < 8; ++i) o = fmaf(inverse ? d.i2[i] : d.f2[i], sh[i * 8 + c], o);
  wave_sync_lds();
  return o;
}

// Orthonormal Haar transform of s[0..n) (n a power of two <= NMAX), in place.
template <int NMAX>
__device__ __forceinline__ void haar_fwd(float* s, int n) {
  const float h = 0.70710678118654752f;
#pragma unroll
  for (int m = NMAX; m >= 2; m >>= 1) {
    if (m <= n) {
      float a[NMAX / 2], d[NMAX / 2];
#pragma unroll
      for (int i = 0; i < m / 2; ++i) {
        a[i] = (s[2 * i] + s[2 * i + 1]) * h;
        d[i] = (s[2 * i] - s[2 * i + 1]) * h;
      }
#pragma unroll
      for (int i = 0; i < m / 2; ++i) {
        s[i] = a[i];
        s[m / 2 + i] = d[i];
      }
    }
  }
}

template <int NMAX>
__device__ __forceinline__ void haar_inv(float* s, int n) {
  const float h = 0.70710678118654752f;
#pragma unroll
  for (int m = 2; m <= NMAX; m <<= 1) {
    if (m <= n) {
      float e[NMAX];
#pragma unroll
      for (int i = 0; i < m / 2; ++i) {
        e[2 * i] = (s[i] + s[m / 2 + i]) * h;
        e[2 * i + 1] = (s[i] - s[m / 2 + i]) * h;
      }
#pragma unroll
      for (int i = 0; i < m; ++i) s[i] = e[i];
    }
  }
}

__device__ __forceinline__ long long to_fix(double v) { return (long long)llrint(v * bm3d::kFix); }

// STAGE 1: hard thresholding of groups cut from `noisy`.
// STAGE 2: Wiener shrinkage of groups cut from `noisy` with the spectrum of
//          the same groups cut from `basic`.
template <int STAGE>
__device__ __forceinline__ void bm3d_filter_tile(int tix, const ImgDev* __restrict__ imgs,
                                                 const RefTile* __restrict__ tiles, const float* __restrict__ noisy,
                                                 const float* __restrict__ basic, const float* __restrict__ sigma,
                                                 const int32_t* __restrict__ groups,
                                                 const int32_t* __restrict__ gate,
                                                 unsigned long long* __restrict__ num,
                                                 unsigned long long* __restrict__ den) {
  using namespace bm3d;
  constexpr int N2 = STAGE == 1 ? kN2Ht : kN2Wie;
  __shared__ unsigned long long acc_num[kFiltWin * kFiltWin];
  __shared__ unsigned long long acc_den[kFiltWin * kFiltWin];
  __shared__ float sh[4][64];
  const RefTile tl = tiles[tix];
  if (gate && gate[1 + tl.img] == 0) return;
  const ImgDev im = imgs[tl.img];
  const float sg = sigma[tl.img];
  if (!(sg > 0.f)) return;
  const int H = im.Hc, W = im.Wc;
  // window of the tile: all member patches of its groups lie inside
  const int wy0 = max(0, bm3d_ref_pos(tl.i0, H) - kHalfWin);
  const int wx0 = max(0, bm3d_ref_pos(tl.j0, W) - kHalfWin);
  const int wy1 = min(H - kN1, bm3d_ref_pos(tl.i0 + tl.ni - 1, H) + kHalfWin) + kN1;
  const int wx1 = min(W - kN1, bm3d_ref_pos(tl.j0 + tl.nj - 1, W) + kHalfWin) + kN1;
  const int wh = wy1 - wy0, ww = wx1 - wx0;
  for (int t = threadIdx.x; t < kFiltWin * kFiltWin; t += 256) {
    acc_num[t] = 0ull;
    acc_den[t] = 0ull;
  }
  __syncthreads();
  const int wave = wave_in_group();
  float* shw = sh[wave];
  const int lane = threadIdx.x & 63, r = lane >> 3, c = lane & 7;
  Dct8Lane dl;
  dct8_lane_init(dl, r, c);
  const float K = c_kaiser8[lane];
  const int nrw = bm3d_nref(W);
  for (int q = wave; q < tl.ni * tl.nj; q += 4) {
    const int ti = q / tl.nj, tj = q - ti * tl.nj;
    const int32_t* g = groups + (tl.ref_base + (int64_t)ti * nrw + tj) * (N2 + 1);
    const int n = g[0];
    int loc[N2];
    float s[N2], b[N2];
#pragma unroll
    for (int j = 0; j < N2; ++j) {
      const int pos = j < n ? g[1 + j] : 0;
      const int py = pos / W, px = pos - py * W;
      loc[j] = (py - wy0 + r) * kFiltWin + (px - wx0 + c);
      const int64_t a = im.out_off + pos + r * W + c;
      s[j] = j < n ? noisy[a] : 0.f;
      if (STAGE == 2) b[j] = j < n ? basic[a] : 0.f;
    }
#pragma unroll
    for (int j = 0; j < N2; ++j) {
      if (j < n) {
        s[j] = dct8_lane(s[j], shw, r, c, dl, false);
        if (STAGE == 2) b[j] = dct8_lane(b[j], shw, r, c, dl, false);
      }
    }
    haar_fwd<N2>(s, n);
    if (STAGE == 2) haar_fwd<N2>(b, n);
    double wgt;
    if (STAGE == 1) {
      const float thr = kLambda * sg;
      int nz = 0;
#pragma unroll
      for (int j = 0; j < N2; ++j) {
        if (j < n) {
          const bool keep = fabsf(s[j]) > thr;
          s[j] = keep ? s[j] : 0.f;
          nz += keep ? 1 : 0;
        }
      }
      for (int o = 32; o > 0; o >>= 1) nz += __shfl_xor(nz, o, 64);
      wgt = 1.0 / (double)(nz > 0 ? nz : 1);
    } else {
      const float s2 = sg * sg;
      float w2 = 0.f;
#pragma unroll
      for (int j = 0; j < N2; ++j) {
        if (j < n) {
          const float bb = b[j] * b[j];
          const float w = bb / (bb + s2);
          s[j] *= w;
          w2 = fmaf(w, w, w2);
        }
      }
      for (int o = 32; o > 0; o >>= 1) w2 += __shfl_xor(w2, o, 64);
      wgt = 1.0 / (double)(w2 > kWFloor ? w2 : kWFloor);
    }
    haar_inv<N2>(s, n);
    const unsigned long long dk = (unsigned long long)to_fix(wgt * (double)K);
#pragma unroll
    for (int j = 0; j < N2; ++j) {
      if (j < n) {
        const float e = dct8_lane(s[j], shw, r, c, dl, true);
        atomicAdd(&acc_num[loc[j]], (unsigned long long)to_fix(wgt * (double)K * (double)e));
        atomicAdd(&acc_den[loc[j]], dk);
      }
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < wh * ww; t += 256) {
    const int rr = t / ww, cc = t - rr * ww;
    const unsigned long long dv = acc_den[rr * kFiltWin + cc];
    if (dv != 0ull) {
      const int64_t a = im.out_off + (int64_t)(wy0 + rr) * W + wx0 + cc;
      atomicAdd(num + a, acc_num[rr * kFiltWin + cc]);
      atomicAdd(den + a, dv);
    }
  }
}

template <int STAGE>
__global__ __launch_bounds__(256) void k_bm3d_filter(const ImgDev* __restrict__ imgs, const RefTile* __restrict__ tiles,
                                                    int ntiles, const float* __restrict__ noisy,
                                                    const float* __restrict__ basic, const float* __restrict__ sigma,
                                                    const int32_t* __restrict__ groups,
                                                    const int32_t* __restrict__ gate,
                                                    unsigned long long* __restrict__ num,
                                                    unsigned long long* __restrict__ den) {
  if (gate && gate[0] == 0) return;
  for (int tix = blockIdx.x; tix < ntiles; tix += gridDim.x) {
    if (tix != (int)blockIdx.x) __syncthreads();  // the previous tile's LDS reads are done
    bm3d_filter_tile<STAGE>(tix, imgs, tiles, noisy, basic, sigma, groups, gate, num, den);
  }
}

// out = num / den for images with sigma > 0, out = in for sigma <= 0, NaN
// for a NaN sigma (no estimate: the matching and filtering kernels skip such
// an image).
__global__ __launch_bounds__(256) void k_bm3d_finish(const ImgDev* __restrict__ imgs, int n_imgs,
                                                    const float* __restrict__ sigma,
                                                    const unsigned long long* __restrict__ num,
                                                    const unsigned long long* __restrict__ den,
                                                    const float* __restrict__ in, float* __restrict__ out,
                                                    int64_t pixels, const int32_t* __restrict__ pix_img,
                                                    const int32_t* __restrict__ gate) {
  if (gate && gate[0] == 0) return;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < pixels; i += (int64_t)gridDim.x * 256) {
    const int im = pix_img[i >> kPixChunkShift];
    if (gate && gate[1 + im] == 0) continue;
    const float sg = sigma[im];
    if (sg > 0.f) {
      out[i] = (float)((double)(long long)num[i] / (double)(long long)den[i]);
    } else if (sg <= 0.f) {
      out[i] = in[i];
    } else {
      out[i] = sg;
    }
  }
}

__global__ __launch_bounds__(256) void k_zero_u64(unsigned long long* __restrict__ p, int64_t n,
                                                 const int32_t* __restrict__ gate) {
  if (gate && gate[0] == 0) return;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = 0ull;
}

}  // namespace abcs
