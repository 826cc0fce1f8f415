// Full-sensing bounds THI and THB (Section IV, Section V-C).
//
// Every DCT coefficient of every block is computed in float64, in the fixed
// order of the definition (as the DD statistic's recheck), so that the
// selections below are decided on exactly the values of that definition:
//
//   THI keeps the M = floor(C_R N) coefficients of largest magnitude over the
//       whole image; ties in magnitude go to the lower block, then the lower
//       zigzag rank.  The M-th largest magnitude T is found by an MSD radix
//       select over the 63-bit pattern of |c| (non-negative doubles order as
//       their bit patterns), 8 digit passes of a histogram kernel over
//       4096-coefficient chunks and a one-wave pick kernel per image.
//   THB keeps the floor(M / n_B) largest of each block (same tie rule), found
//       by a bit-by-bit search of the block's threshold inside one wavefront.
//
// Coefficients live in two planes (high and low 32-bit words of the float64,
// sign included), in rank order per block at the block's decoded-pixel
// offset: image base + raster block index * B^2.  The kept coefficients are
// written as float32 into a dense plane of the same layout, which the masked
// inverse DCT decodes with k_i = B^2.
#pragma once

#include "common.hpp"
#include "transform16.hpp"
#include "generic_kernels.hpp"

namespace abcs {

constexpr int kSelChunk = 4096;  // coefficients per histogram workgroup
constexpr int kSelPasses = 8;

// Digit of pass p over the 63-bit key (bits 62..32 from the high word without
// its sign, 31..0 from the low word): shift and width.
__host__ __device__ constexpr int sel_shift(int p) { return p < 3 ? 55 - 8 * p : (p == 3 ? 32 : 24 - 8 * (p - 4)); }
__host__ __device__ constexpr int sel_width(int p) { return p == 3 ? 7 : 8; }

struct SelChunk {
  int64_t start;  // first coefficient (decoded-pixel index space)
  int32_t len;    // 1 .. kSelChunk
  int32_t img;
};

struct SelState {
  uint64_t prefix;  // decided high bits of T (all 63 after the last pass)
  int64_t need;     // coefficients still to take among those matching prefix
};

template <int B>
struct ThrTables;
template <>
struct ThrTables<8> {
  __device__ static const double* Dd() { return c_D8d; }
  __device__ static int rank(int t) { return c_zzrank8[t]; }
};
template <>
struct ThrTables<16> {
  __device__ static const double* Dd() { return c_D16d; }
  __device__ static int rank(int t) { return c_zzrank16[t]; }
};
template <>
struct ThrTables<32> {
  __device__ static const double* Dd() { return c_D32d; }
  __device__ static int rank(int t) { return c_zzrank32[t]; }
};

__device__ __forceinline__ uint64_t thr_key(uint32_t hi, uint32_t lo) {
  return ((uint64_t)(hi & 0x7fffffffu) << 32) | lo;
}

// C[u][v] = sum_r D[u][r] T[r][v], T[r][v] = sum_j X[r][j] D[v][j], sums in
// ascending index order, every product and sum rounded on its own; written
// as (high, low) words at rank position of (u, v).
template <int B>
__global__ __launch_bounds__(kGroupThreads) void k_thr_coefs(const ImgDev* __restrict__ imgs,
                                                            const Tile* __restrict__ tiles, int ntiles,
                                                            const uint8_t* __restrict__ px,
                                                            uint32_t* __restrict__ khi, uint32_t* __restrict__ klo) {
#pragma clang fp contract(off)
  constexpr int P = B + 1, NN = B * B;
  __shared__ double sD[NN];      // D[u][j] at u B + j
  __shared__ double sDt[NN];     // D[v][j] at j B + v
  __shared__ uint16_t srank[NN];
  __shared__ float sX[kWavesPerGroup][B * P];   // pixels, then high words by rank
  __shared__ double sT[kWavesPerGroup][B * P];
  __shared__ uint32_t sLo[kWavesPerGroup][NN];
  if ((int)blockIdx.x >= ntiles) return;
  for (int t = threadIdx.x; t < NN; t += kGroupThreads) {
    const double d = ThrTables<B>::Dd()[t];
    sD[t] = d;
    sDt[(t % B) * B + t / B] = d;
    srank[t] = (uint16_t)ThrTables<B>::rank(t);
  }
  __syncthreads();
  const Tile tl = tiles[blockIdx.x];
  const ImgDev im = imgs[tl.img];
  const int w = wave_in_group(), lane = threadIdx.x & 63;
  const __amdgpu_buffer_rsrc_t rp = make_rsrc(px + tl.px_base, (B - 1) * im.pitch + B * tl.count);
  float* X = sX[w];
  uint32_t* H = reinterpret_cast<uint32_t*>(sX[w]);
  double* T = sT[w];
  uint32_t* Lo = sLo[w];
  for (int bb = w; bb < tl.count; bb += kWavesPerGroup) {
    gen_load_pixels<B>(rp, im.pitch, bb, X);
    wave_lds_sync();
    for (int idx = lane; idx < NN; idx += 64) {
      const int r = idx / B, v = idx - r * B;
      double s = 0.0;
      for (int j = 0; j < B; ++j) {
        const double p = (double)X[r * P + j] * sDt[j * B + v];
        s = s + p;
      }
      T[r * P + v] = s;
    }
    wave_lds_sync();
    for (int idx = lane; idx < NN; idx += 64) {
      const int u = idx / B, v = idx - u * B;
      double s = 0.0;
      for (int r = 0; r < B; ++r) {
        const double p = sD[u * B + r] * T[r * P + v];
        s = s + p;
      }
      const uint64_t bits = (uint64_t)__double_as_longlong(s);
      const int z = srank[idx];
      H[z] = (uint32_t)(bits >> 32);
      Lo[z] = (uint32_t)bits;
    }
    wave_lds_sync();
    const int64_t dst = im.out_off + (int64_t)(tl.first + bb) * NN;
    for (int z = lane; z < NN; z += 64) {
      khi[dst + z] = H[z];
      klo[dst + z] = Lo[z];
    }
    wave_lds_sync();
  }
}

// need = M of every image, prefix = 0, histograms cleared.
__global__ void k_thr_init(const int64_t* __restrict__ m_total, int n, SelState* __restrict__ st,
                           unsigned long long* __restrict__ hist) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n * 256) hist[i] = 0ull;
  if (i < n) st[i] = SelState{0ull, m_total[i]};
}

// Histogram of pass p's digit over the coefficients whose higher digits
// match the image's decided prefix.
__global__ __launch_bounds__(256) void k_thr_hist(const SelChunk* __restrict__ chunks,
                                                  const uint32_t* __restrict__ khi,
                                                  const uint32_t* __restrict__ klo,
                                                  const SelState* __restrict__ st,
                                                  unsigned long long* __restrict__ hist, int pass) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0u;
  __syncthreads();
  const SelChunk c = chunks[blockIdx.x];
  const SelState s = st[c.img];
  const int shift = sel_shift(pass), width = sel_width(pass);
  const uint64_t above = ~0ull << (shift + width);  // bits of decided digits
  const uint32_t dmask = (1u << width) - 1u;
  const uint32_t phi = (uint32_t)(s.prefix >> 32);
  const uint32_t* hp = khi + c.start;
  const uint32_t* lp = klo + c.start;
  const int lane = threadIdx.x & 63;
  for (int e0 = 0; e0 < c.len; e0 += 256) {
    const int e = e0 + (int)threadIdx.x;
    bool ok = e < c.len;
    uint32_t d = 0;
    if (ok) {
      const uint32_t hi = hp[e] & 0x7fffffffu;
      uint64_t key = (uint64_t)hi << 32;
      if (pass >= 4) {
        ok = hi == phi;
        if (ok) key |= lp[e];
      }
      ok = ok && (key & above) == (s.prefix & above);
      d = (uint32_t)(key >> shift) & dmask;
    }
    if (pass == 0) {
      // the leading digit is the exponent's top: few distinct values per
      // wave, so one LDS add per distinct value instead of one per lane
      uint64_t act = __ballot(ok);
      while (act) {
        const int leader = __ffsll((unsigned long long)act) - 1;
        const uint32_t dl = __shfl(d, leader, 64);
        const uint64_t same = __ballot(ok && d == dl);
        if (lane == leader) atomicAdd(&h[dl], (uint32_t)__popcll(same));
        act &= ~same;
      }
    } else if (ok) {
      atomicAdd(&h[d], 1u);
    }
  }
  __syncthreads();
  const uint32_t v = h[threadIdx.x];
  if (v) atomicAdd(&hist[(int64_t)c.img * 256 + threadIdx.x], (unsigned long long)v);
}

// One wave per image: the digit at which the count of larger keys first
// reaches `need` (lane l holds bins 4l .. 4l + 3); clears the histogram.
__global__ __launch_bounds__(64) void k_thr_pick(unsigned long long* __restrict__ hist, SelState* __restrict__ st,
                                                 int pass) {
  const int img = blockIdx.x, lane = threadIdx.x;
  SelState s = st[img];
  unsigned long long* hb = hist + (int64_t)img * 256 + 4 * lane;
  unsigned long long hv[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    hv[j] = hb[j];
    hb[j] = 0ull;
  }
  const unsigned long long own = hv[0] + hv[1] + hv[2] + hv[3];
  // S_l = sum over lanes >= l
  unsigned long long S = own;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned long long t = __shfl_down(S, o, 64);
    if (lane + o < 64) S += t;
  }
  const uint64_t ge = __ballot(S >= (unsigned long long)s.need);
  const int top = 63 - __clzll((long long)ge);  // ge != 0: keys matching the prefix >= need
  if (lane == top) {
    unsigned long long acc = S - own;  // keys in bins of higher lanes
    int digit = 4 * lane;
    for (int j = 3; j >= 0; --j) {
      if (acc + hv[j] >= (unsigned long long)s.need) {
        digit = 4 * lane + j;
        break;
      }
      acc += hv[j];
    }
    s.need -= (int64_t)acc;
    s.prefix |= (uint64_t)digit << sel_shift(pass);
    st[img] = s;
  }
}

// Per block: keys above T and keys equal to T (THI).
__global__ __launch_bounds__(kGroupThreads) void k_thi_count(const ImgDev* __restrict__ imgs,
                                                            const Tile* __restrict__ tiles, int ntiles,
                                                            const uint32_t* __restrict__ khi,
                                                            const uint32_t* __restrict__ klo,
                                                            const SelState* __restrict__ st,
                                                            int32_t* __restrict__ gt, int32_t* __restrict__ eq) {
  const int tile = blockIdx.x;
  if (tile >= ntiles) return;
  const Tile tl = tiles[tile];
  const ImgDev im = imgs[tl.img];
  const uint64_t T = st[tl.img].prefix;
  const int w = wave_in_group(), lane = threadIdx.x & 63;
  const int NN = im.B * im.B;
  for (int bb = w; bb < tl.count; bb += kWavesPerGroup) {
    const int64_t base = im.out_off + (int64_t)(tl.first + bb) * NN;
    int g = 0, e = 0;
    for (int z = lane; z < NN; z += 64) {
      const uint64_t key = thr_key(khi[base + z], klo[base + z]);
      g += key > T ? 1 : 0;
      e += key == T ? 1 : 0;
    }
    g = wave_sum_i32(g);
    e = wave_sum_i32(e);
    if (lane == 0) {
      gt[im.blk_off + tl.first + bb] = g;
      eq[im.blk_off + tl.first + bb] = e;
    }
  }
}

// One workgroup per image: ties at T go to the lowest blocks; m_i = gt_i +
// ties taken, and eq_i is replaced by the ties block i takes.
__global__ __launch_bounds__(256) void k_thi_ties(const ImgDev* __restrict__ imgs, const SelState* __restrict__ st,
                                                  const int32_t* __restrict__ gt, int32_t* __restrict__ eq,
                                                  int32_t* __restrict__ m) {
  __shared__ int64_t part[256];
  const ImgDev im = imgs[blockIdx.x];
  int64_t left = st[blockIdx.x].need;  // ties still to hand out
  const int tid = threadIdx.x;
  for (int64_t b0 = 0; b0 < im.nB; b0 += 256) {
    const int64_t b = b0 + tid;
    const int64_t blk = im.blk_off + b;
    const int e = b < im.nB ? eq[blk] : 0;
    part[tid] = e;
    __syncthreads();
    // inclusive Hillis-Steele scan
    for (int o = 1; o < 256; o <<= 1) {
      const int64_t t = tid >= o ? part[tid - o] : 0;
      __syncthreads();
      part[tid] += t;
      __syncthreads();
    }
    const int64_t before = part[tid] - e;
    const int64_t total = part[255];
    if (b < im.nB) {
      int64_t take = left - before;
      take = take < 0 ? 0 : (take > e ? e : take);
      eq[blk] = (int32_t)take;
      m[blk] = gt[blk] + (int32_t)take;
    }
    left -= total;
    if (left < 0) left = 0;
    __syncthreads();
  }
}

// Kept coefficients (key > T, or key == T among the block's first `take`
// ties in rank order) as float32, the rest 0.
__global__ __launch_bounds__(kGroupThreads) void k_thi_mask(const ImgDev* __restrict__ imgs,
                                                           const Tile* __restrict__ tiles, int ntiles,
                                                           const uint32_t* __restrict__ khi,
                                                           const uint32_t* __restrict__ klo,
                                                           const SelState* __restrict__ st,
                                                           const int32_t* __restrict__ take,
                                                           float* __restrict__ yfull) {
  const int tile = blockIdx.x;
  if (tile >= ntiles) return;
  const Tile tl = tiles[tile];
  const ImgDev im = imgs[tl.img];
  const uint64_t T = st[tl.img].prefix;
  const int w = wave_in_group(), lane = threadIdx.x & 63;
  const uint64_t below = (1ull << lane) - 1ull;
  const int NN = im.B * im.B;
  for (int bb = w; bb < tl.count; bb += kWavesPerGroup) {
    const int64_t blk = im.blk_off + tl.first + bb;
    const int64_t base = im.out_off + (int64_t)(tl.first + bb) * NN;
    const int tk = take[blk];
    int seen = 0;
    for (int z0 = 0; z0 < NN; z0 += 64) {
      const uint32_t hi = khi[base + z0 + lane], lo = klo[base + z0 + lane];
      const uint64_t key = thr_key(hi, lo);
      const uint64_t tie = __ballot(key == T);
      const int rank_tie = seen + __popcll(tie & below);
      const bool keep = key > T || (key == T && rank_tie < tk);
      const double c = __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
      yfull[base + z0 + lane] = keep ? (float)c : 0.f;
      seen += __popcll(tie);
    }
  }
}

// THB: k = floor(M / n_B) largest of each block; m_i = k.
template <int B>
__global__ __launch_bounds__(kGroupThreads) void k_thb_select(const ImgDev* __restrict__ imgs,
                                                             const Tile* __restrict__ tiles, int ntiles,
                                                             const int64_t* __restrict__ m_total,
                                                             const uint32_t* __restrict__ khi,
                                                             const uint32_t* __restrict__ klo,
                                                             float* __restrict__ yfull, int32_t* __restrict__ m) {
  constexpr int NN = B * B, PER = NN / 64;
  const int tile = blockIdx.x;
  if (tile >= ntiles) return;
  const Tile tl = tiles[tile];
  const ImgDev im = imgs[tl.img];
  const int k = (int)(m_total[tl.img] / im.nB);
  const int w = wave_in_group(), lane = threadIdx.x & 63;
  const uint64_t below = (1ull << lane) - 1ull;
  for (int bb = w; bb < tl.count; bb += kWavesPerGroup) {
    const int64_t base = im.out_off + (int64_t)(tl.first + bb) * NN;
    uint64_t key[PER];
    uint32_t hv[PER], lv[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      hv[j] = khi[base + 64 * j + lane];
      lv[j] = klo[base + 64 * j + lane];
      key[j] = thr_key(hv[j], lv[j]);
    }
    // T = largest key with #(key >= T) >= k, i.e. the k-th largest
    uint64_t T = 0;
    if (k > 0) {
      for (int bit = 62; bit >= 0; --bit) {
        const uint64_t cand = T | (1ull << bit);
        int cnt = 0;
#pragma unroll
        for (int j = 0; j < PER; ++j) cnt += __popcll(__ballot(key[j] >= cand));
        if (cnt >= k) T = cand;
      }
    }
    int gtc = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) gtc += __popcll(__ballot(key[j] > T));
    const int tk = k - gtc;  // ties at T to keep, in rank order
    int seen = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const uint64_t tie = __ballot(key[j] == T);
      const int rank_tie = seen + __popcll(tie & below);
      const bool keep = k > 0 && (key[j] > T || (key[j] == T && rank_tie < tk));
      const double c = __longlong_as_double((long long)(((uint64_t)hv[j] << 32) | lv[j]));
      yfull[base + 64 * j + lane] = keep ? (float)c : 0.f;
      seen += __popcll(tie);
    }
    if (lane == 0) m[im.blk_off + tl.first + bb] = k;
  }
}

// Nearest-ish double of a 128-bit integer (two roundings).
__device__ __forceinline__ double i128_to_f64(__int128 v) {
  const bool neg = v < 0;
  const unsigned __int128 u = neg ? (unsigned __int128)0 - (unsigned __int128)v : (unsigned __int128)v;
  const double r = (double)(uint64_t)(u >> 64) * 18446744073709551616.0 + (double)(uint64_t)u;
  return neg ? -r : r;
}

// Pearson's correlation of two per-block counts over each image's blocks,
// from exact integer moments.
__global__ __launch_bounds__(256) void k_corr(const ImgDev* __restrict__ imgs, const int32_t* __restrict__ a,
                                              const int32_t* __restrict__ b, double* __restrict__ rho) {
  __shared__ long long sh[5][256];
  const ImgDev im = imgs[blockIdx.x];
  long long sa = 0, sb = 0, saa = 0, sbb = 0, sab = 0;
  for (int64_t i = threadIdx.x; i < im.nB; i += 256) {
    const long long x = a[im.blk_off + i], y = b[im.blk_off + i];
    sa += x;
    sb += y;
    saa += x * x;
    sbb += y * y;
    sab += x * y;
  }
  sh[0][threadIdx.x] = sa;
  sh[1][threadIdx.x] = sb;
  sh[2][threadIdx.x] = saa;
  sh[3][threadIdx.x] = sbb;
  sh[4][threadIdx.x] = sab;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
      for (int q = 0; q < 5; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const __int128 n = im.nB;
    const __int128 A = sh[0][0], Bs = sh[1][0];
    const __int128 cov = n * (__int128)sh[4][0] - A * Bs;
    const __int128 va = n * (__int128)sh[2][0] - A * A;
    const __int128 vb = n * (__int128)sh[3][0] - Bs * Bs;
    double r = __builtin_nan("");
    if (va > 0 && vb > 0) r = i128_to_f64(cov) / (sqrt(i128_to_f64(va)) * sqrt(i128_to_f64(vb)));
    rho[blockIdx.x] = r;
  }
}

}  // namespace abcs
