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
//       their bit patterns) with 2048-bin digits: three histogram passes over
//       the high words decide them, the coefficients whose high word equals
//       T's are then gathered into a list, and three passes over that list
//       decide the low word.  A one-workgroup pick kernel per image chooses
//       each digit.
//   THB keeps the floor(M / n_B) largest of each block (same tie rule), found
//       by a bit-by-bit search of the block's threshold inside one wavefront
//       right after the block's coefficients are computed.
//
// Coefficients live in two planes (high and low 32-bit words of the float64,
// sign included), in rank order per block at the block's decoded-pixel
// offset: image base + raster block index * B^2 (THI only).  The kept coefficients are
// written as float32 into a dense plane of the same layout, which the masked
// inverse DCT decodes with k_i = B^2.
#pragma once

#include "common.hpp"
#include "transform16.hpp"
#include "generic_kernels.hpp"

namespace abcs {

constexpr int kSelChunk = 32768;  // coefficients per histogram workgroup (a multiple of every B^2)
constexpr int kSelBins = 2048;
constexpr int kSelPasses = 6;    // 0..2: high words; 3..5: low words of the candidates

// Digit of pass p over the 63-bit key (bits 62..32 from the high word without
// its sign, 31..0 from the low word): shift and width.
__host__ __device__ constexpr int sel_shift(int p) {
  return p == 0 ? 52 : p == 1 ? 42 : p == 2 ? 32 : p == 3 ? 21 : p == 4 ? 10 : 0;
}
__host__ __device__ constexpr int sel_width(int p) { return (p == 0 || p == 3 || p == 4) ? 11 : 10; }

struct SelChunk {
  int64_t start;  // first coefficient (decoded-pixel index space)
  int32_t len;    // 1 .. kSelChunk, a multiple of 64
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

__device__ __forceinline__ float thr_value(uint32_t hi, uint32_t lo) {
  return (float)__longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ void hist_flush(const uint32_t* h, unsigned long long* g) {
  for (int b = threadIdx.x; b < kSelBins; b += blockDim.x) {
    const uint32_t v = h[b];
    if (v) atomicAdd(&g[b], (unsigned long long)v);
  }
}

// THB inside one wavefront: keep the k largest of the block's keys (hi: high
// word without sign, lo: low word; element 64 j + lane in rank order), ties
// to the lower rank.  Threshold (Th, Tl) by a bit-by-bit search, first over
// the high words, then over the low words of the keys whose high word equals
// Th (skipped when all of them are kept).
template <int PER>
__device__ __forceinline__ void thb_keep(const uint32_t (&hv)[PER], const uint32_t (&lv)[PER], int k,
                                         bool (&keep)[PER]) {
  const uint64_t below = (1ull << (threadIdx.x & 63)) - 1ull;
  if (k <= 0) {
#pragma unroll
    for (int j = 0; j < PER; ++j) keep[j] = false;
    return;
  }
  uint32_t Th = 0;
  for (int bit = 30; bit >= 0; --bit) {
    const uint32_t cand = Th | (1u << bit);
    int cnt = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) cnt += __popcll(__ballot(hv[j] >= cand));
    if (cnt >= k) Th = cand;
  }
  int gt = 0, ceq = 0;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    gt += __popcll(__ballot(hv[j] > Th));
    ceq += __popcll(__ballot(hv[j] == Th));
  }
  const int need = k - gt;  // 1 .. ceq
  if (need >= ceq) {
#pragma unroll
    for (int j = 0; j < PER; ++j) keep[j] = hv[j] >= Th;
    return;
  }
  uint32_t Tl = 0;
  for (int bit = 31; bit >= 0; --bit) {
    const uint32_t cand = Tl | (1u << bit);
    int cnt = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) cnt += __popcll(__ballot(hv[j] == Th && lv[j] >= cand));
    if (cnt >= need) Tl = cand;
  }
  int gtl = 0;
#pragma unroll
  for (int j = 0; j < PER; ++j) gtl += __popcll(__ballot(hv[j] == Th && lv[j] > Tl));
  const int tk = need - gtl;  // keys equal to (Th, Tl) to keep, in rank order
  int seen = 0;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const bool tie = hv[j] == Th && lv[j] == Tl;
    const uint64_t tb = __ballot(tie);
    const int r = seen + __popcll(tb & below);
    keep[j] = hv[j] > Th || (hv[j] == Th && lv[j] > Tl) || (tie && r < tk);
    seen += __popcll(tb);
  }
}

constexpr int kRuleTHI = 0, kRuleTHB = 1;

// Register tiling of the float64 transform: each lane computes an R x R
// patch of T and of C, so one LDS load feeds R multiply-adds; a block takes
// LPB lanes and a wave BPW blocks at once.
template <int B>
struct ThrGeom {
  static constexpr int R = B == 8 ? 2 : 4;
  static constexpr int NN = B * B, P = B + 1;
  static constexpr int LPB = NN / (R * R);  // lanes per block
  static constexpr int BPW = 64 / LPB;      // blocks per wave
  static constexpr int SLOTS = kWavesPerGroup * BPW;
};

// Every coefficient of the tile's blocks in float64: C[u][v] = sum_r D[u][r]
// T[r][v], T[r][v] = sum_j X[r][j] D[v][j], sums in ascending index order,
// every product and sum rounded on its own.
//   THI: written as (high, low) words in rank order;
//   THB: the block's selection, written as float32 into yfull, and m_i.
template <int B, int RULE>
__global__ __launch_bounds__(kGroupThreads) void k_thr_coefs(const ImgDev* __restrict__ imgs,
                                                            const Tile* __restrict__ tiles, int ntiles,
                                                            const uint8_t* __restrict__ px,
                                                            uint32_t* __restrict__ khi, uint32_t* __restrict__ klo,
                                                            const int64_t* __restrict__ m_total,
                                                            float* __restrict__ yfull, int32_t* __restrict__ m) {
#pragma clang fp contract(off)
  using G = ThrGeom<B>;
  constexpr int R = G::R, NN = G::NN, P = G::P, PER = NN / 64;
  __shared__ __align__(16) double sDt[NN];   // D[a][b] at b B + a
  __shared__ uint16_t srank[NN];
  __shared__ float sX[G::SLOTS][B * P];      // pixels, then high words by rank
  __shared__ __align__(16) double sT[G::SLOTS][NN];  // T[r][v] at r B + v, then low words
  if ((int)blockIdx.x >= ntiles) return;
  for (int t = threadIdx.x; t < NN; t += kGroupThreads) {
    const double d = ThrTables<B>::Dd()[t];  // D[a][b] at a B + b
    sDt[(t % B) * B + t / B] = d;
    srank[t] = (uint16_t)ThrTables<B>::rank(t);
  }
  __syncthreads();
  const Tile tl = tiles[blockIdx.x];
  const ImgDev im = imgs[tl.img];
  const int w = wave_in_group(), lane = threadIdx.x & 63;
  const int g = lane / G::LPB, li = lane % G::LPB;
  const int a0 = R * (li / (B / R)), b0 = R * (li % (B / R));  // patch origin (row, column)
  const __amdgpu_buffer_rsrc_t rp = make_rsrc(px + tl.px_base, (B - 1) * im.pitch + B * tl.count);
  const int kb = RULE == kRuleTHB ? (int)(m_total[tl.img] / im.nB) : 0;
  for (int base_bb = 0; base_bb < tl.count; base_bb += G::SLOTS) {
    const int first = base_bb + w * G::BPW;  // the wave's first block
    if (first >= tl.count) break;
    for (int q = 0; q < G::BPW; ++q)
      if (first + q < tl.count) gen_load_pixels<B>(rp, im.pitch, first + q, sX[w * G::BPW + q]);
    wave_lds_sync();
    const int slot = w * G::BPW + g;
    const bool active = first + g < tl.count;
    float* X = sX[slot];
    double* T = sT[slot];
    double acc[R][R];
    if (active) {
#pragma unroll
      for (int i = 0; i < R; ++i)
#pragma unroll
        for (int k = 0; k < R; ++k) acc[i][k] = 0.0;
      for (int j = 0; j < B; ++j) {
        double x[R], d[R];
#pragma unroll
        for (int i = 0; i < R; ++i) x[i] = (double)X[(a0 + i) * P + j];
#pragma unroll
        for (int k = 0; k < R; ++k) d[k] = sDt[j * B + b0 + k];
#pragma unroll
        for (int i = 0; i < R; ++i)
#pragma unroll
          for (int k = 0; k < R; ++k) {
            const double p = x[i] * d[k];
            acc[i][k] = acc[i][k] + p;
          }
      }
#pragma unroll
      for (int i = 0; i < R; ++i)
#pragma unroll
        for (int k = 0; k < R; ++k) T[(a0 + i) * B + b0 + k] = acc[i][k];
    }
    wave_lds_sync();
    if (active) {
#pragma unroll
      for (int i = 0; i < R; ++i)
#pragma unroll
        for (int k = 0; k < R; ++k) acc[i][k] = 0.0;
      for (int r = 0; r < B; ++r) {
        double du[R], t[R];
#pragma unroll
        for (int i = 0; i < R; ++i) du[i] = sDt[r * B + a0 + i];
#pragma unroll
        for (int k = 0; k < R; ++k) t[k] = T[r * B + b0 + k];
#pragma unroll
        for (int i = 0; i < R; ++i)
#pragma unroll
          for (int k = 0; k < R; ++k) {
            const double p = du[i] * t[k];
            acc[i][k] = acc[i][k] + p;
          }
      }
    }
    // every lane of the wave has read T before any lane overwrites it
    wave_lds_sync();
    if (active) {
      uint32_t* H = reinterpret_cast<uint32_t*>(X);
      uint32_t* Lo = reinterpret_cast<uint32_t*>(T);
#pragma unroll
      for (int i = 0; i < R; ++i)
#pragma unroll
        for (int k = 0; k < R; ++k) {
          const uint64_t bits = (uint64_t)__double_as_longlong(acc[i][k]);
          const int z = srank[(a0 + i) * B + b0 + k];
          H[z] = (uint32_t)(bits >> 32);
          Lo[z] = (uint32_t)bits;
        }
    }
    wave_lds_sync();
    for (int q = 0; q < G::BPW && first + q < tl.count; ++q) {
      const int bb = first + q;
      const uint32_t* H = reinterpret_cast<const uint32_t*>(sX[w * G::BPW + q]);
      const uint32_t* Lo = reinterpret_cast<const uint32_t*>(sT[w * G::BPW + q]);
      const int64_t dst = im.out_off + (int64_t)(tl.first + bb) * NN;
      if (RULE == kRuleTHI) {
#pragma unroll
        for (int j = 0; j < PER; ++j) {
          khi[dst + 64 * j + lane] = H[64 * j + lane];
          klo[dst + 64 * j + lane] = Lo[64 * j + lane];
        }
      } else {
        uint32_t hv[PER], lv[PER];
        bool keep[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
          hv[j] = H[64 * j + lane] & 0x7fffffffu;
          lv[j] = Lo[64 * j + lane];
        }
        thb_keep<PER>(hv, lv, kb, keep);
#pragma unroll
        for (int j = 0; j < PER; ++j)
          yfull[dst + 64 * j + lane] = keep[j] ? thr_value(H[64 * j + lane], lv[j]) : 0.f;
        if (lane == 0) m[im.blk_off + tl.first + bb] = kb;
      }
    }
    wave_lds_sync();
  }
}

// need = M of every image, prefix = 0; histograms, candidate counts and tie
// counts cleared.
__global__ void k_thr_init(const int64_t* __restrict__ m_total, int n, int64_t blocks, SelState* __restrict__ st,
                           unsigned long long* __restrict__ hist, uint32_t* __restrict__ cnt,
                           int32_t* __restrict__ eq) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < (int64_t)n * kSelBins) hist[i] = 0ull;
  if (i < blocks) eq[i] = 0;
  if (i < n) {
    st[i] = SelState{0ull, m_total[i]};
    cnt[i] = 0u;
  }
}

// Histogram of the first digit (the exponent of |c|).  A wave's magnitudes
// share few exponents, so the LDS histogram has 8 copies (lane l adds to copy
// l % 8), which cuts same-address conflicts of the atomics eightfold.
constexpr int kHist0Copies = 8;
__global__ __launch_bounds__(256) void k_thr_hist0(const SelChunk* __restrict__ chunks,
                                                   const uint32_t* __restrict__ khi,
                                                   unsigned long long* __restrict__ hist) {
  __shared__ uint32_t h[kHist0Copies * kSelBins];
  for (int b = threadIdx.x; b < kHist0Copies * kSelBins; b += 256) h[b] = 0u;
  __syncthreads();
  const SelChunk c = chunks[blockIdx.x];
  const int hs = sel_shift(0) - 32;
  uint32_t* hc = h + (threadIdx.x % kHist0Copies) * kSelBins;
  const uint4* hp = reinterpret_cast<const uint4*>(khi + c.start);
  for (int q = threadIdx.x; 4 * q < c.len; q += 256) {
    const uint4 v = hp[q];
    atomicAdd(&hc[(v.x & 0x7fffffffu) >> hs], 1u);
    atomicAdd(&hc[(v.y & 0x7fffffffu) >> hs], 1u);
    atomicAdd(&hc[(v.z & 0x7fffffffu) >> hs], 1u);
    atomicAdd(&hc[(v.w & 0x7fffffffu) >> hs], 1u);
  }
  __syncthreads();
  unsigned long long* g = hist + (int64_t)c.img * kSelBins;
  for (int b = threadIdx.x; b < kSelBins; b += 256) {
    uint32_t v = 0;
#pragma unroll
    for (int k = 0; k < kHist0Copies; ++k) v += h[k * kSelBins + b];
    if (v) atomicAdd(&g[b], (unsigned long long)v);
  }
}

// Histogram of pass p's digit (p = 1, 2: high words) over the coefficients
// whose higher digits match the image's decided prefix.
__global__ __launch_bounds__(256) void k_thr_hist_hi(const SelChunk* __restrict__ chunks,
                                                     const uint32_t* __restrict__ khi,
                                                     const SelState* __restrict__ st,
                                                     unsigned long long* __restrict__ hist, int pass) {
  __shared__ uint32_t h[kSelBins];
  for (int b = threadIdx.x; b < kSelBins; b += 256) h[b] = 0u;
  __syncthreads();
  const SelChunk c = chunks[blockIdx.x];
  const uint64_t prefix = st[c.img].prefix;
  const int hs = sel_shift(pass) - 32, hw = sel_width(pass);
  const uint32_t above = ~0u << (hs + hw);  // decided bits of the high word (hs + hw <= 21)
  const uint32_t ph = (uint32_t)(prefix >> 32) & above;
  const uint32_t dmask = (1u << hw) - 1u;
  const uint4* hp = reinterpret_cast<const uint4*>(khi + c.start);
  for (int q = threadIdx.x; 4 * q < c.len; q += 256) {
    const uint4 v = hp[q];
    const uint32_t e[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const uint32_t hi = e[t] & 0x7fffffffu;
      if ((hi & above) == ph) atomicAdd(&h[(hi >> hs) & dmask], 1u);
    }
  }
  __syncthreads();
  hist_flush(h, hist + (int64_t)c.img * kSelBins);
}

// Appends the image-relative index of every coefficient whose high word
// equals the decided one (the candidates of the low-word passes) to the
// image's list (cand + out_off, capacity H'W'); order is irrelevant.
__global__ __launch_bounds__(256) void k_thr_collect(const SelChunk* __restrict__ chunks,
                                                     const ImgDev* __restrict__ imgs,
                                                     const uint32_t* __restrict__ khi,
                                                     const SelState* __restrict__ st, uint32_t* __restrict__ cand,
                                                     uint32_t* __restrict__ cnt) {
  const SelChunk c = chunks[blockIdx.x];
  const int64_t base = imgs[c.img].out_off;
  const uint32_t th = (uint32_t)(st[c.img].prefix >> 32);
  const uint4* hp = reinterpret_cast<const uint4*>(khi + c.start);
  const int lane = threadIdx.x & 63;
  const uint64_t below = (1ull << lane) - 1ull;
  const uint32_t rel0 = (uint32_t)(c.start - base);
  // every wave runs the same number of iterations (len is a multiple of 64)
  for (int q0 = 0; 4 * q0 < c.len; q0 += 256) {
    const int q = q0 + (int)threadIdx.x;
    const bool in = 4 * q < c.len;
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (in) v = hp[q];
    const uint32_t e[4] = {v.x, v.y, v.z, v.w};
    uint64_t bal[4];
    int tot = 0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      bal[t] = __ballot(in && (e[t] & 0x7fffffffu) == th);
      tot += __popcll(bal[t]);
    }
    if (tot == 0) continue;
    uint32_t slot = 0;
    if (lane == 0) slot = atomicAdd(&cnt[c.img], (uint32_t)tot);
    slot = __shfl(slot, 0, 64);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if ((bal[t] >> lane) & 1ull) cand[base + slot + __popcll(bal[t] & below)] = rel0 + 4u * q + t;
      slot += __popcll(bal[t]);
    }
  }
}

// Histogram of pass p's digit (p = 3, 4, 5: low words) over the image's
// candidates matching the decided prefix; chunk c covers list positions
// [c.start - out_off, + len).
__global__ __launch_bounds__(256) void k_thr_hist_lo(const SelChunk* __restrict__ chunks,
                                                     const ImgDev* __restrict__ imgs,
                                                     const uint32_t* __restrict__ klo,
                                                     const SelState* __restrict__ st,
                                                     const uint32_t* __restrict__ cand,
                                                     const uint32_t* __restrict__ cnt,
                                                     unsigned long long* __restrict__ hist, int pass) {
  __shared__ uint32_t h[kSelBins];
  const SelChunk c = chunks[blockIdx.x];
  const int64_t base = imgs[c.img].out_off;
  const int64_t r0 = c.start - base;
  const int64_t r1 = min(r0 + (int64_t)c.len, (int64_t)cnt[c.img]);
  if (r0 >= r1) return;
  for (int b = threadIdx.x; b < kSelBins; b += 256) h[b] = 0u;
  __syncthreads();
  const uint64_t prefix = st[c.img].prefix;
  const int ls = sel_shift(pass), lw = sel_width(pass);
  const uint32_t above = (uint32_t)(~0ull << (ls + lw));  // decided bits of the low word
  const uint32_t pl = (uint32_t)prefix & above;
  const uint32_t dmask = (1u << lw) - 1u;
  for (int64_t i = r0 + threadIdx.x; i < r1; i += 256) {
    const uint32_t lo = klo[base + cand[base + i]];
    if ((lo & above) == pl) atomicAdd(&h[(lo >> ls) & dmask], 1u);
  }
  __syncthreads();
  hist_flush(h, hist + (int64_t)c.img * kSelBins);
}

// One workgroup per image: the digit at which the count of larger keys first
// reaches `need` (thread t holds bins 8t .. 8t + 7); clears the histogram.
__global__ __launch_bounds__(256) void k_thr_pick(unsigned long long* __restrict__ hist, SelState* __restrict__ st,
                                                  int pass) {
  __shared__ unsigned long long S[257];
  const int img = blockIdx.x, t = threadIdx.x;
  const SelState s = st[img];
  unsigned long long* hb = hist + (int64_t)img * kSelBins + 8 * t;
  unsigned long long hv[8], own = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    hv[j] = hb[j];
    hb[j] = 0ull;
    own += hv[j];
  }
  // inclusive suffix sums S[t] = sum over threads >= t
  S[t] = own;
  if (t == 0) S[256] = 0ull;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    const unsigned long long add = t + o < 256 ? S[t + o] : 0ull;
    __syncthreads();
    S[t] += add;
    __syncthreads();
  }
  const unsigned long long need = (unsigned long long)s.need;
  // S is non-increasing and S[0] >= need: exactly one thread has S[t] >= need > S[t + 1]
  if (S[t] >= need && S[t + 1] < need) {
    unsigned long long acc = S[t + 1];
    int digit = 8 * t;
    for (int j = 7; j >= 0; --j) {
      if (acc + hv[j] >= need) {
        digit = 8 * t + j;
        break;
      }
      acc += hv[j];
    }
    st[img] = SelState{s.prefix | ((uint64_t)digit << sel_shift(pass)), s.need - (int64_t)acc};
  }
}

// Ties at T per block: candidates whose low word equals T's.
__global__ __launch_bounds__(256) void k_thi_eq(const SelChunk* __restrict__ chunks, const ImgDev* __restrict__ imgs,
                                                const uint32_t* __restrict__ klo, const SelState* __restrict__ st,
                                                const uint32_t* __restrict__ cand, const uint32_t* __restrict__ cnt,
                                                int32_t* __restrict__ eq) {
  const SelChunk c = chunks[blockIdx.x];
  const ImgDev im = imgs[c.img];
  const int64_t r0 = c.start - im.out_off;
  const int64_t r1 = min(r0 + (int64_t)c.len, (int64_t)cnt[c.img]);
  const uint32_t tlo = (uint32_t)st[c.img].prefix;
  const uint32_t nn = (uint32_t)(im.B * im.B);
  for (int64_t i = r0 + threadIdx.x; i < r1; i += 256) {
    const uint32_t idx = cand[im.out_off + i];
    if (klo[im.out_off + idx] == tlo) atomicAdd(&eq[im.blk_off + idx / nn], 1);
  }
}

// One workgroup per image: ties at T go to the lowest blocks; eq_i is
// replaced by the ties block i takes.
__global__ __launch_bounds__(256) void k_thi_ties(const ImgDev* __restrict__ imgs, const SelState* __restrict__ st,
                                                  int32_t* __restrict__ eq) {
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
    }
    left -= total;
    if (left < 0) left = 0;
    __syncthreads();
  }
}

// Per block: m_i = #(key > T) + ties taken; with yfull, the kept
// coefficients (key > T, or key == T among the block's first `take` ties in
// rank order) as float32, the rest 0.
__global__ __launch_bounds__(kGroupThreads) void k_thi_mask(const ImgDev* __restrict__ imgs,
                                                           const Tile* __restrict__ tiles, int ntiles,
                                                           const uint32_t* __restrict__ khi,
                                                           const uint32_t* __restrict__ klo,
                                                           const SelState* __restrict__ st,
                                                           const int32_t* __restrict__ take,
                                                           int32_t* __restrict__ m, float* __restrict__ yfull) {
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
    int seen = 0, gt = 0;
    for (int z0 = 0; z0 < NN; z0 += 64) {
      const uint32_t hi = khi[base + z0 + lane], lo = klo[base + z0 + lane];
      const uint64_t key = thr_key(hi, lo);
      const uint64_t tie = __ballot(key == T);
      const int rank_tie = seen + __popcll(tie & below);
      const bool keep = key > T || (key == T && rank_tie < tk);
      gt += __popcll(__ballot(key > T));
      if (yfull) yfull[base + z0 + lane] = keep ? thr_value(hi, lo) : 0.f;
      seen += __popcll(tie);
    }
    if (lane == 0) m[blk] = gt + tk;
  }
}

// Nearest-ish double of a 128-bit integer (two roundings).
__device__ __forceinline__ double i128_to_f64(__int128 v) {
  const bool neg = v < 0;
  const unsigned __int128 u = neg ? (unsigned __int128)0 - (unsigned __int128)v : (unsigned __int128)v;
  const double r = (double)(uint64_t)(u >> 64) * 18446744073709551616.0 + (double)(uint64_t)u;
  return neg ? -r : r;
}

// Continued fraction of the regularised incomplete beta function I_x(a, b)
// (Abramowitz & Stegun 26.5.8), evaluated with the modified Lentz method;
// converges fast for x < (a + 1) / (a + b + 2).
__device__ inline double betai_cf(double a, double b, double x) {
  const double tiny = 1e-300;
  auto fix = [&](double v) { return fabs(v) < tiny ? tiny : v; };
  double c = 1.0, d = 1.0 / fix(1.0 - (a + b) * x / (a + 1.0)), h = d;
  for (int m = 1; m <= 1000; ++m) {
    const double m2 = 2.0 * m;
    double t = m * (b - m) * x / ((a + m2 - 1.0) * (a + m2));  // even term d_{2m}
    d = 1.0 / fix(1.0 + t * d);
    c = fix(1.0 + t / c);
    h *= d * c;
    t = -(a + m) * (a + b + m) * x / ((a + m2) * (a + m2 + 1.0));  // odd term d_{2m+1}
    d = 1.0 / fix(1.0 + t * d);
    c = fix(1.0 + t / c);
    const double del = d * c;
    h *= del;
    if (fabs(del - 1.0) < 1e-16) break;
  }
  return h;
}

// I_x(a, b) = x^a (1-x)^b / (a B(a, b)) * CF(a, b, x), using
// I_x(a, b) = 1 - I_{1-x}(b, a) where the fraction converges slowly.
__device__ inline double betai(double a, double b, double x) {
  if (x <= 0.0) return 0.0;
  if (x >= 1.0) return 1.0;
  const double lf = lgamma(a + b) - lgamma(a) - lgamma(b) + a * log(x) + b * log1p(-x);
  if (x < (a + 1.0) / (a + b + 2.0)) return exp(lf) * betai_cf(a, b, x) / a;
  return 1.0 - exp(lf) * betai_cf(b, a, 1.0 - x) / b;
}

// Pearson's correlation of two per-block counts over each image's blocks,
// from exact integer moments, and (nullable) the two-sided p-value of rho = 0:
// t = rho sqrt(nu / (1 - rho^2)) with nu = n_B - 2 degrees of freedom,
// P(|T| >= |t|) = I_{1 - rho^2}(nu / 2, 1 / 2).
__global__ __launch_bounds__(256) void k_corr(const ImgDev* __restrict__ imgs, const int32_t* __restrict__ a,
                                              const int32_t* __restrict__ b, double* __restrict__ rho,
                                              double* __restrict__ pval) {
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
    if (pval) {
      double p = __builtin_nan("");
      if (r == r && im.nB >= 3) {
        const double x = (1.0 - r) * (1.0 + r);
        p = x <= 0.0 ? 0.0 : betai(0.5 * (double)(im.nB - 2), 0.5, x);
      }
      pval[blockIdx.x] = p;
    }
  }
}

}  // namespace abcs
