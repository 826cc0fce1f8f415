// Phase-1 statistics and per-image budget apportionment (Section V).
#pragma once

#include "common.hpp"
#include "transform16.hpp"

namespace abcs {

// ---------------------------------------------------------------------------
// BBV_i (eq 19): one thread per block.  With k_j = X0 + j L the block adds the
// absolute differences of horizontally adjacent pixels (k_j - 1, k_j) along
// its top row and of vertically adjacent pixels along its left column; the
// bottom and right terms are the top row of the block below and the left
// column of the block to the right, or the block's own last row / column at
// the image edge.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void bbv_stats_thread(const ImgDev* __restrict__ imgs, const Tile* __restrict__ tiles,
                                                 int ntiles, const uint8_t* __restrict__ px,
                                                 int32_t* __restrict__ stat, int t) {
  const int ti = t / kTileBlocks, b = t % kTileBlocks;
  if (ti >= ntiles) return;
  const Tile tl = tiles[ti];
  if (b >= tl.count) return;
  const ImgDev im = imgs[tl.img];
  const int blk = tl.first + b;
  const int by = tl.by, bx = tl.first - tl.by * im.nbx + b;
  const uint8_t* base = px + im.px_off;
  const int pitch = im.pitch, B = im.B;
  const int r0 = by * B, c0 = bx * B;

  auto row_var = [&](int r, int c) {
    const uint8_t* p = base + (int64_t)r * pitch + c;
    int s = 0;
    for (int j = 0; j < im.nS; ++j) {
      const int k = im.X0 + j * im.L;
      s += abs((int)p[k] - (int)p[k - 1]);
    }
    return s;
  };
  auto col_var = [&](int c, int r) {
    const uint8_t* p = base + (int64_t)r * pitch + c;
    int s = 0;
    for (int j = 0; j < im.nS; ++j) {
      const int k = im.X0 + j * im.L;
      s += abs((int)p[(int64_t)k * pitch] - (int)p[(int64_t)(k - 1) * pitch]);
    }
    return s;
  };
  const int top = row_var(r0, c0);
  const int left = col_var(c0, r0);
  const int bottom = (by + 1 < im.nby) ? row_var(r0 + B, c0) : row_var(r0 + B - 1, c0);
  const int right = (bx + 1 < im.nbx) ? col_var(c0 + B, r0) : col_var(c0 + B - 1, r0);
  stat[im.blk_off + blk] = top + left + bottom + right;
}

// ---------------------------------------------------------------------------
// DD n_i: one wavefront per tile of 16x16 blocks.  A compensated float16
// MFMA transform (dct16_fwd_f16k32) decides |c| > T for every coefficient
// further than kDDGuard from T; the rest are recomputed in float64 from the
// block staged in LDS in one fixed order, T[r] = sum_j X[r][j] D[v][j] (j
// ascending), c = sum_r D[u][r] T[r] (r ascending), every product and sum
// rounded on its own, so the counts are those of the float64 definition
// whatever the screening arithmetic.
//
// kDDGuard bounds the screening error of a coefficient (u = 2^-24 the float32
// unit roundoff, with every float32 sum of n terms taken to err by at most
// n u times the sum of their magnitudes).  Pixels are exact in float16; the
// basis split D = Dhi + Dlo leaves at most 8.4e-8 per entry (|D| <= 0.354,
// float16 unit roundoff 2^-11, subnormal spacing 2^-24).  With |X| <= 255 and
// sum_j |D[v][j]| <= sqrt(16) = 4:
//   stage 1, 32 products of magnitude sum <= 1020.1: 32 u 1020.1 + 16 * 255 *
//     8.4e-8 <= 2.3e-3;
//   stage 2, 48 products of magnitude sum <= 4087: 48 u 4087 = 1.17e-2, plus
//     the stage-1 error times 4 (9.2e-3), the rounding of Tl (|T - Th| <=
//     0.5, 4 * 2.4e-4), the dropped Dlo Tl (16 * 1.73e-4 * 0.5 = 1.4e-3) and
//     the basis residual on T (16 * 8.4e-8 * 1020.5 = 1.4e-3): <= 2.5e-2.
// The guard is twice that.
// ---------------------------------------------------------------------------
constexpr float kDDGuard = 0.05f;
// Undecided coefficients are queued per wave and settled in float64 in
// batches of 64.  A block adds at most m1 <= 128 (C_F >= 1), so the queue is
// flushed before a block whenever fewer than 128 slots are free.
constexpr int kDDListCap = 256;

// Settles queued coefficients in float64, four per pass: the 16 lanes of
// quarter j of the wave take entry base + j, lane r of the quarter forms row
// r's inner sum t_r = sum_y D[v][y] X[r][y] over the columns in order and the
// product D[u][r] t_r, and the products are added over the rows in order
// (read across the quarter by shuffles): the fixed order above, products
// rounded, then added, no contraction.  The count goes to the entry's block
// if |c| > T.  A pass costs a fixed ~200 instructions whatever its number of
// entries, and most tiles queue only a few, so spreading one entry over 16
// lanes beats one entry per lane (a dependent chain of 256 products).  `D`
// is the float64 basis in constant memory: the kernel keeps no LDS copy, so
// that eight workgroups fit on a compute unit.
__device__ __forceinline__ void dd_flush(const uint16_t* list, int n, const uint32_t* st,
                                         const double* __restrict__ D, int T, int32_t* ucnt) {
#pragma clang fp contract(off)
  const int lane = threadIdx.x & 63, j = lane >> 4, r = lane & 15;
  wave_lds_sync();
  for (int base = 0; base < n; base += 4) {
    const bool act = base + j < n;
    const int e = act ? (int)list[base + j] : 0;
    const int b = e >> 8, u = (e >> 4) & 15, v = e & 15;
    double t = 0.0;
    if (act) {
      const uint32_t* row = st + r * (kPxRow / 4) + 4 * b;
      // one column group at a time: four basis values live, not sixteen
#pragma unroll 1
      for (int q = 0; q < 4; ++q) {
        const uint32_t w = row[q];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const double x = (double)((w >> (8 * c)) & 0xffu);
          const double p = x * D[v * 16 + 4 * q + c];
          t = t + p;
        }
      }
    }
    const double pr = D[u * 16 + r] * t;
    double acc = 0.0;
#pragma unroll 1
    for (int i = 0; i < 16; ++i) acc = acc + __shfl(pr, (lane & 48) + i, 64);
    if (act && r == 0 && fabs(acc) > (double)T) atomicAdd(&ucnt[b], 1);
  }
  wave_lds_sync();
}

// LDS of the DD statistics of one workgroup (four waves).
struct DDStatsLds {
  PxStage stage[kWavesPerGroup];
  uint16_t ulist[kWavesPerGroup][kDDListCap];
  int32_t ucount[kWavesPerGroup][kTileBlocks];
};

template <int XF>
__device__ __forceinline__ void dd_stats_group(const ImgDev* __restrict__ imgs, const Tile* __restrict__ tiles,
                                               int ntiles, const uint8_t* __restrict__ px,
                                               int32_t* __restrict__ stat, int group, DDStatsLds& sl) {
  PxStage* stage = sl.stage;
  uint16_t (*ulist)[kDDListCap] = sl.ulist;
  int32_t (*ucount)[kTileBlocks] = sl.ucount;
  const double* Dd = Basis16<XF>::Dd();
  const int wave = group * kWavesPerGroup + wave_in_group();
  if (wave >= ntiles) return;
  const Tile tl = tiles[wave];
  const ImgDev im = imgs[tl.img];
  Lane16 L;
  lane16_init<XF>(L);
  Lane16K32 K;
  lane16k32_init(K, L);
  const int lane = threadIdx.x & 63;
  const float T = (float)im.T;
  const int m1 = im.m1 < 128 ? im.m1 : 128;
  TileIO io;
  io.px = make_rsrc(px + tl.px_base, 15 * im.pitch + 16 * tl.count);
  uint32_t* st = stage[wave_in_group()].w;
  uint16_t* list = ulist[wave_in_group()];
  int32_t* ucnt = ucount[wave_in_group()];
  if (lane < kTileBlocks) ucnt[lane] = 0;
  stage_tile_px(io, im.pitch, tl.count, st);
  wave_lds_sync();
  int32_t my_stat = 0;  // lane b keeps block b's count of coefficients decided in float32
  int nlist = 0;        // wave-uniform length of the queue
  // Lanes whose coefficient r is among the first m1 in zigzag order; the
  // decisions below are wave masks, so each costs two compares per register.
  uint64_t inm[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) inm[r] = __ballot(L.zr[r] < m1);
  const float t_hi = T + kDDGuard, t_lo = T - kDDGuard;
#pragma unroll 2
  for (int b = 0; b < kTileBlocks; ++b) {
    if (nlist > kDDListCap - 128) {
      dd_flush(list, nlist, st, Dd, im.T, ucnt);
      nlist = 0;
    }
    const uint32_t pw = staged_px(st, b, L);
    float a[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) a[c] = (float)((pw >> (8 * c)) & 0xffu);
    const f32x4 C = dct16_fwd_f16k32(a, K);
    int cnt = 0;
    uint64_t un[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float av = fabsf(C[r]);
      const uint64_t gt = __ballot(av > t_hi);
      const uint64_t ge = __ballot(av >= t_lo);
      cnt += __popcll(gt & inm[r]);
      un[r] = ge & ~gt & inm[r];
    }
    if ((un[0] | un[1] | un[2] | un[3]) != 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint64_t um = un[r];
        if (um != 0) {
          const int pos = nlist + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(um >> 32),
                                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)um, 0u));
          if ((um >> lane) & 1) list[pos] = (uint16_t)((b << 8) | ((4 * L.g + r) << 4) | L.n);
          nlist += __popcll(um);
        }
      }
    }
    if (lane == b) my_stat = cnt;
  }
  if (nlist > 0) dd_flush(list, nlist, st, Dd, im.T, ucnt);
  if (lane < kTileBlocks) my_stat += ucnt[lane];
  if (lane < tl.count) stat[im.blk_off + tl.first + lane] = my_stat;
}

// Both phase-1 statistics in one launch, so that the latency-bound BBV
// threads run beside the DD tiles: workgroups below g_bbv take BBV blocks
// (one thread per block of the BBV tile list), the rest take DD tiles of
// 16x16 blocks (one wavefront per tile).
__global__ __launch_bounds__(kGroupThreads) void k_phase1_stats(const ImgDev* __restrict__ imgs,
                                                               const Tile* __restrict__ tiles_bbv, int nt_bbv,
                                                               int g_bbv, const Tile* __restrict__ tiles_dd,
                                                               int nt_dd, const uint8_t* __restrict__ px,
                                                               int32_t* __restrict__ stat) {
  __shared__ DDStatsLds sl;
  if ((int)blockIdx.x < g_bbv)
    bbv_stats_thread(imgs, tiles_bbv, nt_bbv, px, stat, blockIdx.x * kGroupThreads + threadIdx.x);
  else
    dd_stats_group<kXfDCT>(imgs, tiles_dd, nt_dd, px, stat, blockIdx.x - g_bbv, sl);
}

// DD statistics of 16x16 Walsh-Hadamard tiles (one wavefront per tile).
__global__ __launch_bounds__(kGroupThreads) void k_dd_stats16_wht(const ImgDev* __restrict__ imgs,
                                                                 const Tile* __restrict__ tiles, int ntiles,
                                                                 const uint8_t* __restrict__ px,
                                                                 int32_t* __restrict__ stat) {
  __shared__ DDStatsLds sl;
  dd_stats_group<kXfWHT>(imgs, tiles, ntiles, px, stat, blockIdx.x, sl);
}

// ---------------------------------------------------------------------------
// Budget apportionment (eqs 22, 23 and the cap rule after eq 22), one
// workgroup per image, exact integer arithmetic.
//   1. a_i <- undecided for every block (the cap is > 0 for every rule).
//   2. S = sum of undecided weights (all zero -> weight 1 each).
//      q_i = floor(P w_i / S).  If some q_i >= cap: those blocks are fixed at
//      the cap, P shrinks by what they took, repeat 2.
//   3. Otherwise a_i = q_i plus one for the R = P - sum q_i blocks with the
//      largest (P w_i mod S), ties to the lower index (radix select on the
//      remainder, then a rank among equal remainders).
//   4. DD adds the m^1 phase-1 coefficients; offsets = exclusive prefix sum.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_sum_t(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// k_apportion keeps an image's blocks in global memory; it serves images of
// more than kApHistMaxBlocks blocks (1024 threads per image).  Images of at
// most 8192 blocks use k_apportion_reg below, which holds them in registers
// (4 or 8 per thread), and those in between k_apportion_hist, which works on
// a histogram of the weights.

template <int NW, typename T>
__device__ T group_sum(T v, T* sh) {
  v = wave_sum_t(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  T s = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) s += sh[i];
  return s;
}

// Exclusive prefix sum over threads in thread order.
template <typename T>
__device__ T group_exclusive_scan(T v, T* sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  T inc = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const T u = __shfl_up(inc, o, 64);
    if (lane >= o) inc += u;
  }
  __syncthreads();
  if (lane == 63) sh[w] = inc;
  __syncthreads();
  T base = 0;
  for (int i = 0; i < w; ++i) base += sh[i];
  return base + inc - v;
}

__device__ __forceinline__ int32_t wave_max_i32(int32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// Inclusive prefix sum over the 64 lanes of a wavefront on the DPP network
// (vector-ALU latency, no LDS round trips): within each row of 16 lanes by
// shifts of 1, 2, 4 and 8 (lanes without a source add 0), then the last lane
// of row 0 is added to row 1 and 3 and of row 1 (now holding rows 0-1) to
// rows 2 and 3.
__device__ __forceinline__ int32_t wave_incl_scan_dpp(int32_t x) {
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, true);  // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, true);  // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, true);  // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, true);  // row_shr:8
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15 into rows 1, 3
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31 into rows 2, 3
  return x;
}

// floor(pw / S) for 0 <= pw < 2^53 and 0 < S < 2^53: the float64 quotient is
// within one of the exact one, which the integer checks then settle.
__device__ __forceinline__ int64_t floor_div_exact(int64_t pw, int64_t S) {
  int64_t q = (int64_t)((double)pw / (double)S);
  if (q * S > pw) q -= 1;
  if ((q + 1) * S <= pw) q += 1;
  return q;
}

template <int kApThreads>
__global__ __launch_bounds__(kApThreads) void k_apportion(const ImgDev* __restrict__ imgs,
                                                         int32_t* __restrict__ stat_all,
                                                         int32_t* __restrict__ k_all,
                                                         int64_t* __restrict__ off_all) {
  constexpr int kApWaves = kApThreads / 64;
  __shared__ int64_t sh64[kApWaves];
  __shared__ int32_t hist[256];
  __shared__ int64_t sel_sh[2];
  const ImgDev im = imgs[blockIdx.x];
  const int nB = im.nB;
  int32_t* w = stat_all + im.blk_off;
  int32_t* k = k_all + im.blk_off;
  int64_t* off = off_all + im.blk_off;  // also holds the remainders until the offsets are written
  const int tid = threadIdx.x;

  if (im.mode == kModeZZ) {
    for (int i = tid; i < nB; i += kApThreads) {
      k[i] = im.kz;
      w[i] = 0;
      off[i] = im.meas_off + (int64_t)i * im.kz;
    }
    return;
  }

  // Passes without an order over the blocks use interleaved indices
  // (coalesced); the two passes that need index order (ties, offsets) give
  // thread t the contiguous range [t per, t per + per).
  const int64_t cap = im.cap;
  int64_t P = im.pool;
  for (int i = tid; i < nB; i += kApThreads) k[i] = -1;  // undecided

  int64_t S = 0;
  bool uniform = false;
  for (;;) {
    int64_t sw = 0, na = 0;
#pragma unroll 4
    for (int i = tid; i < nB; i += kApThreads)
      if (k[i] < 0) { sw += w[i]; na += 1; }
    S = group_sum<kApWaves>(sw, sh64);
    const int64_t A = group_sum<kApWaves>(na, sh64);
    if (A == 0) break;
    uniform = (S == 0);
    if (uniform) S = A;
    // floor(P w_i / S) >= cap  <=>  P w_i >= cap S: every such block is fixed
    // at its cap with the same P and S, then the split is redone.
    const int64_t capS = cap * S;
    int64_t used = 0;
#pragma unroll 4
    for (int i = tid; i < nB; i += kApThreads) {
      if (k[i] < 0) {
        const int64_t wi = uniform ? 1 : (int64_t)w[i];
        if (P * wi >= capS) { k[i] = (int32_t)cap; used += cap; }
      }
    }
    used = group_sum<kApWaves>(used, sh64);
    if (used == 0) break;
    P -= used;
  }

  // Floors and remainders of the final split, once: k[i] = floor(P w_i / S),
  // off[i] = remainder (-1 for blocks fixed at the cap).
  int64_t sq = 0;
#pragma unroll 4
  for (int i = tid; i < nB; i += kApThreads) {
    if (k[i] < 0) {
      const int64_t wi = uniform ? 1 : (int64_t)w[i];
      const int64_t pw = P * wi;
      const int64_t q = floor_div_exact(pw, S);
      k[i] = (int32_t)q;
      off[i] = pw - q * S;
      sq += q;
    } else {
      off[i] = -1;
    }
  }
  const int64_t R = P - group_sum<kApWaves>(sq, sh64);

  // Radix select of the R-th largest remainder tau (8-bit digits, MSB first).
  int64_t tau = 0, need = R;
  if (R > 0 && S > 1) {
    const int bits = 64 - __clzll((unsigned long long)(S - 1));
    for (int shift = ((bits + 7) / 8) * 8 - 8; shift >= 0; shift -= 8) {
      if (tid < 256) hist[tid] = 0;
      __syncthreads();
      const uint64_t hi_mask = (shift + 8 >= 64) ? 0ull : (~0ull << (shift + 8));
#pragma unroll 4
      for (int i = tid; i < nB; i += kApThreads) {
        const int64_t rem = off[i];
        if (rem >= 0 && ((uint64_t)rem & hi_mask) == ((uint64_t)tau & hi_mask))
          atomicAdd(&hist[((uint64_t)rem >> shift) & 255u], 1);
      }
      __syncthreads();
      // Bin counts summed from the top digit down: the selected digit d is
      // the one where the count of larger-or-equal remainders reaches `need`.
      if (tid == 0) {
        sel_sh[0] = 0;
        sel_sh[1] = need;
      }
      const int32_t bin = tid < 256 ? hist[255 - tid] : 0;
      const int64_t above_incl = group_exclusive_scan((int64_t)bin, sh64) + bin;
      if (tid < 256 && above_incl >= need && above_incl - bin < need) {
        sel_sh[0] = 255 - tid;
        sel_sh[1] = need - (above_incl - bin);
      }
      __syncthreads();
      tau |= (int64_t)sel_sh[0] << shift;
      need = sel_sh[1];
      __syncthreads();
    }
  }

  // Final values: floor + 1 for remainders above tau and for the first `need`
  // (by index) remainders equal to tau; then the offsets, both in index order.
  const int per = (nB + kApThreads - 1) / kApThreads;
  const int i0 = min(nB, tid * per), i1 = min(nB, i0 + per);
  int64_t neq = 0;
  if (R > 0)
    for (int i = i0; i < i1; ++i) neq += (off[i] == tau) ? 1 : 0;
  int64_t rank = group_exclusive_scan(neq, sh64);
  const int32_t add = (im.mode == kModeDD) ? im.m1 : 0;
  int64_t ksum = 0;
  for (int i = i0; i < i1; ++i) {
    int64_t ki = k[i];
    const int64_t rem = off[i];
    if (R > 0 && rem >= 0) {
      if (rem > tau) {
        ki += 1;
      } else if (rem == tau) {
        if (rank < need) ki += 1;
        rank += 1;
      }
    }
    ki += add;
    k[i] = (int32_t)ki;
    ksum += ki;
  }
  int64_t base = group_exclusive_scan(ksum, sh64) + im.meas_off;
  for (int i = i0; i < i1; ++i) {
    off[i] = base;
    base += k[i];
  }
}

// The apportionment over a histogram of the weights, for images of more than
// 8192 blocks.  Every step of k_apportion_reg depends on a block only through
// its weight, except the tie order among equal remainders, so the cap loop,
// the floors and the radix select run on the counts H[w] of blocks per weight
// (kApBins bins; BBV_i <= 4 n_S 255 <= 16,320 with n_S <= B / 2, and
// n_i <= m1 <= B^2 / 2, for B <= 32): the blocks fixed at the cap in one
// round are those with P w >= cap S, i.e. every open weight from
// ceil(cap S / P) up, so the open blocks are always the weights below a
// threshold.  Two passes over the blocks in index order then give the tie
// ranks and the final shares and offsets.  Remainders are kept in int32,
// which holds S for images of up to kApHistMaxBlocks blocks.
constexpr int kApBins = 16384;
constexpr int kApHistMaxBlocks = 131072;
// Images of more than kApTailMinBlocks blocks leave the passes over their
// blocks to workgroups of their own, one per span of blocks (kApSpans spans
// per image):
// k_apportion_hist_count adds the spans' weight counts into the image's slot
// (kept zero between calls: the plan zeroes it, the histogram kernel clears
// it after reading), the histogram kernel writes back each weight's floor
// and remainder and the scalars of the tie rule, and k_apportion_hist_spans
// and k_apportion_hist_tail give the shares and offsets.  Slot layout (int32
// units): floors [kApBins], remainders [kApBins], counts [kApBins], then
// int64: tau, need, R > 0, cap, the added m1, the span, the largest weight
// (int32, kept zero between calls as the counts), 1 spare, each span's
// ties [kApSpans] and each span's sum of shares before the tie rule
// [kApSpans].
constexpr int kApTailMinBlocks = 8192;
constexpr int kApSpans = 64;  // one per lane in k_apportion_hist_tail's scan over spans
static_assert(kApSpans == 64, "k_apportion_hist_tail scans the spans one per lane");
constexpr int kApSlotInts = 3 * kApBins + 2 * (8 + 2 * kApSpans);
constexpr int kApSlotMeta = 3 * kApBins;  // int32 offset of the int64 part
constexpr int kApSlotWmax = 6;            // its int64 entry of the largest weight

// Sums (or exclusive prefix sums in thread order) of two values over the
// workgroup, with one pair of barriers for both.
template <int NW>
__device__ __forceinline__ void group_sum2(int64_t& a, int64_t& b, int64_t* sa, int64_t* sb) {
  a = wave_sum_t(a);
  b = wave_sum_t(b);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    sa[w] = a;
    sb[w] = b;
  }
  __syncthreads();
  a = 0;
  b = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    a += sa[i];
    b += sb[i];
  }
}

template <int NW>
__device__ __forceinline__ void group_exclusive_scan2(int64_t& a, int64_t& b, int64_t* sa, int64_t* sb) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int64_t ia = a, ib = b;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t ua = __shfl_up(ia, o, 64), ub = __shfl_up(ib, o, 64);
    if (lane >= o) {
      ia += ua;
      ib += ub;
    }
  }
  __syncthreads();
  if (lane == 63) {
    sa[w] = ia;
    sb[w] = ib;
  }
  __syncthreads();
  int64_t ba = 0, bb = 0;
  for (int i = 0; i < w; ++i) {
    ba += sa[i];
    bb += sb[i];
  }
  a = ba + ia - a;
  b = bb + ib - b;
}

// One pass of the workgroup radix select after its histogram is complete:
// the first wavefront reads the 256 bins (lane l: bins 255 - 4l .. 252 - 4l,
// so lane order is descending bin order and one DPP scan over lanes counts
// the values above each bin), clears them for the next pass, and writes the
// selected digit and the count still needed to sel_sh.
__device__ __forceinline__ void radix_select_digit_wave(int32_t* hist, int64_t need, int64_t* sel_sh) {
  const int lane = threadIdx.x & 63;
  int32_t c[4], tot = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    c[k] = hist[255 - 4 * lane - k];
    hist[255 - 4 * lane - k] = 0;
    tot += c[k];
  }
  int64_t above = wave_incl_scan_dpp(tot) - tot;
  int sel = -1;
  int64_t nn = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t ai = above + c[k];
    if (sel < 0 && ai >= need && ai - c[k] < need) {
      sel = 255 - 4 * lane - k;
      nn = need - (ai - c[k]);
    }
    above = ai;
  }
  const uint64_t m = __ballot(sel >= 0);
  if (m == 0) {
    if (lane == 0) {
      sel_sh[0] = 0;
      sel_sh[1] = need;
    }
  } else if (lane == __ffsll((unsigned long long)m) - 1) {
    sel_sh[0] = sel;
    sel_sh[1] = nn;
  }
}

// The radix select of tau and need (8 bits a pass, from the top) over one
// wavefront's values val[j] >= 0 (negative: not taking part), each counting
// cnt[j]: tau is the value at which the count of larger values stays below
// need and with it reaches need, and need becomes the count of values equal
// to tau that take one more.  Lane l reads bins
// 255 - 4l .. 252 - 4l of the wavefront's 256-bin histogram in LDS, so lane
// order is descending bin order and one scan over lanes counts the values
// above each bin; nothing waits at a barrier.
template <int N>
__device__ __forceinline__ void wave_radix_select(const int32_t (&val)[N], const int32_t (&cnt)[N], int32_t* hist,
                                                  int64_t S, int64_t& tau, int64_t& need) {
  const int lane = threadIdx.x & 63;
  const int bits = 64 - __clzll((unsigned long long)(S - 1));
  for (int shift = ((bits + 7) / 8) * 8 - 8; shift >= 0; shift -= 8) {
#pragma unroll
    for (int k = 0; k < 4; ++k) hist[4 * lane + k] = 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const uint64_t hi_mask = (shift + 8 >= 64) ? 0ull : (~0ull << (shift + 8));
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const int64_t v = val[j];
      if (v >= 0 && ((uint64_t)v & hi_mask) == ((uint64_t)tau & hi_mask))
        atomicAdd(&hist[((uint64_t)v >> shift) & 255u], cnt[j]);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    int32_t c[4], tot = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      c[k] = hist[255 - 4 * lane - k];
      tot += c[k];
    }
    int64_t above = wave_incl_scan_dpp(tot) - tot;
    int sel = -1;
    int64_t nn = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t ai = above + c[k];
      if (sel < 0 && ai >= need && ai - c[k] < need) {
        sel = 255 - 4 * lane - k;
        nn = need - (ai - c[k]);
      }
      above = ai;
    }
    const uint64_t m = __ballot(sel >= 0);
    if (m != 0) {
      const int src = __ffsll((unsigned long long)m) - 1;
      tau |= (int64_t)__builtin_amdgcn_readlane(sel, src) << shift;
      const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)nn, src);
      const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)nn >> 32), src);
      need = (int64_t)(((uint64_t)hi << 32) | lo);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

// The passes of k_apportion_hist over the weight bins (the cap rule, each
// open weight's floor and remainder, the radix select of tau and need) on
// one wavefront, for weights that span at most kApWaveBins bins: lane l
// holds bins l + 64 j in registers, every sum is a wavefront reduction and
// nothing waits at a barrier.  The integer steps, and so the results, are
// those of the workgroup passes: REM[b] for b < nbins, the floor in H[b]
// where REM[b] >= 0, and out = {R, tau, need} (lane 0 writes it).
constexpr int kApWaveBins = 1024;
__device__ __forceinline__ void ap_bins_wave(int32_t* H, int32_t* REM, int32_t* hist, int nbins, int64_t cap,
                                             int64_t P, int64_t* out) {
  constexpr int kJ = kApWaveBins / 64;
  const int lane = threadIdx.x & 63;
  int32_t h[kJ];
#pragma unroll
  for (int j = 0; j < kJ; ++j) {
    const int b = lane + 64 * j;
    h[j] = b < nbins ? H[b] : 0;
  }
  int64_t S = 0;
  bool uniform = false;
  int wcap = nbins;
  for (;;) {
    int64_t sw = 0, na = 0;
#pragma unroll
    for (int j = 0; j < kJ; ++j) {
      const int b = lane + 64 * j;
      if (b < wcap) {
        sw += (int64_t)h[j] * b;
        na += h[j];
      }
    }
    S = wave_sum_t<int64_t>(sw);
    const int64_t A = wave_sum_t<int64_t>(na);
    if (A == 0) break;
    uniform = (S == 0);
    if (uniform) {
      S = A;
      if (P >= cap * S) {
        P -= cap * A;
        wcap = 0;
      }
      break;
    }
    if (P <= 0) break;
    const int64_t wstar = (cap * S + P - 1) / P;
    if (wstar >= wcap) break;
    int64_t nc = 0;
#pragma unroll
    for (int j = 0; j < kJ; ++j) {
      const int b = lane + 64 * j;
      if (b >= wstar && b < wcap) nc += h[j];
    }
    nc = wave_sum_t<int64_t>(nc);
    if (nc == 0) break;
    wcap = (int)wstar;
    P -= cap * nc;
  }
  int32_t rmv[kJ], qv[kJ];
  int64_t sq = 0;
#pragma unroll
  for (int j = 0; j < kJ; ++j) {
    const int b = lane + 64 * j;
    rmv[j] = -1;
    qv[j] = 0;
    if (b < wcap && h[j] > 0) {
      const int64_t pw = P * (uniform ? 1 : (int64_t)b);
      const int64_t q = floor_div_exact(pw, S);
      rmv[j] = (int32_t)(pw - q * S);
      qv[j] = (int32_t)q;
      sq += h[j] * q;
    }
  }
  const int64_t R = P - wave_sum_t<int64_t>(sq);
  int64_t tau = 0, need = R;
  if (R > 0 && S > 1) wave_radix_select<kJ>(rmv, h, hist, S, tau, need);
#pragma unroll
  for (int j = 0; j < kJ; ++j) {
    const int b = lane + 64 * j;
    if (b < nbins) {
      REM[b] = rmv[j];
      if (rmv[j] >= 0) H[b] = qv[j];
    }
  }
  if (lane == 0) {
    out[0] = R;
    out[1] = tau;
    out[2] = need;
  }
}

__global__ __launch_bounds__(1024) void k_apportion_hist(const ImgDev* __restrict__ imgs,
                                                        int32_t* __restrict__ stat_all,
                                                        int32_t* __restrict__ k_all,
                                                        int64_t* __restrict__ off_all,
                                                        int32_t* __restrict__ ap_tab) {
  constexpr int kThreads = 1024, kWaves = kThreads / 64, kPerBin = kApBins / kThreads;
  __shared__ int64_t sh64[kWaves], sh64b[kWaves];
  __shared__ int32_t hist[256];
  __shared__ int64_t sel_sh[2];
  __shared__ int32_t H[kApBins];    // blocks per weight
  __shared__ int32_t REM[kApBins];  // remainder of an open weight, -1 otherwise
  __shared__ int32_t wmax_sh;       // largest weight present
  __shared__ int64_t res_sh[3];     // R, tau, need from ap_bins_wave
  const ImgDev im = imgs[blockIdx.x];
  const int nB = im.nB;
  int32_t* wg = stat_all + im.blk_off;
  int32_t* kg = k_all + im.blk_off;
  int64_t* og = off_all + im.blk_off;
  const int tid = threadIdx.x;

  if (im.mode == kModeZZ) {
    for (int i = tid; i < nB; i += kThreads) {
      kg[i] = im.kz;
      wg[i] = 0;
      og[i] = im.meas_off + (int64_t)i * im.kz;
    }
    return;
  }

  // Histogram of the weights.  DD weights lie in [0, m1] and many blocks
  // share one: they are counted in kApRep replicas per weight (replica =
  // thread % kApRep, in REM's space, free until the floors), so that equal
  // weights in a wavefront meet at most 64 / kApRep to an LDS address, and
  // the replicas are then added into H.  BBV weights spread over up to
  // 16,320 values and go to H directly.
  constexpr int kApRep = 16;
  const bool slot = im.ap_slot >= 0;
  const bool rep = !slot && im.mode == kModeDD && (im.m1 + 1) * kApRep <= kApBins;
  if (tid == 0) wmax_sh = 0;
  int wmax = 0;
  if (slot) {
    // the counts and the largest weight k_apportion_hist_count left in the
    // slot, which is cleared for the next call
    int32_t* hc = ap_tab + (int64_t)im.ap_slot * kApSlotInts + 2 * kApBins;
    int32_t* top = (int32_t*)(ap_tab + (int64_t)im.ap_slot * kApSlotInts + kApSlotMeta) + 2 * kApSlotWmax;
    wmax = *top;
    for (int b = tid; b <= wmax; b += kThreads) {
      H[b] = hc[b];
      hc[b] = 0;
    }
    __syncthreads();
    if (tid == 0) *top = 0;
  } else {
    for (int b = tid; b < kApBins; b += kThreads) {
      H[b] = 0;
      REM[b] = 0;
    }
    __syncthreads();
#pragma unroll 8
    for (int i = tid; i < nB; i += kThreads) {
      const int w = wg[i] & (kApBins - 1);
      wmax = max(wmax, w);
      if (rep && w <= im.m1)
        atomicAdd(&REM[w * kApRep + (tid & (kApRep - 1))], 1);
      else
        atomicAdd(&H[w], 1);
    }
  }
  wmax = wave_max_i32(wmax);
  if ((tid & 63) == 0) atomicMax(&wmax_sh, wmax);
  __syncthreads();
  if (rep) {
    for (int b = tid; b <= im.m1; b += kThreads) {
      int32_t c = 0;
#pragma unroll
      for (int r = 0; r < kApRep; ++r) c += REM[b * kApRep + r];
      H[b] += c;
    }
    __syncthreads();
  }

  // every pass over the bins stops at the largest weight present
  const int nbins = wmax_sh + 1;
  const int64_t cap = im.cap;
  int64_t R, tau, need;
  if (nbins <= kApWaveBins) {
    if (tid < 64) ap_bins_wave(H, REM, hist, nbins, cap, im.pool, res_sh);
    __syncthreads();
    R = res_sh[0];
    tau = res_sh[1];
    need = res_sh[2];
  } else {
  int64_t P = im.pool;
  int64_t S = 0;
  bool uniform = false;
  int wcap = nbins;  // open weights are those below wcap
  for (;;) {
    int64_t sw = 0, na = 0;
    for (int b = tid; b < wcap; b += kThreads) {
      sw += (int64_t)H[b] * b;
      na += H[b];
    }
    group_sum2<kWaves>(sw, na, sh64, sh64b);
    S = sw;
    const int64_t A = na;
    if (A == 0) break;
    uniform = (S == 0);
    if (uniform) {
      // every open block has weight 0 and counts as weight 1
      S = A;
      if (P >= cap * S) {
        P -= cap * A;
        wcap = 0;
      }
      break;
    }
    if (P <= 0) break;
    const int64_t wstar = (cap * S + P - 1) / P;  // smallest w with P w >= cap S
    if (wstar >= wcap) break;
    int64_t nc = 0;
    for (int b = (int)wstar + tid; b < wcap; b += kThreads) nc += H[b];
    nc = group_sum<kWaves>(nc, sh64);
    if (nc == 0) break;
    wcap = (int)wstar;
    P -= cap * nc;
  }

  // floors and remainders per open weight (and the radix select's bins
  // cleared: each of its passes leaves them so)
  if (tid < 256) hist[tid] = 0;
  int64_t sq = 0;
  for (int b = tid; b < nbins; b += kThreads) {
    int32_t rm = -1;
    if (b < wcap && H[b] > 0) {
      const int64_t pw = P * (uniform ? 1 : (int64_t)b);
      const int64_t q = floor_div_exact(pw, S);
      rm = (int32_t)(pw - q * S);
      sq += H[b] * q;
    }
    REM[b] = rm;
  }
  R = P - group_sum<kWaves>(sq, sh64);

  tau = 0;
  need = R;
  if (R > 0 && S > 1) {
    const int bits = 64 - __clzll((unsigned long long)(S - 1));
    for (int shift = ((bits + 7) / 8) * 8 - 8; shift >= 0; shift -= 8) {
      const uint64_t hi_mask = (shift + 8 >= 64) ? 0ull : (~0ull << (shift + 8));
#pragma unroll
      for (int j = 0; j < kPerBin; ++j) {
        const int b = tid + kThreads * j;
        const int64_t rm = b < nbins ? REM[b] : -1;
        if (rm >= 0 && ((uint64_t)rm & hi_mask) == ((uint64_t)tau & hi_mask))
          atomicAdd(&hist[((uint64_t)rm >> shift) & 255u], H[b]);
      }
      __syncthreads();
      if (tid < 64) radix_select_digit_wave(hist, need, sel_sh);
      __syncthreads();
      tau |= (int64_t)sel_sh[0] << shift;
      need = sel_sh[1];
    }
  }

  // The floor of each open weight's share, in H (its counts are no longer
  // needed): a block's share then takes no division.
  for (int b = tid; b < nbins; b += kThreads)
    if (REM[b] >= 0) H[b] = (int32_t)floor_div_exact(P * (uniform ? 1 : (int64_t)b), S);
  __syncthreads();
  }

  if (im.ap_slot >= 0) {
    // the passes over the blocks go to k_apportion_hist_spans / _tail
    int32_t* tq = ap_tab + (int64_t)im.ap_slot * kApSlotInts;
    int32_t* tr = tq + kApBins;
    int64_t* meta = (int64_t*)(tq + kApSlotMeta);
    for (int b = tid; b < nbins; b += kThreads) {
      tq[b] = H[b];
      tr[b] = REM[b];
    }
    if (tid == 0) {
      meta[0] = tau;
      meta[1] = need;
      meta[2] = R > 0 ? 1 : 0;
      meta[3] = cap;
      meta[4] = (im.mode == kModeDD) ? im.m1 : 0;
      meta[5] = (((nB + kApSpans - 1) / kApSpans) + 63) & ~63;  // span
    }
    return;
  }

  // Blocks in index order, coalesced: wavefront v owns the range
  // [v span, v span + span) and walks it 64 blocks at a time, lane l taking
  // block base + l.  A block's share is its weight's floor, plus one for a
  // remainder above tau or for one of the first `need` remainders equal to
  // tau in index order, or the cap for a capped weight.  The first pass
  // gives each wavefront its count of remainders equal to tau and its sum of
  // shares before the tie rule, so that the wavefronts' first tie ranks and
  // first offsets follow from two scans; the second writes the shares and
  // the offsets (in-wave scans).
  const int lane = tid & 63, wave = tid >> 6;
  const int span = (((nB + kWaves - 1) / kWaves) + 63) & ~63;
  const int v0 = min(nB, wave * span), v1 = min(nB, v0 + span);
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));  // lanes under this one
  const int32_t add = (im.mode == kModeDD) ? im.m1 : 0;
  int64_t s1 = 0, neq = 0;
#pragma unroll 8
  for (int base = v0; base < v1; base += 64) {
    const int i = base + lane;
    const bool valid = i < v1;
    const int w = valid ? (wg[i] & (kApBins - 1)) : 0;
    const int32_t rm = valid ? REM[w] : -1;
    neq += __popcll(__ballot(R > 0 && rm >= 0 && rm == tau));
    if (valid) s1 += (rm >= 0 ? (int64_t)H[w] + ((R > 0 && rm > tau) ? 1 : 0) : cap) + add;
  }
  s1 = wave_sum_t<int64_t>(s1);
  // ranks: wavefronts in order (lane 0 of each holds the wave's count)
  int64_t rank = group_exclusive_scan(lane == 0 ? neq : (int64_t)0, sh64);
  rank = __shfl(rank, 0, 64);
  const int64_t extra = min(max(need - rank, (int64_t)0), neq);  // the wave's ties that take one more
  int64_t obase = group_exclusive_scan(lane == 0 ? s1 + extra : (int64_t)0, sh64);
  obase = __shfl(obase, 0, 64) + im.meas_off;
  // (the weights of eight 64-block chunks are loaded before any is used, as
  // buffer loads that need no branch: past the image they read zero)
  constexpr int kAhead = 8;
  const __amdgpu_buffer_rsrc_t rw = make_rsrc(wg, 4 * nB);
  for (int base0 = v0; base0 < v1; base0 += 64 * kAhead) {
    int32_t wv[kAhead];
#pragma unroll
    for (int u = 0; u < kAhead; ++u) {
      const int i = base0 + 64 * u + lane;
      const int32_t x = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(rw, 4u * (uint32_t)i, 0, 0);
      wv[u] = i < v1 ? (x & (kApBins - 1)) : -1;
    }
#pragma unroll
    for (int u = 0; u < kAhead; ++u) {
      const int i = base0 + 64 * u + lane;
      const bool valid = wv[u] >= 0;
      const int w = valid ? wv[u] : 0;
      const int32_t rm = valid ? REM[w] : -1;
      const bool tie = R > 0 && rm >= 0 && rm == tau;
      const uint64_t eq = __ballot(tie);
      int32_t kv = 0;
      if (valid) {
        int64_t ki = rm >= 0 ? (int64_t)H[w] + ((R > 0 && rm > tau) ? 1 : 0) : cap;
        if (tie && rank + __popcll(eq & below) < need) ki += 1;
        kv = (int32_t)(ki + add);
        kg[i] = kv;
      }
      const int32_t inc = wave_incl_scan_dpp(kv);
      if (valid) og[i] = obase + inc - kv;
      obase += __builtin_amdgcn_readlane(inc, 63);
      rank += __popcll(eq);
    }
  }
}

// The passes of k_apportion_hist over the blocks of an image with a slot,
// on many workgroups: the blocks are cut into kApSpans spans, workgroup
// L kApSpans + v taking span v of large image L with four wavefronts, a
// quarter each.  A block's share before the tie rule and whether its
// remainder ties with tau depend only on its weight (floors and remainders
// read from the slot).

struct ApSpan {
  const int32_t* wg;
  const int32_t* tq;  // floors
  const int32_t* tr;  // remainders (-1: capped)
  int64_t* meta;
  int64_t tau, need, cap;
  bool rpos;
  int32_t add;
  int v0, v1;   // the span
  int w0, w1;   // this wavefront's part
};

__device__ __forceinline__ bool ap_span_init(ApSpan& a, const ImgDev& im, const int32_t* stat_all, int32_t* ap_tab) {
  const int v = blockIdx.x % kApSpans;
  a.wg = stat_all + im.blk_off;
  a.tq = ap_tab + (int64_t)im.ap_slot * kApSlotInts;
  a.tr = a.tq + kApBins;
  a.meta = (int64_t*)(ap_tab + (int64_t)im.ap_slot * kApSlotInts + kApSlotMeta);
  a.tau = a.meta[0];
  a.need = a.meta[1];
  a.rpos = a.meta[2] != 0;
  a.cap = a.meta[3];
  a.add = (int32_t)a.meta[4];
  const int span = (int)a.meta[5];
  a.v0 = min(im.nB, v * span);
  a.v1 = min(im.nB, a.v0 + span);
  const int wave = threadIdx.x >> 6;
  const int sub = (((span + 3) / 4) + 63) & ~63;
  a.w0 = min(a.v1, a.v0 + wave * sub);
  a.w1 = min(a.v1, a.w0 + sub);
  return a.v0 < a.v1;
}

// this wavefront's sum of shares before the tie rule and its count of ties
__device__ __forceinline__ void ap_span_counts(const ApSpan& a, const ImgDev& im, int64_t& s1, int64_t& neq) {
  const int lane = threadIdx.x & 63;
  const __amdgpu_buffer_rsrc_t rw = make_rsrc(a.wg, 4 * im.nB);
  constexpr int kAhead = 4;
  s1 = 0;
  neq = 0;
  for (int base0 = a.w0; base0 < a.w1; base0 += 64 * kAhead) {
    int32_t wv[kAhead];
#pragma unroll
    for (int u = 0; u < kAhead; ++u) {
      const int i = base0 + 64 * u + lane;
      const int32_t x = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(rw, 4u * (uint32_t)i, 0, 0);
      wv[u] = i < a.w1 ? (x & (kApBins - 1)) : -1;
    }
#pragma unroll
    for (int u = 0; u < kAhead; ++u) {
      const bool valid = wv[u] >= 0;
      const int w = valid ? wv[u] : 0;
      const int32_t rm = valid ? a.tr[w] : -1;
      neq += __popcll(__ballot(a.rpos && rm >= 0 && rm == a.tau));
      if (valid) s1 += (rm >= 0 ? (int64_t)a.tq[w] + ((a.rpos && rm > a.tau) ? 1 : 0) : a.cap) + a.add;
    }
  }
  s1 = wave_sum_t<int64_t>(s1);
}

// The weight counts of span v of large image L, added into the image's slot.  They are
// counted in LDS first, DD weights (at most m1) in kApRep replicas per weight
// as in k_apportion_hist, BBV weights one bin per value; the workgroup then
// adds each weight present into the slot with one global atomic.
__global__ __launch_bounds__(256) void k_apportion_hist_count(const ImgDev* __restrict__ imgs,
                                                             const int32_t* __restrict__ large_imgs, int n_large,
                                                             const int32_t* __restrict__ stat_all,
                                                             int32_t* __restrict__ ap_tab) {
  constexpr int kApRep = 16, kMaxW = kApBins / kApRep;  // DD weights kept in replicas: below kMaxW
  __shared__ __align__(16) int32_t cnt[kApBins];
  __shared__ int32_t wmax_sh;
  const int L = blockIdx.x / kApSpans, v = blockIdx.x % kApSpans;
  if (L >= n_large) return;
  const ImgDev im = imgs[large_imgs[L]];
  const int nB = im.nB;
  const int span = (((nB + kApSpans - 1) / kApSpans) + 63) & ~63;
  const int v0 = min(nB, v * span), v1 = min(nB, v0 + span);
  if (v0 >= v1) return;
  const int32_t* wg = stat_all + im.blk_off;
  int32_t* hc = ap_tab + (int64_t)im.ap_slot * kApSlotInts + 2 * kApBins;
  const int tid = threadIdx.x;
  const bool rep = im.mode == kModeDD && im.m1 < kMaxW;
  const int nzero = rep ? (im.m1 + 1) * kApRep : kApBins;
  for (int b = 4 * tid; b < nzero; b += 4 * 256) *(int4*)&cnt[b] = make_int4(0, 0, 0, 0);
  if (tid == 0) wmax_sh = 0;
  __syncthreads();
  int wmax = 0;
#pragma unroll 8
  for (int i = v0 + tid; i < v1; i += 256) {
    const int w = wg[i] & (kApBins - 1);
    wmax = max(wmax, w);
    if (!rep)
      atomicAdd(&cnt[w], 1);
    else if (w <= im.m1)
      atomicAdd(&cnt[w * kApRep + (tid & (kApRep - 1))], 1);
    else
      atomicAdd(&hc[w], 1);  // outside DD's range: not expected
  }
  wmax = wave_max_i32(wmax);
  if ((tid & 63) == 0) atomicMax(&wmax_sh, wmax);
  __syncthreads();
  if (tid == 0)
    atomicMax((int32_t*)(ap_tab + (int64_t)im.ap_slot * kApSlotInts + kApSlotMeta) + 2 * kApSlotWmax, wmax_sh);
  const int wtop = rep ? min(wmax_sh, im.m1) : wmax_sh;
  for (int w = tid; w <= wtop; w += 256) {
    int32_t c = 0;
    if (rep) {
#pragma unroll
      for (int r = 0; r < kApRep; ++r) c += cnt[w * kApRep + r];
    } else {
      c = cnt[w];
    }
    if (c > 0) atomicAdd(&hc[w], c);
  }
}

// Span totals: meta[8 + v] = the span's ties, meta[8 + kApSpans + v] = its
// sum of shares before the tie rule.
__global__ __launch_bounds__(256) void k_apportion_hist_spans(const ImgDev* __restrict__ imgs,
                                                             const int32_t* __restrict__ large_imgs, int n_large,
                                                             const int32_t* __restrict__ stat_all,
                                                             int32_t* __restrict__ ap_tab) {
  __shared__ int64_t sh[2][4];
  const int L = blockIdx.x / kApSpans, v = blockIdx.x % kApSpans;
  if (L >= n_large) return;
  const ImgDev im = imgs[large_imgs[L]];
  ApSpan a;
  const bool any = ap_span_init(a, im, stat_all, ap_tab);
  int64_t s1 = 0, neq = 0;
  if (any) ap_span_counts(a, im, s1, neq);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[0][wave] = neq;
    sh[1][wave] = s1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a.meta[8 + v] = sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3];
    a.meta[8 + kApSpans + v] = sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3];
  }
}

// The shares and offsets of span v: its first tie rank and first offset from
// the totals of the spans before it, each wavefront's from the span's (its
// counts again, then scans), then k_apportion_hist's last pass.
__global__ __launch_bounds__(256) void k_apportion_hist_tail(const ImgDev* __restrict__ imgs,
                                                            const int32_t* __restrict__ large_imgs, int n_large,
                                                            const int32_t* __restrict__ stat_all,
                                                            int32_t* __restrict__ k_all,
                                                            int64_t* __restrict__ off_all,
                                                            int32_t* __restrict__ ap_tab) {
  __shared__ int64_t sh64[4];
  const int L = blockIdx.x / kApSpans, v = blockIdx.x % kApSpans;
  if (L >= n_large) return;
  const ImgDev im = imgs[large_imgs[L]];
  ApSpan a;
  if (!ap_span_init(a, im, stat_all, ap_tab)) return;
  // the spans before this one, lane u taking span u: ties before each span
  // (a scan of the counts, each below 2^31), its extra shares, the totals
  const int lane = threadIdx.x & 63;
  const int32_t nu = lane < v ? (int32_t)a.meta[8 + lane] : 0;
  const int64_t su = lane < v ? a.meta[8 + kApSpans + lane] : 0;
  const int32_t nu_incl = wave_incl_scan_dpp(nu);
  const int64_t xu = min(max(a.need - (int64_t)(nu_incl - nu), (int64_t)0), (int64_t)nu);
  const int64_t rank0 = __builtin_amdgcn_readlane(nu_incl, 63);
  const int64_t obase0 = im.meas_off + wave_sum_t<int64_t>(su + xu);
  int64_t s1, neq;
  ap_span_counts(a, im, s1, neq);
  int64_t rank = group_exclusive_scan(lane == 0 ? neq : (int64_t)0, sh64);
  rank = __shfl(rank, 0, 64) + rank0;
  const int64_t extra = min(max(a.need - rank, (int64_t)0), neq);
  int64_t obase = group_exclusive_scan(lane == 0 ? s1 + extra : (int64_t)0, sh64);
  obase = __shfl(obase, 0, 64) + obase0;
  int32_t* kg = k_all + im.blk_off;
  int64_t* og = off_all + im.blk_off;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const __amdgpu_buffer_rsrc_t rw = make_rsrc(a.wg, 4 * im.nB);
  constexpr int kAhead = 4;
  for (int base0 = a.w0; base0 < a.w1; base0 += 64 * kAhead) {
    int32_t wv[kAhead];
#pragma unroll
    for (int u = 0; u < kAhead; ++u) {
      const int i = base0 + 64 * u + lane;
      const int32_t x = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(rw, 4u * (uint32_t)i, 0, 0);
      wv[u] = i < a.w1 ? (x & (kApBins - 1)) : -1;
    }
#pragma unroll
    for (int u = 0; u < kAhead; ++u) {
      const int i = base0 + 64 * u + lane;
      const bool valid = wv[u] >= 0;
      const int w = valid ? wv[u] : 0;
      const int32_t rm = valid ? a.tr[w] : -1;
      const bool tie = a.rpos && rm >= 0 && rm == a.tau;
      const uint64_t eq = __ballot(tie);
      int32_t kv = 0;
      if (valid) {
        int64_t ki = rm >= 0 ? (int64_t)a.tq[w] + ((a.rpos && rm > a.tau) ? 1 : 0) : a.cap;
        if (tie && rank + __popcll(eq & below) < a.need) ki += 1;
        kv = (int32_t)(ki + a.add);
        kg[i] = kv;
      }
      const int32_t inc = wave_incl_scan_dpp(kv);
      if (valid) og[i] = obase + inc - kv;
      obase += __builtin_amdgcn_readlane(inc, 63);
      rank += __popcll(eq);
    }
  }
}

// The same apportionment with each image's blocks held in registers: thread
// t owns blocks [t kPer, t kPer + kPer), so every pass (the cap loop, the
// floors, the radix select, the ties and the offsets) works on registers and
// LDS only, and global memory is read once and written once.  For images of
// at most kThreads * kPer blocks; the steps and their results are those of
// k_apportion.
template <int kThreads>
struct ApportionLds {
  int64_t sh64[kThreads / 64];
  int64_t sh64b[kThreads / 64];
  int32_t hist[256];
  int64_t sel_sh[2];
};

template <int kThreads, int kPer>
__device__ __forceinline__ void apportion_image_reg(const ImgDev& im, int32_t* __restrict__ stat_all,
                                                    int32_t* __restrict__ k_all, int64_t* __restrict__ off_all,
                                                    ApportionLds<kThreads>& al) {
  constexpr int kWaves = kThreads / 64;
  static_assert(kThreads >= 256, "the radix select reads 256 bins, one per thread");
  int64_t* sh64 = al.sh64;
  int32_t* hist = al.hist;
  int64_t* sel_sh = al.sel_sh;
  const int nB = im.nB;
  int32_t* wg = stat_all + im.blk_off;
  int32_t* kg = k_all + im.blk_off;
  int64_t* og = off_all + im.blk_off;
  const int tid = threadIdx.x;
  const int i0 = tid * kPer;
  const int wave = tid >> 6;

  if (im.mode == kModeZZ) {
    for (int i = tid; i < nB; i += kThreads) {
      kg[i] = im.kz;
      wg[i] = 0;
      og[i] = im.meas_off + (int64_t)i * im.kz;
    }
    return;
  }

  // kv: -1 undecided, else the block's share; blocks past nB are fixed at 0
  // and carry no remainder.
  int32_t wv[kPer], kv[kPer];
  int64_t rem[kPer];
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const bool valid = i0 + j < nB;
    wv[j] = valid ? wg[i0 + j] : 0;
    kv[j] = valid ? -1 : 0;
    rem[j] = -1;
  }
  // the radix select's bins start at zero (each of its passes leaves them
  // so); barriers follow before its first pass
  if (tid < 256) hist[tid] = 0;
  const int64_t cap = im.cap;
  int64_t P = im.pool;
  int64_t S = 0;
  bool uniform = false;
  // A round's capped blocks are the drop in the open count seen by the next
  // round's sums, so the pool shrinks there (cap per block) and a round that
  // caps nothing ends the loop with the same S.
  int64_t A_prev = -1;
  for (;;) {
    int64_t sw = 0, na = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j)
      if (kv[j] < 0) {
        sw += wv[j];
        na += 1;
      }
    group_sum2<kWaves>(sw, na, sh64, al.sh64b);
    S = sw;
    const int64_t A = na;
    if (A_prev >= 0) {
      if (A == A_prev) {
        uniform = (S == 0);
        if (uniform) S = A;
        break;
      }
      P -= cap * (A_prev - A);
    }
    if (A == 0) break;
    uniform = (S == 0);
    if (uniform) S = A;
    const int64_t capS = cap * S;
#pragma unroll
    for (int j = 0; j < kPer; ++j)
      if (kv[j] < 0) {
        const int64_t wi = uniform ? 1 : (int64_t)wv[j];
        if (P * wi >= capS) kv[j] = (int32_t)cap;
      }
    A_prev = A;
  }

  int64_t sq = 0;
#pragma unroll
  for (int j = 0; j < kPer; ++j)
    if (kv[j] < 0) {
      const int64_t wi = uniform ? 1 : (int64_t)wv[j];
      const int64_t pw = P * wi;
      const int64_t q = floor_div_exact(pw, S);
      kv[j] = (int32_t)q;
      rem[j] = pw - q * S;
      sq += q;
    }
  const int64_t R = P - group_sum<kWaves>(sq, sh64);

  int64_t tau = 0, need = R;
  if (R > 0 && S > 1) {
    const int bits = 64 - __clzll((unsigned long long)(S - 1));
    for (int shift = ((bits + 7) / 8) * 8 - 8; shift >= 0; shift -= 8) {
      const uint64_t hi_mask = (shift + 8 >= 64) ? 0ull : (~0ull << (shift + 8));
#pragma unroll
      for (int j = 0; j < kPer; ++j)
        if (rem[j] >= 0 && ((uint64_t)rem[j] & hi_mask) == ((uint64_t)tau & hi_mask))
          atomicAdd(&hist[((uint64_t)rem[j] >> shift) & 255u], 1);
      __syncthreads();
      if (wave == 0) radix_select_digit_wave(hist, need, sel_sh);
      __syncthreads();
      tau |= (int64_t)sel_sh[0] << shift;
      need = sel_sh[1];
    }
  }

  // Ties with tau take one more in index order while `need` lasts.  One
  // paired scan gives each thread its first tie rank and the sum of the
  // shares before it without the tie rule; the ties before it that took one
  // more are min(need, rank) of them.
  int64_t neq = 0, ksum = 0;
  const int32_t add = (im.mode == kModeDD) ? im.m1 : 0;
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    if (R > 0 && rem[j] == tau) neq += 1;
    if (i0 + j < nB) ksum += (int64_t)kv[j] + ((R > 0 && rem[j] >= 0 && rem[j] > tau) ? 1 : 0) + add;
  }
  int64_t rank = neq, kexcl = ksum;
  group_exclusive_scan2<kWaves>(rank, kexcl, sh64, al.sh64b);
  int64_t base = kexcl + min(need, rank) + im.meas_off;
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    int64_t ki = kv[j];
    if (R > 0 && rem[j] >= 0) {
      if (rem[j] > tau) {
        ki += 1;
      } else if (rem[j] == tau) {
        if (rank < need) ki += 1;
        rank += 1;
      }
    }
    ki += add;
    kv[j] = (int32_t)ki;
  }
#pragma unroll
  for (int j = 0; j < kPer; ++j)
    if (i0 + j < nB) {
      kg[i0 + j] = kv[j];
      og[i0 + j] = base;
      base += kv[j];
    }
}

template <int kThreads, int kPer>
__global__ __launch_bounds__(kThreads) void k_apportion_reg(const ImgDev* __restrict__ imgs,
                                                            int32_t* __restrict__ stat_all,
                                                            int32_t* __restrict__ k_all,
                                                            int64_t* __restrict__ off_all) {
  __shared__ ApportionLds<kThreads> al;
  apportion_image_reg<kThreads, kPer>(imgs[blockIdx.x], stat_all, k_all, off_all, al);
}

}  // namespace abcs
