// The whole encoder of a batch in one launch: phase-1 statistics
// (BBV or DD, Section V), the per-image apportionment (eqs 22-23), sensing
// and the decoder's image, for plans whose images are all 16x16 DCT images of
// at most 1024 blocks, in float32.
//
// Each workgroup takes one work item, in one global order given by an atomic
// ticket (so the order does not depend on how the hardware dispatches the
// workgroups): first every statistics item (a group of BBV blocks, four DD
// tiles, or one ZZ image), then every sensing item (four tiles).  (A
// persistent grid looping over items was built first: the compiler keeps
// every phase's per-lane basis values live across the loop, 128 VGPRs, 4 waves
// per SIMD; one item per workgroup needs the largest phase's registers only.)  A statistics item adds the
// blocks it finished to its images' arrival counters; the workgroup whose
// addition completes an image apportions that image at once and then raises
// the image's ready flag.  A sensing wave waits for its image's flag before it
// reads the budgets.  The wait always ends: every flag it can wait on belongs
// to a statistics item with a smaller ticket, already taken by a running
// workgroup that finishes its item, and the apportionment, without waiting on
// anything.  As a guard against a broken invariant the wait gives up after
// kFusedSpinLimit polls, sets the error word and skips the tile.
//
// Memory order: the statistics and budgets are written with ordinary stores;
// a workgroup barrier orders every thread's stores before thread 0, which
// issues one agent-scope release fence before the atomic that publishes them
// (the arrival add, the ready flag).  On the reading side thread 0 watches the
// flag with relaxed loads and issues one agent-scope acquire fence before a
// barrier lets the workgroup's waves read.  An agent-scope fence on this chip
// writes back (release) or invalidates (acquire) the L2 of the XCD it runs
// on, so the kernel issues one per workgroup and handoff, never one per wave
// or per poll.
#pragma once

#include "budget_kernels.hpp"
#include "common.hpp"
#include "sense_kernels.hpp"

namespace abcs {

constexpr int kFusedMaxBlocks = kGroupThreads * 4;  // apportionment in registers, 4 blocks per thread
constexpr int kFusedSpinLimit = 1 << 22;

// Workspace words: [0] ticket, [1] error, [2, 2 + n) arrivals, [2 + n, 2 + 2n)
// ready flags.  Zero on entry (a fill kernel runs first).
__host__ __device__ constexpr int64_t fused_sync_words(int n) { return 2 + 2 * (int64_t)n; }

union FusedLds {
  EncodeLds enc;
  DDStatsLds dd;
  ApportionLds<kGroupThreads> ap;
};

__global__ __launch_bounds__(kGroupThreads, 6) void k_encode_fused(
    const ImgDev* __restrict__ imgs, int n_imgs, const Tile* __restrict__ tiles_bbv, int nt_bbv, int g_bbv,
    const Tile* __restrict__ tiles_dd, int nt_dd, int g_dd, const int32_t* __restrict__ zz_imgs, int n_zz,
    const Tile* __restrict__ tiles_enc, int nt_enc, const uint8_t* __restrict__ px, int32_t* __restrict__ k,
    int64_t* __restrict__ off, int32_t* __restrict__ stat, float* __restrict__ y, float* __restrict__ out,
    int32_t* __restrict__ sync) {
  __shared__ FusedLds u;
  __shared__ int s_item, s_nown;
  __shared__ int s_img[kTileBlocks];  // images of the item's tiles, in tile order
  __shared__ int s_cnt[kTileBlocks];  // blocks the item finished per image
  __shared__ int s_own[kTileBlocks];
  int32_t* ticket = sync;
  int32_t* err = sync + 1;
  int32_t* arrive = sync + 2;
  int32_t* ready = sync + 2 + n_imgs;
  const int g_enc = (nt_enc + kWavesPerGroup - 1) / kWavesPerGroup;
  const int n_a = g_bbv + g_dd + n_zz;
  const int total = n_a + g_enc;
  const int tid = threadIdx.x, lane = tid & 63, wave = wave_in_group();
  {
    if (tid == 0) s_item = atomicAdd(ticket, 1);
    __syncthreads();
    const int item = s_item;
    if (item >= total) return;
    if (item < n_a) {
      // ---- statistics item, then arrivals and the apportionments it completes
      if (tid < kTileBlocks) {
        s_cnt[tid] = 0;
        s_img[tid] = -1;
      }
      if (tid == 0) s_nown = 0;
      // An item's tiles are consecutive entries of one tile list (image order,
      // but the list's images need not be consecutive plan indices): the
      // slot of a tile is the number of image changes before it in the item.
      const Tile* list = nullptr;
      int t0 = 0, ntl = 0, my_tile = -1, my_n = 0;
      if (item < g_bbv) {
        const int t = item * kGroupThreads + tid;
        bbv_stats_thread(imgs, tiles_bbv, nt_bbv, px, stat, t);
        list = tiles_bbv;
        t0 = item * (kGroupThreads / kTileBlocks);
        ntl = nt_bbv;
        const int ti = t / kTileBlocks;
        if (ti < nt_bbv && (t % kTileBlocks) < tiles_bbv[ti].count) {
          my_tile = ti;
          my_n = 1;
        }
      } else if (item < g_bbv + g_dd) {
        const int grp = item - g_bbv;
        dd_stats_group<kXfDCT>(imgs, tiles_dd, nt_dd, px, stat, grp, u.dd);
        list = tiles_dd;
        t0 = grp * kWavesPerGroup;
        ntl = nt_dd;
        const int ti = t0 + wave;
        if (lane == 0 && ti < nt_dd) {
          my_tile = ti;
          my_n = tiles_dd[ti].count;
        }
      } else {
        // an L-DCT-ZZ image: its budget needs no statistic
        const int img = zz_imgs[item - g_bbv - g_dd];
        apportion_image_reg<kGroupThreads, 4>(imgs[img], stat, k, off, u.ap);
        __syncthreads();
        if (tid == 0) {
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
          __hip_atomic_store(&ready[img], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        return;
      }
      __syncthreads();  // s_cnt and s_img are cleared
      if (my_n > 0) {
        int slot = 0;
        for (int j = t0 + 1; j <= my_tile && j < ntl; ++j) slot += list[j].img != list[j - 1].img;
        s_img[slot] = list[my_tile].img;
        atomicAdd(&s_cnt[slot], my_n);
      }
      __syncthreads();  // every thread's statistics and counts precede thread 0's release
      if (tid == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        bool owns = false;
        for (int j = 0; j < kTileBlocks && s_cnt[j] > 0; ++j) {
          const int img = s_img[j];
          const int before = atomicAdd(&arrive[img], s_cnt[j]);
          if (before + s_cnt[j] == imgs[img].nB) {
            s_own[s_nown++] = img;
            owns = true;
          }
        }
        // every other workgroup's statistics of the completed images
        if (owns) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
      __syncthreads();
      const int nown = s_nown;
      for (int j = 0; j < nown; ++j) {
        const int img = s_own[j];
        apportion_image_reg<kGroupThreads, 4>(imgs[img], stat, k, off, u.ap);
        __syncthreads();
        if (tid == 0) {
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
          __hip_atomic_store(&ready[img], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    } else {
      // ---- sensing and decoding: one tile per wave, once its image is ready.
      // Thread 0 polls the ready flags of the group's images and acquires
      // once for the whole group.
      const int ti0 = (item - n_a) * kWavesPerGroup;
      const int ti = ti0 + wave;
      if (tid == 0) {
        int ok = 1, last = -1;
        for (int w = 0; w < kWavesPerGroup && ti0 + w < nt_enc && ok; ++w) {
          const int img = tiles_enc[ti0 + w].img;
          if (img == last) continue;
          last = img;
          int polls = 0;
          while (__hip_atomic_load(&ready[img], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
            if (++polls > kFusedSpinLimit) {
              atomicOr(err, 1);
              ok = 0;
              break;
            }
            __builtin_amdgcn_s_sleep(4);
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s_nown = ok;
      }
      __syncthreads();
      if (ti < nt_enc && s_nown) {
        const Tile tl = tiles_enc[ti];
        encode16_tile<kXfDCT>(imgs[tl.img], tl, px, k, off, y, out, u.enc);
      }
    }
  }
}

}  // namespace abcs
