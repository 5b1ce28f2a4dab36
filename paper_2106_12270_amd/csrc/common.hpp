// Shared constants, workspace layout and small device helpers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "alias_mi355x.h"
#include "dd.hpp"

namespace amdalias {

constexpr int kAggStride = 64;           // prefix sums kept every 64 light/heavy entries
constexpr int kTileThreads = 256;        // partition block
constexpr int kItemsPerThread = 16;
constexpr int kTileItems = kTileThreads * kItemsPerThread;  // 4096 items per tile
constexpr int kReduceThreads = 256;
constexpr int kReduceMaxBlocks = 1024;
constexpr uint32_t kDefaultChunk = 1024;
constexpr uint32_t kMinChunk = 64;
constexpr uint32_t kMaxChunk = 2048;
constexpr int kPackWaves = 4;            // sections per pack block (one wave each)
constexpr int kScanGroup = 1024;         // tiles per block of the tile scan

// One table row in the packed layout: 16 bytes, loaded and stored with a
// single 128-bit access.
struct __attribute__((aligned(16))) TableRow {
  double prob;
  uint32_t alias;
  uint32_t pad;
};

// Per-tile light count and light / heavy weight sums (4096-item tiles).
struct TileSum {
  uint32_t cnt;
  uint32_t pad;
  dd sl, sh;
};

// Exclusive prefix of TileSum over the tiles before a tile.
struct TilePrefix {
  uint64_t l_before;
  uint64_t pad;
  dd pl, ph;
};

struct ReducePart {
  double hi, lo;
  uint32_t bad;
  uint32_t pad;
  double pad2;
};

struct Layout {
  alias_ws_layout pub;
  uint64_t parts;      // ReducePart[reduce_blocks]
  uint64_t tilesum;    // TileSum per tile
  uint64_t tilepre;    // TilePrefix per tile, within its group of 1024 tiles
  uint64_t grpsum;     // TileSum per group of 1024 tiles
  uint64_t grppre;     // TilePrefix per group
  uint32_t chunk;
};

__host__ __device__ inline uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

// Computes the workspace layout; returns false for invalid arguments.
inline bool compute_layout(uint64_t n, const alias_build_opts *o, Layout *L) {
  if (n == 0 || n > 0xFFFFFFFFull) return false;
  uint32_t chunk = kDefaultChunk;
  if (o) {
    if (o->chunk_items) chunk = o->chunk_items;
    if (o->split_method > ALIAS_SPLIT_LEARNED) return false;
    for (int r = 0; r < 2; ++r)
      if (o->reserved[r]) return false;
  }
  if (chunk < kMinChunk || chunk > kMaxChunk || (chunk & (chunk - 1))) return false;
  const uint64_t tiles = (n + kTileItems - 1) / kTileItems;
  const uint64_t s = (n + chunk - 1) / chunk;
  uint64_t rb = (n + (uint64_t)kReduceThreads * 16 - 1) / ((uint64_t)kReduceThreads * 16);
  if (rb > (uint64_t)kReduceMaxBlocks) rb = kReduceMaxBlocks;
  if (rb == 0) rb = 1;
  const uint64_t nagg = n / kAggStride + 2;
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) {
    uint64_t at = off;
    off = align256(off + bytes);
    return at;
  };
  L->pub.header = take(sizeof(alias_ws_header));
  L->parts = take(rb * sizeof(ReducePart));
  const uint64_t groups = (tiles + kScanGroup - 1) / kScanGroup;
  L->tilesum = take(tiles * sizeof(TileSum));
  L->tilepre = take(tiles * sizeof(TilePrefix));
  L->grpsum = take(groups * sizeof(TileSum));
  L->grppre = take(groups * sizeof(TilePrefix));
  L->pub.l_idx = take(n * 4);
  L->pub.h_idx = take(n * 4);
  L->pub.l_w = take(n * 8);
  L->pub.h_w = take(n * 8);
  L->pub.agg_l = take(nagg * 16);
  L->pub.agg_h = take(nagg * 16);
  L->pub.split_i = take((s + 1) * 4);
  L->pub.split_j = take((s + 1) * 4);
  L->pub.spill = take((s + 1) * 16);
  L->pub.total_bytes = off;
  L->pub.sections = (uint32_t)s;
  L->pub.agg_stride = kAggStride;
  L->pub.tiles = (uint32_t)tiles;
  L->pub.reduce_blocks = (uint32_t)rb;
  L->chunk = chunk;
  return true;
}

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------

// Orders this wave's earlier LDS accesses before its later ones, across
// lanes (a compiler barrier plus a wait for outstanding LDS operations).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ dd load_dd(const dd *p) { return *p; }

}  // namespace amdalias
