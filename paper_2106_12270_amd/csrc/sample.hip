// Walker sampling with replacement (arXiv 2106.12270, Sec. 2.2 "Alias
// Tables"; Sec. 5 baseline method: each thread draws independently).
//
// Draw t: one Philox4x32-10 block, counter (t lo, t hi, table, 0), key
// (seed lo, seed hi).  Row k = floor(x * n / 2^64) (64x64 multiply-high) with
// x the first two output words; coin u = the last two words >> 11 (53 bits);
// the draw is k if u * 2^-53 < prob[k], else alias[k].  Integer and exact
// operations only, so every launch shape gives the same bits.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"
#include "philox.hpp"

namespace amdalias {

constexpr int kSampleThreads = 256;
constexpr int kSampleUnroll = 4;

__device__ __forceinline__ void draw_setup(uint64_t t, uint32_t table, uint32_t k0, uint32_t k1,
                                           uint64_t n, uint64_t &row, double &coin) {
  u32x4 c;
  c.x = (uint32_t)t;
  c.y = (uint32_t)(t >> 32);
  c.z = table;
  c.w = 0u;
  const u32x4 r = philox4x32_10(c, k0, k1);
  const uint64_t x = (uint64_t)r.x | ((uint64_t)r.y << 32);
  row = mulhi_u64_u32(x, (uint32_t)n);  // n < 2^32
  const uint64_t u = ((uint64_t)r.z | ((uint64_t)r.w << 32)) >> 11;
  coin = (double)u * 0x1p-53;
}

// Each thread handles kSampleUnroll consecutive grid strides per iteration so
// that several independent row gathers are in flight per lane.
__global__ __launch_bounds__(kSampleThreads) void k_sample(const double *__restrict__ prob,
                                                           const uint32_t *__restrict__ alias,
                                                           uint64_t n, uint64_t count, uint32_t k0,
                                                           uint32_t k1, uint64_t first,
                                                           uint32_t table,
                                                           uint32_t *__restrict__ out) {
  const uint64_t G = (uint64_t)gridDim.x * kSampleThreads;
  uint64_t q = (uint64_t)blockIdx.x * kSampleThreads + threadIdx.x;
  for (; q + (kSampleUnroll - 1) * G < count; q += kSampleUnroll * G) {
    uint64_t row[kSampleUnroll];
    double coin[kSampleUnroll], p[kSampleUnroll];
#pragma unroll
    for (int u = 0; u < kSampleUnroll; ++u) draw_setup(first + q + u * G, table, k0, k1, n, row[u], coin[u]);
#pragma unroll
    for (int u = 0; u < kSampleUnroll; ++u) p[u] = prob[row[u]];
#pragma unroll
    for (int u = 0; u < kSampleUnroll; ++u) {
      const uint32_t o = (coin[u] < p[u]) ? (uint32_t)row[u] : alias[row[u]];
      out[q + u * G] = o;
    }
  }
  for (; q < count; q += G) {
    uint64_t row;
    double coin;
    draw_setup(first + q, table, k0, k1, n, row, coin);
    const double p = prob[row];
    out[q] = (coin < p) ? (uint32_t)row : alias[row];
  }
}

// A row read that is not expected to be reused (a random gather from a
// table much larger than the caches): a non-temporal 128-bit load.
__device__ __forceinline__ TableRow load_row_stream(const TableRow *p) {
  typedef unsigned int u32v4 __attribute__((ext_vector_type(4)));
  const u32v4 v = __builtin_nontemporal_load((const u32v4 *)p);
  TableRow r;
  r.prob = __hiloint2double((int)v.y, (int)v.x);
  r.alias = v.z;
  r.pad = v.w;
  return r;
}

// The same draws from a table of 16-byte rows: one 128-bit gather per draw
// instead of one for prob and another for alias.
__global__ __launch_bounds__(kSampleThreads) void k_sample_rows(const TableRow *__restrict__ rows,
                                                                uint64_t n, uint64_t count,
                                                                uint32_t k0, uint32_t k1,
                                                                uint64_t first, uint32_t table,
                                                                uint32_t *__restrict__ out) {
  const uint64_t G = (uint64_t)gridDim.x * kSampleThreads;
  uint64_t q = (uint64_t)blockIdx.x * kSampleThreads + threadIdx.x;
  for (; q + (kSampleUnroll - 1) * G < count; q += kSampleUnroll * G) {
    uint64_t row[kSampleUnroll];
    double coin[kSampleUnroll];
    TableRow t[kSampleUnroll];
#pragma unroll
    for (int u = 0; u < kSampleUnroll; ++u) draw_setup(first + q + u * G, table, k0, k1, n, row[u], coin[u]);
#pragma unroll
    for (int u = 0; u < kSampleUnroll; ++u) t[u] = load_row_stream(&rows[row[u]]);
#pragma unroll
    for (int u = 0; u < kSampleUnroll; ++u)
      __builtin_nontemporal_store((coin[u] < t[u].prob) ? (uint32_t)row[u] : t[u].alias,
                                  &out[q + u * G]);
  }
  for (; q < count; q += G) {
    uint64_t row;
    double coin;
    draw_setup(first + q, table, k0, k1, n, row, coin);
    const TableRow t = rows[row];
    out[q] = (coin < t.prob) ? (uint32_t)row : t.alias;
  }
}

static uint32_t sample_blocks(uint64_t count) {
  uint64_t blocks = (count + kSampleThreads * 8 - 1) / (kSampleThreads * 8);
  if (blocks > 16384) blocks = 16384;
  if (blocks == 0) blocks = 1;
  return (uint32_t)blocks;
}

int launch_sample(const double *prob, const uint32_t *alias, uint64_t n, uint64_t count,
                  uint64_t seed, uint64_t first, uint32_t table, uint32_t *out, hipStream_t st) {
  if (count == 0) return ALIAS_OK;
  hipLaunchKernelGGL(k_sample, dim3(sample_blocks(count)), dim3(kSampleThreads), 0, st, prob, alias,
                     n, count, (uint32_t)seed, (uint32_t)(seed >> 32), first, table, out);
  return hipGetLastError() == hipSuccess ? ALIAS_OK : ALIAS_EHIP;
}

int launch_sample_rows(const TableRow *rows, uint64_t n, uint64_t count, uint64_t seed,
                       uint64_t first, uint32_t table, uint32_t *out, hipStream_t st) {
  if (count == 0) return ALIAS_OK;
  hipLaunchKernelGGL(k_sample_rows, dim3(sample_blocks(count)), dim3(kSampleThreads), 0, st, rows,
                     n, count, (uint32_t)seed, (uint32_t)(seed >> 32), first, table, out);
  return hipGetLastError() == hipSuccess ? ALIAS_OK : ALIAS_EHIP;
}


// ---------------------------------------------------------------------------
// Batched sampling: T tables back to back (table t owns rows
// [offsets[t], offsets[t+1])); draws [draw_off[t], draw_off[t+1]) belong to
// table t.  Draw d of table t is that table's draw q = d - draw_off[t], made
// exactly as a single-table call with first_draw 0 and table id t would make
// it; the output is the table-local item id.  Draws are handed out in
// contiguous chunks so that a block's draws mostly fall in one table whose
// rows stay in L2.
// ---------------------------------------------------------------------------
constexpr int kBatchPer = 8;  // draws per thread per chunk
constexpr int kBatchChunk = kSampleThreads * kBatchPer;

// largest t in [0, T) with start[t] <= x
__device__ __forceinline__ uint32_t find_first_le(const uint64_t *start, uint32_t T, uint64_t x) {
  uint32_t lo = 0, hi = T;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (start[mid] <= x)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

template <bool kRows>
__device__ __forceinline__ uint32_t batched_draw(const double *__restrict__ prob,
                                                 const uint32_t *__restrict__ alias,
                                                 const TableRow *__restrict__ rows, uint64_t base,
                                                 uint64_t row, double coin) {
  if (kRows) {
    const TableRow r = rows[base + row];
    return (coin < r.prob) ? (uint32_t)row : r.alias;
  }
  return (coin < prob[base + row]) ? (uint32_t)row : alias[base + row];
}

template <bool kRows>
__global__ __launch_bounds__(kSampleThreads) void k_sample_batched(
    const double *__restrict__ prob, const uint32_t *__restrict__ alias,
    const TableRow *__restrict__ rows, const uint64_t *__restrict__ offsets,
    const uint64_t *__restrict__ draw_off, uint32_t T, uint64_t total_items, uint64_t total_draws,
    uint32_t k0, uint32_t k1, uint32_t xcd_classes, uint32_t *__restrict__ out,
    int32_t *status) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const bool ok = draw_off[0] == 0 && draw_off[T] == total_draws && offsets[0] == 0 &&
                    offsets[T] == total_items;
    if (!ok) *status = ALIAS_EINVAL;
  }
  // With small tables the chunks are dealt to eight block classes (block
  // b % 8 runs on one XCD under round-robin dispatch): class c takes the
  // c-th eighth of the draws in order, so a table's draws are served by one
  // XCD and its rows are fetched into one L2 instead of several.  Large
  // tables (gathers from HBM either way) keep the plain grid stride.
  const uint64_t C = (total_draws + kBatchChunk - 1) / kBatchChunk;
  const uint64_t ncls = xcd_classes ? 8 : 1;
  const uint64_t Rg = (C + ncls - 1) / ncls;
  const uint64_t cls = blockIdx.x % ncls, nb = gridDim.x / ncls;
  const uint64_t cend = (cls + 1) * Rg < C ? (cls + 1) * Rg : C;
  for (uint64_t ch = cls * Rg + blockIdx.x / ncls; ch < cend; ch += nb) {
    const uint64_t c0 = ch * kBatchChunk;
    const uint64_t clast = (c0 + kBatchChunk < total_draws ? c0 + kBatchChunk : total_draws) - 1;
    // the chunk's first and last tables (the same for every thread of the block)
    const uint32_t tf = find_first_le(draw_off, T, c0);
    const uint32_t tl = find_first_le(draw_off, T, clast);
    if (tf == tl) {
      // one table serves the whole chunk: its bounds are read once
      const uint64_t a = offsets[tf], b = offsets[tf + 1], ds = draw_off[tf];
      const uint64_t n = b - a;
      const bool valid = !(b < a || b > total_items || n == 0 || n > 0xFFFFFFFFull || c0 < ds);
      uint64_t row[kBatchPer];
      double coin[kBatchPer];
#pragma unroll
      for (int u = 0; u < kBatchPer; ++u) {
        const uint64_t d = c0 + (uint64_t)u * kSampleThreads + threadIdx.x;
        if (valid) draw_setup(d - ds, tf, k0, k1, n, row[u], coin[u]);
      }
#pragma unroll
      for (int u = 0; u < kBatchPer; ++u) {
        const uint64_t d = c0 + (uint64_t)u * kSampleThreads + threadIdx.x;
        if (d > clast) continue;
        if (valid) {
          out[d] = batched_draw<kRows>(prob, alias, rows, a, row[u], coin[u]);
        } else {
          // an empty, oversized or out-of-range table gets no row reads
          out[d] = 0xFFFFFFFFu;
          *status = ALIAS_EINVAL;
        }
      }
      continue;
    }
    // the chunk spans several tables: each draw finds its own
    uint32_t t = tf;
#pragma unroll
    for (int u = 0; u < kBatchPer; ++u) {
      const uint64_t d = c0 + (uint64_t)u * kSampleThreads + threadIdx.x;
      if (d > clast) continue;
      while (t + 1 < T && draw_off[t + 1] <= d) ++t;
      const uint64_t a = offsets[t], b = offsets[t + 1];
      const uint64_t n = b - a;
      if (b < a || b > total_items || n == 0 || n > 0xFFFFFFFFull || d < draw_off[t]) {
        out[d] = 0xFFFFFFFFu;
        *status = ALIAS_EINVAL;
        continue;
      }
      uint64_t row;
      double coin;
      draw_setup(d - draw_off[t], t, k0, k1, n, row, coin);
      out[d] = batched_draw<kRows>(prob, alias, rows, a, row, coin);
    }
  }
}

__global__ void k_set_status(int32_t *status, int32_t v) {
  if (threadIdx.x == 0) *status = v;
}

int launch_sample_batched(const double *prob, const uint32_t *alias, const TableRow *rows,
                          const uint64_t *offsets, const uint64_t *draw_off, uint32_t T,
                          uint64_t total_items, uint64_t total_draws, uint64_t seed,
                          uint32_t *out, int32_t *status, hipStream_t st) {
  uint64_t blocks = (total_draws + kBatchChunk - 1) / kBatchChunk;
  if (blocks > 16384) blocks = 16384;
  blocks = (blocks + 7) / 8 * 8;  // a multiple of the eight block classes
  if (blocks == 0) blocks = 8;
  // block classes when the average table fits well inside one XCD's L2
  const uint32_t classes = (total_items / T) * sizeof(TableRow) <= (1u << 20) ? 1u : 0u;
  hipLaunchKernelGGL(k_set_status, dim3(1), dim3(64), 0, st, status, (int32_t)ALIAS_OK);
  if (rows)
    hipLaunchKernelGGL(k_sample_batched<true>, dim3((uint32_t)blocks), dim3(kSampleThreads), 0, st,
                       nullptr, nullptr, rows, offsets, draw_off, T, total_items, total_draws,
                       (uint32_t)seed, (uint32_t)(seed >> 32), classes, out, status);
  else
    hipLaunchKernelGGL(k_sample_batched<false>, dim3((uint32_t)blocks), dim3(kSampleThreads), 0,
                       st, prob, alias, nullptr, offsets, draw_off, T, total_items, total_draws,
                       (uint32_t)seed, (uint32_t)(seed >> 32), classes, out, status);
  return hipGetLastError() == hipSuccess ? ALIAS_OK : ALIAS_EHIP;
}


}  // namespace amdalias
