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
  row = __umul64hi(x, n);
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
    uint32_t k0, uint32_t k1, uint32_t *__restrict__ out, int32_t *status) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const bool ok = draw_off[0] == 0 && draw_off[T] == total_draws && offsets[0] == 0 &&
                    offsets[T] == total_items;
    if (!ok) *status = ALIAS_EINVAL;
  }
  for (uint64_t c0 = (uint64_t)blockIdx.x * kBatchChunk; c0 < total_draws;
       c0 += (uint64_t)gridDim.x * kBatchChunk) {
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
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(k_set_status, dim3(1), dim3(64), 0, st, status, (int32_t)ALIAS_OK);
  if (rows)
    hipLaunchKernelGGL(k_sample_batched<true>, dim3((uint32_t)blocks), dim3(kSampleThreads), 0, st,
                       nullptr, nullptr, rows, offsets, draw_off, T, total_items, total_draws,
                       (uint32_t)seed, (uint32_t)(seed >> 32), out, status);
  else
    hipLaunchKernelGGL(k_sample_batched<false>, dim3((uint32_t)blocks), dim3(kSampleThreads), 0,
                       st, prob, alias, nullptr, offsets, draw_off, T, total_items, total_draws,
                       (uint32_t)seed, (uint32_t)(seed >> 32), out, status);
  return hipGetLastError() == hipSuccess ? ALIAS_OK : ALIAS_EHIP;
}


// ---------------------------------------------------------------------------
// Sectioned sampling (Sec. 5: many draws served from one cached section of
// the table), with exact per-section counts.  Rows are grouped into
// S = ceil(n / R) sections of R = 2^log2r rows.
//   k_sec_count  the counts: `count` virtual draws, two per Philox block
//                (counter (b lo, b hi, table, 1)), each picking a row exactly
//                as a plain draw does; c_s = virtual draws landing in
//                section s (integer sums: any order gives the same counts);
//   k_sec_scan   exclusive prefix of the counts (output offsets) and of the
//                per-section numbers of work items of kSecItem draws;
//   k_sec_draw   work items: section s's draws j with counter
//                (j lo, j hi, table, 2 + 4 s), row = s R + floor(x R_s / 2^64),
//                the coin as a plain draw, written to out[C_s + j].  All draws
//                of a section read rows of one R-row range, which stays in L2.
// ---------------------------------------------------------------------------
constexpr int kSecThreads = 256;
constexpr uint32_t kSecItem = 8192;       // draws per work item
constexpr uint32_t kSecLdsHist = 16384;   // sections counted in LDS (else in global memory)

struct SecLayout {
  uint64_t counts, offsets, work, total;  // byte offsets in the workspace
  uint64_t S;
};

inline bool sec_layout(uint64_t n, uint64_t count, uint32_t log2r, SecLayout *L) {
  if (n == 0 || n > 0xFFFFFFFFull || log2r < 6 || log2r > 31 || count > (1ull << 40))
    return false;
  const uint64_t R = 1ull << log2r;
  L->S = (n + R - 1) / R;
  if (L->S > (1ull << 20)) return false;
  uint64_t off = 0;
  auto take = [&](uint64_t b) {
    uint64_t at = off;
    off = align256(off + b);
    return at;
  };
  L->counts = take(L->S * 8);
  L->offsets = take((L->S + 1) * 8);
  L->work = take((8 * ((L->S + 7) / 8) + 1) * 8);
  L->total = off;
  return true;
}

__global__ void k_sec_zero(uint64_t *c, uint64_t S) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < S) c[i] = 0;
}

__global__ __launch_bounds__(kSecThreads) void k_sec_count(uint64_t n, uint64_t count,
                                                           uint32_t log2r, uint64_t S,
                                                           uint32_t k0, uint32_t k1,
                                                           uint32_t table,
                                                           unsigned long long *counts) {
  __shared__ uint32_t hist[kSecLdsHist];
  const bool lds = S <= kSecLdsHist;
  if (lds)
    for (uint64_t i = threadIdx.x; i < S; i += kSecThreads) hist[i] = 0;
  __syncthreads();
  const uint64_t pairs = (count + 1) / 2;
  const uint64_t G = (uint64_t)gridDim.x * kSecThreads;
  for (uint64_t b = (uint64_t)blockIdx.x * kSecThreads + threadIdx.x; b < pairs; b += G) {
    u32x4 c;
    c.x = (uint32_t)b;
    c.y = (uint32_t)(b >> 32);
    c.z = table;
    c.w = 1u;
    const u32x4 r = philox4x32_10(c, k0, k1);
    const uint64_t x0 = (uint64_t)r.x | ((uint64_t)r.y << 32);
    const uint64_t x1 = (uint64_t)r.z | ((uint64_t)r.w << 32);
    const uint64_t s0 = __umul64hi(x0, n) >> log2r;
    const bool two = 2 * b + 1 < count;
    const uint64_t s1 = __umul64hi(x1, n) >> log2r;
    if (lds) {
      atomicAdd(&hist[s0], 1u);
      if (two) atomicAdd(&hist[s1], 1u);
    } else {
      atomicAdd(&counts[s0], 1ull);
      if (two) atomicAdd(&counts[s1], 1ull);
    }
  }
  if (lds) {
    __syncthreads();
    for (uint64_t i = threadIdx.x; i < S; i += kSecThreads)
      if (hist[i]) atomicAdd(&counts[i], (unsigned long long)hist[i]);
  }
}

// Sections are served per XCD class: blocks b with b % 8 == c (the
// round-robin dispatch puts them on one XCD) take the work items of the
// sections s with s % 8 == c, so the sections in flight on an XCD stay few
// and their rows stay in that XCD's L2.  Permuted section order: position
// p = c * Sc + k holds section s = 8 k + c (Sc = ceil(S / 8); s >= S is
// empty).
__device__ __forceinline__ uint64_t sec_at(uint64_t p, uint64_t Sc) {
  return (p % Sc) * 8 + p / Sc;
}

__device__ __forceinline__ uint64_t block_excl_u64(uint64_t v, uint64_t *s_w, uint64_t *tot) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint64_t inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t o = __shfl_up(inc, d, 64);
    if (lane >= d) inc += o;
  }
  if (lane == 63) s_w[wave] = inc;
  __syncthreads();
  uint64_t pre = 0, t = 0;
  for (int k = 0; k < 16; ++k) {
    if (k < wave) pre += s_w[k];
    t += s_w[k];
  }
  __syncthreads();
  *tot = t;
  return pre + inc - v;
}

// one block: exclusive prefix of the counts in section order -> offsets[0..S];
// of the work items in the permuted order -> work[0..8 Sc]
__global__ __launch_bounds__(1024) void k_sec_scan(const uint64_t *counts, uint64_t S,
                                                   uint64_t *offsets, uint64_t *work) {
  __shared__ uint64_t s_w[16];
  uint64_t carry = 0;
  for (uint64_t base = 0; base < S; base += 1024) {
    const uint64_t i = base + threadIdx.x;
    const uint64_t c = i < S ? counts[i] : 0;
    uint64_t tot;
    const uint64_t ex = block_excl_u64(c, s_w, &tot);
    if (i < S) offsets[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) offsets[S] = carry;
  const uint64_t Sc = (S + 7) / 8, P = 8 * Sc;
  carry = 0;
  for (uint64_t base = 0; base < P; base += 1024) {
    const uint64_t p = base + threadIdx.x;
    uint64_t wi = 0;
    if (p < P) {
      const uint64_t sec = sec_at(p, Sc);
      if (sec < S) wi = (counts[sec] + kSecItem - 1) / kSecItem;
    }
    uint64_t tot;
    const uint64_t ex = block_excl_u64(wi, s_w, &tot);
    if (p < P) work[p] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) work[P] = carry;
}

// largest p in [lo, hi) with work[p] <= w
__device__ __forceinline__ uint64_t item_pos(const uint64_t *work, uint64_t lo, uint64_t hi,
                                             uint64_t w) {
  while (hi - lo > 1) {
    const uint64_t mid = (lo + hi) >> 1;
    if (work[mid] <= w)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

template <bool kRows>
__global__ __launch_bounds__(kSecThreads) void k_sec_draw(
    const double *__restrict__ prob, const uint32_t *__restrict__ alias,
    const TableRow *__restrict__ rows, uint64_t n, uint32_t log2r, uint64_t S,
    const uint64_t *__restrict__ counts, const uint64_t *__restrict__ offsets,
    const uint64_t *__restrict__ work, uint32_t k0, uint32_t k1, uint32_t table,
    uint32_t *__restrict__ out) {
  const uint64_t Sc = (S + 7) / 8;
  const uint64_t cls = blockIdx.x % 8, nb = gridDim.x / 8;
  const uint64_t p0 = cls * Sc, p1 = p0 + Sc;
  const uint64_t wend = work[p1];
  for (uint64_t w = work[p0] + blockIdx.x / 8; w < wend; w += nb) {
    const uint64_t pp = item_pos(work, p0, p1, w);
    const uint64_t s = sec_at(pp, Sc);
    const uint64_t ws = work[pp];
    const uint64_t c = counts[s];
    const uint64_t j0 = (w - ws) * kSecItem;
    const uint64_t j1 = (j0 + kSecItem < c) ? j0 + kSecItem : c;
    const uint64_t base = s << log2r;
    const uint64_t Rs = (n - base < (1ull << log2r)) ? n - base : (1ull << log2r);
    const uint64_t o = offsets[s];
    constexpr int U = kSecItem / kSecThreads;  // draws per thread
    uint64_t row[U];
    double coin[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t j = j0 + (uint64_t)u * kSecThreads + threadIdx.x;
      u32x4 cc;
      cc.x = (uint32_t)j;
      cc.y = (uint32_t)(j >> 32);
      cc.z = table;
      cc.w = 2u + 4u * (uint32_t)s;
      const u32x4 r = philox4x32_10(cc, k0, k1);
      const uint64_t x = (uint64_t)r.x | ((uint64_t)r.y << 32);
      row[u] = base + __umul64hi(x, Rs);
      const uint64_t uu = ((uint64_t)r.z | ((uint64_t)r.w << 32)) >> 11;
      coin[u] = (double)uu * 0x1p-53;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t j = j0 + (uint64_t)u * kSecThreads + threadIdx.x;
      if (j < j1) {
        uint32_t v;
        if (kRows) {
          const TableRow t = rows[row[u]];
          v = (coin[u] < t.prob) ? (uint32_t)row[u] : t.alias;
        } else {
          v = (coin[u] < prob[row[u]]) ? (uint32_t)row[u] : alias[row[u]];
        }
        out[o + j] = v;
      }
    }
  }
}

size_t sec_workspace_bytes(uint64_t n, uint64_t count, uint32_t log2r) {
  SecLayout L;
  if (!sec_layout(n, count, log2r, &L)) return 0;
  return (size_t)L.total;
}

int launch_sample_sectioned(const double *prob, const uint32_t *alias, const TableRow *rows,
                            uint64_t n, uint64_t count, uint64_t seed, uint32_t table,
                            uint32_t log2r, uint32_t *out, uint64_t *d_counts, void *d_ws,
                            size_t ws_bytes, hipStream_t st) {
  SecLayout L;
  if (!sec_layout(n, count, log2r, &L)) return ALIAS_EINVAL;
  if (ws_bytes < L.total) return ALIAS_EWORKSPACE;
  char *ws = (char *)d_ws;
  uint64_t *counts = d_counts ? d_counts : (uint64_t *)(ws + L.counts);
  uint64_t *offsets = (uint64_t *)(ws + L.offsets), *work = (uint64_t *)(ws + L.work);
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  hipLaunchKernelGGL(k_sec_zero, dim3((uint32_t)((L.S + 255) / 256)), dim3(256), 0, st, counts,
                     L.S);
  uint64_t cb = ((count + 1) / 2 + kSecThreads * 16 - 1) / (kSecThreads * 16);
  if (cb > 2048) cb = 2048;
  if (cb == 0) cb = 1;
  hipLaunchKernelGGL(k_sec_count, dim3((uint32_t)cb), dim3(kSecThreads), 0, st, n, count, log2r,
                     L.S, k0, k1, table, (unsigned long long *)counts);
  hipLaunchKernelGGL(k_sec_scan, dim3(1), dim3(1024), 0, st, counts, L.S, offsets, work);
  // Few blocks (one per CU), each drawing kSecItem samples per work item:
  // the fewer work items in flight, the fewer sections whose rows compete
  // for an XCD's L2 (measured best on the 2^27-row table against 4x-16x
  // more blocks or larger blocks).
  uint64_t db = count / kSecItem + L.S;
  if (db > 256) db = 256;
  db = (db + 7) / 8 * 8;  // eight XCD classes of blocks
  if (db == 0) db = 8;
  if (rows)
    hipLaunchKernelGGL(k_sec_draw<true>, dim3((uint32_t)db), dim3(kSecThreads), 0, st, nullptr,
                       nullptr, rows, n, log2r, L.S, counts, offsets, work, k0, k1, table, out);
  else
    hipLaunchKernelGGL(k_sec_draw<false>, dim3((uint32_t)db), dim3(kSecThreads), 0, st, prob,
                       alias, nullptr, n, log2r, L.S, counts, offsets, work, k0, k1, table, out);
  return hipGetLastError() == hipSuccess ? ALIAS_OK : ALIAS_EHIP;
}

}  // namespace amdalias
