// PSA alias-table construction on gfx950 (Lehmann, Huebschle-Schneider &
// Sanders, arXiv 2106.12270, Sec. 2.2 and Sec. 4), for one table or for a
// batch of T tables of any sizes given by CSR offsets.
//
// Pipeline, one stream, no host synchronisation or readback:
//   k_setup_*        per table: number of 4096-item tiles and of C-row
//                    sections, their prefix sums; table headers reset.
//   k_reduce_tile    per tile: double-double sum of the weights + validation.
//   k_finalize       per table: W, W/N, status (fixed combination order).
//   k_tilesum        per tile: light count, light and heavy weight sums.
//   k_tilescan       per table: exclusive prefix of its tiles' sums.
//   k_partition      per tile: stable light/heavy partition in item order;
//                    entries carry their weight (Sec. 4.2 "Weight in l and h
//                    Arrays"); prefix sums emitted every 64 entries.
//   k_split          per section boundary: lights used, heavies closed and
//                    spill after m = k*C rows (Sec. 2.2; Sec. 4.1 binary
//                    search baseline), or the learned variant.
//   k_pack           one wave per section: the sweep of Sec. 4.2 in LDS.
// A tile, section or boundary finds its table by binary search over the
// per-table prefix arrays.  Every sum is formed in a fixed order, so builds
// are bit-reproducible.  Item ids stored in the light / heavy lists and in
// the alias column are table-local.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"
#include "dd.hpp"
#include "learned.hpp"

namespace amdalias {

// Everything a build kernel needs to know about the batch.
struct Batch {
  const double *w;           // all weights, tables back to back
  const uint64_t *offsets;   // T+1 table starts, or nullptr for one table of n1 items
  uint64_t n1;
  uint64_t total;
  uint32_t T, chunk;
  alias_ws_header *hdr;      // T table headers
  uint64_t *tile_start;      // T+1
  uint64_t *sec_start;       // T+1
  uint32_t *flags;           // [0] != 0: inconsistent batch description
  uint64_t *grp;             // setup scratch
  ReducePart *tilew;
  TileSum *tsum;
  TilePrefix *tpre;
  uint32_t *l_idx, *h_idx;   // table t's lists start at offsets[t]
  double *l_w, *h_w;
  dd *agg_l, *agg_h;         // table t's prefix points start at agg_base(t)
  uint32_t *split_i, *split_j;  // table t's boundaries start at sec_start[t] + t
  dd *spill;
  int32_t *status;           // T status words
  const unsigned char *models;  // learned split: model blobs (or nullptr)
  uint64_t model_bytes, model_stride;
  uint64_t tiles_max, secs_max;
};

__device__ __forceinline__ void table_range(const Batch &B, uint32_t t, uint64_t &off,
                                            uint64_t &n) {
  if (B.offsets) {
    off = B.offsets[t];
    n = B.offsets[t + 1] - off;
  } else {
    off = 0;
    n = B.n1;
  }
}

// prefix points of table t: at least n_t/64 + 2 slots, disjoint across tables
__device__ __forceinline__ uint64_t agg_base(uint64_t off, uint32_t t) {
  return off / kAggStride + 2ull * t;
}

// largest t in [0, T) with start[t] <= x (start nondecreasing, start[T] > x)
__device__ __forceinline__ uint32_t find_table(const uint64_t *start, uint32_t T, uint64_t x) {
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

// the same over boundary indices: table t's boundaries start at sec_start[t] + t
__device__ __forceinline__ uint32_t find_table_bnd(const uint64_t *sec, uint32_t T, uint64_t x) {
  uint32_t lo = 0, hi = T;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (sec[mid] + mid <= x)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// Block reductions (fixed combination order)
// ---------------------------------------------------------------------------
__device__ __forceinline__ dd block_sum_dd(dd v, dd *s_wave /*[blockDim/64]*/) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum(v);
  if (lane == 0) s_wave[wave] = v;
  __syncthreads();
  dd t = s_wave[0];
  for (int k = 1; k < (int)(blockDim.x >> 6); ++k) t = t + s_wave[k];
  __syncthreads();
  return t;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

__device__ __forceinline__ uint64_t wave_incl_u64(uint64_t v, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t o = __shfl_up(v, d, 64);
    if (lane >= d) v += o;
  }
  return v;
}

// ---------------------------------------------------------------------------
// Setup: tiles and sections per table, their exclusive prefixes (two levels
// of kSetupGroup tables), table headers reset.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kSetupGroup) void k_setup_local(Batch B, bool single_group) {
  __shared__ uint64_t s_t[kSetupGroup / 64], s_s[kSetupGroup / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t t = blockIdx.x * kSetupGroup + threadIdx.x;
  uint64_t nt = 0, ns = 0;
  if (t < B.T) {
    uint64_t off, n;
    table_range(B, t, off, n);
    const bool ok = B.offsets ? (B.offsets[t + 1] >= B.offsets[t]) : true;
    if (!ok) atomicOr(&B.flags[0], 1u);
    const bool usable = ok && n >= 1 && n <= 0xFFFFFFFFull;
    if (usable) {
      nt = (n + kTileItems - 1) / kTileItems;
      ns = (n + B.chunk - 1) / B.chunk;
    }
    alias_ws_header h;
    h.W_hi = h.W_lo = h.avg_hi = h.avg_lo = 0.0;
    h.L = h.H = 0;
    h.sl_hi = h.sl_lo = h.sh_hi = h.sh_lo = 0.0;
    h.reserved0[0] = h.reserved0[1] = 0;
    h.status = usable ? ALIAS_OK : ALIAS_EINVAL;
    h.split_fallbacks = 0;
    h.pad[0] = h.pad[1] = h.pad[2] = h.pad[3] = 0;
    B.hdr[t] = h;
    B.status[t] = h.status;
  }
  const uint64_t it = wave_incl_u64(nt, lane), is = wave_incl_u64(ns, lane);
  if (lane == 63) {
    s_t[wave] = it;
    s_s[wave] = is;
  }
  __syncthreads();
  uint64_t ot = 0, os = 0, tt = 0, ts = 0;
  for (int k = 0; k < kSetupGroup / 64; ++k) {
    if (k < wave) {
      ot += s_t[k];
      os += s_s[k];
    }
    tt += s_t[k];
    ts += s_s[k];
  }
  if (t < B.T) {
    B.tile_start[t] = ot + it - nt;
    B.sec_start[t] = os + is - ns;
  }
  if (threadIdx.x == 0) {
    B.grp[2 * blockIdx.x] = tt;
    B.grp[2 * blockIdx.x + 1] = ts;
  }
  if (single_group && threadIdx.x == 0) {
    B.tile_start[B.T] = tt;
    B.sec_start[B.T] = ts;
    const uint64_t last = B.offsets ? B.offsets[B.T] : B.n1;
    const uint64_t first = B.offsets ? B.offsets[0] : 0;
    if (first != 0 || last != B.total || tt > B.tiles_max || ts + B.T > B.secs_max)
      atomicOr(&B.flags[0], 1u);
  }
}

// exclusive prefix over the groups; final entries; consistency checks
__global__ __launch_bounds__(kSetupGroup) void k_setup_groups(Batch B, uint32_t groups) {
  __shared__ uint64_t s_t[kSetupGroup / 64], s_s[kSetupGroup / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t g = threadIdx.x;
  const uint64_t nt = g < groups ? B.grp[2 * g] : 0, ns = g < groups ? B.grp[2 * g + 1] : 0;
  const uint64_t it = wave_incl_u64(nt, lane), is = wave_incl_u64(ns, lane);
  if (lane == 63) {
    s_t[wave] = it;
    s_s[wave] = is;
  }
  __syncthreads();
  uint64_t ot = 0, os = 0, tt = 0, ts = 0;
  for (int k = 0; k < kSetupGroup / 64; ++k) {
    if (k < wave) {
      ot += s_t[k];
      os += s_s[k];
    }
    tt += s_t[k];
    ts += s_s[k];
  }
  __syncthreads();
  if (g < groups) {
    B.grp[2 * g] = ot + it - nt;  // now the group's exclusive prefix
    B.grp[2 * g + 1] = os + is - ns;
  }
  if (g == 0) {
    B.tile_start[B.T] = tt;
    B.sec_start[B.T] = ts;
    if (B.offsets[0] != 0 || B.offsets[B.T] != B.total || tt > B.tiles_max ||
        ts + B.T > B.secs_max)
      atomicOr(&B.flags[0], 1u);
  }
}

__global__ __launch_bounds__(kSetupGroup) void k_setup_add(Batch B) {
  const uint32_t t = blockIdx.x * kSetupGroup + threadIdx.x;
  if (t >= B.T) return;
  B.tile_start[t] += B.grp[2 * blockIdx.x];
  B.sec_start[t] += B.grp[2 * blockIdx.x + 1];
}

// ---------------------------------------------------------------------------
// k_reduce_tile: dd sum of one tile's weights and the validation flag
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kTileThreads) void k_reduce_tile(Batch B) {
  __shared__ dd s_wave[kTileThreads / 64];
  __shared__ uint32_t s_t;
  __shared__ uint32_t s_bad[kTileThreads / 64];
  if (B.flags[0]) return;
  const uint64_t tile = blockIdx.x;
  if (tile >= B.tile_start[B.T]) return;
  if (threadIdx.x == 0) s_t = find_table(B.tile_start, B.T, tile);
  __syncthreads();
  const uint32_t t = s_t;
  uint64_t off, n;
  table_range(B, t, off, n);
  const uint64_t lbase = (tile - B.tile_start[t]) * kTileItems;
  dd s = dd_make(0.0, 0.0);
  uint32_t bad = 0;
#pragma unroll 4
  for (int k = 0; k < kItemsPerThread; ++k) {
    const uint64_t li = lbase + (uint64_t)k * kTileThreads + threadIdx.x;
    if (li < n) {
      const double x = B.w[off + li];
      bad |= !(x >= 0.0) | (x == INFINITY);
      s = add_d(s, x);
    }
  }
  bad = __any(bad) ? 1u : 0u;
  if ((threadIdx.x & 63) == 0) s_bad[threadIdx.x >> 6] = bad;
  const dd tot = block_sum_dd(s, s_wave);
  if (threadIdx.x == 0) {
    ReducePart p;
    p.hi = tot.hi;
    p.lo = tot.lo;
    p.bad = s_bad[0] | s_bad[1] | s_bad[2] | s_bad[3];
    p.pad = 0;
    p.pad2 = 0.0;
    B.tilew[tile] = p;
  }
}

// ---------------------------------------------------------------------------
// k_finalize: per table W, W/N, status (one block per table)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_finalize(Batch B) {
  __shared__ dd s_wave[16];
  __shared__ uint32_t s_bad;
  const uint32_t t = blockIdx.x;
  if (B.flags[0]) {  // inconsistent batch description: every table fails, nothing is built
    if (threadIdx.x == 0) {
      B.hdr[t].status = ALIAS_EINVAL;
      B.status[t] = ALIAS_EINVAL;
    }
    return;
  }
  if (B.hdr[t].status != ALIAS_OK) return;
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  const uint64_t t0 = B.tile_start[t], t1 = B.tile_start[t + 1];
  dd s = dd_make(0.0, 0.0);
  uint32_t bad = 0;
  for (uint64_t k = t0 + threadIdx.x; k < t1; k += blockDim.x) {
    const ReducePart p = B.tilew[k];
    s = s + dd_make(p.hi, p.lo);
    bad |= p.bad;
  }
  if (bad) atomicOr(&s_bad, 1u);
  const dd W = block_sum_dd(s, s_wave);
  if (threadIdx.x == 0) {
    uint64_t off, n;
    table_range(B, t, off, n);
    const bool ok = !s_bad && (W.hi > 0.0) && (W.hi < INFINITY);
    const dd avg = ok ? div_d(W, (double)n) : dd_make(0.0, 0.0);
    alias_ws_header *h = &B.hdr[t];
    h->W_hi = W.hi;
    h->W_lo = W.lo;
    h->avg_hi = avg.hi;
    h->avg_lo = avg.lo;
    h->status = ok ? ALIAS_OK : ALIAS_EWEIGHTS;
    B.status[t] = h->status;
    const uint64_t ab = agg_base(off, t);
    B.agg_l[ab] = dd_make(0.0, 0.0);
    B.agg_h[ab] = dd_make(0.0, 0.0);
  }
}

// ---------------------------------------------------------------------------
// k_tilesum: per tile, the number of light items and the light and heavy
// weight sums
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kTileThreads) void k_tilesum(Batch B) {
  __shared__ dd s_l[kTileThreads / 64], s_h[kTileThreads / 64];
  __shared__ uint32_t s_c[kTileThreads / 64];
  __shared__ uint32_t s_t;
  if (B.flags[0]) return;
  const uint64_t tile = blockIdx.x;
  if (tile >= B.tile_start[B.T]) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) s_t = find_table(B.tile_start, B.T, tile);
  __syncthreads();
  const uint32_t t = s_t;
  if (B.hdr[t].status != ALIAS_OK) return;
  uint64_t off, n;
  table_range(B, t, off, n);
  const uint64_t lbase = (tile - B.tile_start[t]) * kTileItems;
  const dd avg = dd_make(B.hdr[t].avg_hi, B.hdr[t].avg_lo);
  dd acc_l = dd_make(0.0, 0.0), acc_h = dd_make(0.0, 0.0);
  uint32_t cnt = 0;
#pragma unroll 4
  for (int k = 0; k < kItemsPerThread; ++k) {
    const uint64_t li = lbase + (uint64_t)k * kTileThreads + tid;
    if (li < n) {
      const double x = B.w[off + li];
      const bool light = le(dd_make(x, 0.0), avg);
      dd a = light ? acc_l : acc_h;
      a = add_d(a, x);
      if (light)
        acc_l = a;
      else
        acc_h = a;
      cnt += light;
    }
  }
  acc_l = wave_sum(acc_l);
  acc_h = wave_sum(acc_h);
  cnt = wave_sum_u32(cnt);
  if (lane == 0) {
    s_l[wave] = acc_l;
    s_h[wave] = acc_h;
    s_c[wave] = cnt;
  }
  __syncthreads();
  if (tid == 0) {
    dd tl = s_l[0], th = s_h[0];
    uint32_t c = s_c[0];
    for (int k = 1; k < kTileThreads / 64; ++k) {
      tl = tl + s_l[k];
      th = th + s_h[k];
      c += s_c[k];
    }
    TileSum ts;
    ts.cnt = c;
    ts.pad = 0;
    ts.sl = tl;
    ts.sh = th;
    B.tsum[tile] = ts;
  }
}

// ---------------------------------------------------------------------------
// k_tilescan: per table (one block), exclusive prefix of its tiles' sums in
// chunks of 4 tiles per thread; table totals; the final prefix-sum points
// when a list length is a multiple of the stride.
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 1024;
constexpr int kScanPer = 4;

struct ScanVal {
  uint64_t c;
  dd l, h;
};

__device__ __forceinline__ ScanVal sv_zero() {
  ScanVal v;
  v.c = 0;
  v.l = dd_make(0.0, 0.0);
  v.h = dd_make(0.0, 0.0);
  return v;
}

__device__ __forceinline__ ScanVal sv_add(const ScanVal &a, const ScanVal &b) {
  ScanVal r;
  r.c = a.c + b.c;
  r.l = a.l + b.l;
  r.h = a.h + b.h;
  return r;
}

__device__ __forceinline__ ScanVal sv_of(const TileSum &ts) {
  ScanVal v;
  v.c = ts.cnt;
  v.l = ts.sl;
  v.h = ts.sh;
  return v;
}

// exclusive scan over a 1024-thread block; *total gets the block total
__device__ __forceinline__ ScanVal block_exscan(ScanVal v, ScanVal *s_w /*[16]*/, ScanVal *total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  ScanVal inc;
  inc.l = wave_inclusive_scan(v.l, lane);
  inc.h = wave_inclusive_scan(v.h, lane);
  inc.c = wave_incl_u64(v.c, lane);
  if (lane == 63) s_w[wave] = inc;
  ScanVal ex;
  ex.l = shfl_up(inc.l, 1);
  ex.h = shfl_up(inc.h, 1);
  ex.c = __shfl_up(inc.c, 1, 64);
  if (lane == 0) ex = sv_zero();
  __syncthreads();
  ScanVal off = sv_zero(), tot = sv_zero();
  for (int k = 0; k < kScanThreads / 64; ++k) {
    if (k < wave) off = sv_add(off, s_w[k]);
    tot = sv_add(tot, s_w[k]);
  }
  __syncthreads();
  *total = tot;
  return sv_add(off, ex);
}

__global__ __launch_bounds__(kScanThreads) void k_tilescan(Batch B) {
  __shared__ ScanVal s_w[kScanThreads / 64];
  if (B.flags[0]) return;
  const uint32_t t = blockIdx.x;
  if (B.hdr[t].status != ALIAS_OK) return;
  const uint64_t t0 = B.tile_start[t], t1 = B.tile_start[t + 1];
  ScanVal carry = sv_zero();
  for (uint64_t c0 = t0; c0 < t1; c0 += (uint64_t)kScanThreads * kScanPer) {
    const uint64_t b = c0 + (uint64_t)threadIdx.x * kScanPer;
    ScanVal mine = sv_zero();
    for (int u = 0; u < kScanPer; ++u)
      if (b + u < t1) mine = sv_add(mine, sv_of(B.tsum[b + u]));
    ScanVal tot;
    ScanVal run = sv_add(carry, block_exscan(mine, s_w, &tot));
    for (int u = 0; u < kScanPer; ++u) {
      if (b + u < t1) {
        TilePrefix p;
        p.l_before = run.c;
        p.pad = 0;
        p.pl = run.l;
        p.ph = run.h;
        B.tpre[b + u] = p;
        run = sv_add(run, sv_of(B.tsum[b + u]));
      }
    }
    carry = sv_add(carry, tot);
  }
  if (threadIdx.x == 0) {
    uint64_t off, n;
    table_range(B, t, off, n);
    const uint64_t L = carry.c, H = n - carry.c;
    alias_ws_header *h = &B.hdr[t];
    h->L = L;
    h->H = H;
    h->sl_hi = carry.l.hi;
    h->sl_lo = carry.l.lo;
    h->sh_hi = carry.h.hi;
    h->sh_lo = carry.h.lo;
    const uint64_t ab = agg_base(off, t);
    if ((L & (kAggStride - 1)) == 0) B.agg_l[ab + L / kAggStride] = carry.l;
    if ((H & (kAggStride - 1)) == 0) B.agg_h[ab + H / kAggStride] = carry.h;
  }
}

// ---------------------------------------------------------------------------
// k_partition: stable partition of one tile with known offsets
// ---------------------------------------------------------------------------
struct PartShared {
  double val[kTileItems + kTileItems / 16];  // staging (padded for the transpose)
  uint32_t idx[kTileItems];
  dd wl[4], wh[4];
  uint32_t cl[4], ch[4];
  uint32_t t;
};

__device__ __forceinline__ int spos(int i) { return i + (i >> 4); }

__global__ __launch_bounds__(kTileThreads) void k_partition(Batch B) {
  __shared__ PartShared S;
  if (B.flags[0]) return;
  const uint64_t tile = blockIdx.x;
  if (tile >= B.tile_start[B.T]) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) S.t = find_table(B.tile_start, B.T, tile);
  __syncthreads();
  const uint32_t t = S.t;
  if (B.hdr[t].status != ALIAS_OK) return;
  uint64_t off, n;
  table_range(B, t, off, n);
  const uint64_t lbase = (tile - B.tile_start[t]) * kTileItems;  // table-local first item
  const dd avg = dd_make(B.hdr[t].avg_hi, B.hdr[t].avg_lo);

  // 1. striped, coalesced load into the staging area
#pragma unroll
  for (int k = 0; k < kItemsPerThread; ++k) {
    const int e = k * kTileThreads + tid;
    const uint64_t li = lbase + e;
    S.val[spos(e)] = (li < n) ? B.w[off + li] : 0.0;
  }
  __syncthreads();

  // 2. blocked view: this thread owns items tid*16 .. tid*16+15
  double x[kItemsPerThread];
  uint32_t lmask = 0, vmask = 0;
#pragma unroll
  for (int u = 0; u < kItemsPerThread; ++u) {
    const int e = tid * kItemsPerThread + u;
    x[u] = S.val[spos(e)];
    const bool valid = lbase + e < n;
    const bool light = valid && le(dd_make(x[u], 0.0), avg);
    vmask |= (uint32_t)valid << u;
    lmask |= (uint32_t)light << u;
  }
  const uint32_t hmask = vmask & ~lmask;
  dd acc_l = dd_make(0.0, 0.0), acc_h = dd_make(0.0, 0.0);
#pragma unroll
  for (int u = 0; u < kItemsPerThread; ++u) {
    const bool light = (lmask >> u) & 1u;
    dd a = light ? acc_l : acc_h;
    a = add_d(a, ((vmask >> u) & 1u) ? x[u] : 0.0);
    if (light)
      acc_l = a;
    else
      acc_h = a;
  }
  const uint32_t nl = __popc(lmask), nh = __popc(hmask);

  // 3. block exclusive scans of the counts and sums
  uint32_t cl_inc = nl, ch_inc = nh;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t a = __shfl_up(cl_inc, d, 64), b = __shfl_up(ch_inc, d, 64);
    if (lane >= d) {
      cl_inc += a;
      ch_inc += b;
    }
  }
  dd sl_inc = wave_inclusive_scan(acc_l, lane);
  dd sh_inc = wave_inclusive_scan(acc_h, lane);
  if (lane == 63) {
    S.cl[wave] = cl_inc;
    S.ch[wave] = ch_inc;
    S.wl[wave] = sl_inc;
    S.wh[wave] = sh_inc;
  }
  __syncthreads();  // also: every thread has its x[] in registers
  uint32_t cl_off = 0, ch_off = 0, Lt = 0;
  dd sl_off = dd_make(0.0, 0.0), sh_off = dd_make(0.0, 0.0);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (k < wave) {
      cl_off += S.cl[k];
      ch_off += S.ch[k];
      sl_off = sl_off + S.wl[k];
      sh_off = sh_off + S.wh[k];
    }
    Lt += S.cl[k];
  }
  dd sl_lane = shfl_up(sl_inc, 1), sh_lane = shfl_up(sh_inc, 1);
  if (lane == 0) {
    sl_lane = dd_make(0.0, 0.0);
    sh_lane = dd_make(0.0, 0.0);
  }
  const TilePrefix tp = B.tpre[tile];
  const uint64_t l_before = tp.l_before;          // table-local
  const uint64_t h_before = lbase - l_before;     // table-local
  const dd pl_thr = tp.pl + (sl_off + sl_lane);
  const dd ph_thr = tp.ph + (sh_off + sh_lane);
  const uint64_t ab = agg_base(off, t);
  uint32_t rl = cl_off + cl_inc - nl;
  uint32_t rh = Lt + ch_off + ch_inc - nh;

  // 4. stage entries at their tile-local ranks; emit prefix sums every 64
  dd run_l = dd_make(0.0, 0.0), run_h = dd_make(0.0, 0.0);
#pragma unroll
  for (int u = 0; u < kItemsPerThread; ++u) {
    const uint32_t li = (uint32_t)(lbase + (uint64_t)tid * kItemsPerThread + u);
    if ((lmask >> u) & 1u) {
      const uint64_t g = l_before + rl;
      S.idx[rl] = li;
      S.val[rl] = x[u];
      if ((g & (kAggStride - 1)) == 0) B.agg_l[ab + g / kAggStride] = pl_thr + run_l;
      run_l = add_d(run_l, x[u]);
      ++rl;
    } else if ((hmask >> u) & 1u) {
      const uint64_t g = h_before + (rh - Lt);
      S.idx[rh] = li;
      S.val[rh] = x[u];
      if ((g & (kAggStride - 1)) == 0) B.agg_h[ab + g / kAggStride] = ph_thr + run_h;
      run_h = add_d(run_h, x[u]);
      ++rh;
    }
  }
  __syncthreads();

  // 5. coalesced write-out of both lists
  const uint32_t cnt = (uint32_t)((n - lbase < (uint64_t)kTileItems) ? n - lbase : kTileItems);
  for (uint32_t e = tid; e < cnt; e += kTileThreads) {
    if (e < Lt) {
      B.l_idx[off + l_before + e] = S.idx[e];
      B.l_w[off + l_before + e] = S.val[e];
    } else {
      B.h_idx[off + h_before + (e - Lt)] = S.idx[e];
      B.h_w[off + h_before + (e - Lt)] = S.val[e];
    }
  }
}

// ---------------------------------------------------------------------------
// Split search (Sec. 2.2: the sweep's state after m rows is the largest j
// with sigma_l[m-j] + sigma_h[j] <= m*avg; f is strictly increasing in j).
// ---------------------------------------------------------------------------
struct SplitCtx {
  const dd *agg_l, *agg_h;  // this table's prefix points
  const double *l_w, *h_w;  // this table's lists
  uint64_t L, H, m;
  dd mavg, sl_tot;
};

// P(64q): prefix sums at aggregate points (m is a multiple of 64)
__device__ __forceinline__ bool pred_q(const SplitCtx &c, uint64_t q) {
  const dd f = c.agg_l[(c.m - q * kAggStride) / kAggStride] + c.agg_h[q];
  return le(f, c.mavg);
}

// Fine phase: given the largest aggregate point q* with P true (or q* < qa
// meaning none), walk entry by entry.  Returns j and writes the spill.
__device__ __forceinline__ uint64_t split_fine(const SplitCtx &c, int64_t qstar, uint64_t qa,
                                               uint64_t jlo, uint64_t jhi, dd *spill) {
  uint64_t ja, jb;
  dd g;
  if (qstar >= (int64_t)qa) {
    ja = (uint64_t)qstar * kAggStride;
    jb = ja + (kAggStride - 1);
    g = c.agg_l[(c.m - ja) / kAggStride] + c.agg_h[qstar];
  } else {
    ja = jlo;
    jb = qa * kAggStride - 1;
    // sigma_l[m - jlo]: m - jlo is either m (jlo == 0, a multiple of 64) or L
    const dd sl = (jlo == 0) ? c.agg_l[c.m / kAggStride] : c.sl_tot;
    const uint64_t qb0 = ja / kAggStride;
    dd sh = c.agg_h[qb0];
    for (uint64_t t = qb0 * kAggStride; t < ja; ++t) sh = add_d(sh, c.h_w[t]);
    g = sl + sh;
  }
  if (jb > jhi) jb = jhi;
  // walk entry by entry; the weights are fetched 8 at a time so that one
  // memory round trip serves 8 steps
  uint64_t j = ja;
  bool stop = false;
  while (!stop && j < jb) {
    double hw[8], lw[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const bool in = j + u < jb;
      hw[u] = in ? c.h_w[j + u] : 0.0;
      lw[u] = in ? c.l_w[c.m - j - u - 1] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (stop || j >= jb) break;
      const dd g2 = add_d(add_d(g, hw[u]), -lw[u]);
      if (!le(g2, c.mavg)) {
        stop = true;
        break;
      }
      g = g2;
      ++j;
    }
  }
  *spill = (j < c.H) ? add_d(g, c.h_w[j]) - c.mavg : dd_make(0.0, 0.0);
  return j;
}

__global__ __launch_bounds__(256) void k_split(Batch B) {
  if (B.flags[0]) return;
  const uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B.sec_start[B.T] + B.T) return;
  const uint32_t t = find_table_bnd(B.sec_start, B.T, b);
  const alias_ws_header &h = B.hdr[t];
  if (h.status != ALIAS_OK) return;
  const uint64_t k = b - (B.sec_start[t] + t);  // table-local boundary
  uint64_t off, n;
  table_range(B, t, off, n);
  const SplitModel *model = nullptr;
  if (B.models) {
    model = (const SplitModel *)(B.models + (uint64_t)t * B.model_stride);
    if (!model_usable(model, B.model_bytes)) {
      // an unusable model is never read past its header; the split falls back
      if (k < B.sec_start[t + 1] - B.sec_start[t]) atomicAdd(&B.hdr[t].split_fallbacks, 1u);
      model = nullptr;
    }
  }
  const uint64_t ab = agg_base(off, t);
  SplitCtx c;
  c.agg_l = B.agg_l + ab;
  c.agg_h = B.agg_h + ab;
  c.l_w = B.l_w + off;
  c.h_w = B.h_w + off;
  c.L = h.L;
  c.H = h.H;
  c.m = (k * B.chunk < n) ? k * B.chunk : n;
  const dd avg = dd_make(h.avg_hi, h.avg_lo);
  c.sl_tot = dd_make(h.sl_hi, h.sl_lo);
  if (c.m == n) {
    B.split_i[b] = (uint32_t)c.L;
    B.split_j[b] = (uint32_t)c.H;
    B.spill[b] = dd_make(0.0, 0.0);
    return;
  }
  c.mavg = mul_d(avg, (double)c.m);
  const uint64_t jlo = c.m > c.L ? c.m - c.L : 0;
  const uint64_t jhi = c.m < c.H ? c.m : c.H;
  const uint64_t qa = (jlo + kAggStride - 1) / kAggStride;
  const int64_t qb = (int64_t)(jhi / kAggStride);
  int64_t lo = (int64_t)qa - 1, hi = qb;  // answer in [qa-1, qb]
  if (model) {
    // learned: bracket [p - eps, p + eps] around the model's prediction
    const int64_t p = learned_predict_q(model, c.m, n, c.H);
    const int64_t e = model->eps_q;
    int64_t blo = p - e, bhi = p + e;
    if (blo < lo) blo = lo;
    if (bhi > hi) bhi = hi;
    bool ok = blo <= bhi;
    if (ok && blo >= (int64_t)qa) ok = pred_q(c, (uint64_t)blo);
    if (ok && bhi < qb) ok = !pred_q(c, (uint64_t)(bhi + 1));
    if (ok) {
      lo = blo;
      hi = bhi;
    } else {
      atomicAdd(&B.hdr[t].split_fallbacks, 1u);
    }
  }
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo + 1) / 2;
    if (pred_q(c, (uint64_t)mid))
      lo = mid;
    else
      hi = mid - 1;
  }
  dd sp;
  const uint64_t j = split_fine(c, lo, qa, jlo, jhi, &sp);
  B.split_i[b] = (uint32_t)(c.m - j);
  B.split_j[b] = (uint32_t)j;
  B.spill[b] = sp;
}

// ---------------------------------------------------------------------------
// k_pack: one wave per section of C rows (Sec. 4.2).
//   1. stage the section's light and heavy entries (weight, id) in LDS with
//      coalesced loads (the paper's shared-memory pack with weights in l/h);
//   2. prefix sums every S = min(16, C/64) entries of both lists;
//   3. each lane finds its start state at local row G*lane (G = C/64) by a
//      search on those sums and a walk of fewer than S entries;
//   4. each lane sweeps its G rows in LDS: a light row records its alias, a
//      closing heavy records the light index at which it closed; the
//      residual advances by (incoming weight - W/N) either way;
//   5. heavy rows are finished in parallel: residual at closing from the
//      prefix sums, prob = residual / (W/N), alias = next heavy;
//   6. light rows are written in light (near item) order: prob = w / (W/N)
//      and the recorded alias.  Every table row is written exactly once.
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ int ppos(int e) { return e + (e >> 4); }  // padded LDS index

struct PackLds {
  uint32_t w_off, q_off, ix_off, ao_off, bytes, nq;
};

__host__ __device__ inline int pack_stride(uint32_t chunk) {
  const int G = (int)(chunk >> 6);
  return G < 16 ? G : 16;
}

__host__ __device__ inline PackLds pack_lds(uint32_t chunk) {
  PackLds p;
  const uint32_t nw = (uint32_t)ppos((int)chunk + 2) + 1;
  p.nq = chunk / (uint32_t)pack_stride(chunk) + 2;
  p.w_off = 0;
  p.q_off = (8u * nw + 15u) & ~15u;
  p.ix_off = p.q_off + 16u * 2u * p.nq;
  p.ao_off = p.ix_off + 4u * nw;
  p.bytes = (p.ao_off + 4u * nw + 15u) & ~15u;
  return p;
}

// Prefix sums every S entries of one staged list: Q[q] = sum of the first
// min(q*S, cnt) entries, for q = 0 .. C/S.  Lane t owns entries [tG, tG+G).
__device__ __forceinline__ void pack_prefix(const double *Wv, int off, int cnt, dd *Q, int G,
                                            int S, int lane) {
  const int b = lane * G;
  dd acc = dd_make(0.0, 0.0);
  dd part[2];  // partial sums at the lane's stride points (G/S <= 2)
  const int per = G / S;
  for (int u = 0; u < G; ++u) {
    if ((u % S) == 0 && (u / S) < 2) part[u / S] = acc;
    if (b + u < cnt) acc = add_d(acc, Wv[ppos(off + b + u)]);
  }
  const dd inc = wave_inclusive_scan(acc, lane);
  dd ex = shfl_up(inc, 1);
  if (lane == 0) ex = dd_make(0.0, 0.0);
  for (int k = 0; k < per && k < 2; ++k) Q[(b / S) + k] = ex + part[k];
  if (lane == 63) Q[(64 * G) / S] = inc;
}

// sigma of the first p entries of a staged list, from the stride points and
// fewer than S entries.
__device__ __forceinline__ dd pack_sigma(const double *Wv, int off, const dd *Q, int S, int p) {
  const int q = p / S;
  dd sgm = Q[q];
  for (int e = q * S; e < p; ++e) sgm = add_d(sgm, Wv[ppos(off + e)]);
  return sgm;
}

// Table output: two arrays (prob, alias) or one array of 16-byte rows.
struct TableOut {
  double *prob;
  uint32_t *alias;
  TableRow *rows;
};

template <bool kRows>
__device__ __forceinline__ void put_row(const TableOut &t, uint64_t item, double p, uint32_t a) {
  if (kRows) {
    TableRow r;
    r.prob = p;
    r.alias = a;
    r.pad = 0u;
    t.rows[item] = r;
  } else {
    t.prob[item] = p;
    t.alias[item] = a;
  }
}

template <bool kRows>
__global__ __launch_bounds__(64 * kPackWaves) void k_pack(Batch B, TableOut out) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  if (B.flags[0]) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t gsec = (uint64_t)blockIdx.x * (blockDim.x >> 6) + wave;
  if (gsec >= B.sec_start[B.T]) return;
  const uint32_t t = find_table(B.sec_start, B.T, gsec);
  const alias_ws_header &hdr = B.hdr[t];
  if (hdr.status != ALIAS_OK) return;
  const uint32_t chunk = B.chunk;
  const PackLds PLy = pack_lds(chunk);
  unsigned char *base = smem_raw + (size_t)wave * PLy.bytes;
  double *Wv = (double *)(base + PLy.w_off);
  dd *QL = (dd *)(base + PLy.q_off);
  dd *QH = QL + PLy.nq;
  uint32_t *Ix = (uint32_t *)(base + PLy.ix_off);
  uint32_t *Ao = (uint32_t *)(base + PLy.ao_off);

  uint64_t off, n;
  table_range(B, t, off, n);
  const uint64_t bnd = gsec + t;  // this section's first boundary: sec_start[t] + t + local
  const uint32_t *l_idx = B.l_idx + off, *h_idx = B.h_idx + off;
  const double *l_w = B.l_w + off, *h_w = B.h_w + off;
  const uint64_t H = hdr.H;
  const dd avg = dd_make(hdr.avg_hi, hdr.avg_lo);
  const uint64_t i0 = B.split_i[bnd], j0 = B.split_j[bnd];
  const uint64_t i1 = B.split_i[bnd + 1], j1 = B.split_j[bnd + 1];
  const int nl = (int)((int64_t)i1 - (int64_t)i0), nh = (int)((int64_t)j1 - (int64_t)j0);
  // i + j = m at every boundary, so nl + nh is the section's row count; a
  // negative part would mean inconsistent splits: report, write nothing.
  if (nl < 0 || nh < 0 || nl + nh > (int)chunk) {
    if (lane == 0) B.status[t] = ALIAS_EINTERNAL;
    return;
  }
  const Divisor dv = make_divisor(avg);
  if (j0 >= H) {  // no heavy item left: remaining lights keep their whole row
    for (int e = lane; e < nl; e += 64) {
      const uint32_t l = l_idx[i0 + e];
      put_row<kRows>(out, off + l, clamp01(quot_fast(dd_make(l_w[i0 + e], 0.0), dv)), l);
    }
    return;
  }
  const int nhl = (nh + 1 < (int)(H - j0)) ? nh + 1 : (int)(H - j0);
  const int G = (int)(chunk >> 6);  // rows per lane
  const int S = pack_stride(chunk);  // prefix-sum stride

  // 1. stage lights in slots [0, nl), heavies in [nl, nl + nhl)
  for (int e = lane; e < nl; e += 64) {
    Wv[ppos(e)] = l_w[i0 + e];
    Ix[ppos(e)] = l_idx[i0 + e];
  }
  for (int e = lane; e < nhl; e += 64) {
    Wv[ppos(nl + e)] = h_w[j0 + e];
    Ix[ppos(nl + e)] = h_idx[j0 + e];
  }
  wave_lds_sync();

  // 2. prefix sums every S entries
  pack_prefix(Wv, 0, nl, QL, G, S, lane);
  pack_prefix(Wv, nl, nhl, QH, G, S, lane);
  wave_lds_sync();

  const dd sp0 = B.spill[bnd];
  const dd Bo = sp0 - dd_make(Wv[ppos(nl)], 0.0);  // local f(i, j) + Bo - m*avg = global f - m*avg
  const int total = nl + nh;

  // 3. this lane's start state at local row m = G*lane
  int i, j;
  dd r = dd_make(0.0, 0.0);
  {
    const int m = G * lane;
    if (m >= total) {
      i = nl;
      j = nh;
    } else if (m == 0) {
      i = 0;
      j = 0;
      r = sp0;
    } else {
      const dd target = mul_d(avg, (double)m) - Bo;
      const int jlo = (m > nl) ? m - nl : 0;
      const int jhi = (m < nh) ? m : nh;
      const int qa = (jlo + S - 1) / S, qb = jhi / S;
      const int mq = m / S;
      int lo = qa - 1, hi = qb;
      while (lo < hi) {
        const int mid = lo + (hi - lo + 1) / 2;
        if (le(QL[mq - mid] + QH[mid], target))
          lo = mid;
        else
          hi = mid - 1;
      }
      int ja, jb;
      dd g;
      if (lo >= qa) {
        ja = lo * S;
        jb = ja + S - 1;
        g = QL[mq - lo] + QH[lo];
      } else {
        ja = jlo;
        jb = qa * S - 1;
        g = pack_sigma(Wv, 0, QL, S, m - jlo) + pack_sigma(Wv, nl, QH, S, jlo);
      }
      if (jb > jhi) jb = jhi;
      int jj = ja;
      while (jj < jb) {
        const dd g2 = add_d(add_d(g, Wv[ppos(nl + jj)]), -Wv[ppos(m - jj - 1)]);
        if (!le(g2, target)) break;
        g = g2;
        ++jj;
      }
      j = jj;
      i = m - jj;
      if (j0 + (uint64_t)j < H) r = (add_d(g, Wv[ppos(nl + j)]) + Bo) - mul_d(avg, (double)m);
    }
  }
  int ie = __shfl_down(i, 1, 64), je = __shfl_down(j, 1, 64);
  if (lane == 63) {
    ie = nl;
    je = nh;
  }

  // 4. the sweep: lights record their alias, closing heavies their light index
  const dd navg = -avg;
  while (i < ie || j < je) {
    const uint64_t jg = j0 + (uint64_t)j;
    const bool closing = (j < je) && (i == ie || le(r, avg));
    double x;
    if (closing) {
      Ao[ppos(nl + j)] = (uint32_t)i;
      x = (jg + 1 < H) ? Wv[ppos(nl + j + 1)] : 0.0;
    } else {
      Ao[ppos(i)] = (jg < H) ? Ix[ppos(nl + j)] : Ix[ppos(i)];
      x = Wv[ppos(i)];
    }
    r = add_fast(r, add_d(navg, x));  // residual += incoming weight - W/N
    i += closing ? 0 : 1;
    j += closing ? 1 : 0;
  }
  wave_lds_sync();

  // 5. heavy rows: residual at closing from the prefix sums
  for (int e = lane; e < nh; e += 64) {
    const int ic = (int)Ao[ppos(nl + e)];
    const dd rc = (pack_sigma(Wv, 0, QL, S, ic) + pack_sigma(Wv, nl, QH, S, e + 1) + Bo) -
                  mul_d(avg, (double)(ic + e));
    const uint32_t hh = Ix[ppos(nl + e)];
    put_row<kRows>(out, off + hh, clamp01(quot_fast(rc, dv)),
                   (j0 + (uint64_t)e + 1 < H) ? Ix[ppos(nl + e + 1)] : hh);
  }

  // 6. light rows, in light (near item) order: own share w/avg and alias
  for (int e = lane; e < nl; e += 64)
    put_row<kRows>(out, off + Ix[ppos(e)], clamp01(quot_fast(dd_make(Wv[ppos(e)], 0.0), dv)),
                   Ao[ppos(e)]);
}

__global__ void k_reset_fallbacks(Batch B) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < B.T) B.hdr[t].split_fallbacks = 0;
}

__global__ void k_clear_flags(uint32_t *flags) {
  if (threadIdx.x < 16) flags[threadIdx.x] = 0;
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

// Largest dynamic LDS allocation one block may make on the current device
// (queried once per device; the attribute query does not synchronise).
static size_t device_max_lds_per_block() {
  static size_t cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 65536;
  if (!cache[dev]) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        v <= 0)
      v = 65536;
    cache[dev] = (size_t)v;
  }
  return cache[dev];
}

static Batch make_batch(const double *d_w, const uint64_t *d_offsets, uint64_t n1, void *d_ws,
                        int32_t *d_status, const Layout &Lo, const unsigned char *models,
                        uint64_t model_bytes, uint64_t model_stride) {
  char *ws = (char *)d_ws;
  Batch B;
  B.w = d_w;
  B.offsets = d_offsets;
  B.n1 = n1;
  B.total = Lo.total;
  B.T = Lo.T;
  B.chunk = Lo.chunk;
  B.hdr = (alias_ws_header *)(ws + Lo.pub.header);
  B.tile_start = (uint64_t *)(ws + Lo.tile_start);
  B.sec_start = (uint64_t *)(ws + Lo.sec_start);
  B.flags = (uint32_t *)(ws + Lo.flags);
  B.grp = (uint64_t *)(ws + Lo.grp);
  B.tilew = (ReducePart *)(ws + Lo.tilew);
  B.tsum = (TileSum *)(ws + Lo.tilesum);
  B.tpre = (TilePrefix *)(ws + Lo.tilepre);
  B.l_idx = (uint32_t *)(ws + Lo.pub.l_idx);
  B.h_idx = (uint32_t *)(ws + Lo.pub.h_idx);
  B.l_w = (double *)(ws + Lo.pub.l_w);
  B.h_w = (double *)(ws + Lo.pub.h_w);
  B.agg_l = (dd *)(ws + Lo.pub.agg_l);
  B.agg_h = (dd *)(ws + Lo.pub.agg_h);
  B.split_i = (uint32_t *)(ws + Lo.pub.split_i);
  B.split_j = (uint32_t *)(ws + Lo.pub.split_j);
  B.spill = (dd *)(ws + Lo.pub.spill);
  B.status = d_status;
  B.models = models;
  B.model_bytes = model_bytes;
  B.model_stride = model_stride;
  B.tiles_max = Lo.tiles_max;
  B.secs_max = Lo.secs_max;
  return B;
}

static void launch_setup(const Batch &B, hipStream_t st) {
  hipLaunchKernelGGL(k_clear_flags, dim3(1), dim3(64), 0, st, B.flags);
  const uint32_t groups = (B.T + kSetupGroup - 1) / kSetupGroup;
  hipLaunchKernelGGL(k_setup_local, dim3(groups), dim3(kSetupGroup), 0, st, B, groups == 1);
  if (groups > 1) {
    hipLaunchKernelGGL(k_setup_groups, dim3(1), dim3(kSetupGroup), 0, st, B, groups);
    hipLaunchKernelGGL(k_setup_add, dim3(groups), dim3(kSetupGroup), 0, st, B);
  }
}

static void launch_split(const Batch &B, hipStream_t st) {
  const uint64_t nb = B.secs_max;  // >= section boundaries of all tables
  hipLaunchKernelGGL(k_split, dim3((uint32_t)((nb + 255) / 256)), dim3(256), 0, st, B);
}

int launch_build_batch(const double *d_w, const uint64_t *d_offsets, uint64_t n1, double *d_prob,
                       uint32_t *d_alias, TableRow *d_rows, void *d_ws, int32_t *d_status,
                       const Layout &Lo, const unsigned char *models, uint64_t model_bytes,
                       uint64_t model_stride, hipStream_t st) {
  const Batch B =
      make_batch(d_w, d_offsets, n1, d_ws, d_status, Lo, models, model_bytes, model_stride);
  const uint32_t tiles = (uint32_t)Lo.tiles_max;
  launch_setup(B, st);
  hipLaunchKernelGGL(k_reduce_tile, dim3(tiles), dim3(kTileThreads), 0, st, B);
  hipLaunchKernelGGL(k_finalize, dim3(B.T), dim3(1024), 0, st, B);
  hipLaunchKernelGGL(k_tilesum, dim3(tiles), dim3(kTileThreads), 0, st, B);
  hipLaunchKernelGGL(k_tilescan, dim3(B.T), dim3(kScanThreads), 0, st, B);
  hipLaunchKernelGGL(k_partition, dim3(tiles), dim3(kTileThreads), 0, st, B);
  launch_split(B, st);
  // one wave per section; as many waves per block as the LDS allows (<= 4)
  const size_t per_wave = pack_lds(Lo.chunk).bytes;
  const size_t max_lds = device_max_lds_per_block();
  size_t waves = max_lds / per_wave;
  if (waves > (size_t)kPackWaves) waves = kPackWaves;
  if (Lo.pack_waves && Lo.pack_waves < waves) waves = Lo.pack_waves;
  if (waves == 0) return ALIAS_EINVAL;
  TableOut out;
  out.prob = d_prob;
  out.alias = d_alias;
  out.rows = d_rows;
  const uint32_t pblocks = (uint32_t)((Lo.secs_max + waves - 1) / waves);
  if (d_rows)
    hipLaunchKernelGGL(k_pack<true>, dim3(pblocks), dim3(64 * waves), waves * per_wave, st, B, out);
  else
    hipLaunchKernelGGL(k_pack<false>, dim3(pblocks), dim3(64 * waves), waves * per_wave, st, B,
                       out);
  return hipGetLastError() == hipSuccess ? ALIAS_OK : ALIAS_EHIP;
}

int launch_build(const double *d_w, uint64_t n, double *d_prob, uint32_t *d_alias,
                 TableRow *d_rows, void *d_ws, int32_t *d_status, const Layout &Lo,
                 const SplitModel *model, uint64_t model_bytes, hipStream_t st) {
  return launch_build_batch(d_w, nullptr, n, d_prob, d_alias, d_rows, d_ws, d_status, Lo,
                            (const unsigned char *)model, model_bytes, 0, st);
}

// Recompute the splits of a finished build (binary or learned); the pack is
// not rerun.  Used to compare split methods on the same partition.
int launch_split_only(void *d_ws, const uint64_t *d_offsets, uint64_t n1, const Layout &Lo,
                      const unsigned char *models, uint64_t model_bytes, uint64_t model_stride,
                      hipStream_t st) {
  char *ws = (char *)d_ws;
  alias_ws_header *hdr = (alias_ws_header *)(ws + Lo.pub.header);
  // status words are not written by the split; point them at the headers
  Batch B = make_batch(nullptr, d_offsets, n1, d_ws, &hdr->status, Lo, models, model_bytes,
                       model_stride);
  hipLaunchKernelGGL(k_reset_fallbacks, dim3((Lo.T + 255) / 256), dim3(256), 0, st, B);
  launch_split(B, st);
  return hipGetLastError() == hipSuccess ? ALIAS_OK : ALIAS_EHIP;
}

}  // namespace amdalias
