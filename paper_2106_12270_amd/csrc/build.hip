// PSA alias-table construction on gfx950 (Lehmann, Huebschle-Schneider &
// Sanders, arXiv 2106.12270, Sec. 2.2 and Sec. 4).
//
// Pipeline, one stream, no host synchronisation or readback:
//   k_reduce    per-block double-double sums of the weights + validation.
//   k_finalize  W, W/N, status; resets the counters the later kernels use.
//   k_tilesum   per 4096-item tile: light count, light and heavy weight sums.
//   k_tilescan, k_groupscan  exclusive prefix over the tiles in two levels.
//   k_partition stable light/heavy partition in item order with the tile
//               offsets known; entries carry their weight (Sec. 4.2 "Weight
//               in l and h Arrays"); prefix sums of the light / heavy weights
//               emitted every 64 entries.
//   Every sum is formed in a fixed order, so builds are bit-reproducible.
//   k_split     state (lights used, heavies closed, spill) after m_k = k*C
//               rows for every section boundary (Sec. 2.2; Sec. 4.1 binary
//               search baseline), or the learned variant.
//   k_pack      one wave per section: stages the section's prefix sums in
//               LDS, splits the section among the 64 lanes there, and each
//               lane runs the sequential sweep over its rows (Sec. 4.2).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"
#include "dd.hpp"
#include "learned.hpp"

namespace amdalias {

// ---------------------------------------------------------------------------
// Block reductions and scans (fixed combination order: results never depend
// on timing, so builds are bit-reproducible)
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

// ---------------------------------------------------------------------------
// k_reduce: per-block dd partial sums of w and the validation flag
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kReduceThreads) void k_reduce(const double *__restrict__ w, uint64_t n,
                                                           ReducePart *__restrict__ parts) {
  __shared__ dd s_wave[kReduceThreads / 64];
  __shared__ uint32_t s_bad;
  const uint64_t G = (uint64_t)gridDim.x * kReduceThreads;
  const uint64_t g = (uint64_t)blockIdx.x * kReduceThreads + threadIdx.x;
  if (threadIdx.x == 0) s_bad = 0;
  dd s = dd_make(0.0, 0.0);
  uint32_t bad = 0;
  uint64_t i = g;
  for (; i + 3 * G < n; i += 4 * G) {
    double x0 = w[i], x1 = w[i + G], x2 = w[i + 2 * G], x3 = w[i + 3 * G];
    bad |= !(x0 >= 0.0) | (x0 == INFINITY);
    bad |= !(x1 >= 0.0) | (x1 == INFINITY);
    bad |= !(x2 >= 0.0) | (x2 == INFINITY);
    bad |= !(x3 >= 0.0) | (x3 == INFINITY);
    s = add_d(add_d(add_d(add_d(s, x0), x1), x2), x3);
  }
  for (; i < n; i += G) {
    double x = w[i];
    bad |= !(x >= 0.0) | (x == INFINITY);
    s = add_d(s, x);
  }
  __syncthreads();
  if (bad) atomicOr(&s_bad, 1u);
  dd tot = block_sum_dd(s, s_wave);
  if (threadIdx.x == 0) {
    parts[blockIdx.x].hi = tot.hi;
    parts[blockIdx.x].lo = tot.lo;
    parts[blockIdx.x].bad = s_bad;
  }
}

// ---------------------------------------------------------------------------
// k_finalize: W, W/N, status, counters (one block)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_finalize(const ReducePart *__restrict__ parts, uint32_t nparts,
                                                  uint64_t n, alias_ws_header *hdr, dd *agg_l,
                                                  dd *agg_h, int32_t *d_status) {
  __shared__ dd s_wave[4];
  __shared__ uint32_t s_bad;
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  dd s = dd_make(0.0, 0.0);
  uint32_t bad = 0;
  for (uint32_t k = threadIdx.x; k < nparts; k += blockDim.x) {
    s = s + dd_make(parts[k].hi, parts[k].lo);
    bad |= parts[k].bad;
  }
  if (bad) atomicOr(&s_bad, 1u);
  dd W = block_sum_dd(s, s_wave);
  if (threadIdx.x == 0) {
    bool ok = !s_bad && (W.hi > 0.0) && (W.hi < INFINITY);
    dd avg = ok ? div_d(W, (double)n) : dd_make(0.0, 0.0);
    hdr->W_hi = W.hi;
    hdr->W_lo = W.lo;
    hdr->avg_hi = avg.hi;
    hdr->avg_lo = avg.lo;
    hdr->L = 0;
    hdr->H = 0;
    hdr->sl_hi = hdr->sl_lo = hdr->sh_hi = hdr->sh_lo = 0.0;
    hdr->reserved0[0] = hdr->reserved0[1] = 0;
    hdr->status = ok ? ALIAS_OK : ALIAS_EWEIGHTS;
    hdr->split_fallbacks = 0;
    agg_l[0] = dd_make(0.0, 0.0);
    agg_h[0] = dd_make(0.0, 0.0);
    *d_status = ok ? ALIAS_OK : ALIAS_EWEIGHTS;
  }
}

// ---------------------------------------------------------------------------
// k_tilesum: per tile of 4096 items, the number of light items and the light
// and heavy weight sums.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kTileThreads) void k_tilesum(const double *__restrict__ w, uint64_t n,
                                                          const alias_ws_header *hdr,
                                                          TileSum *__restrict__ sums) {
  __shared__ dd s_l[kTileThreads / 64], s_h[kTileThreads / 64];
  __shared__ uint32_t s_c[kTileThreads / 64];
  if (hdr->status != ALIAS_OK) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t base = (uint64_t)blockIdx.x * kTileItems;
  const dd avg = dd_make(hdr->avg_hi, hdr->avg_lo);
  dd acc_l = dd_make(0.0, 0.0), acc_h = dd_make(0.0, 0.0);
  uint32_t cnt = 0;
#pragma unroll 4
  for (int k = 0; k < kItemsPerThread; ++k) {
    const uint64_t gi = base + (uint64_t)k * kTileThreads + tid;
    if (gi < n) {
      const double x = w[gi];
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
    TileSum t;
    t.cnt = c;
    t.pad = 0;
    t.sl = tl;
    t.sh = th;
    sums[blockIdx.x] = t;
  }
}

// ---------------------------------------------------------------------------
// Tile scan in two levels, fixed combination order throughout:
//   k_tilescan   one block per group of 1024 tiles: exclusive prefix of the
//                tile sums within the group, and the group total;
//   k_groupscan  one block: exclusive prefix over the groups, the totals, and
//                the final prefix-sum points when a list length is a
//                multiple of the aggregate stride.
// ---------------------------------------------------------------------------
struct ScanVal {
  uint64_t c;
  dd l, h;
};

__device__ __forceinline__ ScanVal sv_add(const ScanVal &a, const ScanVal &b) {
  ScanVal r;
  r.c = a.c + b.c;
  r.l = a.l + b.l;
  r.h = a.h + b.h;
  return r;
}

// exclusive scan over a 1024-thread block; *total gets the block total
__device__ __forceinline__ ScanVal block_exscan_1024(ScanVal v, ScanVal *s_w /*[16]*/,
                                                     ScanVal *total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  ScanVal inc;
  inc.l = wave_inclusive_scan(v.l, lane);
  inc.h = wave_inclusive_scan(v.h, lane);
  inc.c = v.c;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint64_t o = __shfl_up(inc.c, d, 64);
    if (lane >= d) inc.c += o;
  }
  if (lane == 63) s_w[wave] = inc;
  ScanVal ex;
  ex.l = shfl_up(inc.l, 1);
  ex.h = shfl_up(inc.h, 1);
  ex.c = __shfl_up(inc.c, 1, 64);
  if (lane == 0) {
    ex.c = 0;
    ex.l = dd_make(0.0, 0.0);
    ex.h = dd_make(0.0, 0.0);
  }
  __syncthreads();
  ScanVal off;
  off.c = 0;
  off.l = dd_make(0.0, 0.0);
  off.h = dd_make(0.0, 0.0);
  ScanVal tot = off;
  for (int k = 0; k < 16; ++k) {
    if (k < wave) off = sv_add(off, s_w[k]);
    tot = sv_add(tot, s_w[k]);
  }
  *total = tot;
  return sv_add(off, ex);
}

__global__ __launch_bounds__(kScanGroup) void k_tilescan(const TileSum *__restrict__ sums,
                                                         uint32_t tiles, const alias_ws_header *hdr,
                                                         TilePrefix *__restrict__ pre,
                                                         TileSum *__restrict__ grp) {
  __shared__ ScanVal s_w[16];
  if (hdr->status != ALIAS_OK) return;
  const uint32_t t = blockIdx.x * kScanGroup + threadIdx.x;
  ScanVal v;
  v.c = 0;
  v.l = dd_make(0.0, 0.0);
  v.h = dd_make(0.0, 0.0);
  if (t < tiles) {
    const TileSum ts = sums[t];
    v.c = ts.cnt;
    v.l = ts.sl;
    v.h = ts.sh;
  }
  ScanVal tot;
  const ScanVal ex = block_exscan_1024(v, s_w, &tot);
  if (t < tiles) {
    TilePrefix p;
    p.l_before = ex.c;
    p.pad = 0;
    p.pl = ex.l;
    p.ph = ex.h;
    pre[t] = p;
  }
  if (threadIdx.x == 0) {
    TileSum g;
    g.cnt = (uint32_t)tot.c;
    g.pad = 0;
    g.sl = tot.l;
    g.sh = tot.h;
    grp[blockIdx.x] = g;
  }
}

__global__ __launch_bounds__(kScanGroup) void k_groupscan(const TileSum *__restrict__ grp,
                                                          uint32_t groups, uint64_t n,
                                                          alias_ws_header *hdr,
                                                          TilePrefix *__restrict__ gpre,
                                                          dd *__restrict__ agg_l,
                                                          dd *__restrict__ agg_h) {
  __shared__ ScanVal s_w[16];
  if (hdr->status != ALIAS_OK) return;
  const uint32_t g = threadIdx.x;
  ScanVal v;
  v.c = 0;
  v.l = dd_make(0.0, 0.0);
  v.h = dd_make(0.0, 0.0);
  if (g < groups) {
    const TileSum ts = grp[g];
    v.c = ts.cnt;
    v.l = ts.sl;
    v.h = ts.sh;
  }
  ScanVal tot;
  const ScanVal ex = block_exscan_1024(v, s_w, &tot);
  if (g < groups) {
    TilePrefix p;
    p.l_before = ex.c;
    p.pad = 0;
    p.pl = ex.l;
    p.ph = ex.h;
    gpre[g] = p;
  }
  if (threadIdx.x == 0) {
    const uint64_t L = tot.c, H = n - tot.c;
    hdr->L = L;
    hdr->H = H;
    hdr->sl_hi = tot.l.hi;
    hdr->sl_lo = tot.l.lo;
    hdr->sh_hi = tot.h.hi;
    hdr->sh_lo = tot.h.lo;
    if ((L & (kAggStride - 1)) == 0) agg_l[L / kAggStride] = tot.l;
    if ((H & (kAggStride - 1)) == 0) agg_h[H / kAggStride] = tot.h;
  }
}

// ---------------------------------------------------------------------------
// k_partition: stable partition with known tile offsets
// ---------------------------------------------------------------------------
struct PartShared {
  double val[kTileItems + kTileItems / 16];  // staging (padded for the transpose)
  uint32_t idx[kTileItems];
  dd wl[4], wh[4];
  uint32_t cl[4], ch[4];
};

__device__ __forceinline__ int spos(int i) { return i + (i >> 4); }

__global__ __launch_bounds__(kTileThreads) void k_partition(
    const double *__restrict__ w, uint64_t n, const alias_ws_header *hdr,
    const TilePrefix *__restrict__ pre, const TilePrefix *__restrict__ gpre,
    uint32_t *__restrict__ l_idx, double *__restrict__ l_w,
    uint32_t *__restrict__ h_idx, double *__restrict__ h_w, dd *__restrict__ agg_l,
    dd *__restrict__ agg_h) {
  __shared__ PartShared S;
  if (hdr->status != ALIAS_OK) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t tile = blockIdx.x;
  const uint64_t base = (uint64_t)tile * kTileItems;
  const dd avg = dd_make(hdr->avg_hi, hdr->avg_lo);

  // 1. striped, coalesced load into the staging area
#pragma unroll
  for (int k = 0; k < kItemsPerThread; ++k) {
    const int e = k * kTileThreads + tid;
    const uint64_t gi = base + e;
    S.val[spos(e)] = (gi < n) ? w[gi] : 0.0;
  }
  __syncthreads();

  // 2. blocked view: this thread owns items tid*16 .. tid*16+15
  double x[kItemsPerThread];
  uint32_t lmask = 0, vmask = 0;
#pragma unroll
  for (int u = 0; u < kItemsPerThread; ++u) {
    const int e = tid * kItemsPerThread + u;
    x[u] = S.val[spos(e)];
    const bool valid = base + e < n;
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
  const TilePrefix tp = pre[tile], gp = gpre[tile / kScanGroup];
  const uint64_t l_before = gp.l_before + tp.l_before;
  const uint64_t h_before = base - l_before;
  const dd pl_thr = (gp.pl + tp.pl) + (sl_off + sl_lane);
  const dd ph_thr = (gp.ph + tp.ph) + (sh_off + sh_lane);
  uint32_t rl = cl_off + cl_inc - nl;
  uint32_t rh = Lt + ch_off + ch_inc - nh;

  // 4. stage entries at their tile-local ranks; emit prefix sums every 64
  dd run_l = dd_make(0.0, 0.0), run_h = dd_make(0.0, 0.0);
#pragma unroll
  for (int u = 0; u < kItemsPerThread; ++u) {
    const uint32_t gi = (uint32_t)(base + (uint64_t)tid * kItemsPerThread + u);
    if ((lmask >> u) & 1u) {
      const uint64_t g = l_before + rl;
      S.idx[rl] = gi;
      S.val[rl] = x[u];
      if ((g & (kAggStride - 1)) == 0) agg_l[g / kAggStride] = pl_thr + run_l;
      run_l = add_d(run_l, x[u]);
      ++rl;
    } else if ((hmask >> u) & 1u) {
      const uint64_t g = h_before + (rh - Lt);
      S.idx[rh] = gi;
      S.val[rh] = x[u];
      if ((g & (kAggStride - 1)) == 0) agg_h[g / kAggStride] = ph_thr + run_h;
      run_h = add_d(run_h, x[u]);
      ++rh;
    }
  }
  __syncthreads();

  // 5. coalesced write-out of both lists
  const uint32_t cnt = (uint32_t)((n - base < (uint64_t)kTileItems) ? n - base : kTileItems);
  for (uint32_t e = tid; e < cnt; e += kTileThreads) {
    if (e < Lt) {
      l_idx[l_before + e] = S.idx[e];
      l_w[l_before + e] = S.val[e];
    } else {
      h_idx[h_before + (e - Lt)] = S.idx[e];
      h_w[h_before + (e - Lt)] = S.val[e];
    }
  }
}

// ---------------------------------------------------------------------------
// Split search (Sec. 2.2: the sweep's state after m rows is the largest j
// with sigma_l[m-j] + sigma_h[j] <= m*avg; f is strictly increasing in j).
// ---------------------------------------------------------------------------
struct SplitCtx {
  const dd *agg_l, *agg_h;
  const double *l_w, *h_w;
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

__global__ __launch_bounds__(256) void k_split(const alias_ws_header *hdr, const dd *__restrict__ agg_l,
                                               const dd *__restrict__ agg_h,
                                               const double *__restrict__ l_w,
                                               const double *__restrict__ h_w, uint32_t s,
                                               uint32_t chunk, uint64_t n, uint32_t *split_i,
                                               uint32_t *split_j, dd *spill,
                                               const SplitModel *model, uint64_t model_bytes,
                                               uint32_t *fallbacks) {
  const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k > s || hdr->status != ALIAS_OK) return;
  if (model && !model_usable(model, model_bytes)) {
    // an unusable model is never read past its header; every split falls back
    if (k < s) atomicAdd(fallbacks, 1u);
    model = nullptr;
  }
  SplitCtx c;
  c.agg_l = agg_l;
  c.agg_h = agg_h;
  c.l_w = l_w;
  c.h_w = h_w;
  c.L = hdr->L;
  c.H = hdr->H;
  c.m = (k * chunk < n) ? k * chunk : n;
  const dd avg = dd_make(hdr->avg_hi, hdr->avg_lo);
  c.sl_tot = dd_make(hdr->sl_hi, hdr->sl_lo);
  if (c.m == n) {
    split_i[k] = (uint32_t)c.L;
    split_j[k] = (uint32_t)c.H;
    spill[k] = dd_make(0.0, 0.0);
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
    int64_t p = learned_predict_q(model, c.m, n, c.H);
    int64_t e = model->eps_q;
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
      atomicAdd(fallbacks, 1u);
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
  split_i[k] = (uint32_t)(c.m - j);
  split_j[k] = (uint32_t)j;
  spill[k] = sp;
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
__device__ __forceinline__ void put_row(const TableOut &t, uint32_t item, double p, uint32_t a) {
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
__global__ __launch_bounds__(64 * kPackWaves) void k_pack(
    const alias_ws_header *hdr, const uint32_t *__restrict__ l_idx, const double *__restrict__ l_w,
    const uint32_t *__restrict__ h_idx, const double *__restrict__ h_w,
    const uint32_t *__restrict__ split_i, const uint32_t *__restrict__ split_j,
    const dd *__restrict__ spill, uint32_t s, uint32_t chunk, TableOut out, int32_t *d_status) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t k = blockIdx.x * (blockDim.x >> 6) + wave;
  if (k >= s || hdr->status != ALIAS_OK) return;
  const PackLds PLy = pack_lds(chunk);
  unsigned char *base = smem_raw + (size_t)wave * PLy.bytes;
  double *Wv = (double *)(base + PLy.w_off);
  dd *QL = (dd *)(base + PLy.q_off);
  dd *QH = QL + PLy.nq;
  uint32_t *Ix = (uint32_t *)(base + PLy.ix_off);
  uint32_t *Ao = (uint32_t *)(base + PLy.ao_off);

  const uint64_t H = hdr->H;
  const dd avg = dd_make(hdr->avg_hi, hdr->avg_lo);
  const uint64_t i0 = split_i[k], j0 = split_j[k], i1 = split_i[k + 1], j1 = split_j[k + 1];
  const int nl = (int)((int64_t)i1 - (int64_t)i0), nh = (int)((int64_t)j1 - (int64_t)j0);
  // i + j = m at every boundary, so nl + nh is the section's row count; a
  // negative part would mean inconsistent splits: report, write nothing.
  if (nl < 0 || nh < 0 || nl + nh > (int)chunk) {
    if (lane == 0) *d_status = ALIAS_EINTERNAL;
    return;
  }
  const Divisor dv = make_divisor(avg);
  if (j0 >= H) {  // no heavy item left: remaining lights keep their whole row
    for (int e = lane; e < nl; e += 64) {
      const uint32_t l = l_idx[i0 + e];
      put_row<kRows>(out, l, clamp01(quot_fast(dd_make(l_w[i0 + e], 0.0), dv)), l);
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

  const dd sp0 = spill[k];
  const dd B = sp0 - dd_make(Wv[ppos(nl)], 0.0);  // local f(i, j) + B - m*avg = global f - m*avg
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
      const dd target = mul_d(avg, (double)m) - B;
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
      if (j0 + (uint64_t)j < H) r = (add_d(g, Wv[ppos(nl + j)]) + B) - mul_d(avg, (double)m);
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
    const dd rc = (pack_sigma(Wv, 0, QL, S, ic) + pack_sigma(Wv, nl, QH, S, e + 1) + B) -
                  mul_d(avg, (double)(ic + e));
    const uint32_t h = Ix[ppos(nl + e)];
    put_row<kRows>(out, h, clamp01(quot_fast(rc, dv)),
                   (j0 + (uint64_t)e + 1 < H) ? Ix[ppos(nl + e + 1)] : h);
  }

  // 6. light rows, in light (near item) order: own share w/avg and alias
  for (int e = lane; e < nl; e += 64)
    put_row<kRows>(out, Ix[ppos(e)], clamp01(quot_fast(dd_make(Wv[ppos(e)], 0.0), dv)),
                   Ao[ppos(e)]);
}

__global__ void k_reset_fallbacks(alias_ws_header *hdr) {
  if (threadIdx.x == 0 && blockIdx.x == 0) hdr->split_fallbacks = 0;
}

// Recompute the splits of a finished build (binary or learned); the pack is
// not rerun.  Used to compare split methods on the same partition.
int launch_split_only(void *d_ws, uint64_t n, const Layout &Lo, const SplitModel *model,
                      uint64_t model_bytes, hipStream_t st) {
  char *ws = (char *)d_ws;
  alias_ws_header *hdr = (alias_ws_header *)(ws + Lo.pub.header);
  const uint32_t s = Lo.pub.sections;
  hipLaunchKernelGGL(k_reset_fallbacks, dim3(1), dim3(64), 0, st, hdr);
  hipLaunchKernelGGL(k_split, dim3((s + 1 + 255) / 256), dim3(256), 0, st, hdr,
                     (const dd *)(ws + Lo.pub.agg_l), (const dd *)(ws + Lo.pub.agg_h),
                     (const double *)(ws + Lo.pub.l_w), (const double *)(ws + Lo.pub.h_w), s,
                     Lo.chunk, n, (uint32_t *)(ws + Lo.pub.split_i),
                     (uint32_t *)(ws + Lo.pub.split_j), (dd *)(ws + Lo.pub.spill), model,
                     model_bytes, &hdr->split_fallbacks);
  return hipGetLastError() == hipSuccess ? ALIAS_OK : ALIAS_EHIP;
}

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

int launch_build(const double *d_w, uint64_t n, double *d_prob, uint32_t *d_alias,
                 TableRow *d_rows, void *d_ws, int32_t *d_status, const Layout &Lo,
                 const SplitModel *model, uint64_t model_bytes, hipStream_t st) {
  char *ws = (char *)d_ws;
  alias_ws_header *hdr = (alias_ws_header *)(ws + Lo.pub.header);
  ReducePart *parts = (ReducePart *)(ws + Lo.parts);
  TileSum *tsum = (TileSum *)(ws + Lo.tilesum);
  TilePrefix *tpre = (TilePrefix *)(ws + Lo.tilepre);
  TileSum *gsum = (TileSum *)(ws + Lo.grpsum);
  TilePrefix *gpre = (TilePrefix *)(ws + Lo.grppre);
  const uint32_t groups = (Lo.pub.tiles + kScanGroup - 1) / kScanGroup;
  uint32_t *l_idx = (uint32_t *)(ws + Lo.pub.l_idx);
  uint32_t *h_idx = (uint32_t *)(ws + Lo.pub.h_idx);
  double *l_w = (double *)(ws + Lo.pub.l_w);
  double *h_w = (double *)(ws + Lo.pub.h_w);
  dd *agg_l = (dd *)(ws + Lo.pub.agg_l);
  dd *agg_h = (dd *)(ws + Lo.pub.agg_h);
  uint32_t *sp_i = (uint32_t *)(ws + Lo.pub.split_i);
  uint32_t *sp_j = (uint32_t *)(ws + Lo.pub.split_j);
  dd *spill = (dd *)(ws + Lo.pub.spill);
  const uint32_t tiles = Lo.pub.tiles, s = Lo.pub.sections, rb = Lo.pub.reduce_blocks;

  hipLaunchKernelGGL(k_reduce, dim3(rb), dim3(kReduceThreads), 0, st, d_w, n, parts);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, st, parts, rb, n, hdr, agg_l, agg_h,
                     d_status);
  hipLaunchKernelGGL(k_tilesum, dim3(tiles), dim3(kTileThreads), 0, st, d_w, n, hdr, tsum);
  hipLaunchKernelGGL(k_tilescan, dim3(groups), dim3(kScanGroup), 0, st, tsum, tiles, hdr, tpre,
                     gsum);
  hipLaunchKernelGGL(k_groupscan, dim3(1), dim3(kScanGroup), 0, st, gsum, groups, n, hdr, gpre,
                     agg_l, agg_h);
  hipLaunchKernelGGL(k_partition, dim3(tiles), dim3(kTileThreads), 0, st, d_w, n, hdr, tpre, gpre,
                     l_idx, l_w, h_idx, h_w, agg_l, agg_h);
  hipLaunchKernelGGL(k_split, dim3((s + 1 + 255) / 256), dim3(256), 0, st, hdr, agg_l, agg_h, l_w,
                     h_w, s, Lo.chunk, n, sp_i, sp_j, spill, model, model_bytes,
                     &hdr->split_fallbacks);
  // one wave per section; as many waves per block as the LDS allows (<= 4)
  const size_t per_wave = pack_lds(Lo.chunk).bytes;
  const size_t max_lds = device_max_lds_per_block();
  size_t waves = max_lds / per_wave;
  if (waves > (size_t)kPackWaves) waves = kPackWaves;
  if (waves == 0) return ALIAS_EINVAL;
  TableOut out;
  out.prob = d_prob;
  out.alias = d_alias;
  out.rows = d_rows;
  if (d_rows)
    hipLaunchKernelGGL(k_pack<true>, dim3((s + waves - 1) / waves), dim3(64 * waves),
                       waves * per_wave, st, hdr, l_idx, l_w, h_idx, h_w, sp_i, sp_j, spill, s,
                       Lo.chunk, out, d_status);
  else
    hipLaunchKernelGGL(k_pack<false>, dim3((s + waves - 1) / waves), dim3(64 * waves),
                       waves * per_wave, st, hdr, l_idx, l_w, h_idx, h_w, sp_i, sp_j, spill, s,
                       Lo.chunk, out, d_status);
  return hipGetLastError() == hipSuccess ? ALIAS_OK : ALIAS_EHIP;
}

}  // namespace amdalias
