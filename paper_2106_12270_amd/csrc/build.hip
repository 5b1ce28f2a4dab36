// PSA alias-table construction on gfx950 (Lehmann, Huebschle-Schneider &
// Sanders, arXiv 2106.12270, Sec. 2.2 and Sec. 4).
//
// Pipeline, one stream, no host synchronisation or readback:
//   k_reduce    per-block double-double sums of the weights + validation;
//               also clears the partition's look-back flags.
//   k_finalize  W, W/N, status; resets the counters the later kernels use.
//   k_partition stable light/heavy partition in item order, entries carry
//               their weight (Sec. 4.2 "Weight in l and h Arrays"), light
//               probabilities written in item order, and prefix sums of the
//               light / heavy weights emitted every 64 entries.  Single pass:
//               tiles take ids from a ticket and find their offsets by a
//               decoupled look-back (Merrill & Garland) whose carries are
//               exact 128-bit fixed-point integers, so the result does not
//               depend on timing.
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

typedef __int128 i128;
typedef unsigned __int128 u128;

// ---------------------------------------------------------------------------
// Fixed-point helpers for the look-back carry
// ---------------------------------------------------------------------------

// trunc(x * 2^-E) as a signed 128-bit integer (|x * 2^-E| < 2^126 assumed).
__device__ __forceinline__ i128 fx_from_double(double x, int E) {
  if (x == 0.0) return 0;
  int e;
  double m = frexp(x, &e);  // x = m * 2^e, 0.5 <= |m| < 1
  int sh = e - E;           // |x| * 2^-E = |m| * 2^sh
  if (sh <= 0) return 0;
  long long M = (long long)(m * 9007199254740992.0);  // m * 2^53, exact
  bool neg = M < 0;
  u128 A = (u128)(unsigned long long)(neg ? -M : M);
  u128 U = (sh >= 53) ? (A << (sh - 53)) : (A >> (53 - sh));
  i128 r = (i128)U;
  return neg ? -r : r;
}

__device__ __forceinline__ i128 fx_from_dd(dd v, int E) {
  return fx_from_double(v.hi, E) + fx_from_double(v.lo, E);
}

__device__ __forceinline__ double u128_to_double(u128 U) {
  unsigned long long hi = (unsigned long long)(U >> 64);
  unsigned long long lo = (unsigned long long)U;
  return (double)hi * 18446744073709551616.0 + (double)lo;
}

__device__ __forceinline__ double i128_to_double(i128 V) {
  return V < 0 ? -u128_to_double((u128)(-V)) : u128_to_double((u128)V);
}

__device__ __forceinline__ dd fx_to_dd(i128 V, int E) {
  double a = i128_to_double(V);
  i128 R = V - fx_from_double(a, 0);
  double b = i128_to_double(R);
  dd r = quick_two_sum(a, b);
  r.hi = ldexp(r.hi, E);
  r.lo = ldexp(r.lo, E);
  return r;
}

__device__ __forceinline__ i128 u128_pack(uint64_t lo, uint64_t hi) {
  return (i128)(((u128)hi << 64) | (u128)lo);
}

__device__ __forceinline__ void st_relaxed(uint64_t *p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_relaxed(const uint64_t *p) {
  return __hip_atomic_load(const_cast<uint64_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Publish a tile descriptor: the value words go out with cache-bypassing
// atomic stores, then (after all of them have completed) the flag.  Only
// ordering is needed, not an L2 writeback, because every word is itself
// coherent.
__device__ __forceinline__ void publish(TileWords *slot, uint32_t *flag, uint32_t fval, uint64_t cnt,
                                        i128 sl, i128 sh) {
  st_relaxed(&slot->cnt, cnt);
  st_relaxed(&slot->sl_lo, (uint64_t)(u128)sl);
  st_relaxed(&slot->sl_hi, (uint64_t)((u128)sl >> 64));
  st_relaxed(&slot->sh_lo, (uint64_t)(u128)sh);
  st_relaxed(&slot->sh_hi, (uint64_t)((u128)sh >> 64));
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_waitcnt(0);
  __hip_atomic_store(flag, fval, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned long long shfl_xor_u64(unsigned long long v, int m) {
  return __shfl_xor(v, m, 64);
}

__device__ __forceinline__ i128 wave_sum_i128(i128 v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    u128 u = (u128)v;
    unsigned long long lo = shfl_xor_u64((unsigned long long)u, m);
    unsigned long long hi = shfl_xor_u64((unsigned long long)(u >> 64), m);
    v += u128_pack(lo, hi);
  }
  return v;
}

// ---------------------------------------------------------------------------
// Block reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ dd block_sum_dd(dd v, dd *s_wave /*[4]*/) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum(v);
  if (lane == 0) s_wave[wave] = v;
  __syncthreads();
  dd t = s_wave[0];
  for (int k = 1; k < (int)(blockDim.x >> 6); ++k) t = t + s_wave[k];
  __syncthreads();
  return t;
}

// ---------------------------------------------------------------------------
// k_reduce: per-block dd partial sums of w and the validation flag
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kReduceThreads) void k_reduce(const double *__restrict__ w, uint64_t n,
                                                           ReducePart *__restrict__ parts,
                                                           uint32_t *__restrict__ flags,
                                                           uint32_t tiles) {
  __shared__ dd s_wave[kReduceThreads / 64];
  __shared__ uint32_t s_bad;
  const uint64_t G = (uint64_t)gridDim.x * kReduceThreads;
  const uint64_t g = (uint64_t)blockIdx.x * kReduceThreads + threadIdx.x;
  for (uint64_t t = g; t < tiles; t += G) flags[t] = 0u;
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
    hdr->tile_ticket = 0;
    hdr->fx_exp = ok ? (ilogb(W.hi) - 125) : 0;
    hdr->status = ok ? ALIAS_OK : ALIAS_EWEIGHTS;
    hdr->split_fallbacks = 0;
    agg_l[0] = dd_make(0.0, 0.0);
    agg_h[0] = dd_make(0.0, 0.0);
    *d_status = ok ? ALIAS_OK : ALIAS_EWEIGHTS;
  }
}

// ---------------------------------------------------------------------------
// k_partition
// ---------------------------------------------------------------------------
struct PartShared {
  double val[kTileItems + kTileItems / 16];  // staging (padded for the transpose)
  uint32_t idx[kTileItems];
  dd wl[4], wh[4];
  uint32_t cl[4], ch[4];
  uint32_t tile;
  uint32_t pad;
  uint64_t l_before;
  dd pl, ph;
};

__device__ __forceinline__ int spos(int i) { return i + (i >> 4); }

__global__ __launch_bounds__(kTileThreads) void k_partition(
    const double *__restrict__ w, uint64_t n, alias_ws_header *hdr, uint32_t *flags,
    TileWords *tile_a, TileWords *tile_p, uint32_t tiles, uint32_t *__restrict__ l_idx,
    double *__restrict__ l_w, uint32_t *__restrict__ h_idx, double *__restrict__ h_w,
    dd *__restrict__ agg_l, dd *__restrict__ agg_h, double *__restrict__ prob) {
  __shared__ PartShared S;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (hdr->status != ALIAS_OK) return;
  if (tid == 0) S.tile = atomicAdd(&hdr->tile_ticket, 1u);
  __syncthreads();
  const uint32_t tile = S.tile;
  const uint64_t base = (uint64_t)tile * kTileItems;
  const dd avg = dd_make(hdr->avg_hi, hdr->avg_lo);
  const int E = hdr->fx_exp;

  // 1. striped, coalesced load; light probabilities written in item order
#pragma unroll
  for (int k = 0; k < kItemsPerThread; ++k) {
    const int e = k * kTileThreads + tid;
    const uint64_t gi = base + e;
    double x = 0.0;
    if (gi < n) {
      x = w[gi];
      prob[gi] = clamp01(quot(dd_make(x, 0.0), avg));  // heavies are rewritten by k_pack
    }
    S.val[spos(e)] = x;
  }
  __syncthreads();

  // 2. blocked view: thread owns items tid*16 .. tid*16+15
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
  // running sums before each item, for the item's own list
  dd before[kItemsPerThread];
  dd acc_l = dd_make(0.0, 0.0), acc_h = dd_make(0.0, 0.0);
#pragma unroll
  for (int u = 0; u < kItemsPerThread; ++u) {
    const bool light = (lmask >> u) & 1u;
    dd a = light ? acc_l : acc_h;
    before[u] = a;
    a = add_d(a, ((vmask >> u) & 1u) ? x[u] : 0.0);
    if (light)
      acc_l = a;
    else
      acc_h = a;
  }
  const uint32_t nl = __popc(lmask), nh = __popc(hmask);

  // 3. block exclusive scans: counts (int) and sums (dd), fixed pattern
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
  __syncthreads();
  uint32_t cl_off = 0, ch_off = 0, Lt = 0, Ht = 0;
  dd sl_off = dd_make(0.0, 0.0), sh_off = dd_make(0.0, 0.0);
  dd Slt = dd_make(0.0, 0.0), Sht = dd_make(0.0, 0.0);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (k < wave) {
      cl_off += S.cl[k];
      ch_off += S.ch[k];
      sl_off = sl_off + S.wl[k];
      sh_off = sh_off + S.wh[k];
    }
    Lt += S.cl[k];
    Ht += S.ch[k];
    Slt = Slt + S.wl[k];
    Sht = Sht + S.wh[k];
  }
  const uint32_t l_ex = cl_off + cl_inc - nl;  // tile-local rank of this thread's first light
  const uint32_t h_ex = ch_off + ch_inc - nh;
  // exclusive dd prefix within the tile: wave offset + lanes before
  dd sl_lane = shfl_up(sl_inc, 1), sh_lane = shfl_up(sh_inc, 1);
  if (lane == 0) {
    sl_lane = dd_make(0.0, 0.0);
    sh_lane = dd_make(0.0, 0.0);
  }
  const dd sl_ex = sl_off + sl_lane;
  const dd sh_ex = sh_off + sh_lane;

  // 4. decoupled look-back (wave 0) for the tile's global offsets
  if (wave == 0) {
    const i128 agg_sl = fx_from_dd(Slt, E), agg_sh = fx_from_dd(Sht, E);
    uint64_t ex_cnt = 0;
    i128 ex_sl = 0, ex_sh = 0;
    if (tile == 0) {
      if (lane == 0) publish(&tile_p[0], &flags[0], 2u, Lt, agg_sl, agg_sh);
    } else {
      if (lane == 0) publish(&tile_a[tile], &flags[tile], 1u, Lt, agg_sl, agg_sh);
      int64_t p_end = tile;
      while (true) {
        const int64_t p = p_end - 1 - lane;
        uint32_t f = 2u;
        uint64_t c = 0;
        i128 a = 0, b = 0;
        if (p >= 0) {
          f = __hip_atomic_load(&flags[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          while (f == 0u) {
            __builtin_amdgcn_s_sleep(1);
            f = __hip_atomic_load(&flags[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
          __builtin_amdgcn_s_waitcnt(0);
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
          const TileWords *src = (f == 2u) ? &tile_p[p] : &tile_a[p];
          c = ld_relaxed(&src->cnt);
          a = u128_pack(ld_relaxed(&src->sl_lo), ld_relaxed(&src->sl_hi));
          b = u128_pack(ld_relaxed(&src->sh_lo), ld_relaxed(&src->sh_hi));
        }
        const unsigned long long done = __ballot(f == 2u);
        const int first = done ? (__ffsll((long long)done) - 1) : 64;
        if (lane > first) {
          c = 0;
          a = 0;
          b = 0;
        }
        // counts fit in 64 bits; reuse the 128-bit reduction for all three
        ex_cnt += (uint64_t)wave_sum_i128((i128)c);
        ex_sl += wave_sum_i128(a);
        ex_sh += wave_sum_i128(b);
        if (done) break;
        p_end -= 64;
      }
      if (lane == 0)
        publish(&tile_p[tile], &flags[tile], 2u, ex_cnt + Lt, ex_sl + agg_sl, ex_sh + agg_sh);
    }
    if (lane == 0) {
      S.l_before = ex_cnt;
      S.pl = fx_to_dd(ex_sl, E);
      S.ph = fx_to_dd(ex_sh, E);
    }
  }
  __syncthreads();  // also: every thread has read S.val into x[]

  const uint64_t l_before = S.l_before;
  const uint64_t h_before = base - l_before;
  const dd pl_thr = S.pl + sl_ex;
  const dd ph_thr = S.ph + sh_ex;

  // 5. stage entries at their tile-local ranks; emit prefix sums every 64
  uint32_t rl = l_ex, rh = Lt + h_ex;
#pragma unroll
  for (int u = 0; u < kItemsPerThread; ++u) {
    const uint64_t gi = base + (uint64_t)tid * kItemsPerThread + u;
    if ((lmask >> u) & 1u) {
      const uint64_t g = l_before + rl;
      S.idx[rl] = (uint32_t)gi;
      S.val[rl] = x[u];
      if ((g & (kAggStride - 1)) == 0) agg_l[g / kAggStride] = pl_thr + before[u];
      ++rl;
    } else if ((hmask >> u) & 1u) {
      const uint64_t g = h_before + (rh - Lt);
      S.idx[rh] = (uint32_t)gi;
      S.val[rh] = x[u];
      if ((g & (kAggStride - 1)) == 0) agg_h[g / kAggStride] = ph_thr + before[u];
      ++rh;
    }
  }
  __syncthreads();

  // 6. coalesced write-out of both lists
  const uint32_t cnt = Lt + Ht;
  for (uint32_t e = tid; e < cnt; e += kTileThreads) {
    if (e < Lt) {
      l_idx[l_before + e] = S.idx[e];
      l_w[l_before + e] = S.val[e];
    } else {
      h_idx[h_before + (e - Lt)] = S.idx[e];
      h_w[h_before + (e - Lt)] = S.val[e];
    }
  }

  // 7. the last tile records the totals
  if (tile == tiles - 1 && tid == 0) {
    const uint64_t L = l_before + Lt, H = h_before + Ht;
    const dd slt = S.pl + Slt, sht = S.ph + Sht;
    hdr->L = L;
    hdr->H = H;
    hdr->sl_hi = slt.hi;
    hdr->sl_lo = slt.lo;
    hdr->sh_hi = sht.hi;
    hdr->sh_lo = sht.lo;
    if ((L & (kAggStride - 1)) == 0) agg_l[L / kAggStride] = slt;
    if ((H & (kAggStride - 1)) == 0) agg_h[H / kAggStride] = sht;
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
  uint64_t j = ja;
  while (j < jb) {
    const dd g2 = add_d(add_d(g, c.h_w[j]), -c.l_w[c.m - j - 1]);
    if (!le(g2, c.mavg)) break;
    g = g2;
    ++j;
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
// k_pack: one wave per section
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ int ppos(int e) { return e + (e >> 4); }  // padded LDS index

// P[ppos(0)] = 0 and P[ppos(e+1)] = src[0] + ... + src[e] for e < cnt.
__device__ void wave_prefix(const double *__restrict__ src, int cnt, dd *P, int lane) {
  for (int e = lane; e < cnt; e += 64) P[ppos(e + 1)] = dd_make(src[e], 0.0);
  if (lane == 0) P[ppos(0)] = dd_make(0.0, 0.0);
  wave_lds_sync();
  const int per = (cnt + 63) >> 6;
  const int b = lane * per;
  const int en = (b + per < cnt) ? b + per : cnt;
  dd acc = dd_make(0.0, 0.0);
  for (int e = b; e < en; ++e) acc = add_d(acc, P[ppos(e + 1)].hi);
  dd inc = wave_inclusive_scan(acc, lane);
  dd run = shfl_up(inc, 1);
  if (lane == 0) run = dd_make(0.0, 0.0);
  for (int e = b; e < en; ++e) {
    run = add_d(run, P[ppos(e + 1)].hi);
    P[ppos(e + 1)] = run;
  }
  wave_lds_sync();
}

__global__ __launch_bounds__(64 * kPackWaves) void k_pack(
    const alias_ws_header *hdr, const uint32_t *__restrict__ l_idx, const double *__restrict__ l_w,
    const uint32_t *__restrict__ h_idx, const double *__restrict__ h_w,
    const uint32_t *__restrict__ split_i, const uint32_t *__restrict__ split_j,
    const dd *__restrict__ spill, uint32_t s, uint32_t chunk, double *__restrict__ prob,
    uint32_t *__restrict__ alias, int32_t *d_status) {
  extern __shared__ dd smem[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t k = blockIdx.x * (blockDim.x >> 6) + wave;
  if (k >= s || hdr->status != ALIAS_OK) return;
  const int stride = ppos((int)chunk + 3) + 1;
  dd *P = smem + wave * stride;

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

  if (j0 >= H) {  // no heavy item left: remaining lights keep their whole row
    for (int e = lane; e < nl; e += 64) {
      const uint32_t l = l_idx[i0 + e];
      alias[l] = l;
    }
    return;
  }
  const int nhl = (nh + 1 < (int)(H - j0)) ? nh + 1 : (int)(H - j0);
  dd *PL = P;                    // ppos(0 .. nl)
  dd *PH = P + ppos(nl + 1);     // ppos(0 .. nhl), relative
  wave_prefix(l_w + i0, nl, PL, lane);
  wave_prefix(h_w + j0, nhl, PH, lane);

  const dd sp0 = spill[k];
  const dd B = sp0 - PH[ppos(1)];  // sigma offset: f_local(i,j) = PL[i] + PH[j] + B - m*avg
  const int total = nl + nh;
  const int rpl = (int)(chunk >> 6);

  // sub-split at local row m: largest j with PL[m-j] + PH[j] + B <= m*avg
  auto subsplit = [&](int m, int &io, int &jo) {
    if (m <= 0) {
      io = 0;
      jo = 0;
      return;
    }
    if (m >= total) {
      io = nl;
      jo = nh;
      return;
    }
    const dd target = mul_d(avg, (double)m) - B;
    int lo = (m > nl) ? m - nl : 0;
    int hi = (m < nh) ? m : nh;
    while (lo < hi) {
      const int mid = lo + (hi - lo + 1) / 2;
      if (le(PL[ppos(m - mid)] + PH[ppos(mid)], target))
        lo = mid;
      else
        hi = mid - 1;
    }
    io = m - lo;
    jo = lo;
  };
  int i, j, ie, je;
  subsplit(lane * rpl, i, j);
  subsplit((lane + 1) * rpl, ie, je);
  if (lane * rpl >= total) return;

  dd r = dd_make(0.0, 0.0);
  if (j0 + (uint64_t)j < H) {
    const int m = i + j;
    r = (B + PL[ppos(i)] + PH[ppos(j + 1)]) - mul_d(avg, (double)m);
  }
  while (i < ie || j < je) {
    const uint64_t jj = j0 + (uint64_t)j;
    if (j < je && (le(r, avg) || i == ie)) {
      const uint32_t h = h_idx[jj];
      const bool next = jj + 1 < H;
      prob[h] = clamp01(quot(r, avg));
      alias[h] = next ? h_idx[jj + 1] : h;
      if (next) r = add_d(r - avg, h_w[jj + 1]);
      ++j;
    } else {
      const uint32_t l = l_idx[i0 + i];
      if (jj < H) {
        alias[l] = h_idx[jj];
        r = r - add_d(avg, -l_w[i0 + i]);
      } else {
        alias[l] = l;
      }
      ++i;
    }
  }
}

// ---------------------------------------------------------------------------
// Host launcher
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

int launch_build(const double *d_w, uint64_t n, double *d_prob, uint32_t *d_alias, void *d_ws,
                 int32_t *d_status, const Layout &Lo, const SplitModel *model, uint64_t model_bytes,
                 hipStream_t st) {
  char *ws = (char *)d_ws;
  alias_ws_header *hdr = (alias_ws_header *)(ws + Lo.pub.header);
  ReducePart *parts = (ReducePart *)(ws + Lo.parts);
  uint32_t *flags = (uint32_t *)(ws + Lo.flags);
  TileWords *ta = (TileWords *)(ws + Lo.tile_a);
  TileWords *tp = (TileWords *)(ws + Lo.tile_p);
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

  hipLaunchKernelGGL(k_reduce, dim3(rb), dim3(kReduceThreads), 0, st, d_w, n, parts, flags, tiles);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, st, parts, rb, n, hdr, agg_l, agg_h,
                     d_status);
  hipLaunchKernelGGL(k_partition, dim3(tiles), dim3(kTileThreads), 0, st, d_w, n, hdr, flags, ta,
                     tp, tiles, l_idx, l_w, h_idx, h_w, agg_l, agg_h, d_prob);
  hipLaunchKernelGGL(k_split, dim3((s + 1 + 255) / 256), dim3(256), 0, st, hdr, agg_l, agg_h, l_w,
                     h_w, s, Lo.chunk, n, sp_i, sp_j, spill, model, model_bytes,
                     &hdr->split_fallbacks);
  // one wave per section; as many waves per block as the LDS allows (<= 4)
  const size_t per_wave = (size_t)(ppos((int)Lo.chunk + 3) + 1) * sizeof(dd);
  const size_t max_lds = device_max_lds_per_block();
  size_t waves = max_lds / per_wave;
  if (waves > (size_t)kPackWaves) waves = kPackWaves;
  if (waves == 0) return ALIAS_EINVAL;
  hipLaunchKernelGGL(k_pack, dim3((s + waves - 1) / waves), dim3(64 * waves), waves * per_wave, st,
                     hdr, l_idx, l_w, h_idx, h_w, sp_i, sp_j, spill, s, Lo.chunk, d_prob, d_alias,
                     d_status);
  return hipGetLastError() == hipSuccess ? ALIAS_OK : ALIAS_EHIP;
}

}  // namespace amdalias
