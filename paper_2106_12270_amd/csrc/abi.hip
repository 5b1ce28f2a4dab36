// C entry points of the alias-table library (declared in alias_mi355x.h).
// Argument checking and launch plumbing only: all work happens in the
// kernels of build.hip and sample.hip.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "alias_mi355x.h"
#include "common.hpp"
#include "learned.hpp"

namespace amdalias {
int launch_build(const double *d_w, uint64_t n, double *d_prob, uint32_t *d_alias,
                 TableRow *d_rows, void *d_ws, int32_t *d_status, const Layout &Lo,
                 const SplitModel *model, uint64_t model_bytes, hipStream_t st);
int launch_build_batch(const double *d_w, const uint64_t *d_offsets, uint64_t n1, double *d_prob,
                       uint32_t *d_alias, TableRow *d_rows, void *d_ws, int32_t *d_status,
                       const Layout &Lo, const unsigned char *models, uint64_t model_bytes,
                       uint64_t model_stride, hipStream_t st);
int launch_sample_batched(const double *prob, const uint32_t *alias, const TableRow *rows,
                          const uint64_t *offsets, const uint64_t *draw_off, uint32_t T,
                          uint64_t total_items, uint64_t total_draws, uint64_t seed,
                          uint32_t *out, int32_t *status, hipStream_t st);
int launch_sample(const double *prob, const uint32_t *alias, uint64_t n, uint64_t count,
                  uint64_t seed, uint64_t first, uint32_t table, uint32_t *out, hipStream_t st);
int launch_sample_rows(const TableRow *rows, uint64_t n, uint64_t count, uint64_t seed,
                       uint64_t first, uint32_t table, uint32_t *out, hipStream_t st);
}  // namespace amdalias

using namespace amdalias;

static bool aligned(const void *p, uintptr_t a) { return ((uintptr_t)p & (a - 1)) == 0; }

extern "C" {

size_t alias_build_workspace_bytes(uint64_t n, const alias_build_opts *opts) {
  Layout L;
  if (!compute_layout(n, opts, &L)) return 0;
  return (size_t)L.pub.total_bytes;
}

int alias_workspace_layout(uint64_t n, const alias_build_opts *opts, alias_ws_layout *out) {
  if (!out) return ALIAS_EINVAL;
  Layout L;
  if (!compute_layout(n, opts, &L)) return ALIAS_EINVAL;
  *out = L.pub;
  return ALIAS_OK;
}

// Shared argument checks of the two build entry points.
static int build_common(const double *d_w, uint64_t n, void *d_ws, size_t ws_bytes,
                        int32_t *d_status, const alias_build_opts *opts, Layout *L,
                        const SplitModel **model, uint64_t *model_bytes) {
  if (!d_w || !d_ws || !d_status) return ALIAS_EINVAL;
  if (!aligned(d_w, 8) || !aligned(d_ws, 256) || !aligned(d_status, 4)) return ALIAS_EINVAL;
  if (!compute_layout(n, opts, L)) return ALIAS_EINVAL;
  if (ws_bytes < L->pub.total_bytes) return ALIAS_EWORKSPACE;
  *model = nullptr;
  *model_bytes = 0;
  if (opts && opts->split_method == ALIAS_SPLIT_LEARNED) {
    if (!opts->split_model || opts->split_model_bytes < 16 || !aligned(opts->split_model, 4))
      return ALIAS_EMODEL;
    *model = (const SplitModel *)opts->split_model;
    *model_bytes = opts->split_model_bytes;
  }
  return ALIAS_OK;
}

int alias_build(const double *d_w, uint64_t n, double *d_prob, uint32_t *d_alias, void *d_ws,
                size_t ws_bytes, int32_t *d_status, const alias_build_opts *opts, void *stream) {
  Layout L;
  const SplitModel *model;
  uint64_t model_bytes;
  if (!d_prob || !d_alias || !aligned(d_prob, 8) || !aligned(d_alias, 4)) return ALIAS_EINVAL;
  const int st = build_common(d_w, n, d_ws, ws_bytes, d_status, opts, &L, &model, &model_bytes);
  if (st) return st;
  return launch_build(d_w, n, d_prob, d_alias, nullptr, d_ws, d_status, L, model, model_bytes,
                      (hipStream_t)stream);
}

int alias_build_rows(const double *d_w, uint64_t n, void *d_rows, void *d_ws, size_t ws_bytes,
                     int32_t *d_status, const alias_build_opts *opts, void *stream) {
  Layout L;
  const SplitModel *model;
  uint64_t model_bytes;
  if (!d_rows || !aligned(d_rows, 16)) return ALIAS_EINVAL;
  const int st = build_common(d_w, n, d_ws, ws_bytes, d_status, opts, &L, &model, &model_bytes);
  if (st) return st;
  return launch_build(d_w, n, nullptr, nullptr, (TableRow *)d_rows, d_ws, d_status, L, model,
                      model_bytes, (hipStream_t)stream);
}

int alias_sample(const double *d_prob, const uint32_t *d_alias, uint64_t n, uint64_t count,
                 uint64_t seed, uint64_t first_draw, uint32_t table_id, uint32_t *d_out,
                 void *stream) {
  if (n == 0 || n > 0xFFFFFFFFull) return ALIAS_EINVAL;
  if (count == 0) return ALIAS_OK;
  if (!d_prob || !d_alias || !d_out) return ALIAS_EINVAL;
  if (!aligned(d_prob, 8) || !aligned(d_alias, 4) || !aligned(d_out, 4)) return ALIAS_EINVAL;
  if (first_draw + count < first_draw) return ALIAS_EINVAL;  // counter range wraps
  return launch_sample(d_prob, d_alias, n, count, seed, first_draw, table_id, d_out,
                       (hipStream_t)stream);
}

int alias_sample_rows(const void *d_rows, uint64_t n, uint64_t count, uint64_t seed,
                      uint64_t first_draw, uint32_t table_id, uint32_t *d_out, void *stream) {
  if (n == 0 || n > 0xFFFFFFFFull) return ALIAS_EINVAL;
  if (count == 0) return ALIAS_OK;
  if (!d_rows || !d_out || !aligned(d_rows, 16) || !aligned(d_out, 4)) return ALIAS_EINVAL;
  if (first_draw + count < first_draw) return ALIAS_EINVAL;
  return launch_sample_rows((const TableRow *)d_rows, n, count, seed, first_draw, table_id, d_out,
                            (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// Batched tables
// ---------------------------------------------------------------------------
size_t alias_build_batched_workspace_bytes(uint32_t T, uint64_t total_items,
                                           const alias_build_opts *opts) {
  Layout L;
  if (!compute_layout_batch(T, total_items, opts, &L)) return 0;
  return (size_t)L.pub.total_bytes;
}

static int batched_common(const double *d_w, const uint64_t *d_offsets, uint32_t T,
                          uint64_t total_items, void *d_ws, size_t ws_bytes, int32_t *d_status,
                          const alias_build_opts *opts, Layout *L, const unsigned char **models,
                          uint64_t *model_bytes, uint64_t *model_stride) {
  if (!d_w || !d_offsets || !d_ws || !d_status) return ALIAS_EINVAL;
  if (!aligned(d_w, 8) || !aligned(d_offsets, 8) || !aligned(d_ws, 256) || !aligned(d_status, 4))
    return ALIAS_EINVAL;
  if (!compute_layout_batch(T, total_items, opts, L)) return ALIAS_EINVAL;
  if (ws_bytes < L->pub.total_bytes) return ALIAS_EWORKSPACE;
  *models = nullptr;
  *model_bytes = 0;
  *model_stride = 0;
  if (opts && opts->split_method == ALIAS_SPLIT_LEARNED) {
    if (!opts->split_model || opts->split_model_bytes < 16 || !aligned(opts->split_model, 4))
      return ALIAS_EMODEL;
    if (opts->split_model_stride != 0 &&
        (opts->split_model_stride < opts->split_model_bytes || (opts->split_model_stride & 3)))
      return ALIAS_EMODEL;
    *models = (const unsigned char *)opts->split_model;
    *model_bytes = opts->split_model_bytes;
    *model_stride = opts->split_model_stride;
  }
  return ALIAS_OK;
}

int alias_build_batched(const double *d_w, const uint64_t *d_offsets, uint32_t T,
                        uint64_t total_items, double *d_prob, uint32_t *d_alias, void *d_ws,
                        size_t ws_bytes, int32_t *d_status, const alias_build_opts *opts,
                        void *stream) {
  Layout L;
  const unsigned char *models;
  uint64_t mb, ms;
  if (!d_prob || !d_alias || !aligned(d_prob, 8) || !aligned(d_alias, 4)) return ALIAS_EINVAL;
  const int st = batched_common(d_w, d_offsets, T, total_items, d_ws, ws_bytes, d_status, opts,
                                &L, &models, &mb, &ms);
  if (st) return st;
  return launch_build_batch(d_w, d_offsets, 0, d_prob, d_alias, nullptr, d_ws, d_status, L,
                            models, mb, ms, (hipStream_t)stream);
}

int alias_build_batched_rows(const double *d_w, const uint64_t *d_offsets, uint32_t T,
                             uint64_t total_items, void *d_rows, void *d_ws, size_t ws_bytes,
                             int32_t *d_status, const alias_build_opts *opts, void *stream) {
  Layout L;
  const unsigned char *models;
  uint64_t mb, ms;
  if (!d_rows || !aligned(d_rows, 16)) return ALIAS_EINVAL;
  const int st = batched_common(d_w, d_offsets, T, total_items, d_ws, ws_bytes, d_status, opts,
                                &L, &models, &mb, &ms);
  if (st) return st;
  return launch_build_batch(d_w, d_offsets, 0, nullptr, nullptr, (TableRow *)d_rows, d_ws,
                            d_status, L, models, mb, ms, (hipStream_t)stream);
}

static int sample_batched_common(const uint64_t *d_offsets, uint32_t T, uint64_t total_items,
                                 const uint64_t *d_draw_offsets, uint64_t total_draws,
                                 const uint32_t *d_out, const int32_t *d_status) {
  if (T == 0 || T > kMaxTables || total_items == 0 || total_items > (1ull << 40))
    return ALIAS_EINVAL;
  if (!d_offsets || !d_draw_offsets || !d_out || !d_status) return ALIAS_EINVAL;
  if (!aligned(d_offsets, 8) || !aligned(d_draw_offsets, 8) || !aligned(d_out, 4) ||
      !aligned(d_status, 4))
    return ALIAS_EINVAL;
  if (total_draws > (1ull << 40)) return ALIAS_EINVAL;
  return ALIAS_OK;
}

int alias_sample_batched(const double *d_prob, const uint32_t *d_alias, const uint64_t *d_offsets,
                         uint32_t T, uint64_t total_items, const uint64_t *d_draw_offsets,
                         uint64_t total_draws, uint64_t seed, uint32_t *d_out,
                         int32_t *d_status, void *stream) {
  if (!d_prob || !d_alias || !aligned(d_prob, 8) || !aligned(d_alias, 4)) return ALIAS_EINVAL;
  const int st = sample_batched_common(d_offsets, T, total_items, d_draw_offsets, total_draws,
                                       d_out, d_status);
  if (st) return st;
  return launch_sample_batched(d_prob, d_alias, nullptr, d_offsets, d_draw_offsets, T,
                               total_items, total_draws, seed, d_out, d_status,
                               (hipStream_t)stream);
}

int alias_sample_batched_rows(const void *d_rows, const uint64_t *d_offsets, uint32_t T,
                              uint64_t total_items, const uint64_t *d_draw_offsets,
                              uint64_t total_draws, uint64_t seed, uint32_t *d_out,
                              int32_t *d_status, void *stream) {
  if (!d_rows || !aligned(d_rows, 16)) return ALIAS_EINVAL;
  const int st = sample_batched_common(d_offsets, T, total_items, d_draw_offsets, total_draws,
                                       d_out, d_status);
  if (st) return st;
  return launch_sample_batched(nullptr, nullptr, (const TableRow *)d_rows, d_offsets,
                               d_draw_offsets, T, total_items, total_draws, seed, d_out, d_status,
                               (hipStream_t)stream);
}

const char *alias_status_str(int code) {
  switch (code) {
    case ALIAS_OK: return "ok";
    case ALIAS_EINVAL: return "invalid argument";
    case ALIAS_EWEIGHTS: return "invalid weights (negative, NaN, infinite, or zero total)";
    case ALIAS_EWORKSPACE: return "workspace too small";
    case ALIAS_EHIP: return "HIP launch failed";
    case ALIAS_EMODEL: return "learned split requested without a usable model";
    case ALIAS_EINTERNAL: return "internal consistency check failed";
    default: return "unknown status";
  }
}

const char *alias_version(void) { return "alias_mi355x 0.1 (gfx950)"; }

}  // extern "C"
