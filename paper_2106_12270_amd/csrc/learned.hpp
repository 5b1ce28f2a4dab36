// Learned split predictor: a small model that maps a section boundary's row
// position x = m/n to the fraction y = j/H of heavy items closed by then.
// The split search only has to confirm the prediction inside a bracket of
// +-eps_q aggregate points; when the bracket check fails it falls back to
// the full binary search, so the splits stay exact whatever the model says.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace amdalias {

enum : uint32_t { kModelPWL = 1, kModelMLP = 2 };
constexpr int kMlpHidden = 32;
// MLP 1 -> 32 -> 32 -> 1 with tanh: W1[32], b1[32], W2[32*32], b2[32], W3[32], b3[1]
constexpr int kMlpParams = 32 + 32 + 32 * 32 + 32 + 32 + 1;

struct SplitModel {
  uint32_t kind;      // kModelPWL or kModelMLP
  uint32_t segments;  // PWL: number of segments K (K+1 knot values follow)
  int32_t eps_q;      // bracket half-width in units of 64 heavy entries
  uint32_t nparams;   // number of float parameters that follow
  float params[1];    // PWL: y at x = 0, 1/K, ..., 1; MLP: kMlpParams floats
};

// Header fields are checked against the blob size before any parameter is read.
__device__ __forceinline__ bool model_usable(const SplitModel *M, uint64_t bytes) {
  if (bytes < 16) return false;
  uint64_t need;
  if (M->kind == kModelPWL) {
    if (M->segments < 1 || M->nparams != M->segments + 1) return false;
    need = 16 + 4ull * M->nparams;
  } else if (M->kind == kModelMLP) {
    if (M->nparams != (uint32_t)kMlpParams) return false;
    need = 16 + 4ull * kMlpParams;
  } else {
    return false;
  }
  return need <= bytes && M->eps_q >= 0;
}

__device__ __forceinline__ float mlp_forward(const float *p, float x) {
  const float *W1 = p, *b1 = p + 32, *W2 = p + 64, *b2 = p + 64 + 1024, *W3 = p + 64 + 1024 + 32;
  const float b3 = p[64 + 1024 + 64];
  float h1[kMlpHidden];
#pragma unroll
  for (int a = 0; a < kMlpHidden; ++a) h1[a] = tanhf(W1[a] * x + b1[a]);
  float y = b3;
  for (int b = 0; b < kMlpHidden; ++b) {
    float z = b2[b];
#pragma unroll
    for (int a = 0; a < kMlpHidden; ++a) z += W2[b * kMlpHidden + a] * h1[a];
    y += W3[b] * tanhf(z);
  }
  return y;
}

__device__ __forceinline__ float pwl_forward(const float *p, uint32_t K, float x) {
  float t = x * (float)K;
  int s = (int)t;
  if (s < 0) s = 0;
  if (s > (int)K - 1) s = (int)K - 1;
  const float f = t - (float)s;
  return p[s] + f * (p[s + 1] - p[s]);
}

// Predicted aggregate index q = floor(j_hat / 64) for the boundary after m
// rows, from the parameters P of a model of the given kind.
__device__ __forceinline__ int64_t predict_q(const float *P, uint32_t kind, uint32_t segments,
                                             uint64_t m, uint64_t n, uint64_t H) {
  const float x = (float)((double)m / (double)n);
  const float y = (kind == kModelPWL) ? pwl_forward(P, segments, x) : mlp_forward(P, x);
  const double jhat = (double)y * (double)H;
  return (int64_t)floor(jhat / 64.0);
}

__device__ __forceinline__ int64_t learned_predict_q(const SplitModel *M, uint64_t m, uint64_t n,
                                                     uint64_t H) {
  return predict_q(M->params, M->kind, M->segments, m, n, H);
}

}  // namespace amdalias
