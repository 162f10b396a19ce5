// learned.cpp -- learned-rank form: the MLP entry points of the C interface
// and the per-level rank prediction used by the factorization.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/lrsp.h"
#include "learned.hpp"
#include "runtime.hpp"

using namespace lrsp;
using namespace lrsp::rt;

namespace lrsp {
namespace rt {

lrsp_status predict_level(LevelDev* L, int level, double tol, const float* d_params, hipStream_t st,
                          std::vector<double>* feat, std::vector<float>* pred) {
  const LevelPlan& p = L->plan;
  const int M = p.M;
  std::vector<FeatItem> items(M);
  std::vector<FeatSeg> segs;
  std::vector<size_t> seg0(M);
  double* W = at<double>(L->work, 0);
  const int32_t* WI = at<int32_t>(L->wints, 0);
  for (int s = 0; s < M; ++s) {
    seg0[s] = segs.size();
    int bsum = 0, nbefore = 0;
    for (int y : p.wlist[s]) bsum += p.m[y];
    for (int y : p.adj[s]) nbefore += p.pos[y] < p.pos[s] ? 1 : 0;
    for (int y : p.adj[s]) {
      FeatSeg g{};
      g.y = y;
      g.my = p.m[y];
      g.Dy = W + p.d_off[y];
      const bool s_first = p.pos[s] < p.pos[y];
      const uint64_t key = s_first ? pkey(s, y) : pkey(y, s);
      g.H = W + p.hf_off.at(key);
      g.zl = WI + p.zl_off.at(key);
      g.ncols = (int)p.zfin.at(key).size();
      g.ld = s_first ? p.m[s] : p.m[y];
      g.orient = s_first ? 0 : 1;
      if (p.m[s] > 0 && p.m[y] > 0) segs.push_back(g);
    }
    const double before = (double)nbefore / (double)std::max<size_t>(1, p.adj[s].size());
    items[s] = FeatItem{W + p.d_off[s], nullptr, before, p.m[s], (int)(segs.size() - seg0[s]), s, bsum};
  }
  DevBuf dseg, ditem, dfeat, dpred;
  const size_t bs = std::max<size_t>(1, segs.size()) * sizeof(FeatSeg);
  HIPCHK(dalloc(&dseg, bs, st));
  if (!segs.empty())
    HIPCHK(hipMemcpyAsync(dseg.p, segs.data(), segs.size() * sizeof(FeatSeg), hipMemcpyHostToDevice, st));
  for (int s = 0; s < M; ++s) items[s].seg = at<FeatSeg>(dseg, (int64_t)seg0[s]);
  if (lrsp_status e = upload(&ditem, items.data(), items.size() * sizeof(FeatItem), st)) return e;
  HIPCHK(dalloc(&dfeat, (size_t)M * kMlpFeatures * (sizeof(double) + sizeof(float)), st));
  HIPCHK(dalloc(&dpred, (size_t)M * sizeof(float), st));
  double* f64 = at<double>(dfeat, 0);
  float* f32 = reinterpret_cast<float*>(f64 + (size_t)M * kMlpFeatures);
  launch_rank_features(at<FeatItem>(ditem, 0), M, L->max_m, level, kSketchSeed, f64, f32, st);
  launch_mlp_predict(d_params, f32, M, at<float>(dpred, 0), st);
  HIPCHK(hipGetLastError());
  feat->resize((size_t)M * kMlpFeatures);
  pred->resize(M);
  HIPCHK(hipMemcpyAsync(feat->data(), f64, feat->size() * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(pred->data(), dpred.p, pred->size() * 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  dfree(&dseg, st);
  dfree(&ditem, st);
  dfree(&dfeat, st);
  dfree(&dpred, st);
  return LRSP_OK;
}

std::vector<int> rank_caps(const std::vector<float>& pred) {
  std::vector<int> caps(pred.size());
  for (size_t s = 0; s < pred.size(); ++s) {
    const double y = std::isfinite(pred[s]) ? std::max(0.0f, pred[s]) : 1e9;
    caps[s] = (int)std::min(1e9, std::ceil(kRankCapScale * y + kRankCapSlack));
  }
  return caps;
}

}  // namespace rt
}  // namespace lrsp

extern "C" {

int32_t lrsp_mlp_nparams(void) { return kMlpParams; }

lrsp_status lrsp_mlp_init(float* params, const float* X, const float* t, int64_t n, uint64_t seed,
                          void* stream) {
  if (!params || !X || !t || n < 1) return fail(LRSP_ERR_ARG, "invalid argument");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  launch_mlp_init(params, X, t, n, seed, st);
  HIPCHK(hipGetLastError());
  return LRSP_OK;
}

lrsp_status lrsp_mlp_loss_grad(const float* params, const float* X, const float* t, int64_t n,
                               float* grad, float* loss, void* stream) {
  if (!params || !X || !t || !grad || n < 1) return fail(LRSP_ERR_ARG, "invalid argument");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  DevBuf part;
  HIPCHK(dalloc(&part, sizeof(float) * (size_t)mlp_partial_floats(n), st));
  launch_mlp_grad(params, X, t, n, at<float>(part, 0), grad, loss, st);
  HIPCHK(hipGetLastError());
  dfree(&part, st);
  return LRSP_OK;
}

lrsp_status lrsp_mlp_train(float* params, const float* X, const float* t, int64_t n, int32_t steps,
                           float lr, float* loss_trace, void* stream) {
  if (!params || !X || !t || n < 1 || steps < 0 || !(lr > 0.0f)) return fail(LRSP_ERR_ARG, "invalid argument");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  DevBuf part, work;
  HIPCHK(dalloc(&part, sizeof(float) * (size_t)mlp_partial_floats(n), st));
  HIPCHK(dalloc(&work, sizeof(float) * 3 * kMlpParams, st));
  float* grad = at<float>(work, 0);
  float* m1 = grad + kMlpParams;
  float* m2 = m1 + kMlpParams;
  launch_zero_i32(reinterpret_cast<int32_t*>(m1), 2 * kMlpParams, st);
  for (int s = 0; s < steps; ++s) {
    launch_mlp_grad(params, X, t, n, at<float>(part, 0), grad, loss_trace ? loss_trace + s : nullptr, st);
    launch_mlp_adam(params, grad, m1, m2, lr, s + 1, st);
  }
  HIPCHK(hipGetLastError());
  dfree(&part, st);
  dfree(&work, st);
  return LRSP_OK;
}

lrsp_status lrsp_mlp_predict(const float* params, const float* X, int64_t n, float* y, void* stream) {
  if (!params || !X || !y || n < 0) return fail(LRSP_ERR_ARG, "invalid argument");
  launch_mlp_predict(params, X, n, y, reinterpret_cast<hipStream_t>(stream));
  HIPCHK(hipGetLastError());
  return LRSP_OK;
}

}  // extern "C"
