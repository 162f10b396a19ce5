// learned.hpp -- launchers of the learned-rank kernels (see learned.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "desc.hpp"

namespace lrsp {

constexpr int kMlpFeatures = 12;
constexpr int kMlpHidden = 64;
constexpr int kMlpParams = 2 * kMlpFeatures + kMlpHidden * kMlpFeatures + kMlpHidden +
                           kMlpHidden * kMlpHidden + kMlpHidden + kMlpHidden + 1;
constexpr uint32_t kSketchSeed = 0x5EED1811u;

// Features [nitems][12] (fp64 and fp32 copies) of the level-start clusters.
void launch_rank_features(const FeatItem* items, int nitems, int max_m, int level, uint32_t seed,
                          double* feat, float* featf, hipStream_t st);
void launch_mlp_predict(const float* params, const float* X, int64_t n, float* y, hipStream_t st);
// Gradient (kMlpParams floats) and mean loss; part: mlp_partial_floats(n) floats.
void launch_mlp_grad(const float* params, const float* X, const float* t, int64_t n, float* part,
                     float* grad, float* loss, hipStream_t st);
int mlp_partial_floats(int64_t n);
void launch_mlp_adam(float* params, const float* grad, float* m1, float* m2, float lr, int step,
                     hipStream_t st);
void launch_mlp_init(float* params, const float* X, const float* t, int64_t n, uint64_t seed,
                     hipStream_t st);

}  // namespace lrsp
