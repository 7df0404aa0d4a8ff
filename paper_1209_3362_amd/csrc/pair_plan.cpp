// Launch planning of the pair kernel (see pair_plan.hpp).
#include "pair_plan.hpp"

#include <algorithm>
#include <limits>

namespace nfs {
namespace {
size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
}  // namespace

int pair_simd_load(int count, int waves) {
  const int base = count / waves, extra = count % waves;
  int worst = 0;
  for (int simd = 0; simd < 4; ++simd) {
    int load = 0;
    for (int w = simd; w < waves; w += 4) load += base + (w < extra ? 1 : 0);
    worst = std::max(worst, load);
  }
  return worst;
}

bool plan_group(const std::vector<int32_t>& lags, int first, int count,
                       LagGroup* g) {
  g->first = first;
  g->count = count;
  g->max_lag = lags[first + count - 1];
  g->modes = 0;
  // Two workgroups per CU hide each other's barrier and LDS waits: the first
  // choice is 16 modes per workgroup with LDS for two workgroups, then 16 or
  // 8 modes with LDS for one (the 8-wave kernels with 16 or 8 modes fit the
  // registers of two workgroups per CU).
  const int S = kPairChunk;
  const int H = int(round_up(size_t(g->max_lag + 2 * S), S));
  const struct { int K; size_t budget; } choices[] = {
      {16, size_t(kLdsBytes) / 2}, {16, size_t(kLdsBytes)}, {8, size_t(kLdsBytes)}};
  for (const auto& ch : choices) {
    const size_t lds = size_t(H + kPairMirror) * ch.K * 8;
    if (lds <= ch.budget) {
      g->modes = ch.K;
      g->hist = H;
      g->lds = lds;
      break;
    }
  }
  if (!g->modes) return false;
  // The lags are split over W waves in contiguous slices whose lengths
  // differ by at most one; waves w, w + 4, w + 8 share a SIMD, so pick the
  // W whose busiest SIMD has the fewest lags; ties go to more waves (more
  // waves per SIMD hide each other's LDS and barrier waits: measured on
  // 32-lag groups with one and with two workgroups per CU).
  int best_w = 0, best_cost = std::numeric_limits<int>::max();
  for (int W = 1; W <= kMaxPairWaves; ++W) {
    const int per = (count + W - 1) / W;
    if (per > kMaxLagsPerWave) continue;
    // Workgroups of 12 waves are built for 6 or more lags per wave only.
    if (W > 8 && per < 6) continue;
    const int cost = pair_simd_load(count, W);
    if (cost <= best_cost) {
      best_cost = cost;
      best_w = W;
    }
  }
  g->waves = best_w;
  g->per_wave = best_w ? (count + best_w - 1) / best_w : 0;
  return best_w > 0;
}

std::vector<LagGroup> group_candidates(const std::vector<int32_t>& lags, int first, int count) {
  std::vector<LagGroup> out;
  const int S = kPairChunk;
  const int max_lag = lags[first + count - 1];
  const int H = int(round_up(size_t(max_lag + 2 * S), S));
  for (int K : {16, 8}) {
    const size_t lds = size_t(H + kPairMirror) * K * 8;
    if (lds > size_t(kLdsBytes)) continue;
    for (int W = 1; W <= kMaxPairWaves; ++W) {
      const int per = (count + W - 1) / W;
      if (per > kMaxLagsPerWave) continue;
      if (W > 8 && per < 6) continue;
      LagGroup g;
      g.first = first;
      g.count = count;
      g.max_lag = max_lag;
      g.modes = K;
      g.hist = H;
      g.lds = lds;
      g.waves = W;
      g.per_wave = per;
      out.push_back(g);
    }
  }
  return out;
}

}  // namespace nfs
