// Launch planning of the pair kernel: its compile-time shape constants, the
// lag groups one launch handles, and how a group's lags are split over the
// waves of a workgroup. Host-only, no HIP dependency.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

namespace nfs {

// Frames of the time series handled per step of the pair kernel (with K
// modes per workgroup every lane holds 32 * K / 64 target frames).
constexpr int kPairChunk = 32;
// Most lags one wave of the pair kernel accumulates at once, and most waves
// per workgroup; a launch handles at most their product.
constexpr int kMaxLagsPerWave = 8;
constexpr int kMaxPairWaves = 12;
// LDS rows mirrored after the pair kernel's history ring: from a row of the
// ring a lane reads up to S + kMaxLagsPerWave - 2 rows further on.
constexpr int kPairMirror = kPairChunk + kMaxLagsPerWave;
// LDS a workgroup may allocate on gfx950.
constexpr int kLdsBytes = 160 * 1024;
// Largest delay the pair kernel's on-chip history supports (K = 8 modes);
// groups of longer delays run the global-memory kernel (modes == 0), up to
// kGlobalLags delays per launch.
constexpr int kMaxLag = 2400;
constexpr int kGlobalLags = 8;

// Lags of the busiest SIMD when `count` lags are split over `waves` waves
// in contiguous slices whose lengths differ by at most one (the first
// count % waves waves take one more) and wave w runs on SIMD w % 4.
int pair_simd_load(int count, int waves);

// One group of lags handled by one launch of the pair kernel.
struct LagGroup {
  int first = 0;      // index of the group's first lag in the lag list
  int count = 0;      // lags in the group
  int max_lag = 0;    // largest lag of the group
  int modes = 0;      // K: modes per workgroup; 0: the global-memory kernel
  int hist = 0;       // H: history rows kept in LDS (multiple of the chunk)
  int waves = 0;      // waves that sum lags (the launch has 8, or 12 if more)
  int per_wave = 0;   // most lags of one wave (<= kMaxLagsPerWave)
  size_t lds = 0;     // dynamic LDS bytes
};

// Launch shape for lags[first .. first + count): 16 modes per workgroup with
// LDS for two workgroups per CU if the history allows, else 16 or 8 with LDS
// for one; the wave count whose busiest SIMD has the fewest lags. False when
// the history fits no shape.
bool plan_group(const std::vector<int32_t>& lags, int first, int count, LagGroup* g);

// Every launch shape the pair kernel can run a lag group of `count` lags
// from lags[first] with: 16 or 8 modes per workgroup (LDS for two
// workgroups per CU, or for one), and each wave count whose slices fit
// (at most kMaxLagsPerWave lags per wave; 12-wave workgroups for 6 or more).
std::vector<LagGroup> group_candidates(const std::vector<int32_t>& lags, int first, int count);

}  // namespace nfs
