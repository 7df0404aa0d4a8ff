// Lag-pair accumulator: for every stored mode m and every lag tau of the
// plan, S_tau(m) += |I_t(m) - I_{t-tau}(m)|^2 summed over target frames t.
// These are the square moduli of transform differences that the paper
// evaluates for every pair and averages per delay (processing section,
// "differences area" of Fig. 2); the average itself is taken when binning.
//
// One workgroup owns K consecutive modes and walks the time axis in chunks
// of S = 32 frames. The last H frames of its modes live in an LDS ring, so
// every spectrum value is read from HBM exactly once per launch, however
// many lags use it; waves split the lag list, and within a wave each lane
// owns one mode and S*K/64 consecutive target frames. Per pair and mode the
// inner loop is one LDS read (the older frame), two subtractions and two
// FMAs. The first S rows of the LDS ring are mirrored after its end so a
// lane's run of older rows never wraps.
#include "nfs_device.hpp"
#include "nfs_host.hpp"
#include "nfs_kernels.hpp"

namespace nfs {
namespace {

constexpr int S = kPairChunk;
constexpr int MAXLW = kMaxLagsPerWave;

template <int K>
__global__ __launch_bounds__(1024) void pair_kernel(
    const float2* __restrict__ ring, int64_t n_modes, int64_t mode_stride, int64_t capacity,
    int64_t T0, int64_t T1, const int32_t* __restrict__ lags, int n_lags, int max_lag,
    float* __restrict__ acc, int H, int per_wave) {
  constexpr int G = 64 / K;       // lanes sharing one mode inside a wave
  constexpr int RPT = S / G;      // target rows per lane per chunk
  constexpr int V4 = K / 2;       // float4 (two modes) per ring row of the tile
  // float4 per thread per chunk; launches have at least 4 waves.
  constexpr int MAXPF = (S * V4 / 256) > 0 ? (S * V4 / 256) : 1;
  extern __shared__ float4 hist4[];
  float2* hist = reinterpret_cast<float2*>(hist4);

  const int nthreads = blockDim.x;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int m = lane % K, g = lane / K;
  const int64_t m0 = int64_t(blockIdx.x) * K;

  const int l_begin = wave * per_wave;
  const int l_count = max(0, min(per_wave, n_lags - l_begin));
  int tau[MAXLW];
#pragma unroll
  for (int s = 0; s < MAXLW; ++s) tau[s] = s < l_count ? lags[l_begin + s] : 0;

  // Time t lives in LDS row (t - Tb) mod H, Tb = T0 - max_lag.
  const int64_t Tb = T0 - max_lag;
  auto slot_row = [&](int64_t slot) -> const float4* {
    return reinterpret_cast<const float4*>(ring + slot * mode_stride + m0);
  };
  auto put_row = [&](int row, int col2, float4 val) {
    hist4[(row * K) / 2 + col2] = val;
    if (row < S) hist4[((row + H) * K) / 2 + col2] = val;
  };

  // History from earlier windows: frames [max(0, T0 - max_lag), T0).
  {
    const int64_t r0 = T0 - max_lag > 0 ? T0 - max_lag : 0;
    const int64_t nrows = T0 - r0;
    for (int64_t e = threadIdx.x; e < nrows * V4; e += nthreads) {
      const int64_t t = r0 + e / V4;
      const int col2 = int(e % V4);
      put_row(int((t - Tb) % H), col2, slot_row(t % capacity)[col2]);
    }
  }

  float4 pf[MAXPF];
  const int n_el = S * V4;  // float4 per chunk
  // Chunk c's first frame is in ring slot cslot; slots of the chunk wrap once.
  auto prefetch = [&](int64_t c, int64_t cslot) {
#pragma unroll
    for (int i = 0; i < MAXPF; ++i) {
      const int e = threadIdx.x + i * nthreads;
      pf[i] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (e < n_el) {
        const int dt = e / V4;
        if (c + dt < T1) {
          int64_t slot = cslot + dt;
          if (slot >= capacity) slot -= capacity;
          pf[i] = slot_row(slot)[e % V4];
        }
      }
    }
  };
  auto commit = [&](int64_t c, int crow) {
#pragma unroll
    for (int i = 0; i < MAXPF; ++i) {
      const int e = threadIdx.x + i * nthreads;
      if (e < n_el) {
        int row = crow + e / V4;
        if (row >= H) row -= H;
        put_row(row, e % V4, pf[i]);
      }
    }
  };

  float ax[MAXLW], ay[MAXLW];
#pragma unroll
  for (int s = 0; s < MAXLW; ++s) ax[s] = ay[s] = 0.f;

  int crow = int((T0 - Tb) % H);  // LDS row of the chunk's first frame
  int64_t cslot = T0 % capacity;  // ring slot of the chunk's first frame
  prefetch(T0, cslot);
  for (int64_t c = T0; c < T1; c += S) {
    commit(c, crow);
    __syncthreads();
    cslot += S;
    if (cslot >= capacity) cslot -= capacity;
    if (c + S < T1) prefetch(c + S, cslot);

    const int rb = crow + g * RPT;  // < H + S: reads stay inside the mirror
    float2 cur[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) cur[i] = hist[(rb + i) * K + m];
    const bool full = c + S <= T1;
#pragma unroll
    for (int s = 0; s < MAXLW; ++s) {
      if (s < l_count) {
        const int ts = tau[s];
        if (c + S > ts) {  // some target frame of the chunk has a partner
          int ob = rb - ts;
          if (ob < 0) ob += H;
          const float2* old = hist + ob * K + m;
          if (full && c >= ts) {
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
              const float2 o = old[i * K];
              const float dx = cur[i].x - o.x, dy = cur[i].y - o.y;
              ax[s] = fmaf(dx, dx, ax[s]);
              ay[s] = fmaf(dy, dy, ay[s]);
            }
          } else {
            const int64_t tb = c + g * RPT;
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
              const int64_t t = tb + i;
              if (t - ts >= 0 && t < T1) {
                const float2 o = old[i * K];
                const float dx = cur[i].x - o.x, dy = cur[i].y - o.y;
                ax[s] = fmaf(dx, dx, ax[s]);
                ay[s] = fmaf(dy, dy, ay[s]);
              }
            }
          }
        }
      }
    }
    crow += S;
    if (crow >= H) crow -= H;
  }

  // Lanes g = 0..G-1 of one mode hold partial sums over disjoint frames.
  const bool mode_ok = m0 + m < n_modes;
#pragma unroll
  for (int s = 0; s < MAXLW; ++s) {
    if (s < l_count) {
      float v = ax[s] + ay[s];
#pragma unroll
      for (int o = K; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
      if (g == 0 && mode_ok) {
        float* p = acc + int64_t(l_begin + s) * mode_stride + m0 + m;
        *p += v;
      }
    }
  }
}

template <int K>
hipError_t pair_launch(const float2* ring, int64_t n_modes, int64_t mode_stride,
                       int64_t capacity, int64_t T0, int64_t T1, const int32_t* lags,
                       int n_lags, int max_lag, float* acc, int hist, int waves,
                       int per_wave, size_t lds, hipStream_t s) {
  // Allow the LDS history beyond the default dynamic limit; a failure here
  // shows up as a launch error below.
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&pair_kernel<K>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
  const int64_t blocks = (n_modes + K - 1) / K;
  const int launched = waves < 4 ? 4 : waves;  // extra waves only help load
  hipLaunchKernelGGL(pair_kernel<K>, dim3(unsigned(blocks)), dim3(64 * launched), lds, s, ring,
                     n_modes, mode_stride, capacity, T0, T1, lags, n_lags, max_lag, acc,
                     hist, per_wave);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_pairs(const float2* ring, int64_t n_modes, int64_t mode_stride,
                        int64_t capacity, int64_t T0, int64_t T1, const int32_t* lags,
                        int n_lags, int max_lag, float* acc, int modes, int hist, int waves,
                        int per_wave, size_t lds, hipStream_t s) {
  switch (modes) {
    case 64: return pair_launch<64>(ring, n_modes, mode_stride, capacity, T0, T1, lags, n_lags,
                                    max_lag, acc, hist, waves, per_wave, lds, s);
    case 32: return pair_launch<32>(ring, n_modes, mode_stride, capacity, T0, T1, lags, n_lags,
                                    max_lag, acc, hist, waves, per_wave, lds, s);
    case 16: return pair_launch<16>(ring, n_modes, mode_stride, capacity, T0, T1, lags, n_lags,
                                    max_lag, acc, hist, waves, per_wave, lds, s);
    case 8: return pair_launch<8>(ring, n_modes, mode_stride, capacity, T0, T1, lags, n_lags,
                                  max_lag, acc, hist, waves, per_wave, lds, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace nfs
