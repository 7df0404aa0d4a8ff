// Lag-pair accumulator: for every stored mode m and every lag tau of the
// plan, S_tau(m) += |I_t(m) - I_{t-tau}(m)|^2 summed over target frames t.
// These are the square moduli of transform differences that the paper
// evaluates for every pair and averages per delay (processing section,
// "differences area" of Fig. 2); the average itself is taken when binning.
//
// One workgroup owns K consecutive modes and walks the time axis in chunks
// of S frames. The last H frames of its modes live in an LDS ring, so every
// spectrum value is read from HBM exactly once per launch, however many lags
// use it; waves split the lag list, and within a wave each lane owns one
// mode and S*K/64 consecutive target frames. Per pair and mode the inner
// loop is one LDS read (the older frame), two subtractions and two FMAs; a
// wave whose lags are consecutive integers reads one register window of
// older frames shared by all its lags instead. The first rows of the LDS
// ring are mirrored after its end so a lane's run of rows never wraps.
//
// A ring slot holds sigma_t F[frame_t - reference]; the spectrum the pairs
// use is that plus (sigma_t - sigma_ref) F[reference], i.e. the normalised
// transform minus the constant sigma_ref F[reference], which cancels in
// every difference. The correction is applied once per (frame, mode) as the
// slot is copied into LDS.
#include "nfs_device.hpp"
#include "nfs_host.hpp"
#include "nfs_kernels.hpp"

namespace nfs {
namespace {

// K modes per workgroup, MAXLW lag slots per wave: the lag list is split
// into lag_waves contiguous slices of near-equal length, one per wave;
// slots past a slice's end read harmless rows and are not summed.
template <int K, int MAXLW>
__global__ __launch_bounds__(64 * kMaxPairWaves) void pair_kernel(
    const float2* __restrict__ ring, const float2* __restrict__ refspec,
    const float2* __restrict__ fscale, int64_t n_modes, int64_t mode_stride, int64_t capacity,
    int64_t T0, int64_t T1, const int32_t* __restrict__ lags, int n_lags, int max_lag,
    float* __restrict__ acc, int acc_pitch, int H, int lag_waves) {
  constexpr int S = pair_chunk(K);  // frames per chunk
  constexpr int G = 64 / K;         // lanes sharing one mode inside a wave
  constexpr int RPT = S / G;        // target rows per lane per chunk
  constexpr int V4 = K / 2;         // float4 (two modes) per ring row of the tile
  constexpr int WIN = RPT + MAXLW - 1;  // register window of a run of consecutive lags
  constexpr int MR = pair_mirror(K);    // rows mirrored past the end of the LDS ring
  static_assert(MR >= S && MR >= WIN - 1, "mirror too short for a lane's row run");
  // float4 per thread per chunk; launches have at least 4 waves.
  constexpr int MAXPF = (S * V4 / 256) > 0 ? (S * V4 / 256) : 1;
  extern __shared__ float4 hist4[];
  float2* hist = reinterpret_cast<float2*>(hist4);

  const int nthreads = blockDim.x;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int m = lane % K, g = lane / K;
  const int64_t m0 = int64_t(blockIdx.x) * K;
  const int len = int(T1 - T0);  // frames in this window (< capacity)

  // This wave's lags, in scalar registers: the first n_lags % lag_waves
  // waves take one lag more than the others (waves past lag_waves none). A
  // target frame at window offset u has a partner for lag tau[s] iff
  // u >= first[s].
  const int base = n_lags / lag_waves, extra = n_lags % lag_waves;
  const int l_begin = wave * base + min(wave, extra);
  const int l_count = wave < lag_waves ? base + (wave < extra ? 1 : 0) : 0;
  int tau[MAXLW], first[MAXLW];
#pragma unroll
  for (int s = 0; s < MAXLW; ++s) {
    const int ts = s < l_count ? lags[l_begin + s] : 0;
    tau[s] = __builtin_amdgcn_readfirstlane(ts);
    const int64_t f = int64_t(ts) - T0;
    first[s] = __builtin_amdgcn_readfirstlane(int(f > 0 ? f : 0));
  }
  // Consecutive lags tau[0], tau[0]+1, ... share one register window.
  bool consecutive = MAXLW > 1 && l_count > 1;
#pragma unroll
  for (int s = 1; s < MAXLW; ++s)
    if (s < l_count && tau[s] != tau[0] + s) consecutive = false;

  // Window offset u lives in LDS row (u + max_lag) mod H.
  auto slot_row = [&](int64_t slot) -> const float4* {
    return reinterpret_cast<const float4*>(ring + slot * mode_stride + m0);
  };
  auto put_row = [&](int row, int col2, float4 val) {
    hist4[(row * K) / 2 + col2] = val;
    if (row < MR) hist4[((row + H) * K) / 2 + col2] = val;
  };
  // Slot value v of two modes plus d * F[reference] of the same modes.
  const float4* ref4 = reinterpret_cast<const float4*>(refspec + m0);
  auto corrected = [](float4 v, float d, float4 R) {
    return make_float4(fmaf(d, R.x, v.x), fmaf(d, R.y, v.y), fmaf(d, R.z, v.z),
                       fmaf(d, R.w, v.w));
  };

  // History from earlier windows: frames [max(0, T0 - max_lag), T0).
  {
    const int pre = int(T0 - max_lag > 0 ? max_lag : T0);
    int64_t slot = (T0 - pre) % capacity;
    for (int r = 0; r < pre; ++r) {
      const float d = fscale[slot].y;
      for (int col2 = threadIdx.x; col2 < V4; col2 += nthreads)
        put_row((max_lag - pre + r) % H, col2, corrected(slot_row(slot)[col2], d, ref4[col2]));
      if (++slot == capacity) slot = 0;
    }
  }

  // Each thread copies the same two modes of every chunk row it handles, so
  // their reference values stay in registers.
  float4 pf[MAXPF], rr[MAXPF];
  float pd[MAXPF];
  const int n_el = S * V4;  // float4 per chunk
#pragma unroll
  for (int i = 0; i < MAXPF; ++i) {
    const int e = threadIdx.x + i * nthreads;
    rr[i] = e < n_el ? ref4[e % V4] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
  // Chunk at window offset c starts in ring slot cslot; slots wrap once.
  auto prefetch = [&](int c, int64_t cslot) {
#pragma unroll
    for (int i = 0; i < MAXPF; ++i) {
      const int e = threadIdx.x + i * nthreads;
      pf[i] = make_float4(0.f, 0.f, 0.f, 0.f);
      pd[i] = 0.f;
      if (e < n_el) {
        const int dt = e / V4;
        if (c + dt < len) {
          int64_t slot = cslot + dt;
          if (slot >= capacity) slot -= capacity;
          pf[i] = slot_row(slot)[e % V4];
          pd[i] = fscale[slot].y;
        }
      }
    }
  };
  auto commit = [&](int crow) {
#pragma unroll
    for (int i = 0; i < MAXPF; ++i) {
      const int e = threadIdx.x + i * nthreads;
      if (e < n_el) {
        int row = crow + e / V4;
        if (row >= H) row -= H;
        put_row(row, e % V4, corrected(pf[i], pd[i], rr[i]));
      }
    }
  };

  float ax[MAXLW], ay[MAXLW];
#pragma unroll
  for (int s = 0; s < MAXLW; ++s) ax[s] = ay[s] = 0.f;

  // |cur[i] - old[i]|^2 into lag slot s.
  auto acc_plain = [&](const float2* cur, const float2* old, int s) {
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const float dx = cur[i].x - old[i].x, dy = cur[i].y - old[i].y;
      ax[s] = fmaf(dx, dx, ax[s]);
      ay[s] = fmaf(dy, dy, ay[s]);
    }
  };
  // The same with targets that have no partner yet (u < first) or lie past
  // the window end zeroed by selects, not branches.
  auto acc_masked = [&](const float2* cur, const float2* old, int s, int ub) {
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int u = ub + i;
      const bool ok = (u >= first[s]) & (u < len);
      const float dx = ok ? cur[i].x - old[i].x : 0.f;
      const float dy = ok ? cur[i].y - old[i].y : 0.f;
      ax[s] = fmaf(dx, dx, ax[s]);
      ay[s] = fmaf(dy, dy, ay[s]);
    }
  };
  int first_max = 0;
#pragma unroll
  for (int s = 0; s < MAXLW; ++s)
    if (s < l_count) first_max = max(first_max, first[s]);

  int crow = max_lag % H;         // LDS row of the chunk's first frame
  int64_t cslot = T0 % capacity;  // ring slot of the chunk's first frame
  prefetch(0, cslot);
  for (int c = 0; c < len; c += S) {
    commit(crow);
    __syncthreads();
    cslot += S;
    if (cslot >= capacity) cslot -= capacity;
    if (c + S < len) prefetch(c + S, cslot);

    const int rb = crow + g * RPT;  // reads stay inside the ring and its mirror
    const int ub = c + g * RPT;     // window offset of this lane's first target
    const bool full = c + S <= len;
    float2 cur[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) cur[i] = hist[(rb + i) * K + m];
    auto older = [&](int ts) {
      int r = rb - ts;
      if (r < 0) r += H;
      return hist + r * K + m;
    };

    // Older rows of a lag slot; slots past l_count have tau = 0 and read the
    // current rows, so every read is in bounds and unconditional.
    auto load_old = [&](float2 (&o)[RPT], int ts) {
      const float2* src = older(ts);
#pragma unroll
      for (int i = 0; i < RPT; ++i) o[i] = src[i * K];
    };
    if (consecutive && full && c >= first_max) {
      // Every target of the chunk has a partner for every lag of the run:
      // rows rb - tau[0] - (MAXLW-1) .. rb - tau[0] + RPT - 1 serve them
      // all, lag tau[0] + s reads win[MAXLW - 1 - s + i].
      float2 win[WIN];
      const float2* src = older(tau[0] + MAXLW - 1);
#pragma unroll
      for (int i = 0; i < WIN; ++i) win[i] = src[i * K];
      dev::static_for<MAXLW>([&](auto SS) {
        constexpr int s = decltype(SS)::value;
        if (s < l_count) acc_plain(cur, win + (MAXLW - 1 - s), s);
      });
    } else {
      // Per lag slot (wave-uniform): every target of the chunk has a
      // partner (plain sums), some do (masked sums) or none (skipped). The
      // older rows of slot s+1 are read while slot s is summed.
      auto sum_slot = [&](const float2* o, int s) {
        if (s < l_count) {
          if (full && c >= first[s])
            acc_plain(cur, o, s);
          else if (c + S > first[s])
            acc_masked(cur, o, s, ub);
        }
      };
      float2 o0[RPT], o1[RPT];
      load_old(o0, tau[0]);
      dev::static_for<MAXLW>([&](auto SS) {
        constexpr int s = decltype(SS)::value;
        constexpr int nx = s + 1 < MAXLW ? s + 1 : s;
        if constexpr ((s & 1) == 0) {
          if constexpr (s + 1 < MAXLW) load_old(o1, tau[nx]);
          sum_slot(o0, s);
        } else {
          if constexpr (s + 1 < MAXLW) load_old(o0, tau[nx]);
          sum_slot(o1, s);
        }
      });
    }
    crow += S;
    if (crow >= H) crow -= H;
  }

  // Lanes g = 0..G-1 of one mode hold partial sums over disjoint frames;
  // their total goes through LDS so the workgroup adds its K x n_lags block
  // to the mode-major sums acc[mode][lag] with contiguous accesses.
  __syncthreads();  // every wave is done with the history
  float* blk = reinterpret_cast<float*>(hist4);  // [K][n_lags]
#pragma unroll
  for (int s = 0; s < MAXLW; ++s) {
    if (s < l_count) {
      float v = ax[s] + ay[s];
#pragma unroll
      for (int o = K; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
      if (g == 0) blk[m * n_lags + l_begin + s] = v;
    }
  }
  __syncthreads();
  const int64_t kmax = n_modes - m0 < K ? n_modes - m0 : K;
  const int nel = int(kmax) * n_lags;
  for (int e = threadIdx.x; e < nel; e += nthreads) {
    const int mm = e / n_lags, l = e - mm * n_lags;
    acc[(m0 + mm) * acc_pitch + l] += blk[e];
  }
}

template <int K, int P>
hipError_t pair_launch(const float2* ring, const float2* refspec, const float2* fscale,
                       int64_t n_modes, int64_t mode_stride,
                       int64_t capacity, int64_t T0, int64_t T1, const int32_t* lags,
                       int n_lags, int max_lag, float* acc, int acc_pitch, int hist, int waves,
                       size_t lds, hipStream_t s) {
  // Allow the LDS history beyond the default dynamic limit; a failure here
  // shows up as a launch error below.
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&pair_kernel<K, P>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
  const int64_t blocks = (n_modes + K - 1) / K;
  const int launched = waves < 4 ? 4 : waves;  // extra waves only help load
  hipLaunchKernelGGL((pair_kernel<K, P>), dim3(unsigned(blocks)), dim3(64 * launched), lds, s,
                     ring, refspec, fscale, n_modes, mode_stride, capacity, T0, T1, lags, n_lags,
                     max_lag, acc, acc_pitch, hist, waves);
  return hipGetLastError();
}

template <int K>
hipError_t pair_dispatch(int per_wave, const float2* ring, const float2* refspec,
                         const float2* fscale, int64_t n_modes,
                         int64_t mode_stride, int64_t capacity, int64_t T0, int64_t T1,
                         const int32_t* lags, int n_lags, int max_lag, float* acc,
                         int acc_pitch, int hist, int waves, size_t lds, hipStream_t s) {
#define NFS_PAIR_P(PP)                                                                     \
  case PP:                                                                                 \
    return pair_launch<K, PP>(ring, refspec, fscale, n_modes, mode_stride, capacity, T0,  \
                              T1, lags, n_lags, max_lag, acc, acc_pitch, hist, waves, lds, \
                              s);
  switch (per_wave) {
    NFS_PAIR_P(1)
    NFS_PAIR_P(2)
    NFS_PAIR_P(3)
    NFS_PAIR_P(4)
    NFS_PAIR_P(5)
    NFS_PAIR_P(6)
    NFS_PAIR_P(7)
    NFS_PAIR_P(8)
    default: return hipErrorInvalidValue;
  }
#undef NFS_PAIR_P
}

}  // namespace

hipError_t launch_pairs(const float2* ring, const float2* refspec, const float2* fscale,
                        int64_t n_modes, int64_t mode_stride,
                        int64_t capacity, int64_t T0, int64_t T1, const int32_t* lags,
                        int n_lags, int max_lag, float* acc, int acc_pitch, int modes, int hist,
                        int waves, int per_wave, size_t lds, hipStream_t s) {
#define NFS_PAIR_CASE(KK)                                                                  \
  case KK:                                                                                 \
    return pair_dispatch<KK>(per_wave, ring, refspec, fscale, n_modes, mode_stride,        \
                             capacity, T0, T1, lags, n_lags, max_lag, acc, acc_pitch, hist, \
                             waves, lds, s);
  switch (modes) {
    NFS_PAIR_CASE(64)
    NFS_PAIR_CASE(32)
    NFS_PAIR_CASE(16)
    NFS_PAIR_CASE(8)
    default: return hipErrorInvalidValue;
  }
#undef NFS_PAIR_CASE
}

}  // namespace nfs
