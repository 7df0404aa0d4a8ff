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
// ring are mirrored after its end so a lane's run of rows never wraps. With
// 16 modes per workgroup the history of lags up to about 500 frames fits
// half the LDS, so two workgroups share a CU and each covers the other's
// barrier and LDS waits.
//
// A ring slot holds sigma_t F[frame_t - reference]; the spectrum the pairs
// use is that plus (sigma_t - sigma_ref) F[reference], i.e. the normalised
// transform minus the constant sigma_ref F[reference], which cancels in
// every difference. The correction is applied once per (frame, mode) as the
// slot is copied into LDS.
#include "nfs_device.hpp"
#include "pair_plan.hpp"
#include "nfs_kernels.hpp"

namespace nfs {
namespace {
using dev::kSpecBF16;
using dev::kSpecF32;
using dev::unpack_bf16;
using dev::unpack_f16;

// Window total v of one (mode, lag) into the running sum: stored (and the
// compensation cleared) for the first window after a reset, else added
// with Kahan compensation kept in comp across windows, so long streams
// summed in many ring windows keep the compensated accuracy.
__device__ __forceinline__ void kahan_window_add(float* sum, float* comp, float v, bool assign) {
  if (assign) {
    *sum = v;
    *comp = 0.f;
    return;
  }
  const float c = *comp, a = *sum;
  const float y = v - c;
  const float t = a + y;
  *comp = (t - a) - y;
  *sum = t;
}

// K modes per workgroup, MAXLW lag slots per wave, NW waves launched: the
// lag list is split into lag_waves <= NW contiguous slices of near-equal
// length, one per wave; slots past a slice's end read harmless rows and are
// not summed. NW = 8 leaves each wave 256 registers, NW = 12 170. KAHAN: each
// lag's terms of a chunk are summed in FP32 and the chunk sums added with
// Kahan compensation. `spec` is the ring's storage type (uniform): FP32
// pairs, or BF16 / FP16 pairs decoded (and FP16 scaled by fscale[slot].z)
// as a slot is copied into LDS.
template <int K, int MAXLW, int NW, bool KAHAN>
__global__ __launch_bounds__(64 * NW) void pair_kernel(
    const char* __restrict__ ring, int spec, const float2* __restrict__ refspec,
    const float4* __restrict__ fscale, int64_t n_modes, int64_t mode_stride, int64_t capacity,
    int64_t T0, int64_t T1, const int32_t* __restrict__ lags, int n_lags, int max_lag,
    float* __restrict__ acc, int acc_pitch, bool assign, int H, int lag_waves,
    unsigned long long* __restrict__ work, float* __restrict__ comp) {
  static_assert(K == 16 || K == 8, "16 or 8 modes per workgroup");
  constexpr int S = kPairChunk;  // frames per chunk
  constexpr int G = 64 / K;         // lanes sharing one mode inside a wave
  constexpr int RPT = S / G;        // target rows per lane per chunk
  constexpr int V4 = K / 2;         // float4 (two modes) per ring row of the tile
  constexpr int MR = kPairMirror;  // rows mirrored past the end of the LDS ring
  // A wrapped row r < H plus a lane's run (at most S + MAXLW - 2 rows on)
  // must stay below H + MR.
  static_assert(MR >= S + MAXLW - 2, "mirror too short for a lane's row run");
  // A chunk's rows are S * V4 float4: at most one per thread.
  static_assert(S * V4 <= 64 * NW && (S * V4) % 64 == 0, "one float4 per loading thread");
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

  // Ring slot bytes and the two modes m0 + 2 col2, m0 + 2 col2 + 1 of a slot:
  // one float4 (FP32) or one 8-byte word pair (16-bit storage), kept raw in
  // a float4 until decoded.
  const bool f32 = spec == kSpecF32;
  const int64_t mode_bytes = f32 ? 8 : 4;
  const int64_t slot_bytes = mode_stride * mode_bytes;
  const char* ring_m0 = ring + m0 * mode_bytes;
  auto load_raw = [&](const char* p) -> float4 {
    if (f32) return *reinterpret_cast<const float4*>(p);
    const uint2 w = *reinterpret_cast<const uint2*>(p);
    return make_float4(__uint_as_float(w.x), __uint_as_float(w.y), 0.f, 0.f);
  };
  auto decode = [&](float4 raw, float inv_scale) -> float4 {
    if (f32) return raw;
    const uint32_t w0 = __float_as_uint(raw.x), w1 = __float_as_uint(raw.y);
    const float2 a = spec == kSpecBF16 ? unpack_bf16(w0) : unpack_f16(w0);
    const float2 b = spec == kSpecBF16 ? unpack_bf16(w1) : unpack_f16(w1);
    return make_float4(a.x * inv_scale, a.y * inv_scale, b.x * inv_scale, b.y * inv_scale);
  };
  // Window offset u lives in LDS row (u + max_lag) mod H.
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

  // History from earlier windows: frames [max(0, T0 - max_lag), T0), all
  // threads copying float4 elements in parallel (unrolled by 4 so several
  // loads are in flight). Frame T0 - pre + r goes to LDS row
  // (max_lag - pre + r) mod H.
  {
    const int pre = int(T0 - max_lag > 0 ? max_lag : T0);
    const int slot0 = int((T0 - pre) % capacity);
    const int total = pre * V4;
    const int cap0 = int(capacity);
    auto copy_one = [&](int e) {
      const int r = e / V4, col2 = e % V4;
      int slot = slot0 + r;
      if (slot >= cap0) slot -= cap0;
      const float4 raw = load_raw(ring_m0 + slot * slot_bytes + col2 * 2 * mode_bytes);
      const float4 sc = fscale[slot];
      put_row((max_lag - pre + r) % H, col2, corrected(decode(raw, sc.z), sc.y, ref4[col2]));
    };
    int e = threadIdx.x;
    for (; e + 3 * nthreads < total; e += 4 * nthreads) {
#pragma unroll
      for (int u = 0; u < 4; ++u) copy_one(e + u * nthreads);
    }
    for (; e < total; e += nthreads) copy_one(e);
  }

  // Thread e < S * V4 copies float4 column e % V4 of chunk row e / V4 (whole
  // waves take part or not), so its two modes' reference values stay in
  // registers. Slot arithmetic is 32-bit (capacity < 2^31).
  const int cap = int(capacity);
  const int n_el = S * V4;
  const bool loader = int(threadIdx.x) < n_el;
  const int pdt = int(threadIdx.x) / V4, pcol = int(threadIdx.x) % V4;
  const char* pbase = ring_m0 + pcol * 2 * mode_bytes;
  const float4 rr = loader ? ref4[pcol] : make_float4(0.f, 0.f, 0.f, 0.f);
  float4 pf = make_float4(0.f, 0.f, 0.f, 0.f);
  float pd = 0.f, ps = 1.f;
  // Rows of the chunk at window offset c, starting in ring slot cslot. A
  // row past the window end loads the chunk's first slot instead (only
  // masked targets ever meet it); every other row is a frame of the window
  // (len <= capacity), so c + dt < len <= cap and one wrap of cslot + dt
  // lands in [0, cap).
  const uint32_t ucap = uint32_t(cap), ulen = uint32_t(len), updt = uint32_t(pdt);
  auto prefetch = [&](int c, int cslot) {
    if (loader) {
      const uint32_t dt = uint32_t(c) + updt < ulen ? updt : 0u;
      uint32_t slot = uint32_t(cslot) + dt;
      slot = slot >= ucap ? slot - ucap : slot;
      pf = load_raw(pbase + size_t(slot) * size_t(slot_bytes));
      const float4 sc = fscale[slot];
      pd = sc.y;
      ps = sc.z;
    }
  };
  auto commit = [&](int crow) {
    if (loader) {
      int row = crow + pdt;
      if (row >= H) row -= H;
      put_row(row, pcol, corrected(decode(pf, ps), pd, rr));
    }
  };

  // Plain: running sums of dx^2 (ax) and dy^2 (ay). KAHAN: running sum
  // (ax) and compensation (ay) of the chunk sums.
  float ax[MAXLW], ay[MAXLW];
#pragma unroll
  for (int s = 0; s < MAXLW; ++s) ax[s] = ay[s] = 0.f;
  auto add_chunk = [&](int s, float v) {
    const float y = v - ay[s];
    const float t = ax[s] + y;
    ay[s] = (t - ax[s]) - y;
    ax[s] = t;
  };

  // |cur[i] - old[i]|^2 into lag slot s.
  auto acc_plain = [&](const float2* cur, const float2* old, int s) {
    if constexpr (KAHAN) {
      float px = 0.f, py = 0.f;
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const float dx = cur[i].x - old[i].x, dy = cur[i].y - old[i].y;
        px = fmaf(dx, dx, px);
        py = fmaf(dy, dy, py);
      }
      add_chunk(s, px + py);
    } else {
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const float dx = cur[i].x - old[i].x, dy = cur[i].y - old[i].y;
        ax[s] = fmaf(dx, dx, ax[s]);
        ay[s] = fmaf(dy, dy, ay[s]);
      }
    }
  };
  // The same with targets that have no partner yet (u < first) or lie past
  // the window end zeroed by selects, not branches.
  auto acc_masked = [&](const float2* cur, const float2* old, int s, int ub) {
    float px = 0.f, py = 0.f;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int u = ub + i;
      const bool ok = (u >= first[s]) & (u < len);
      const float dx = ok ? cur[i].x - old[i].x : 0.f;
      const float dy = ok ? cur[i].y - old[i].y : 0.f;
      if constexpr (KAHAN) {
        px = fmaf(dx, dx, px);
        py = fmaf(dy, dy, py);
      } else {
        ax[s] = fmaf(dx, dx, ax[s]);
        ay[s] = fmaf(dy, dy, ay[s]);
      }
    }
    if constexpr (KAHAN) add_chunk(s, px + py);
  };
  int first_max = 0;
#pragma unroll
  for (int s = 0; s < MAXLW; ++s)
    if (s < l_count) first_max = max(first_max, first[s]);


  // Lane (m, g) reads rows r + g * RPT + i of column m for a ring row r.
  const float2* lane_hist = hist + g * RPT * K + m;
  int crow = max_lag % H;          // LDS row of the chunk's first frame
  int cslot = int(T0 % capacity);  // ring slot of the chunk's first frame
  prefetch(0, cslot);

  // One chunk: copy its rows (prefetched one chunk earlier) into the LDS
  // ring, start loading the next chunk, then sum the wave's lags. Every
  // wave runs every chunk once, in order, so the barriers pair up.
  auto chunk = [&](int c, auto&& body) {
    commit(crow);
    __syncthreads();
    cslot += S;
    if (cslot >= cap) cslot -= cap;
    if (c + S < len) prefetch(c + S, cslot);
    // Rows of lag ts: the chunk's first row moved back by ts and wrapped
    // once, all in scalar registers (crow and ts are wave-uniform); a
    // lane's run then stays inside the ring and its mirror.
    auto rows = [&](int ts) -> const float2* {
      int r = crow - ts;
      if (r < 0) r += H;
      return lane_hist + r * K;
    };
    float2 cur[RPT];
    {
      const float2* src = lane_hist + crow * K;
#pragma unroll
      for (int i = 0; i < RPT; ++i) cur[i] = src[i * K];
    }
    body(c, cur, rows);
    crow += S;
    if (crow >= H) crow -= H;
  };

  auto load_rows = [&](float2 (&o)[RPT], const float2* src) {
#pragma unroll
    for (int i = 0; i < RPT; ++i) o[i] = src[i * K];
  };
  // Chunks where some target lacks a partner, or past the window end. Per
  // lag slot (wave-uniform): every target of the chunk has a partner (plain
  // sums), some do (masked sums) or none (skipped).
  auto generic = [&](int c, const float2* cur, auto&& rows) {
    const int ub = c + g * RPT;  // window offset of this lane's first target
    const bool full = c + S <= len;
    auto sum_slot = [&](const float2* o, int s) {
      if (s < l_count) {
        if (full && c >= first[s]) {
          acc_plain(cur, o, s);
        } else if (c + S > first[s]) {
          // Targets [lo, hi) of the chunk have partners. When both ends fall
          // on lane boundaries every lane's run is wholly in or out: plain
          // sums on the lanes that are in; otherwise per-target selects.
          const int lo = max(first[s] - c, 0), hi = min(len - c, S);
          if (lo % RPT == 0 && hi % RPT == 0) {
            if (g * RPT >= lo && g * RPT < hi) acc_plain(cur, o, s);
          } else {
            acc_masked(cur, o, s, ub);
          }
        }
      }
    };
    // Older rows are read only for lag slots with some target that has a
    // partner in this chunk (the same wave-uniform test sum_slot makes).
    auto wanted = [&](int s) { return s < l_count && c + S > first[s]; };
    float2 o0[RPT], o1[RPT];
    if (wanted(0)) load_rows(o0, rows(tau[0]));
    dev::static_for<MAXLW>([&](auto SS) {
      constexpr int s = decltype(SS)::value;
      constexpr int nx = s + 1 < MAXLW ? s + 1 : s;
      if constexpr ((s & 1) == 0) {
        if constexpr (s + 1 < MAXLW)
          if (wanted(nx)) load_rows(o1, rows(tau[nx]));
        sum_slot(o0, s);
      } else {
        if constexpr (s + 1 < MAXLW)
          if (wanted(nx)) load_rows(o0, rows(tau[nx]));
        sum_slot(o1, s);
      }
    });
  };
  // A full chunk in which every target has a partner for each of the
  // wave's L lags: no masks and no per-lag branches.
  auto full_chunk = [&](auto NL, auto CONSEC, const float2* cur, auto&& rows) {
    constexpr int L = decltype(NL)::value;
    constexpr bool CONS = decltype(CONSEC)::value;
    {
      if constexpr (CONS) {
        // Rows of lags tau[0] .. tau[0] + L - 1 overlap: one register
        // window serves them all, lag tau[0] + s reads win[L - 1 - s + i].
        constexpr int WL = RPT + L - 1;
        float2 win[WL];
        const float2* src = rows(tau[L - 1]);
#pragma unroll
        for (int i = 0; i < WL; ++i) win[i] = src[i * K];
        dev::static_for<L>([&](auto SS) {
          constexpr int s = decltype(SS)::value;
          acc_plain(cur, win + (L - 1 - s), s);
        });
      } else {
        // The older rows of lag s+1 are read while lag s is summed.
        float2 o0[RPT], o1[RPT];
        load_rows(o0, rows(tau[0]));
        dev::static_for<L>([&](auto SS) {
          constexpr int s = decltype(SS)::value;
          if constexpr ((s & 1) == 0) {
            if constexpr (s + 1 < L) load_rows(o1, rows(tau[s + 1]));
            acc_plain(cur, o0, s);
          } else {
            if constexpr (s + 1 < L) load_rows(o0, rows(tau[s + 1]));
            acc_plain(cur, o1, s);
          }
        });
      }
    }
  };

  // Chunks [0, ca): some target of the wave's lags may lack a partner;
  // [ca, lenS): full chunks; [lenS, len): the partial last chunk. A wave
  // has MAXLW or MAXLW - 1 lags (helper waves none); the full-chunk loop is
  // specialised on that count and on consecutive lags, so the wave's
  // accumulators stay in place through each loop.
  const int lenS = (len / S) * S;
  int ca = (first_max + S - 1) / S * S;
  if (ca > lenS) ca = lenS;
  int c = 0;
  for (; c < ca; c += S) chunk(c, generic);
  constexpr int LS = MAXLW > 1 ? MAXLW - 1 : 1;
  using LMax = std::integral_constant<int, MAXLW>;
  using LLess = std::integral_constant<int, LS>;
  using Yes = std::true_type;
  using No = std::false_type;
  if (l_count == MAXLW && consecutive) {
    for (; c < lenS; c += S)
      chunk(c, [&](int, const float2* cur, auto&& rows) { full_chunk(LMax{}, Yes{}, cur, rows); });
  } else if (l_count == MAXLW) {
    for (; c < lenS; c += S)
      chunk(c, [&](int, const float2* cur, auto&& rows) { full_chunk(LMax{}, No{}, cur, rows); });
  } else if (MAXLW > 1 && l_count == LS && consecutive) {
    for (; c < lenS; c += S)
      chunk(c, [&](int, const float2* cur, auto&& rows) { full_chunk(LLess{}, Yes{}, cur, rows); });
  } else if (MAXLW > 1 && l_count == LS) {
    for (; c < lenS; c += S)
      chunk(c, [&](int, const float2* cur, auto&& rows) { full_chunk(LLess{}, No{}, cur, rows); });
  } else {
    // Waves without lags only copy rows.
    for (; c < lenS; c += S) chunk(c, [](int, const float2*, auto&&) {});
  }
  for (; c < len; c += S) chunk(c, generic);

  // Work counter: the (target, lag) pairs this wave summed, from the same
  // per-lag first partnered offsets and window length that bound its masks.
  if (work && blockIdx.x == 0 && lane == 0 && l_count > 0) {
    unsigned long long npairs = 0;
#pragma unroll
    for (int s = 0; s < MAXLW; ++s)
      if (s < l_count && len > first[s]) npairs += static_cast<unsigned long long>(len - first[s]);
    atomicAdd(work, npairs);
  }

  // Lanes g = 0..G-1 of one mode hold partial sums over disjoint frames;
  // their total goes through LDS so the workgroup adds its K x n_lags block
  // to the mode-major sums acc[mode][lag] with contiguous accesses (or
  // stores it, `assign`, for the first window after the sums were reset).
  __syncthreads();  // every wave is done with the history
  float* blk = reinterpret_cast<float*>(hist4);  // [K][n_lags]
#pragma unroll
  for (int s = 0; s < MAXLW; ++s) {
    if (s < l_count) {
      float v = KAHAN ? ax[s] - ay[s] : ax[s] + ay[s];
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
    const int64_t at = (m0 + mm) * acc_pitch + l;
    if (KAHAN && comp)
      kahan_window_add(acc + at, comp + at, blk[e], assign);
    else
      acc[at] = assign ? blk[e] : acc[at] + blk[e];
  }
}

template <int K, int P, int NW, bool KAHAN>
hipError_t pair_launch(const char* ring, int spec, const float2* refspec, const float4* fscale,
                       int64_t n_modes, int64_t mode_stride, int64_t capacity, int64_t T0,
                       int64_t T1, const int32_t* lags, int n_lags, int max_lag, float* acc,
                       int acc_pitch, bool assign, int hist, int waves, size_t lds,
                       unsigned long long* work, float* comp, hipStream_t s) {
  // Allow the LDS history beyond the default dynamic limit; a failure here
  // shows up as a launch error below.
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&pair_kernel<K, P, NW, KAHAN>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
  const int64_t blocks = (n_modes + K - 1) / K;
  hipLaunchKernelGGL((pair_kernel<K, P, NW, KAHAN>), dim3(unsigned(blocks)), dim3(64 * NW), lds,
                     s, ring, spec, refspec, fscale, n_modes, mode_stride, capacity, T0, T1,
                     lags, n_lags, max_lag, acc, acc_pitch, assign, hist, waves, work, comp);
  return hipGetLastError();
}

// Long delays, whose history does not fit the LDS ring: one thread per mode
// (256 consecutive modes per workgroup, loads coalesced across modes),
// walking the window's targets t in order; the target's value is read
// once and each lag's older frame t - tau comes from the ring in memory
// (L2 or HBM), decoded and corrected as the LDS copy does. Up to
// kGlobalLags lags per launch. KAHAN: each lag's terms of 32 consecutive
// targets are summed in FP32 and the chunk sums added with Kahan
// compensation; the running sum minus the compensation is the result.
template <bool KAHAN>
__global__ __launch_bounds__(256) void pair_global_kernel(
    const char* __restrict__ ring, int spec, const float2* __restrict__ refspec,
    const float4* __restrict__ fscale, int64_t n_modes, int64_t mode_stride, int64_t capacity,
    int64_t T0, int64_t T1, const int32_t* __restrict__ lags, int n_lags,
    float* __restrict__ acc, int acc_pitch, bool assign, unsigned long long* __restrict__ work,
    float* __restrict__ comp) {
  constexpr int GL = kGlobalLags;
  const int64_t m = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (m >= n_modes) return;  // no barrier below
  const bool f32 = spec == kSpecF32;
  const int64_t mode_bytes = f32 ? 8 : 4;
  const float2 R = refspec[m];
  auto value = [&](int64_t slot) -> float2 {
    const float4 sc = fscale[slot];
    const char* p = ring + (slot * mode_stride + m) * mode_bytes;
    float2 a;
    if (f32) {
      a = *reinterpret_cast<const float2*>(p);
    } else {
      const uint32_t w = *reinterpret_cast<const uint32_t*>(p);
      a = spec == kSpecBF16 ? unpack_bf16(w) : unpack_f16(w);
      a = make_float2(a.x * sc.z, a.y * sc.z);
    }
    return make_float2(fmaf(sc.y, R.x, a.x), fmaf(sc.y, R.y, a.y));
  };
  int tau[GL];
#pragma unroll
  for (int s = 0; s < GL; ++s) tau[s] = __builtin_amdgcn_readfirstlane(s < n_lags ? lags[s] : 0);
  float run[GL], cmp[GL], part[GL];
#pragma unroll
  for (int s = 0; s < GL; ++s) run[s] = cmp[s] = part[s] = 0.f;
  int64_t slot = T0 % capacity;
  for (int64_t t = T0; t < T1; ++t) {
    const float2 at = value(slot);
#pragma unroll
    for (int s = 0; s < GL; ++s) {
      if (s < n_lags && t >= tau[s]) {
        const int64_t so = slot >= tau[s] ? slot - tau[s] : slot - tau[s] + capacity;
        const float2 o = value(so);
        const float dx = at.x - o.x, dy = at.y - o.y;
        part[s] = fmaf(dx, dx, fmaf(dy, dy, part[s]));
      }
    }
    if (KAHAN && ((t - T0) % 32 == 31 || t + 1 == T1)) {
#pragma unroll
      for (int s = 0; s < GL; ++s) {
        const float y = part[s] - cmp[s];
        const float z = run[s] + y;
        cmp[s] = (z - run[s]) - y;
        run[s] = z;
        part[s] = 0.f;
      }
    }
    if (++slot == capacity) slot = 0;
  }
  // Work counter: the (target, lag) pairs summed, targets t in [T0, T1) with
  // t >= tau (the bounds of the loop above).
  if (work && m == 0) {
    unsigned long long npairs = 0;
    for (int s = 0; s < n_lags && s < GL; ++s) {
      const int64_t from = T0 > tau[s] ? T0 : int64_t(tau[s]);
      if (T1 > from) npairs += static_cast<unsigned long long>(T1 - from);
    }
    atomicAdd(work, npairs);
  }
#pragma unroll
  for (int s = 0; s < GL; ++s) {
    if (s < n_lags) {
      const float total = KAHAN ? run[s] - cmp[s] : part[s];
      const int64_t at = m * acc_pitch + s;
      if (KAHAN && comp)
        kahan_window_add(acc + at, comp + at, total, assign);
      else
        acc[at] = assign ? total : acc[at] + total;
    }
  }
}

// Up to 8 lag waves run in 8-wave workgroups; more (only with 6 or more
// lags per wave) in 12-wave ones.
template <int K, bool KAHAN>
hipError_t pair_dispatch(int per_wave, const char* ring, int spec, const float2* refspec,
                         const float4* fscale, int64_t n_modes, int64_t mode_stride,
                         int64_t capacity, int64_t T0, int64_t T1, const int32_t* lags,
                         int n_lags, int max_lag, float* acc, int acc_pitch, bool assign,
                         int hist, int waves, size_t lds, unsigned long long* work,
                         float* comp, hipStream_t s) {
#define NFS_PAIR_P(PP, NWW)                                                                 \
  return pair_launch<K, PP, NWW, KAHAN>(ring, spec, refspec, fscale, n_modes, mode_stride, \
                                        capacity, T0, T1, lags, n_lags, max_lag, acc,       \
                                        acc_pitch, assign, hist, waves, lds, work, comp, s)
  if (waves <= 8) {
    switch (per_wave) {
      case 1: NFS_PAIR_P(1, 8);
      case 2: NFS_PAIR_P(2, 8);
      case 3: NFS_PAIR_P(3, 8);
      case 4: NFS_PAIR_P(4, 8);
      case 5: NFS_PAIR_P(5, 8);
      case 6: NFS_PAIR_P(6, 8);
      case 7: NFS_PAIR_P(7, 8);
      case 8: NFS_PAIR_P(8, 8);
      default: return hipErrorInvalidValue;
    }
  }
  if (waves <= 12) {
    switch (per_wave) {
      case 6: NFS_PAIR_P(6, 12);
      case 7: NFS_PAIR_P(7, 12);
      case 8: NFS_PAIR_P(8, 12);
      default: return hipErrorInvalidValue;
    }
  }
  return hipErrorInvalidValue;
#undef NFS_PAIR_P
}

}  // namespace

hipError_t launch_pairs(const void* ring, int spec, bool kahan, const float2* refspec,
                        const float4* fscale, int64_t n_modes, int64_t mode_stride,
                        int64_t capacity, int64_t T0, int64_t T1, const int32_t* lags,
                        int n_lags, int max_lag, float* acc, int acc_pitch, bool assign,
                        int modes, int hist, int waves, int per_wave, size_t lds,
                        unsigned long long* work, float* comp, hipStream_t s) {
  const char* r = static_cast<const char*>(ring);
  if (modes == 0) {  // the global-memory kernel (long delays)
    if (n_lags < 1 || n_lags > kGlobalLags) return hipErrorInvalidValue;
    const dim3 grid(unsigned((n_modes + 255) / 256));
    if (kahan)
      hipLaunchKernelGGL(pair_global_kernel<true>, grid, dim3(256), 0, s, r, spec, refspec,
                         fscale, n_modes, mode_stride, capacity, T0, T1, lags, n_lags, acc,
                         acc_pitch, assign, work, comp);
    else
      hipLaunchKernelGGL(pair_global_kernel<false>, grid, dim3(256), 0, s, r, spec, refspec,
                         fscale, n_modes, mode_stride, capacity, T0, T1, lags, n_lags, acc,
                         acc_pitch, assign, work, comp);
    return hipGetLastError();
  }
#define NFS_PAIR_CASE(KK, KH)                                                              \
  return pair_dispatch<KK, KH>(per_wave, r, spec, refspec, fscale, n_modes, mode_stride,  \
                               capacity, T0, T1, lags, n_lags, max_lag, acc, acc_pitch,   \
                               assign, hist, waves, lds, work, comp, s)
  if (modes == 16) {
    if (kahan) NFS_PAIR_CASE(16, true);
    NFS_PAIR_CASE(16, false);
  }
  if (modes == 8) {
    if (kahan) NFS_PAIR_CASE(8, true);
    NFS_PAIR_CASE(8, false);
  }
  return hipErrorInvalidValue;
#undef NFS_PAIR_CASE
}

}  // namespace nfs
