// Per-image 2D real-to-complex transform, split into a row pass and a column
// pass. The paper transforms every image once and differences transforms
// instead of transforming every image difference (processing section:
// linearity of the Fourier transform); it normalises by dividing each
// transform by its zero-frequency value, which is what the column pass's
// epilogue does with the exact pixel sum from the row pass.
//
// Both passes use a two-level (P1 x P2) decomposition of each 1D transform:
// every thread does one P-point DFT in registers, the partial results are
// twiddled and exchanged once through LDS, and a second register DFT
// finishes the transform. Twiddles of the register DFTs are compile-time
// constants built in double; the exchange twiddles come from a table built
// in double on the host and rounded once to float, kept in LDS with one
// pad entry per 8 (fewer bank conflicts for strided reads).
//
// The intermediate between the passes is [frame][tiles][n rows][TWD]: tiles
// of the columns one column-pass workgroup transforms (8 up to n = 1024; at
// least 2), so a row pass wave writes runs of 4 rows x TWD columns and a
// column pass wave reads 8 rows x 8 columns contiguously.
#include "fft_common.hpp"
#include "nfs_device.hpp"
#include "nfs_kernels.hpp"

namespace nfs {
using namespace dev;

namespace {

// Orders a wave's LDS writes before later LDS reads of other lanes of the
// same wave: the exchanges of the row pass never leave a wave, so no
// workgroup barrier is needed.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int N>
struct RowCfg {
  static constexpr int H = N / 2;                    // complex points per row
  static constexpr int P1 = 1 << (ilog2(H) / 2);     // H = P1 * P2, P2 in {P1, 2 P1}
  static constexpr int P2 = H / P1;
  static constexpr int Q = P2 / P1;
  static constexpr int PITCH = P2 * (P1 + 1) + 4;    // LDS complex values per row
  static constexpr int R0 = fit_rows(256 / P1, PITCH, tw_len(N) * 8);
  static constexpr int R = R0 < N ? R0 : N;          // rows per workgroup
  static constexpr int THREADS = R * P1;
  static constexpr int RB = N / R;                   // row blocks per frame
  // The intermediate is cut into the column pass's tiles.
  static constexpr int TWD = ColCfg<N>::TWD;
  static constexpr int TILES = ColCfg<N>::TILES;
  static_assert(64 % P1 == 0, "a row's threads must sit in one wave");
};


// Two row-pass workgroups per CU where a thread's state fits the register
// budget of two waves per SIMD without spilling (integer pixels, no window,
// up to 1024 pixels per row).
template <int N, typename T, bool WIN, bool ABS>
constexpr int row_min_waves() {
  return N <= 512 || (N == 1024 && std::is_same<T, uint16_t>::value && !WIN) ? 2 : 1;
}

template <typename T>
struct RawPair;  // two neighbouring pixels as loaded
template <>
struct RawPair<uint16_t> {
  using type = uint32_t;
};
template <>
struct RawPair<float> {
  using type = float2;
};

template <typename T>
__device__ __forceinline__ typename RawPair<T>::type load_pair(const T* p) {
  return *reinterpret_cast<const typename RawPair<T>::type*>(p);
}

// ---------------------------------------------------------------------------
// Row pass. Real row u of N pixels (minus the reference row, times the
// window) -> z[j] = u[2j] + i u[2j+1] (H points), Z = DFT_H(z), then
// X[k] = (Z[k] + conj Z[H-k])/2 - i W_N^k (Z[k] - conj Z[H-k])/2 for
// k = 0..H-1 (the real-input split; X[H], never binned, is written to
// nyq[f][y] only for full half-plane plans, nyq not null). A row's P1
// threads sit in one wave and only they touch the row's LDS, so the frame
// loop has no workgroup barrier. A workgroup owns R rows and loops over up
// to `per_group` frames of the batch, loading the next frame's pixels while
// it transforms the current one. ABS: also write rowabs[f][y], the row's sum
// of |what is transformed| (bounds every coefficient of the frame).
template <int N, typename T, bool WIN, bool ABS>
__global__ __launch_bounds__(RowCfg<N>::THREADS, (row_min_waves<N, T, WIN, ABS>())) void row_pass_kernel(
    const T* __restrict__ frames, const T* __restrict__ ref, const float* __restrict__ window,
    int nframes, int per_group, float2* __restrict__ inter, double* __restrict__ rowsum,
    double* __restrict__ rowabs, float* __restrict__ nyq, const float2* __restrict__ tw) {
  using C = RowCfg<N>;
  using Raw = typename RawPair<T>::type;
  constexpr bool U16 = std::is_same<T, uint16_t>::value;
  constexpr int H = C::H, P1 = C::P1, P2 = C::P2, Q = C::Q, R = C::R, RB = C::RB;
  constexpr int PITCH = C::PITCH, THREADS = C::THREADS, TILES = C::TILES, TWD = C::TWD;
  __shared__ float2 lds[R * PITCH];
  __shared__ float2 twl[tw_len(N)];

  const int tid = threadIdx.x;
  const int rl = tid / P1, j1 = tid % P1;
  const int rblk = blockIdx.x % RB;
  const int f_begin = (blockIdx.x / RB) * per_group;
  const int f_end = min(nframes, f_begin + per_group);
  const int y = rblk * R + rl;
  float2* row_lds = lds + rl * PITCH;

  for (int i = tid; i < N; i += THREADS) twl[tw_skew(i)] = tw[i];

  // Up to 32 pixel pairs per thread the reference row stays in registers and
  // the next frame is prefetched; larger rows reload both from cache.
  constexpr bool CACHE = P2 <= 32;
  constexpr int NC = CACHE ? P2 : 1;
  Raw refv[NC], raw[NC];
  auto ref_pair = [&](int j2) -> Raw {
    if (!ref) {
      if constexpr (U16) return 0u; else return make_float2(0.f, 0.f);
    }
    return load_pair(ref + int64_t(y) * N + 2 * (j1 + P1 * j2));
  };
  auto raw_pair = [&](int f, int j2) -> Raw {
    return load_pair(frames + (int64_t(f) * N + y) * N + 2 * (j1 + P1 * j2));
  };
  auto load_raw = [&](int f) {
#pragma unroll
    for (int j2 = 0; j2 < NC; ++j2) raw[j2] = raw_pair(f, j2);
  };
  if constexpr (CACHE) {
#pragma unroll
    for (int j2 = 0; j2 < P2; ++j2) refv[j2] = ref_pair(j2);
    if (f_begin < f_end) load_raw(f_begin);
  }
  __syncthreads();  // the twiddle table is shared by all rows

  for (int f = f_begin; f < f_end; ++f) {
    float2 v[P2];
    int si = 0, sia = 0;
    double sd = 0.0, sda = 0.0;
#pragma unroll
    for (int j2 = 0; j2 < P2; ++j2) {
      float a, b;
      Raw rp, px;
      if constexpr (CACHE) {
        rp = refv[j2];
        px = raw[j2];
      } else {
        rp = ref_pair(j2);
        px = raw_pair(f, j2);
      }
      if constexpr (U16) {
        // Integer difference from the reference: exact, and summed exactly.
        const int da = int(px & 0xffffu) - int(rp & 0xffffu);
        const int db = int(px >> 16) - int(rp >> 16);
        a = float(da);
        b = float(db);
        if constexpr (!WIN) si += da + db;
        if constexpr (ABS && !WIN) sia += abs(da) + abs(db);
      } else {
        a = px.x - rp.x;
        b = px.y - rp.y;
      }
      if constexpr (WIN) {
        const float2 ww =
            *reinterpret_cast<const float2*>(window + int64_t(y) * N + 2 * (j1 + P1 * j2));
        a *= ww.x;
        b *= ww.y;
      }
      if constexpr (!U16 || WIN) sd += double(a) + double(b);
      if constexpr (ABS && (!U16 || WIN)) sda += double(fabsf(a)) + double(fabsf(b));
      v[j2] = make_float2(a, b);
    }
    // Next frame's pixels are in flight while this one is transformed.
    if constexpr (CACHE) {
      if (f + 1 < f_end) load_raw(f + 1);
    }
    // Row sum of what is transformed, butterfly over the row's P1 lanes.
    double s;
    if constexpr (U16 && !WIN) {
#pragma unroll
      for (int o = P1 / 2; o >= 1; o >>= 1) si += __shfl_xor(si, o, P1);
      s = double(si);
    } else {
#pragma unroll
      for (int o = P1 / 2; o >= 1; o >>= 1) sd += __shfl_xor(sd, o, P1);
      s = sd;
    }
    if (j1 == 0) rowsum[int64_t(f) * N + y] = s;
    if constexpr (ABS) {
      double sa;
      if constexpr (U16 && !WIN) {
#pragma unroll
        for (int o = P1 / 2; o >= 1; o >>= 1) sia += __shfl_xor(sia, o, P1);
        sa = double(sia);
      } else {
#pragma unroll
        for (int o = P1 / 2; o >= 1; o >>= 1) sda += __shfl_xor(sda, o, P1);
        sa = sda;
      }
      if (j1 == 0) rowabs[int64_t(f) * N + y] = sa;
    }

    // First level: DFT over j2 of z[j1 + P1 j2], twiddle W_H^{j1 k2} = W_N^{2 j1 k2}.
    dft<P2>(v);
    static_for<P2>([&](auto K2) {
      constexpr int k2 = decltype(K2)::value;
      float2 yv = v[bitrev<P2>(k2)];
      if constexpr (k2 != 0) yv = cmul(yv, twl[tw_skew((2 * j1 * k2) & (N - 1))]);
      row_lds[k2 * (P1 + 1) + j1] = yv;
    });
    wave_lds_sync();

    // Second level: for k2 = j1 + q P1, DFT over j1 gives Z[k2 + P2 k1].
    float2 z[Q][P1];
    static_for<Q>([&](auto QQ) {
      constexpr int q = decltype(QQ)::value;
      const int k2 = j1 + q * P1;
      float2 w[P1];
#pragma unroll
      for (int j = 0; j < P1; ++j) w[j] = row_lds[k2 * (P1 + 1) + j];
      dft<P1>(w);
      static_for<P1>([&](auto K1) {
        constexpr int k1 = decltype(K1)::value;
        z[q][k1] = w[bitrev<P1>(k1)];
      });
    });
    wave_lds_sync();
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int k1 = 0; k1 < P1; ++k1) row_lds[(j1 + q * P1) + P2 * k1] = z[q][k1];
    wave_lds_sync();

    // k_x = n/2 (full half-plane plans): X[H] = Re Z[0] - Im Z[0], real.
    if (nyq && j1 == 0) {
      const float2 z0 = row_lds[0];
      nyq[int64_t(f) * N + y] = z0.x - z0.y;
    }
    // Real-input split of this thread's outputs k = j1 + P1 i, stored into
    // the intermediate: column k % TWD of row y of tile k / TWD.
    float2* frame_out = inter + int64_t(f) * TILES * N * TWD;
    // When TWD divides P1, output i of this thread is a fixed stride from
    // output 0 (one base pointer, compile-time offsets).
    float2* out0 = frame_out + (int64_t(j1 / TWD) * N + y) * TWD + (j1 % TWD);
#pragma unroll
    for (int i = 0; i < P2; ++i) {
      const int k = j1 + P1 * i;
      const float2 zk = row_lds[k];
      const float2 zm = row_lds[(H - k) & (H - 1)];
      const float2 e = make_float2(zk.x + zm.x, zk.y - zm.y);   // Z[k] + conj Z[H-k]
      const float2 d = make_float2(zk.x - zm.x, zk.y + zm.y);   // Z[k] - conj Z[H-k]
      const float2 wd = cmul(d, twl[tw_skew(k)]);
      const float2 X = make_float2(0.5f * (e.x + wd.y), 0.5f * (e.y - wd.x));
      if constexpr (P1 % TWD == 0)
        out0[int64_t(i) * (P1 / TWD) * N * TWD] = X;
      else
        frame_out[(int64_t(k / TWD) * N + y) * TWD + (k % TWD)] = X;
    }
    wave_lds_sync();  // the row's LDS is rewritten by the next frame
  }
}

// ---------------------------------------------------------------------------
// Scale of the reference image from its row sums, in a fixed order
// (strided partial sums, butterfly per wave, waves in index order):
// refscal = {S_ref, n^2/S_ref}, sigma 0 (and bit 0 of *status) when S_ref
// is not positive and finite. Frames' scales are formed in the column pass.
__global__ __launch_bounds__(256) void ref_scale_kernel(int n, const double* __restrict__ rowsum,
                                                        double* __restrict__ refscal,
                                                        int32_t* __restrict__ status) {
  __shared__ double red[4];
  const int tid = threadIdx.x;
  double s = 0.0;
  for (int y = tid; y < n; y += 256) s += rowsum[y];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  if (tid == 0) {
    const double total = ((red[0] + red[1]) + red[2]) + red[3];
    const bool bad = !(total > 0.0) || !isfinite(total);
    refscal[0] = total;
    refscal[1] = bad ? 0.0 : double(n) * double(n) / total;
    if (bad) atomicOr(status, 1);
  }
}

// ---------------------------------------------------------------------------
// Column pass over CW columns: DFT_N over the rows of each frame of the
// group. REF: store the reference transform F[reference] unscaled in
// refspec. Otherwise the rows were (frame - reference) of frame t0 + f:
// every workgroup of the frame forms S = S_ref + (sum of its row sums) in
// the same fixed order (strided partial sums, butterfly per wave, waves in
// index order) and sigma = n^2 / S, stores sigma * X (X = F[frame -
// reference]) into ring slot (t0 + f) mod capacity, and the frame's first
// column group writes fscale[slot] = {sigma, sigma - sigma_ref}; a frame
// whose S is not positive and finite gets sigma = 0 and sets bit 0 of
// *status. Both store 0 at k = 0 and fill the slots of the tiled layout
// (ring_slot; n_modes slots); the pair kernel adds (sigma - sigma_ref) * refspec when it
// reads a slot. SPEC (ring storage type): FP32 pairs; BF16 pairs rounded
// once; FP16 pairs of sigma * 2^e * X with e the largest exponent for which
// 2^e * sigma * (sum of the frame's rowabs) <= 65504, 2^-e written as
// fscale[slot].z (1 otherwise). Per-thread store offsets are computed once;
// the next frame's columns are loaded during the second level.
template <int N, bool REF, int SPEC>
__global__ __launch_bounds__(ColCfg<N>::THREADS, ColCfg<N>::MINW) void col_pass_kernel(
    const float2* __restrict__ inter, const double* __restrict__ rowsum,
    const double* __restrict__ rowabs, const double* __restrict__ refscal,
    float4* __restrict__ fscale, int32_t* __restrict__ status, int nframes, int per_group,
    int64_t t0, int64_t capacity, int64_t mode_stride, int64_t n_modes,
    const int32_t* __restrict__ tiles, const float2* __restrict__ tw, char* __restrict__ ring,
    float2* __restrict__ refspec, unsigned long long* __restrict__ work) {
  static_assert(!REF || SPEC == kSpecF32, "the reference transform is kept in FP32");
  constexpr bool F16 = SPEC == kSpecF16;
  constexpr uint32_t MODE_BYTES = SPEC == kSpecF32 ? 8u : 4u;
  using C = ColCfg<N>;
  constexpr int P1 = C::P1, P2 = C::P2, Q = C::Q, CP = C::CP, CW = C::CW;
  constexpr int THREADS = C::THREADS, GROUPS = C::GROUPS, TILES = C::TILES, TWD = C::TWD;
  constexpr int WW = THREADS < 64 ? THREADS : 64;  // lanes of a (possibly partial) wave
  constexpr int NWAVES = (THREADS + 63) / 64;
  __shared__ float2 lds[CW * CP];
  __shared__ float2 twl[C::TWL];
  __shared__ double red[NWAVES];
  __shared__ double red_abs[F16 ? NWAVES : 1];

  // Workgroups are dispatched round-robin over the 8 XCDs; renumber them so
  // neighbouring column groups of a frame (which write the two halves of
  // the same 128-byte lines of the stored rows) share an XCD and its L2.
  int bid = blockIdx.x;
  if (gridDim.x % 8 == 0) bid = (bid % 8) * int(gridDim.x / 8) + bid / 8;
  const int grp = bid % GROUPS;
  const int f_begin = (bid / GROUPS) * per_group;
  const int f_end = min(nframes, f_begin + per_group);
  const int kx0 = grp * CW;
  const int tid = threadIdx.x;
  const int c = tid % CW, j1 = tid / CW;
  const int kx = kx0 + c;

  load_col_twiddles<N>(twl, tw, tid, THREADS);

  // Outputs of this thread: rows r = (j1 + q P1) + P2 k1 of column kx,
  // stored at byte offset 8 ring_slot(r, kx) of the spectrum (tiled slot
  // layout: a workgroup's columns fill one contiguous block), or not at all
  // (kDropOffset) when the row is not kept in the column's tile. Up to 32
  // outputs per thread the offsets stay in registers across frames; more
  // are looked up again per frame.
  constexpr bool CACHE = Q * P1 <= 32;
  constexpr int QC = CACHE ? Q : 1, PC = CACHE ? P1 : 1;
  auto store_offset = [&](int q, int k1) -> uint32_t {
    const int r = (j1 + q * P1) + P2 * k1;
    const int slot = ring_slot(N, tiles, r, kx);
    return slot >= 0 ? uint32_t(slot) * 8u : kDropOffset;
  };
  uint32_t at[QC][PC];
  if constexpr (CACHE) {
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int k1 = 0; k1 < P1; ++k1) at[q][k1] = store_offset(q, k1);
  }

  auto load_cols = [&](float2 (&v)[P2], int f) {
    // Column kx is column kx % TWD of tile kx / TWD of the intermediate.
    const float2* src = inter + (int64_t(f) * TILES + kx / TWD) * N * TWD + kx % TWD;
#pragma unroll
    for (int j2 = 0; j2 < P2; ++j2) v[j2] = src[(j1 + P1 * j2) * TWD];
  };
  float2 v[P2];
  if (CACHE && f_begin < f_end) load_cols(v, f_begin);
  float2* col_lds = lds + c * CP;
  int64_t slot = (t0 + f_begin) % capacity;
  const uint32_t spec_bytes = uint32_t(n_modes) * MODE_BYTES;
  double s_ref = 0.0, sigma_ref = 0.0;
  if constexpr (!REF) {
    s_ref = refscal[0];
    sigma_ref = refscal[1];
  }
  __syncthreads();

  for (int f = f_begin; f < f_end; ++f) {
    // This thread's share of the frame's pixel sum (loads issued early).
    double part = 0.0, part_abs = 0.0;
    if constexpr (!REF) {
      for (int y = tid; y < N; y += THREADS) part += rowsum[int64_t(f) * N + y];
    }
    if constexpr (F16) {
      for (int y = tid; y < N; y += THREADS) part_abs += rowabs[int64_t(f) * N + y];
    }
    if constexpr (!CACHE) load_cols(v, f);
    dft<P2>(v);
    static_for<P2>([&](auto K2) {
      constexpr int k2 = decltype(K2)::value;
      float2 yv = v[bitrev<P2>(k2)];
      if constexpr (k2 != 0) yv = cmul(yv, col_twiddle<N>(twl, tw, (j1 * k2) & (N - 1)));
      col_lds[k2 * (P1 + 1) + j1] = yv;
    });
    if constexpr (!REF) {
#pragma unroll
      for (int o = WW / 2; o >= 1; o >>= 1) part += __shfl_xor(part, o, WW);
      if ((tid & 63) == 0) red[tid >> 6] = part;
    }
    if constexpr (F16) {
#pragma unroll
      for (int o = WW / 2; o >= 1; o >>= 1) part_abs += __shfl_xor(part_abs, o, WW);
      if ((tid & 63) == 0) red_abs[tid >> 6] = part_abs;
    }
    __syncthreads();
    if constexpr (CACHE) {
      if (f + 1 < f_end) load_cols(v, f + 1);
    }

    float scale = 1.f;
    if constexpr (!REF) {
      double tot = red[0];
#pragma unroll
      for (int w = 1; w < NWAVES; ++w) tot += red[w];
      const double S = s_ref + tot;
      const bool bad = !(S > 0.0) || !isfinite(S);
      const double sigma = bad ? 0.0 : double(N) * double(N) / S;
      int e = 0;
      if constexpr (F16) {
        double l1 = red_abs[0];
#pragma unroll
        for (int w = 1; w < NWAVES; ++w) l1 += red_abs[w];
        e = f16_exponent(sigma * l1);  // bounds every |sigma * X(k)|
      }
      scale = float(ldexp(sigma, e));
      if (grp == 0 && tid == 0) {
        fscale[slot] =
            make_float4(float(sigma), float(sigma - sigma_ref), float(ldexp(1.0, -e)), 0.f);
        if (bad) atomicOr(status, 1);
        if (work) atomicAdd(work, 1ull);  // work counter: frames transformed
      }
    }
    const BufferRsrc dst =
        make_buffer(REF ? static_cast<void*>(refspec)
                        : static_cast<void*>(ring + slot * mode_stride * int64_t(MODE_BYTES)),
                    spec_bytes);
    static_for<Q>([&](auto QQ) {
      constexpr int q = decltype(QQ)::value;
      const int k2 = j1 + q * P1;
      float2 w[P1];
#pragma unroll
      for (int j = 0; j < P1; ++j) w[j] = col_lds[k2 * (P1 + 1) + j];
      dft<P1>(w);
      static_for<P1>([&](auto K1) {
        constexpr int k1 = decltype(K1)::value;
        uint32_t o;
        if constexpr (CACHE) o = at[q][k1]; else o = store_offset(q, k1);
        float2 X = w[bitrev<P1>(k1)];
        if constexpr (!REF) {
          X.x *= scale;
          X.y *= scale;
        }
        // Only output (q, k1) = (0, 0) of thread 0 of group 0 is k = 0.
        if constexpr (q == 0 && k1 == 0) {
          if (o == 0) X = make_float2(0.f, 0.f);
        }
        if constexpr (SPEC == kSpecF32) {
          buffer_store(X, dst, o);
        } else {
          // Offsets were computed for 8-byte modes; halving keeps the drop
          // value out of range.
          buffer_store_u32(SPEC == kSpecBF16 ? pack_bf16(X) : pack_f16(X), dst, o >> 1);
        }
      });
    });
    if (++slot == capacity) slot = 0;
    __syncthreads();  // LDS is rewritten by the next frame
  }
}

// ---------------------------------------------------------------------------
// The k_x = n/2 column of full half-plane plans, one workgroup per frame:
// Y(k_y) = sum_y x[y] W_n^{k_y y} of the row pass's real values x[y] =
// X_y(n/2), by an iterative radix-2 transform in LDS (bit-reversed load,
// log2 n butterfly stages, twiddles from the plan's table), stored at slot
// nyq_slot + r of the frame's spectrum, r = k_y mod n. REF: the reference
// frame's values, unscaled FP32 into refspec. Otherwise frame t0 + f,
// scaled and encoded exactly as the column pass did its other modes, with
// sigma and the FP16 scale that pass wrote to fscale[slot] (it runs first
// on the stream): sigma 2^e = fscale.x / fscale.z.
template <bool REF, int SPEC>
__global__ __launch_bounds__(256) void nyquist_col_kernel(
    int n, const float* __restrict__ nyq, const float2* __restrict__ tw,
    const float4* __restrict__ fscale, int64_t t0, int64_t capacity, int64_t mode_stride,
    int64_t nyq_slot, char* __restrict__ ring, float2* __restrict__ refspec) {
  extern __shared__ float2 buf[];
  const int f = blockIdx.x;
  const int lg = __builtin_ctz(uint32_t(n));
  for (int y = threadIdx.x; y < n; y += blockDim.x) {
    const int rv = int(__brev(uint32_t(y)) >> (32 - lg));
    buf[rv] = make_float2(nyq[int64_t(f) * n + y], 0.f);
  }
  __syncthreads();
  for (int half = 1; half < n; half <<= 1) {
    const int step = n / (2 * half);  // twiddle W_n^{j step} = W_{2 half}^j
    for (int b = threadIdx.x; b < n / 2; b += blockDim.x) {
      const int j = b % half;
      const int i0 = (b / half) * 2 * half + j;
      const float2 a = buf[i0];
      const float2 c = cmul(buf[i0 + half], tw[j * step]);
      buf[i0] = make_float2(a.x + c.x, a.y + c.y);
      buf[i0 + half] = make_float2(a.x - c.x, a.y - c.y);
    }
    __syncthreads();
  }
  if constexpr (REF) {
    for (int r = threadIdx.x; r < n; r += blockDim.x) refspec[nyq_slot + r] = buf[r];
  } else {
    const int64_t slot = (t0 + f) % capacity;
    const float4 sc = fscale[slot];
    const float scale = sc.x == 0.f ? 0.f : sc.x / sc.z;  // sigma 0: degenerate frame
    char* base = ring + slot * mode_stride * int64_t(SPEC == kSpecF32 ? 8 : 4);
    for (int r = threadIdx.x; r < n; r += blockDim.x) {
      const float2 X = make_float2(buf[r].x * scale, buf[r].y * scale);
      if constexpr (SPEC == kSpecF32)
        reinterpret_cast<float2*>(base)[nyq_slot + r] = X;
      else
        reinterpret_cast<uint32_t*>(base)[nyq_slot + r] =
            SPEC == kSpecBF16 ? pack_bf16(X) : pack_f16(X);
    }
  }
}

// ---------------------------------------------------------------------------
// Fused transform: the row and column passes of a batch in one persistent
// launch, with the row-to-column intermediate of a frame handed over inside
// one XCD. Frame j belongs to XCD j mod 8 (workgroups are dispatched to the
// 8 XCDs round robin, and each reads the XCD it runs on from the XCC_ID
// register). Each XCD has its own task queue: its s-th frame, j = x + 8 s,
// is job slot s, made of RB row tasks (16 rows each) followed by GROUPS
// column tasks (8 columns each). Row tasks write the first `keep` column
// tiles of their rows to the XCD's L2-sized buffer A and the others to
// buffer B; column tasks read them back. Only workgroups of one XCD touch its
// buffers and counters, so the hand-off needs no L2 writeback: a row task
// waits for its stores to reach L2 (vmcnt 0) before counting itself done,
// and a column task, after seeing every row task of its job done,
// invalidates its L1 (buffer_inv sc0) before loading.
//
// Scheduler state (cleared before the launch): per XCD a task counter and,
// per job slot, rows done and columns done. Every access to them is an
// atomic read-modify-write at agent scope (polls add an opaque zero, so the
// compiler keeps them atomics instead of turning them into loads, which
// would not see the counts the atomics keep in the XCD's L2). A worker
// claims task k = s * TPJ + i of its XCD's queue and stops when slot s has
// no frame. Every wait is for tasks claimed earlier (smaller k) by running
// workers: the row tasks of s (column tasks), the column tasks of s - 1
// (row tasks: buffers A and B are reused), so the waits end whatever the
// number of resident workers. Waits are bounded by spin_limit polls; past
// it the worker sets bit 1 of *status and stops (the result is then
// incomplete).
constexpr int kFusedLine = 64;  // ints per XCD counter (one 256-byte line)

__device__ __forceinline__ int sched_add(int* p, int v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int sched_peek(int* p) {
  int zero = 0;
  asm volatile("" : "+v"(zero));
  return sched_add(p, zero);
}
// Poll *p until pred(value) or spin_limit polls; returns the last value.
template <class Pred>
__device__ __forceinline__ int sched_wait(int* p, Pred pred, unsigned spin_limit, bool* timed_out) {
  int v = sched_peek(p);
  for (unsigned it = 0; !pred(v); ++it) {
    if (it >= spin_limit) {
      *timed_out = true;
      return v;
    }
    __builtin_amdgcn_s_sleep(2);
    v = sched_peek(p);
  }
  return v;
}

template <int N, typename T, bool WIN, bool ABS, int SPEC>
__global__ __launch_bounds__(256, 2) void fused_transform_kernel(
    const T* __restrict__ frames, const T* __restrict__ ref, const float* __restrict__ window,
    int nframes, double* __restrict__ rowsum, double* __restrict__ rowabs,
    float2* __restrict__ bufA, float2* __restrict__ bufB, int keep, int* __restrict__ sched,
    int slots, unsigned spin_limit, const double* __restrict__ refscal,
    float4* __restrict__ fscale, int32_t* __restrict__ status, int64_t t0, int64_t capacity,
    int64_t mode_stride, int64_t n_modes, const int32_t* __restrict__ tiles,
    const float2* __restrict__ tw, char* __restrict__ ring, unsigned long long* __restrict__ work) {
  using RC = RowCfg<N>;
  using CC = ColCfg<N>;
  using Raw = typename RawPair<T>::type;
  constexpr bool U16 = std::is_same<T, uint16_t>::value;
  constexpr bool F16 = SPEC == kSpecF16;
  constexpr uint32_t MODE_BYTES = SPEC == kSpecF32 ? 8u : 4u;
  constexpr int H = RC::H, RP1 = RC::P1, RP2 = RC::P2, RQ = RC::Q, R = RC::R, RB = RC::RB;
  constexpr int PITCH = RC::PITCH;
  constexpr int CP1 = CC::P1, CP2 = CC::P2, CQ = CC::Q, CP = CC::CP, CW = CC::CW;
  constexpr int GROUPS = CC::GROUPS, TILES = CC::TILES, TWD = CC::TWD;
  constexpr int TPJ = RB + GROUPS;  // tasks per job
  static_assert(RC::THREADS == 256 && CC::THREADS == 256, "both tasks use 256 threads");
  static_assert(TWD == CW && TWD == 8 && RP1 % TWD == 0 && CC::TW_LDS,
                "one column tile per column task; row outputs at fixed tile strides");
  constexpr int SMEM = R * PITCH > CW * CP ? R * PITCH : CW * CP;
  __shared__ float2 smem[SMEM];
  __shared__ float2 twl[tw_len(N)];
  __shared__ double red[4];
  __shared__ double red_abs[F16 ? 4 : 1];
  __shared__ int bcast[2];

  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += 256) twl[tw_skew(i)] = tw[i];
  // The XCD this workgroup runs on (constant for its lifetime).
  const int xcd = __builtin_amdgcn_readfirstlane(
      __builtin_amdgcn_s_getreg((20) | (0 << 6) | (15 << 11)) & 7);
  int* next_task = sched + xcd * kFusedLine;
  int* rdone = sched + 8 * kFusedLine + xcd * slots;
  int* cdone = rdone + 8 * slots;
  float2* myA = bufA + int64_t(xcd) * keep * N * TWD;
  float2* myB = bufB + int64_t(xcd) * (TILES - keep) * N * TWD;
  double s_ref = refscal[0], sigma_ref = refscal[1];
  const uint32_t spec_bytes = uint32_t(n_modes) * MODE_BYTES;
  __syncthreads();

  for (;;) {
    if (tid == 0) {
      bool timed_out = false;
      const int k = sched_add(next_task, 1);
      const int sl = k / TPJ, i = k - sl * TPJ;
      const int64_t j = int64_t(xcd) + 8 * int64_t(sl);
      int f = j < nframes ? int(j) : -1;
      if (f >= 0 && sl >= slots) timed_out = true;  // cannot happen: slots >= ceil(nframes / 8)
      if (f >= 0 && !timed_out) {
        if (i < RB) {
          if (sl > 0) sched_wait(cdone + sl - 1, [](int v) { return v >= GROUPS; }, spin_limit,
                                 &timed_out);
        } else {
          sched_wait(rdone + sl, [](int v) { return v >= RB; }, spin_limit, &timed_out);
        }
      }
      if (timed_out) {
        atomicOr(status, 2);
        f = -1;
      }
      bcast[0] = f;
      bcast[1] = (sl << 8) | i;
    }
    __syncthreads();
    const int f = bcast[0];
    const int sl = bcast[1] >> 8, task = bcast[1] & 255;
    __syncthreads();  // bcast is rewritten by the next claim
    if (f < 0) break;

    // The thread index goes through an empty asm statement so that the
    // addresses derived from it are computed per task, not hoisted out of
    // the task loop and kept live across both task bodies (which spills).
    int lt = tid;
    asm volatile("" : "+v"(lt));
    if (task < RB) {
      // ---- row task: rows [task * R, task * R + R) of frame f ----
      const int rl = lt / RP1, j1 = lt % RP1;
      const int y = task * R + rl;
      float2* row_lds = smem + rl * PITCH;
      float2 v[RP2];
      int si = 0, sia = 0;
      double sd = 0.0, sda = 0.0;
      const T* frow = frames + (int64_t(f) * N + y) * N + 2 * j1;
      const T* rrow = ref + int64_t(y) * N + 2 * j1;  // the reference is always set here
#pragma unroll
      for (int j2 = 0; j2 < RP2; ++j2) {
        const Raw pxj = load_pair(frow + 2 * RP1 * j2);
        const Raw rpj = load_pair(rrow + 2 * RP1 * j2);
        float a, b;
        if constexpr (U16) {
          const int da = int(pxj & 0xffffu) - int(rpj & 0xffffu);
          const int db = int(pxj >> 16) - int(rpj >> 16);
          a = float(da);
          b = float(db);
          if constexpr (!WIN) si += da + db;
          if constexpr (ABS && !WIN) sia += abs(da) + abs(db);
        } else {
          a = pxj.x - rpj.x;
          b = pxj.y - rpj.y;
        }
        if constexpr (WIN) {
          const float2 ww =
              *reinterpret_cast<const float2*>(window + int64_t(y) * N + 2 * (j1 + RP1 * j2));
          a *= ww.x;
          b *= ww.y;
        }
        if constexpr (!U16 || WIN) sd += double(a) + double(b);
        if constexpr (ABS && (!U16 || WIN)) sda += double(fabsf(a)) + double(fabsf(b));
        v[j2] = make_float2(a, b);
      }
      double rs;
      if constexpr (U16 && !WIN) {
#pragma unroll
        for (int o = RP1 / 2; o >= 1; o >>= 1) si += __shfl_xor(si, o, RP1);
        rs = double(si);
      } else {
#pragma unroll
        for (int o = RP1 / 2; o >= 1; o >>= 1) sd += __shfl_xor(sd, o, RP1);
        rs = sd;
      }
      if (j1 == 0) rowsum[int64_t(f) * N + y] = rs;
      if constexpr (ABS) {
        double sa;
        if constexpr (U16 && !WIN) {
#pragma unroll
          for (int o = RP1 / 2; o >= 1; o >>= 1) sia += __shfl_xor(sia, o, RP1);
          sa = double(sia);
        } else {
#pragma unroll
          for (int o = RP1 / 2; o >= 1; o >>= 1) sda += __shfl_xor(sda, o, RP1);
          sa = sda;
        }
        if (j1 == 0) rowabs[int64_t(f) * N + y] = sa;
      }
      dft<RP2>(v);
      static_for<RP2>([&](auto K2) {
        constexpr int k2 = decltype(K2)::value;
        float2 yv = v[bitrev<RP2>(k2)];
        if constexpr (k2 != 0) yv = cmul(yv, twl[tw_skew((2 * j1 * k2) & (N - 1))]);
        row_lds[k2 * (RP1 + 1) + j1] = yv;
      });
      wave_lds_sync();
      float2 z[RQ][RP1];
      static_for<RQ>([&](auto QQ) {
        constexpr int q = decltype(QQ)::value;
        const int k2 = j1 + q * RP1;
        float2 w[RP1];
#pragma unroll
        for (int j = 0; j < RP1; ++j) w[j] = row_lds[k2 * (RP1 + 1) + j];
        dft<RP1>(w);
        static_for<RP1>([&](auto K1) {
          constexpr int k1 = decltype(K1)::value;
          z[q][k1] = w[bitrev<RP1>(k1)];
        });
      });
      wave_lds_sync();
#pragma unroll
      for (int q = 0; q < RQ; ++q)
#pragma unroll
        for (int k1 = 0; k1 < RP1; ++k1) row_lds[(j1 + q * RP1) + RP2 * k1] = z[q][k1];
      wave_lds_sync();
      // Output i of this thread is k = j1 + RP1 i, in tile 2 i + j1 / 8 (RP1 =
      // 16, 8 columns per tile), column j1 % 8, row y; with `keep` even it
      // lies in buffer A exactly when i < keep / 2.
      static_assert(RP1 == 2 * TWD, "two tiles per row-task output step");
      float2* outA = myA + (int64_t(j1 / TWD) * N + y) * TWD + (j1 % TWD);
      float2* outB = myB + (int64_t(j1 / TWD) * N + y) * TWD + (j1 % TWD);
      const int half_keep = keep / 2;
#pragma unroll
      for (int i = 0; i < RP2; ++i) {
        const int k = j1 + RP1 * i;
        const float2 zk = row_lds[k];
        const float2 zm = row_lds[(H - k) & (H - 1)];
        const float2 e = make_float2(zk.x + zm.x, zk.y - zm.y);
        const float2 d = make_float2(zk.x - zm.x, zk.y + zm.y);
        const float2 wd = cmul(d, twl[tw_skew(k)]);
        const float2 X = make_float2(0.5f * (e.x + wd.y), 0.5f * (e.y - wd.x));
        if (i < half_keep)
          outA[int64_t(i) * 2 * N * TWD] = X;
        else
          outB[int64_t(i - half_keep) * 2 * N * TWD] = X;
      }
      // Stores of this task reach L2 before the task counts as done.
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();
      if (tid == 0) sched_add(rdone + sl, 1);
    } else {
      // ---- column task: columns [8 g, 8 g + 8) of frame f ----
      const int grp = task - RB;
      const int c = lt % CW, j1 = lt / CW;
      const int kx = grp * CW + c;
      // Rows written by other workgroups of this XCD are in its L2; drop
      // any stale copies from this CU's L1 first.
      asm volatile("buffer_inv sc0" ::: "memory");
      const float2* src = (grp < keep ? myA + int64_t(grp) * N * TWD
                                      : myB + int64_t(grp - keep) * N * TWD) + c;
      float2 v[CP2];
#pragma unroll
      for (int j2 = 0; j2 < CP2; ++j2) v[j2] = src[(j1 + CP1 * j2) * TWD];
      double part = 0.0, part_abs = 0.0;
      for (int yy = tid; yy < N; yy += 256) part += rowsum[int64_t(f) * N + yy];
      if constexpr (F16)
        for (int yy = tid; yy < N; yy += 256) part_abs += rowabs[int64_t(f) * N + yy];
      float2* col_lds = smem + c * CP;
      dft<CP2>(v);
      static_for<CP2>([&](auto K2) {
        constexpr int k2 = decltype(K2)::value;
        float2 yv = v[bitrev<CP2>(k2)];
        if constexpr (k2 != 0) yv = cmul(yv, col_twiddle<N>(twl, tw, (j1 * k2) & (N - 1)));
        col_lds[k2 * (CP1 + 1) + j1] = yv;
      });
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) part += __shfl_xor(part, o, 64);
      if ((tid & 63) == 0) red[tid >> 6] = part;
      if constexpr (F16) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) part_abs += __shfl_xor(part_abs, o, 64);
        if ((tid & 63) == 0) red_abs[tid >> 6] = part_abs;
      }
      __syncthreads();
      const double S = s_ref + (((red[0] + red[1]) + red[2]) + red[3]);
      const bool bad = !(S > 0.0) || !isfinite(S);
      const double sigma = bad ? 0.0 : double(N) * double(N) / S;
      int e = 0;
      if constexpr (F16) e = f16_exponent(sigma * (((red_abs[0] + red_abs[1]) + red_abs[2]) + red_abs[3]));
      const float scale = float(ldexp(sigma, e));
      const int64_t slot = (t0 + f) % capacity;
      if (grp == 0 && tid == 0) {
        fscale[slot] =
            make_float4(float(sigma), float(sigma - sigma_ref), float(ldexp(1.0, -e)), 0.f);
        if (bad) atomicOr(status, 1);
        if (work) atomicAdd(work, 1ull);  // work counter: frames transformed
      }
      const BufferRsrc dst = make_buffer(ring + slot * mode_stride * int64_t(MODE_BYTES), spec_bytes);
      static_for<CQ>([&](auto QQ) {
        constexpr int q = decltype(QQ)::value;
        const int k2 = j1 + q * CP1;
        float2 w[CP1];
#pragma unroll
        for (int j = 0; j < CP1; ++j) w[j] = col_lds[k2 * (CP1 + 1) + j];
        dft<CP1>(w);
        static_for<CP1>([&](auto K1) {
          constexpr int k1 = decltype(K1)::value;
          const int r = (j1 + q * CP1) + CP2 * k1;
          const int sl2 = ring_slot(N, tiles, r, kx);
          uint32_t o = sl2 >= 0 ? uint32_t(sl2) * 8u : kDropOffset;
          float2 X = w[bitrev<CP1>(k1)];
          X.x *= scale;
          X.y *= scale;
          if constexpr (q == 0 && k1 == 0) {
            if (o == 0) X = make_float2(0.f, 0.f);
          }
          if constexpr (SPEC == kSpecF32)
            buffer_store(X, dst, o);
          else
            buffer_store_u32(SPEC == kSpecBF16 ? pack_bf16(X) : pack_f16(X), dst, o >> 1);
        });
      });
      __syncthreads();  // every read of this task's buffer tile is done; LDS free
      if (tid == 0) sched_add(cdone + sl, 1);
    }
  }
}

template <int N, typename T, bool WIN>
hipError_t row_launch(const void* frames, const void* ref, const float* window, int nframes,
                      float2* inter, double* rowsum, double* rowabs, float* nyq,
                      const float2* tw, hipStream_t s) {
  using C = RowCfg<N>;
  const int per = frames_per_group(nframes, C::RB);
  const int64_t blocks = int64_t(C::RB) * ((nframes + per - 1) / per);
  if (rowabs) {
    hipLaunchKernelGGL((row_pass_kernel<N, T, WIN, true>), dim3(unsigned(blocks)),
                       dim3(C::THREADS), 0, s, static_cast<const T*>(frames),
                       static_cast<const T*>(ref), window, nframes, per, inter, rowsum, rowabs,
                       nyq, tw);
  } else {
    hipLaunchKernelGGL((row_pass_kernel<N, T, WIN, false>), dim3(unsigned(blocks)),
                       dim3(C::THREADS), 0, s, static_cast<const T*>(frames),
                       static_cast<const T*>(ref), window, nframes, per, inter, rowsum, rowabs,
                       nyq, tw);
  }
  return hipGetLastError();
}

template <int N>
hipError_t row_dispatch(int in_dtype, const void* frames, const void* ref, const float* window,
                        int nframes, float2* inter, double* rowsum, double* rowabs, float* nyq,
                        const float2* tw, hipStream_t s) {
  if (in_dtype == 0) {
    return window ? row_launch<N, uint16_t, true>(frames, ref, window, nframes, inter, rowsum,
                                                  rowabs, nyq, tw, s)
                  : row_launch<N, uint16_t, false>(frames, ref, window, nframes, inter, rowsum,
                                                   rowabs, nyq, tw, s);
  }
  return window ? row_launch<N, float, true>(frames, ref, window, nframes, inter, rowsum,
                                             rowabs, nyq, tw, s)
                : row_launch<N, float, false>(frames, ref, window, nframes, inter, rowsum,
                                              rowabs, nyq, tw, s);
}

template <int N>
hipError_t col_launch(bool reference, int spec, const float2* inter, const double* rowsum,
                      const double* rowabs, int nframes, int64_t t0, int64_t capacity,
                      int64_t mode_stride, int64_t n_modes, const int32_t* tiles,
                      const float2* tw, void* ring, float2* refspec,
                      double* refscal, float4* fscale, int32_t* status,
                      unsigned long long* work, hipStream_t s) {
  using C = ColCfg<N>;
  const int per = frames_per_group(nframes, C::GROUPS);
  const int64_t blocks = int64_t(C::GROUPS) * ((nframes + per - 1) / per);
  char* ringb = static_cast<char*>(ring);
#define NFS_COL_GO(REFV, SPECV)                                                                \
  hipLaunchKernelGGL((col_pass_kernel<N, REFV, SPECV>), dim3(unsigned(blocks)),               \
                     dim3(C::THREADS), 0, s, inter, rowsum, rowabs, refscal, fscale, status,   \
                     nframes, per, t0, capacity, mode_stride, n_modes, tiles, tw, ringb,     \
                     refspec, work)
  if (reference) {
    hipLaunchKernelGGL(ref_scale_kernel, dim3(1), dim3(256), 0, s, N, rowsum, refscal, status);
    NFS_COL_GO(true, kSpecF32);
  } else if (spec == kSpecBF16) {
    NFS_COL_GO(false, kSpecBF16);
  } else if (spec == kSpecF16) {
    NFS_COL_GO(false, kSpecF16);
  } else {
    NFS_COL_GO(false, kSpecF32);
  }
#undef NFS_COL_GO
  return hipGetLastError();
}

}  // namespace

hipError_t launch_row_pass(int n, int in_dtype, const void* frames, const void* ref,
                           const float* window, int nframes, float2* inter, double* rowsum,
                           double* rowabs, float* nyq, const float2* tw, hipStream_t s) {
#define NFS_ROW_CASE(NN)                                                                    \
  case NN:                                                                                  \
    return row_dispatch<NN>(in_dtype, frames, ref, window, nframes, inter, rowsum, rowabs, \
                            nyq, tw, s);
  switch (n) {
    NFS_ROW_CASE(16)
    NFS_ROW_CASE(32)
    NFS_ROW_CASE(64)
    NFS_ROW_CASE(128)
    NFS_ROW_CASE(256)
    NFS_ROW_CASE(512)
    NFS_ROW_CASE(1024)
    NFS_ROW_CASE(2048)
    NFS_ROW_CASE(4096)
    default: return hipErrorInvalidValue;
  }
#undef NFS_ROW_CASE
}

hipError_t launch_fused_transform(int n, int in_dtype, int spec, const void* frames,
                                  const void* ref, const float* window, int nframes,
                                  double* rowsum, double* rowabs, float2* bufA, float2* bufB,
                                  int keep, int* sched, int slots, int workers,
                                  unsigned spin_limit, const double* refscal, float4* fscale,
                                  int32_t* status, int64_t t0, int64_t capacity,
                                  int64_t mode_stride, int64_t n_modes, const int32_t* tiles,
                                  const float2* tw, void* ring, unsigned long long* work,
                                  hipStream_t s) {
  if (n != 1024 || nframes < 1 || keep < 0 || keep > 64 || keep % 2 || workers < 8 ||
      workers % 8 || slots < (nframes + 7) / 8)
    return hipErrorInvalidValue;
  constexpr int N = 1024;
  char* ringb = static_cast<char*>(ring);
  const dim3 grid = dim3(unsigned(workers)), block = dim3(256);
#define NFS_FUSED_GO(TT, WINV, ABSV, SPECV)                                                    \
  hipLaunchKernelGGL((fused_transform_kernel<N, TT, WINV, ABSV, SPECV>), grid, block, 0, s,    \
                     static_cast<const TT*>(frames), static_cast<const TT*>(ref), window,     \
                     nframes, rowsum, rowabs, bufA, bufB, keep, sched, slots, spin_limit,     \
                     refscal, fscale, status, t0, capacity, mode_stride, n_modes, tiles, tw,  \
                     ringb, work)
#define NFS_FUSED_SPEC(TT, WINV)                                                                \
  if (spec == kSpecF16) NFS_FUSED_GO(TT, WINV, true, kSpecF16);                                \
  else if (spec == kSpecBF16) NFS_FUSED_GO(TT, WINV, false, kSpecBF16);                        \
  else NFS_FUSED_GO(TT, WINV, false, kSpecF32);
  if (in_dtype == 0) {
    if (window) { NFS_FUSED_SPEC(uint16_t, true) } else { NFS_FUSED_SPEC(uint16_t, false) }
  } else {
    if (window) { NFS_FUSED_SPEC(float, true) } else { NFS_FUSED_SPEC(float, false) }
  }
#undef NFS_FUSED_SPEC
#undef NFS_FUSED_GO
  return hipGetLastError();
}

hipError_t launch_nyquist_col(int n, bool reference, int spec, const float* nyq, int nframes,
                              int64_t t0, int64_t capacity, int64_t mode_stride,
                              int64_t nyq_slot, const float2* tw, const float4* fscale,
                              void* ring, float2* refspec, hipStream_t s) {
  if (nframes < 1) return hipSuccess;
  const size_t lds = size_t(n) * sizeof(float2);
  char* ringb = static_cast<char*>(ring);
#define NFS_NYQ_GO(REFV, SPECV)                                                                \
  hipLaunchKernelGGL((nyquist_col_kernel<REFV, SPECV>), dim3(unsigned(nframes)), dim3(256),  \
                     lds, s, n, nyq, tw, fscale, t0, capacity, mode_stride, nyq_slot, ringb, \
                     refspec)
  if (reference)
    NFS_NYQ_GO(true, kSpecF32);
  else if (spec == kSpecBF16)
    NFS_NYQ_GO(false, kSpecBF16);
  else if (spec == kSpecF16)
    NFS_NYQ_GO(false, kSpecF16);
  else
    NFS_NYQ_GO(false, kSpecF32);
#undef NFS_NYQ_GO
  return hipGetLastError();
}

hipError_t launch_col_pass(int n, bool reference, int spec, const float2* inter,
                           const double* rowsum, const double* rowabs, int nframes, int64_t t0,
                           int64_t capacity, int64_t mode_stride, int64_t n_modes,
                           const int32_t* tiles, const float2* tw, void* ring,
                           float2* refspec, double* refscal, float4* fscale, int32_t* status,
                           unsigned long long* work, hipStream_t s) {
#define NFS_COL_CASE(NN)                                                                   \
  case NN:                                                                                 \
    return col_launch<NN>(reference, spec, inter, rowsum, rowabs, nframes, t0, capacity,  \
                          mode_stride, n_modes, tiles, tw, ring, refspec,                 \
                          refscal, fscale, status, work, s);
  switch (n) {
    NFS_COL_CASE(16)
    NFS_COL_CASE(32)
    NFS_COL_CASE(64)
    NFS_COL_CASE(128)
    NFS_COL_CASE(256)
    NFS_COL_CASE(512)
    NFS_COL_CASE(1024)
    NFS_COL_CASE(2048)
    NFS_COL_CASE(4096)
    default: return hipErrorInvalidValue;
  }
#undef NFS_COL_CASE
}

}  // namespace nfs
