// Shared shape of the n-point complex transforms: the column pass of the
// forward 2D transform and the inverse transforms of the gradient use the
// same two-level P1 x P2 decomposition, LDS pitch and twiddle table.
#pragma once

#include "nfs_device.hpp"

namespace nfs {

constexpr int kLdsBudget = 80 * 1024;  // per workgroup, so two fit per CU

// Exchange twiddle table in LDS: entry m at m + m/8.
__host__ __device__ constexpr int tw_skew(int m) { return m + (m >> 3); }
constexpr int tw_len(int n) { return n + n / 8; }

constexpr int fit_rows(int r, int pitch, int fixed) {
  while (r > 1 && r * pitch * 8 + fixed > kLdsBudget) r /= 2;
  return r;
}
// LDS column pitch congruent to 2 mod 16 complex values, so 8 columns x 2
// rows of 8-byte accesses fall in 16 distinct bank pairs.
constexpr int pad_2mod16(int v) { return v + ((2 - v % 16) + 16) % 16; }
constexpr int fit_cols(int pitch, int fixed) {
  int c = 8;
  while (c > 1 && c * pitch * 8 + fixed > kLdsBudget) c /= 2;
  return c;
}

template <int N>
struct ColCfg {
  static constexpr int P1 = 1 << (dev::ilog2(N) / 2);  // N = P1 * P2, P2 in {P1, 2 P1}
  static constexpr int P2 = N / P1;
  static constexpr int Q = P2 / P1;
  static constexpr int CP = pad_2mod16(P2 * (P1 + 1));
  // Up to n = 1024 the exchange twiddles sit in LDS; from 2048 on a column
  // alone takes 16 KB of LDS, so the table is read through the L1 cache
  // instead and the freed LDS holds twice the columns per workgroup.
  static constexpr bool TW_LDS = N < 2048;
  static constexpr int TWL = TW_LDS ? tw_len(N) : 1;     // LDS twiddle entries
  static constexpr int CW = fit_cols(CP, TW_LDS ? tw_len(N) * 8 : 0);  // columns per workgroup
  static constexpr int THREADS = CW * P1;
  static constexpr int GROUPS = (N / 2) / CW;        // column groups per frame
  // The intermediate is cut into tiles of TWD = max(CW, 2) columns (whole
  // groups of this pass, or two one-column groups).
  static constexpr int TWD = CW > 2 ? CW : 2;
  static constexpr int TILES = (N / 2) / TWD;
  // Two workgroups per CU while the per-thread store offsets fit the
  // register budget of two waves per SIMD.
  static constexpr int MINW = Q * P1 <= 32 ? 2 : 1;
};

// One n-point complex DFT per vector, CW vectors per workgroup, P1 threads
// per vector (thread j1 of vector c): X[k] = sum_j x[j] W_N^{jk}, in two
// halves so a caller can load the next vector between them.
// dft_first: v[j2] holds x[j1 + P1 * j2] (j2 < P2); DFT_P2 in registers,
// exchange twiddles, write to vec_lds (this vector's CP values of LDS; twl:
// the twiddle table in LDS, tw: the global one, see col_twiddle). Then a
// workgroup barrier.
// dft_second: store(k, X[k]) for k = (j1 + q P1) + P2 k1 (q < Q, k1 < P1).
// A barrier must separate dft_second from the next write of vec_lds.
// Exchange twiddle W_N^i of the column transforms: from the LDS table
// (tw_skew layout) or, when ColCfg<N>::TW_LDS is false, from the global one.
template <int N>
__device__ __forceinline__ float2 col_twiddle(const float2* twl, const float2* tw, int i) {
  if constexpr (ColCfg<N>::TW_LDS) return twl[tw_skew(i)];
  else return tw[i];
}

// Fill the LDS twiddle table (nothing when the global table is used).
template <int N>
__device__ __forceinline__ void load_col_twiddles(float2* twl, const float2* tw, int tid,
                                                  int threads) {
  if constexpr (ColCfg<N>::TW_LDS)
    for (int i = tid; i < N; i += threads) twl[tw_skew(i)] = tw[i];
}

template <int N>
__device__ __forceinline__ void dft_first(float2 (&v)[ColCfg<N>::P2], float2* vec_lds,
                                          const float2* twl, const float2* tw, int j1) {
  using namespace dev;
  using C = ColCfg<N>;
  constexpr int P1 = C::P1, P2 = C::P2;
  dft<P2>(v);
  static_for<P2>([&](auto K2) {
    constexpr int k2 = decltype(K2)::value;
    float2 yv = v[bitrev<P2>(k2)];
    if constexpr (k2 != 0) yv = cmul(yv, col_twiddle<N>(twl, tw, (j1 * k2) & (N - 1)));
    vec_lds[k2 * (P1 + 1) + j1] = yv;
  });
}

template <int N, class Store>
__device__ __forceinline__ void dft_second(const float2* vec_lds, int j1, Store&& store) {
  using namespace dev;
  using C = ColCfg<N>;
  constexpr int P1 = C::P1, P2 = C::P2, Q = C::Q;
  static_for<Q>([&](auto QQ) {
    constexpr int q = decltype(QQ)::value;
    const int k2 = j1 + q * P1;
    float2 w[P1];
#pragma unroll
    for (int j = 0; j < P1; ++j) w[j] = vec_lds[k2 * (P1 + 1) + j];
    dft<P1>(w);
    static_for<P1>([&](auto K1) {
      constexpr int k1 = decltype(K1)::value;
      store(k2 + P2 * k1, w[bitrev<P1>(k1)]);
    });
  });
}

// Frames one workgroup of a pass loops over: enough workgroups to give
// every CU two, and at most 8 frames each.
inline int frames_per_group(int nframes, int groups_per_frame) {
  int f = (nframes * groups_per_frame) / 512;
  if (f < 1) f = 1;
  if (f > 8) f = 8;
  return f;
}

}  // namespace nfs
