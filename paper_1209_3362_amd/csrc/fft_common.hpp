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
  static constexpr int CW = fit_cols(CP, tw_len(N) * 8);  // columns per workgroup
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
// per vector (thread j1 of vector c): X[k] = sum_j x[j] W_N^{jk}.
// load(j) returns x[j] for j = j1 + P1 * j2 (j2 < P2); store(k, X[k]) is
// called for k = (j1 + q P1) + P2 k1 (q < Q, k1 < P1). vec_lds: this
// vector's CP values of LDS; twl: the twiddle table in LDS (tw_skew
// layout). Contains one workgroup barrier; the caller separates reuse of
// vec_lds by another barrier.
template <int N, class Load, class Store>
__device__ __forceinline__ void dft_vector(float2* vec_lds, const float2* twl, int j1,
                                           Load&& load, Store&& store) {
  using namespace dev;
  using C = ColCfg<N>;
  constexpr int P1 = C::P1, P2 = C::P2, Q = C::Q;
  float2 v[P2];
#pragma unroll
  for (int j2 = 0; j2 < P2; ++j2) v[j2] = load(j1 + P1 * j2);
  dft<P2>(v);
  static_for<P2>([&](auto K2) {
    constexpr int k2 = decltype(K2)::value;
    float2 yv = v[bitrev<P2>(k2)];
    if constexpr (k2 != 0) yv = cmul(yv, twl[tw_skew((j1 * k2) & (N - 1))]);
    vec_lds[k2 * (P1 + 1) + j1] = yv;
  });
  __syncthreads();
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

}  // namespace nfs
