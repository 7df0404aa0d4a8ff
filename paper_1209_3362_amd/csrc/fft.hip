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
// in double on the host and rounded once to float.
#include "nfs_device.hpp"
#include "nfs_kernels.hpp"

namespace nfs {
using namespace dev;

namespace {

constexpr int kLdsBudget = 80 * 1024;  // per workgroup, so two fit per CU

constexpr int fit_rows(int r, int pitch) {
  while (r > 1 && r * pitch * 8 > kLdsBudget) r /= 2;
  return r;
}
// LDS column pitch congruent to 2 mod 16 complex values, so 8 columns x 2
// rows of 8-byte accesses fall in 16 distinct bank pairs.
constexpr int pad_2mod16(int v) { return v + ((2 - v % 16) + 16) % 16; }
constexpr int fit_cols(int pitch) {
  int c = 8;
  while (c > 1 && c * pitch * 8 > kLdsBudget) c /= 2;
  return c;
}

template <int N>
struct RowCfg {
  static constexpr int H = N / 2;                    // complex points per row
  static constexpr int P1 = 1 << (ilog2(H) / 2);     // H = P1 * P2, P2 in {P1, 2 P1}
  static constexpr int P2 = H / P1;
  static constexpr int Q = P2 / P1;
  static constexpr int PITCH = P2 * (P1 + 1) + 4;    // LDS complex values per row
  static constexpr int R = fit_rows(256 / P1, PITCH);
  static constexpr int THREADS = R * P1;
  static constexpr int TILES = H / 8;                // 8-column tiles of the intermediate
};

template <int N>
struct ColCfg {
  static constexpr int P1 = 1 << (ilog2(N) / 2);     // N = P1 * P2, P2 in {P1, 2 P1}
  static constexpr int P2 = N / P1;
  static constexpr int Q = P2 / P1;
  static constexpr int CP = pad_2mod16(P2 * (P1 + 1));
  static constexpr int CW = fit_cols(CP);            // columns per workgroup
  static constexpr int THREADS = CW * P1;
  static constexpr int GROUPS = (N / 2) / CW;        // column groups per frame
  static constexpr int TILES = N / 16;
};

// ---------------------------------------------------------------------------
// Row pass. Real row u of N pixels -> z[j] = u[2j] + i u[2j+1] (H points),
// Z = DFT_H(z), then X[k] = (Z[k] + conj Z[H-k])/2 - i W_N^k (Z[k] - conj Z[H-k])/2
// for k = 0..H-1 (the real-input split; X[H] is never binned).
template <int N, typename T, bool WIN>
__global__ __launch_bounds__(RowCfg<N>::THREADS) void row_pass_kernel(
    const T* __restrict__ frames, const T* __restrict__ ref, const float* __restrict__ window,
    int64_t total_rows, float2* __restrict__ inter, double* __restrict__ rowsum,
    const float2* __restrict__ tw) {
  using C = RowCfg<N>;
  constexpr int H = C::H, P1 = C::P1, P2 = C::P2, Q = C::Q, R = C::R;
  constexpr int PITCH = C::PITCH, THREADS = C::THREADS, TILES = C::TILES;
  __shared__ float2 lds[R * PITCH];

  const int tid = threadIdx.x;
  const int rl = tid / P1, j1 = tid % P1;
  const int64_t g0 = int64_t(blockIdx.x) * R;
  const int64_t grow = g0 + rl;
  const bool valid = grow < total_rows;
  const int y = int(grow & (N - 1));
  float2* row_lds = lds + rl * PITCH;

  float2 v[P2];
  double s = 0.0;
  const T* src = frames + grow * N;
#pragma unroll
  for (int j2 = 0; j2 < P2; ++j2) {
    const int j = j1 + P1 * j2;
    float a = 0.f, b = 0.f;
    if (valid) {
      if constexpr (std::is_same<T, uint16_t>::value) {
        const uint32_t w = *reinterpret_cast<const uint32_t*>(src + 2 * j);
        a = float(w & 0xffffu);
        b = float(w >> 16);
        if (ref) {  // integer difference: exact in FP32
          const uint32_t r = *reinterpret_cast<const uint32_t*>(ref + int64_t(y) * N + 2 * j);
          a -= float(r & 0xffffu);
          b -= float(r >> 16);
        }
      } else {
        const float2 w = *reinterpret_cast<const float2*>(src + 2 * j);
        a = w.x;
        b = w.y;
        if (ref) {
          const float2 r = *reinterpret_cast<const float2*>(ref + int64_t(y) * N + 2 * j);
          a -= r.x;
          b -= r.y;
        }
      }
      if constexpr (WIN) {
        const float2 ww = *reinterpret_cast<const float2*>(window + int64_t(y) * N + 2 * j);
        a *= ww.x;
        b *= ww.y;
      }
    }
    v[j2] = make_float2(a, b);
    s += double(a) + double(b);
  }
  // Row sum of what was transformed (exact in double for integer pixels),
  // butterfly over the P1 lanes of the row: every lane ends with the same
  // value.
#pragma unroll
  for (int o = P1 / 2; o >= 1; o >>= 1) s += __shfl_xor(s, o, P1);
  if (valid && j1 == 0) rowsum[grow] = s;

  // First level: DFT over j2 of z[j1 + P1 j2], twiddle W_H^{j1 k2} = W_N^{2 j1 k2}.
  dft<P2>(v);
  static_for<P2>([&](auto K2) {
    constexpr int k2 = decltype(K2)::value;
    float2 yv = v[bitrev<P2>(k2)];
    if constexpr (k2 != 0) yv = cmul(yv, tw[(2 * j1 * k2) & (N - 1)]);
    row_lds[k2 * (P1 + 1) + j1] = yv;
  });
  __syncthreads();

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
  __syncthreads();
#pragma unroll
  for (int q = 0; q < Q; ++q)
#pragma unroll
    for (int k1 = 0; k1 < P1; ++k1) row_lds[(j1 + q * P1) + P2 * k1] = z[q][k1];
  __syncthreads();

  // Real-input split and store into 8-column tiles: for tile T the rows of
  // this workgroup are contiguous in the intermediate.
#pragma unroll
  for (int i = 0; i < P2; ++i) {
    const int idx = tid + i * THREADS;
    const int c = idx & 7;
    const int rr = (idx >> 3) & (R - 1);
    const int tile = idx / (8 * R);
    const int k = tile * 8 + c;
    const int64_t g = g0 + rr;
    if (g < total_rows) {
      const float2 zk = lds[rr * PITCH + k];
      const float2 zm = lds[rr * PITCH + ((H - k) & (H - 1))];
      const float2 e = make_float2(zk.x + zm.x, zk.y - zm.y);   // Z[k] + conj Z[H-k]
      const float2 d = make_float2(zk.x - zm.x, zk.y + zm.y);   // Z[k] - conj Z[H-k]
      const float2 wd = cmul(d, tw[k]);
      const float2 X = make_float2(0.5f * (e.x + wd.y), 0.5f * (e.y - wd.x));
      const int64_t f = g / N;
      const int yy = int(g & (N - 1));
      inter[((f * TILES + tile) * N + yy) * 8 + c] = X;
    }
  }
}

// ---------------------------------------------------------------------------
// Column pass over CW columns of one frame: DFT_N over the rows, scale by
// n^2 / sum(u) (the zero-frequency value of the row-pass output), set
// I(0) = n^2 exactly and store the modes with k_x < row_width[r].
template <int N, bool REF>
__global__ __launch_bounds__(ColCfg<N>::THREADS) void col_pass_kernel(
    const float2* __restrict__ inter, const double* __restrict__ rowsum, int64_t t0,
    int64_t capacity, int64_t mode_stride, const int32_t* __restrict__ row_width,
    const int32_t* __restrict__ row_offset, const float2* __restrict__ tw,
    float2* __restrict__ ring, float2* __restrict__ refspec, double* __restrict__ refscal,
    int32_t* __restrict__ status) {
  using C = ColCfg<N>;
  constexpr int P1 = C::P1, P2 = C::P2, Q = C::Q, CP = C::CP, CW = C::CW;
  constexpr int THREADS = C::THREADS, GROUPS = C::GROUPS, TILES = C::TILES;
  constexpr int WAVE = THREADS < 64 ? THREADS : 64;
  constexpr int NWAVES = (THREADS + 63) / 64;
  __shared__ float2 lds[CW * CP];
  __shared__ double red[NWAVES];

  const int f = blockIdx.x / GROUPS;
  const int grp = blockIdx.x % GROUPS;
  const int kx0 = grp * CW;
  const int tile = kx0 / 8, c0 = kx0 % 8;
  const int tid = threadIdx.x;
  const int c = tid % CW, j1 = tid / CW;

  // Frame sum in a fixed order: strided partial sums, butterfly within the
  // wave, waves added in index order. Every workgroup of the frame gets the
  // same value.
  double s = 0.0;
  for (int yy = tid; yy < N; yy += THREADS) s += rowsum[int64_t(f) * N + yy];
#pragma unroll
  for (int o = WAVE / 2; o >= 1; o >>= 1) s += __shfl_xor(s, o, WAVE);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  double part = 0.0;
#pragma unroll
  for (int w = 0; w < NWAVES; ++w) part += red[w];
  // REF: the rows were the reference image itself; its transform is stored
  // unscaled in refspec and its sum S_ref and scale n^2/S_ref in refscal.
  // Otherwise the rows were (image - reference): the image sum is
  // S_ref + part, sigma = n^2 / sum, and the stored value is
  // sigma * F[image - reference] + (sigma - sigma_ref) * F[reference]
  // = I_t - sigma_ref * F[reference], fluctuation-sized.
  const double total = REF ? part : refscal[0] + part;
  const bool bad = !(total > 0.0) || !isfinite(total);
  const double sigma = bad ? 0.0 : double(N) * double(N) / total;
  float scale, dscale;
  if constexpr (REF) {
    scale = 1.f;
    dscale = 0.f;
    if (blockIdx.x == 0 && tid == 0) {
      refscal[0] = total;
      refscal[1] = sigma;
    }
  } else {
    scale = float(sigma);
    dscale = float(sigma - refscal[1]);
    if (bad && tid == 0) atomicOr(status, 1);
  }

  const float2* src = inter + (int64_t(f) * TILES + tile) * N * 8 + c0 + c;
  float2 v[P2];
#pragma unroll
  for (int j2 = 0; j2 < P2; ++j2) v[j2] = src[(j1 + P1 * j2) * 8];
  dft<P2>(v);
  float2* col_lds = lds + c * CP;
  static_for<P2>([&](auto K2) {
    constexpr int k2 = decltype(K2)::value;
    float2 yv = v[bitrev<P2>(k2)];
    if constexpr (k2 != 0) yv = cmul(yv, tw[(j1 * k2) & (N - 1)]);
    col_lds[k2 * (P1 + 1) + j1] = yv;
  });
  __syncthreads();

  float2* dst = REF ? refspec : ring + ((t0 + f) % capacity) * mode_stride;
  const int kx = kx0 + c;
  static_for<Q>([&](auto QQ) {
    constexpr int q = decltype(QQ)::value;
    const int k2 = j1 + q * P1;
    float2 w[P1];
#pragma unroll
    for (int j = 0; j < P1; ++j) w[j] = col_lds[k2 * (P1 + 1) + j];
    dft<P1>(w);
    static_for<P1>([&](auto K1) {
      constexpr int k1 = decltype(K1)::value;
      const int r = k2 + P2 * k1;
      float2 X = w[bitrev<P1>(k1)];
      if (kx < row_width[r]) {
        const int64_t at = row_offset[r] + kx;
        if constexpr (!REF) {
          const float2 R = refspec[at];
          X.x = fmaf(dscale, R.x, scale * X.x);
          X.y = fmaf(dscale, R.y, scale * X.y);
          // I_t(0) = n^2 for every frame, so its offset from the reference is 0.
          if (at == 0) X = make_float2(0.f, 0.f);
        }
        dst[at] = X;
      }
    });
  });
}

template <int N, typename T, bool WIN>
hipError_t row_launch(const void* frames, const void* ref, const float* window, int nframes,
                      float2* inter, double* rowsum, const float2* tw, hipStream_t s) {
  using C = RowCfg<N>;
  const int64_t rows = int64_t(nframes) * N;
  const int64_t blocks = (rows + C::R - 1) / C::R;
  hipLaunchKernelGGL((row_pass_kernel<N, T, WIN>), dim3(unsigned(blocks)), dim3(C::THREADS),
                     0, s, static_cast<const T*>(frames), static_cast<const T*>(ref), window,
                     rows, inter, rowsum, tw);
  return hipGetLastError();
}

template <int N>
hipError_t row_dispatch(int in_dtype, const void* frames, const void* ref, const float* window,
                        int nframes, float2* inter, double* rowsum, const float2* tw,
                        hipStream_t s) {
  if (in_dtype == 0) {
    return window ? row_launch<N, uint16_t, true>(frames, ref, window, nframes, inter, rowsum,
                                                  tw, s)
                  : row_launch<N, uint16_t, false>(frames, ref, window, nframes, inter, rowsum,
                                                   tw, s);
  }
  return window ? row_launch<N, float, true>(frames, ref, window, nframes, inter, rowsum, tw, s)
                : row_launch<N, float, false>(frames, ref, window, nframes, inter, rowsum, tw, s);
}

template <int N>
hipError_t col_launch(bool reference, const float2* inter, const double* rowsum, int nframes,
                      int64_t t0, int64_t capacity, int64_t mode_stride,
                      const int32_t* row_width, const int32_t* row_offset, const float2* tw,
                      float2* ring, float2* refspec, double* refscal, int32_t* status,
                      hipStream_t s) {
  using C = ColCfg<N>;
  const int64_t blocks = int64_t(nframes) * C::GROUPS;
  if (reference) {
    hipLaunchKernelGGL((col_pass_kernel<N, true>), dim3(unsigned(blocks)), dim3(C::THREADS), 0,
                       s, inter, rowsum, t0, capacity, mode_stride, row_width, row_offset, tw,
                       ring, refspec, refscal, status);
  } else {
    hipLaunchKernelGGL((col_pass_kernel<N, false>), dim3(unsigned(blocks)), dim3(C::THREADS), 0,
                       s, inter, rowsum, t0, capacity, mode_stride, row_width, row_offset, tw,
                       ring, refspec, refscal, status);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_row_pass(int n, int in_dtype, const void* frames, const void* ref,
                           const float* window, int nframes, float2* inter, double* rowsum,
                           const float2* tw, hipStream_t s) {
#define NFS_ROW_CASE(NN) \
  case NN:               \
    return row_dispatch<NN>(in_dtype, frames, ref, window, nframes, inter, rowsum, tw, s);
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

hipError_t launch_col_pass(int n, bool reference, const float2* inter, const double* rowsum,
                           int nframes, int64_t t0, int64_t capacity, int64_t mode_stride,
                           const int32_t* row_width, const int32_t* row_offset,
                           const float2* tw, float2* ring, float2* refspec, double* refscal,
                           int32_t* status, hipStream_t s) {
#define NFS_COL_CASE(NN)                                                                   \
  case NN:                                                                                 \
    return col_launch<NN>(reference, inter, rowsum, nframes, t0, capacity, mode_stride,   \
                          row_width, row_offset, tw, ring, refspec, refscal, status, s);
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
