// Azimuthal average of the per-lag sums into rings of |q| (text after
// Eq. 1 and Fig. 1e-f), and the average over pairs per delay (processing
// section: the average for every delay is stored).
//
// One workgroup per ring b. Ring b is the set of modes with
// lo_b <= |k|^2 < hi_b, so on row k_y its half-plane modes are the run
// k_x in [ceil_sqrt(lo_b - k_y^2), ceil_sqrt(hi_b - k_y^2)): the workgroup
// walks the ring row by row with no per-mode table. Each half-plane mode
// stands for itself and its mirror -k (weight 2) except on k_x = 0, where
// both k and -k are stored (weight 1). Sums are FP64 in a fixed order
// (per-thread rows, a fixed butterfly per wave, waves in index order), so D
// is bitwise reproducible.
#include "nfs.h"
#include "nfs_device.hpp"
#include "nfs_kernels.hpp"

namespace nfs {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kMaxRowsPerThread = 16;  // 2 * 2047 + 1 rows at n = 4096
constexpr int kLagChunk = 8;           // lags summed per pass over the ring

// Sum over the 64 lanes of a wave in a fixed butterfly order; every lane
// gets the same value.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ __launch_bounds__(kThreads) void bin_kernel(
    int n, int nb, const float* __restrict__ acc, int64_t mode_stride,
    const int32_t* __restrict__ row_offset, const int32_t* __restrict__ lags, int n_lags,
    int64_t n_frames, const int32_t* __restrict__ status, double* __restrict__ D,
    int64_t* __restrict__ counts, int64_t* __restrict__ pairs, int32_t* __restrict__ status_out) {
  using namespace dev;
  __shared__ double red[kWaves][kLagChunk];
  __shared__ long long redc[kWaves];
  const int b = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;

  int64_t lo, hi;
  ring_bounds_dev(n, nb, b, &lo, &hi);
  const int R = int(isqrt_dev(uint64_t(hi - 1)));  // |k_y| <= R on the ring
  const int nrows = 2 * R + 1;

  int roff[kMaxRowsPerThread], kxa[kMaxRowsPerThread], kxb[kMaxRowsPerThread];
  long long cnt = 0;
#pragma unroll
  for (int i = 0; i < kMaxRowsPerThread; ++i) {
    const int row = tid + i * kThreads;
    roff[i] = 0;
    kxa[i] = kxb[i] = 0;
    if (row < nrows) {
      const int ky = row - R;
      const int64_t ky2 = int64_t(ky) * ky;
      const int a = int(ceil_sqrt_dev(lo - ky2));
      const int e = int(ceil_sqrt_dev(hi - ky2));
      if (e > a) {
        roff[i] = row_offset[ky >= 0 ? ky : ky + n];
        kxa[i] = a;
        kxb[i] = e;
        cnt += (a == 0) ? 1 + 2 * (e - 1) : 2 * (e - a);
      }
    }
  }
  cnt = wave_sum(cnt);
  if (lane == 0) redc[wave] = cnt;
  __syncthreads();
  long long C = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) C += redc[w];
  if (tid == 0 && counts) counts[b] = C;

  for (int l0 = 0; l0 < n_lags; l0 += kLagChunk) {
    double s[kLagChunk];
#pragma unroll
    for (int j = 0; j < kLagChunk; ++j) s[j] = 0.0;
#pragma unroll
    for (int i = 0; i < kMaxRowsPerThread; ++i) {
      for (int kx = kxa[i]; kx < kxb[i]; ++kx) {
        const double wgt = kx == 0 ? 1.0 : 2.0;
        const float* src = acc + int64_t(l0) * mode_stride + roff[i] + kx;
#pragma unroll
        for (int j = 0; j < kLagChunk; ++j)
          if (l0 + j < n_lags) s[j] += wgt * double(src[int64_t(j) * mode_stride]);
      }
    }
#pragma unroll
    for (int j = 0; j < kLagChunk; ++j) {
      const double v = wave_sum(s[j]);
      if (lane == 0) red[wave][j] = v;
    }
    __syncthreads();
    if (tid < kLagChunk && l0 + tid < n_lags) {
      double tot = 0.0;
#pragma unroll
      for (int w = 0; w < kWaves; ++w) tot += red[w][tid];
      const int l = l0 + tid;
      const int64_t np = n_frames - lags[l] > 0 ? n_frames - lags[l] : 0;
      D[int64_t(l) * nb + b] = (np > 0 && C > 0) ? tot / (double(C) * double(np))
                                                 : __builtin_nan("");
    }
    __syncthreads();  // red[] is reused by the next chunk
  }

  if (b == 0) {
    for (int l = tid; l < n_lags; l += kThreads) {
      const int64_t np = n_frames - lags[l];
      if (pairs) pairs[l] = np > 0 ? np : 0;
    }
    if (tid == 0 && status_out) status_out[0] = (status[0] & 1) ? NFS_E_DEGENERATE_FRAME : NFS_OK;
  }
}

}  // namespace

hipError_t launch_bins(int n, int n_bins, const float* acc, int64_t mode_stride,
                       const int32_t* row_offset, const int32_t* lags, int n_lags,
                       int64_t n_frames, const int32_t* status, double* D, int64_t* counts,
                       int64_t* pairs, int32_t* status_out, hipStream_t s) {
  hipLaunchKernelGGL(bin_kernel, dim3(unsigned(n_bins)), dim3(kThreads), 0, s, n, n_bins, acc,
                     mode_stride, row_offset, lags, n_lags, n_frames, status, D, counts, pairs,
                     status_out);
  return hipGetLastError();
}

}  // namespace nfs
