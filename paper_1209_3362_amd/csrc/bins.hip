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
// (per-thread rows, then a fixed LDS tree), so D is bitwise reproducible.
#include "nfs.h"
#include "nfs_device.hpp"
#include "nfs_kernels.hpp"

namespace nfs {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxRowsPerThread = 16;  // 2 * 2047 + 1 rows at n = 4096

__global__ __launch_bounds__(kThreads) void bin_kernel(
    int n, int nb, const float* __restrict__ acc, int64_t mode_stride,
    const int32_t* __restrict__ row_offset, const int32_t* __restrict__ lags, int n_lags,
    int64_t n_frames, const int32_t* __restrict__ status, double* __restrict__ D,
    int64_t* __restrict__ counts, int64_t* __restrict__ pairs, int32_t* __restrict__ status_out) {
  using namespace dev;
  __shared__ double red[kThreads];
  __shared__ long long redc[kThreads];
  const int b = blockIdx.x;
  const int tid = threadIdx.x;

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
  redc[tid] = cnt;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (tid < w) redc[tid] += redc[tid + w];
    __syncthreads();
  }
  const long long C = redc[0];
  if (tid == 0 && counts) counts[b] = C;

  for (int l = 0; l < n_lags; ++l) {
    const float* src = acc + int64_t(l) * mode_stride;
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kMaxRowsPerThread; ++i) {
      for (int kx = kxa[i]; kx < kxb[i]; ++kx) {
        const double v = double(src[roff[i] + kx]);
        s += kx == 0 ? v : 2.0 * v;
      }
    }
    __syncthreads();  // red[] of the previous lag has been read
    red[tid] = s;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    if (tid == 0) {
      const int64_t np = n_frames - lags[l] > 0 ? n_frames - lags[l] : 0;
      D[int64_t(l) * nb + b] = (np > 0 && C > 0) ? red[0] / (double(C) * double(np))
                                                 : __builtin_nan("");
    }
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
