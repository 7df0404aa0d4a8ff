// Azimuthal average of the per-lag sums into rings of |q| (text after
// Eq. 1 and Fig. 1e-f), and the average over pairs per delay (processing
// section: the average for every delay is stored).
//
// Ring b is the set of modes with lo_b <= |k|^2 < hi_b, so on row k_y its
// half-plane modes are the run k_x in [ceil_sqrt(lo_b - k_y^2),
// ceil_sqrt(hi_b - k_y^2)): the rings are walked row by row with no
// per-mode table. Each half-plane mode stands for itself and its mirror -k
// (weight 2) except on k_x = 0, where both k and -k are stored (weight 1).
//
// The sums are mode-major per slot of the tiled layout (ring_slot).
// The rows of ring b are cut into segments of kSegRows rows. One
// workgroup sums one segment: lanes are lags, so each mode's lag sums are
// one contiguous read of the mode-major sums. A second kernel adds the
// segments of each ring in order. All sums are FP64 in a fixed order, so D
// is bitwise reproducible.
#include "nfs.h"
#include "nfs_device.hpp"
#include "nfs_host.hpp"
#include "nfs_kernels.hpp"

namespace nfs {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

__global__ __launch_bounds__(kThreads) void bin_segment_kernel(
    int n, int nb, const float* __restrict__ acc, int n_lags,
    const int32_t* __restrict__ tiles, const int32_t* __restrict__ seg_bin,
    const int32_t* __restrict__ seg_row0, double* __restrict__ part,
    long long* __restrict__ part_cnt) {
  using namespace dev;
  __shared__ double red[kWaves][64];
  __shared__ long long redc[kWaves];
  // The slot table (2 n/16 + 1 entries, at most 513) in LDS: it is read
  // once per mode.
  __shared__ int32_t tl[2 * (4096 / 16) + 1];
  for (int i = threadIdx.x; i < 2 * (n / 16) + 1; i += kThreads) tl[i] = tiles[i];
  __syncthreads();
  const int seg = blockIdx.x;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int b = seg_bin[seg];
  int64_t lo, hi;
  ring_bounds_dev(n, nb, b, &lo, &hi);
  const int R = int(isqrt_dev(uint64_t(hi - 1)));  // |k_y| <= R on the ring
  const int ky0 = seg_row0[seg];
  const int ky1 = min(ky0 + kSegRows, R + 1);

  long long cnt = 0;
  for (int l0 = 0; l0 < n_lags; l0 += 64) {
    const int l = l0 + lane;
    const bool lag_ok = l < n_lags;
    double s = 0.0;
    for (int ky = ky0 + wave; ky < ky1; ky += kWaves) {
      const int64_t ky2 = int64_t(ky) * ky;
      const int a = int(ceil_sqrt_dev(lo - ky2));
      const int e = int(ceil_sqrt_dev(hi - ky2));
      if (e <= a) continue;
      if (l0 == 0) cnt += (a == 0) ? 1 + 2 * (e - 1) : 2 * (e - a);
      const int r = ky >= 0 ? ky : ky + n;
      const float* src = acc + l;
      auto at = [&](int x) { return int64_t(ring_slot(n, tl, r, x)) * n_lags; };
      int kx = a;
      if (kx == 0) {
        if (lag_ok) s += double(src[at(0)]);
        kx = 1;
      }
      // weight 2 for k_x > 0; four independent loads per step
      for (; kx + 4 <= e; kx += 4) {
        float v0 = 0.f, v1 = 0.f, v2 = 0.f, v3 = 0.f;
        if (lag_ok) {
          v0 = src[at(kx)];
          v1 = src[at(kx + 1)];
          v2 = src[at(kx + 2)];
          v3 = src[at(kx + 3)];
        }
        s += 2.0 * double(v0);
        s += 2.0 * double(v1);
        s += 2.0 * double(v2);
        s += 2.0 * double(v3);
      }
      for (; kx < e; ++kx)
        if (lag_ok) s += 2.0 * double(src[at(kx)]);
    }
    red[wave][lane] = s;
    if (l0 == 0 && lane == 0) redc[wave] = cnt;
    __syncthreads();
    if (wave == 0 && lag_ok) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < kWaves; ++w) t += red[w][lane];
      part[int64_t(seg) * n_lags + l] = t;
    }
    if (l0 == 0 && threadIdx.x == 0) {
      long long c = 0;
#pragma unroll
      for (int w = 0; w < kWaves; ++w) c += redc[w];
      part_cnt[seg] = c;
    }
    __syncthreads();
  }
}

__global__ void bin_final_kernel(int nb, int n_lags, const double* __restrict__ part,
                                 const long long* __restrict__ part_cnt,
                                 const int32_t* __restrict__ bin_seg0,
                                 const int32_t* __restrict__ lags, int64_t n_frames,
                                 const int32_t* __restrict__ status, double* __restrict__ D,
                                 int64_t* __restrict__ counts, int64_t* __restrict__ pairs,
                                 int32_t* __restrict__ status_out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(nb) * n_lags) return;
  const int b = int(i / n_lags), l = int(i % n_lags);
  const int s0 = bin_seg0[b], s1 = bin_seg0[b + 1];
  double sum = 0.0;
  long long C = 0;
  for (int s = s0; s < s1; ++s) {
    sum += part[int64_t(s) * n_lags + l];
    C += part_cnt[s];
  }
  const int64_t np = n_frames - lags[l] > 0 ? n_frames - lags[l] : 0;
  D[int64_t(l) * nb + b] = (np > 0 && C > 0) ? sum / (double(C) * double(np))
                                             : __builtin_nan("");
  if (l == 0 && counts) counts[b] = C;
  if (b == 0) {
    if (pairs) pairs[l] = np;
    if (l == 0 && status_out) status_out[0] = (status[0] & 1) ? NFS_E_DEGENERATE_FRAME : NFS_OK;
  }
}

}  // namespace

hipError_t launch_bins(int n, int n_bins, const float* acc, int n_lags,
                       const int32_t* tiles, const int32_t* seg_bin,
                       const int32_t* seg_row0, int n_segs, const int32_t* bin_seg0,
                       double* part, long long* part_cnt, const int32_t* lags,
                       int64_t n_frames, const int32_t* status, double* D, int64_t* counts,
                       int64_t* pairs, int32_t* status_out, hipStream_t s) {
  hipLaunchKernelGGL(bin_segment_kernel, dim3(unsigned(n_segs)), dim3(kThreads), 0, s, n,
                     n_bins, acc, n_lags, tiles, seg_bin, seg_row0, part, part_cnt);
  const int64_t items = int64_t(n_bins) * n_lags;
  hipLaunchKernelGGL(bin_final_kernel, dim3(unsigned((items + 255) / 256)), dim3(256), 0, s,
                     n_bins, n_lags, part, part_cnt, bin_seg0, lags, n_frames, status, D,
                     counts, pairs, status_out);
  return hipGetLastError();
}

}  // namespace nfs
