// Azimuthal average of the per-lag sums into rings of |q| (text after
// Eq. 1 and Fig. 1e-f), and the average over pairs per delay (processing
// section: the average for every delay is stored).
//
// Ring b is the set of modes with lo_b <= |k|^2 < hi_b. Each half-plane
// mode stands for itself and its mirror -k (weight 2) except on k_x = 0,
// where both k and -k are stored (weight 1). The plan lists the slots of
// every ring's stored modes with their weights (the binning table) and cuts
// each ring's list into segments of at most kSegModes modes.
//
// The sums are mode-major per slot, so each mode's lag sums are one
// contiguous read. One workgroup sums one segment: each wave takes 64
// consecutive table entries (one per lane), then walks them with the slot
// broadcast from its lane and the lags on the lanes, eight reads in
// flight. A second kernel adds the segments of each ring in order. All
// sums are FP64 in a fixed order, so D is bitwise reproducible.
#include "nfs.h"
#include "nfs_device.hpp"
#include "nfs_host.hpp"
#include "nfs_kernels.hpp"

namespace nfs {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
static_assert(kSegModes == 64 * kWaves, "one table entry per thread of a segment");

__global__ __launch_bounds__(kThreads) void bin_segment_kernel(
    const float* __restrict__ acc, int n_lags, const int32_t* __restrict__ bin_slots,
    const int32_t* __restrict__ seg_first, double* __restrict__ part,
    long long* __restrict__ part_cnt) {
  __shared__ double red[kWaves][64];
  __shared__ long long redc[kWaves];
  const int seg = blockIdx.x;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int i0 = seg_first[seg] + wave * 64;
  const int i1 = seg_first[seg + 1];
  const int cnt = __builtin_amdgcn_readfirstlane(max(0, min(64, i1 - i0)));
  const int code = lane < cnt ? bin_slots[i0 + lane] : 0;
  int wsum = lane < cnt ? ((code & 1) ? 2 : 1) : 0;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) wsum += __shfl_xor(wsum, o, 64);
  if (lane == 0) redc[wave] = wsum;
  for (int l0 = 0; l0 < n_lags; l0 += 64) {
    const int l = l0 + lane;
    const bool lag_ok = l < n_lags;
    double s = 0.0;
    for (int j = 0; j < cnt; j += 8) {
      float v[8];
      int c8[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        c8[u] = j + u < cnt ? __builtin_amdgcn_readlane(code, j + u) : 0;
        const int64_t slot = c8[u] >> 1;
        v[u] = (j + u < cnt && lag_ok) ? acc[slot * n_lags + l] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) s += ((c8[u] & 1) ? 2.0 : 1.0) * double(v[u]);
    }
    red[wave][lane] = s;
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
    if (l == 0 && status_out)
      status_out[0] = (status[0] & 2)   ? NFS_E_TIMEOUT
                      : (status[0] & 1) ? NFS_E_DEGENERATE_FRAME
                                        : NFS_OK;
  }
}

}  // namespace

hipError_t launch_bins(int n_bins, const float* acc, int n_lags, const int32_t* bin_slots,
                       const int32_t* seg_first, int n_segs, const int32_t* bin_seg0,
                       double* part, long long* part_cnt, const int32_t* lags,
                       int64_t n_frames, const int32_t* status, double* D, int64_t* counts,
                       int64_t* pairs, int32_t* status_out, hipStream_t s) {
  hipLaunchKernelGGL(bin_segment_kernel, dim3(unsigned(n_segs)), dim3(kThreads), 0, s, acc,
                     n_lags, bin_slots, seg_first, part, part_cnt);
  const int64_t items = int64_t(n_bins) * n_lags;
  hipLaunchKernelGGL(bin_final_kernel, dim3(unsigned((items + 255) / 256)), dim3(256), 0, s,
                     n_bins, n_lags, part, part_cnt, bin_seg0, lags, n_frames, status, D,
                     counts, pairs, status_out);
  return hipGetLastError();
}

}  // namespace nfs
