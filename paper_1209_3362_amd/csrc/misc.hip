// Small utility kernels: fills (used instead of memset nodes so the work
// can be captured in a graph), the bin map and spectrum expansion used for
// inspection.
#include "nfs_device.hpp"
#include "nfs_kernels.hpp"

namespace nfs {
namespace {

__global__ void fill_u32_kernel(uint32_t* __restrict__ dst, size_t words, uint32_t value) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < words;
       i += size_t(gridDim.x) * blockDim.x)
    dst[i] = value;
}

__global__ void bin_map_kernel(int n, int nb, int32_t* __restrict__ map) {
  const int h = n / 2;
  const int64_t total = int64_t(n) * h;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int r = int(i / h), kx = int(i % h);
    const int ky = r < h ? r : r - n;
    map[i] = dev::bin_of_dev(n, nb, ky, kx);
  }
}

// I_t = decoded stored value + sigma_t * F[reference] on the stored modes,
// I_t(0) = n^2, zero elsewhere. The slot holds FP32 pairs, or BF16 / FP16
// pairs (FP16 scaled by 1 / fscale.z).
__global__ void expand_kernel(int n, const char* __restrict__ spec_base, int spec,
                              const int32_t* __restrict__ row_width,
                              const int32_t* __restrict__ tiles,
                              const float2* __restrict__ refspec,
                              const float4* __restrict__ fscale_slot, float2* __restrict__ out) {
  const int h = n / 2;
  const int64_t total = int64_t(n) * h;
  const float4 sc = *fscale_slot;
  const float sigma = sc.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int r = int(i / h), kx = int(i % h);
    float2 v = make_float2(0.f, 0.f);
    if (kx < row_width[r]) {
      const int64_t at = dev::ring_slot(n, tiles, r, kx);
      float2 a;
      if (spec == dev::kSpecF32) {
        a = reinterpret_cast<const float2*>(spec_base)[at];
      } else {
        const uint32_t w = reinterpret_cast<const uint32_t*>(spec_base)[at];
        a = spec == dev::kSpecBF16 ? dev::unpack_bf16(w) : dev::unpack_f16(w);
        a = make_float2(a.x * sc.z, a.y * sc.z);
      }
      const float2 R = refspec[at];
      v = make_float2(fmaf(sigma, R.x, a.x), fmaf(sigma, R.y, a.y));
      if (at == 0) v = make_float2(float(n) * float(n), 0.f);
    }
    out[i] = v;
  }
}

// P_tau(k) = S_tau(k) / (N - tau) from the mode-major sums acc[mode][lag]
// onto [n_lags][n][n/2 + 1]; 0 where no mode is stored, NaN for a delay
// without pairs. nyq_slot >= 0: the k_x = n/2 column is stored, row r in
// slot nyq_slot + r.
__global__ void power_kernel(int n, int n_lags, const float* __restrict__ acc,
                             const int32_t* __restrict__ row_width,
                             const int32_t* __restrict__ tiles, int64_t nyq_slot,
                             const int32_t* __restrict__ lags, int64_t n_frames,
                             float* __restrict__ out) {
  const int h = n / 2, w = h + 1;
  const int64_t plane = int64_t(n) * w;
  const int64_t total = int64_t(n_lags) * plane;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int l = int(i / plane);
    const int64_t rem = i - int64_t(l) * plane;
    const int r = int(rem / w), kx = int(rem % w);
    const int64_t pairs = n_frames - lags[l];
    float v = 0.f;
    if (pairs <= 0) {
      v = __builtin_nanf("");
    } else if (kx < h && kx < row_width[r]) {
      const int64_t m = dev::ring_slot(n, tiles, r, kx);
      v = float(double(acc[m * n_lags + l]) / double(pairs));
    } else if (kx == h && nyq_slot >= 0) {
      v = float(double(acc[(nyq_slot + r) * n_lags + l]) / double(pairs));
    }
    out[i] = v;
  }
}

// Memory-bandwidth probes over `vecs` 16-byte vectors: copy src to dst,
// read src (a per-workgroup checksum goes to dst so the loads are kept), or
// write dst. Grid-stride loops, four independent vectors in flight per
// thread.
template <int MODE>
__global__ __launch_bounds__(256) void probe_kernel(const uint4* __restrict__ src,
                                                    uint4* __restrict__ dst, size_t vecs) {
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  uint32_t x = 0;
  for (; i + 3 * stride < vecs; i += 4 * stride) {
    uint4 v[4];
    if constexpr (MODE != 2) {
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = src[i + u * stride];
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = make_uint4(uint32_t(i + u), 1u, 2u, 3u);
    }
    if constexpr (MODE == 1) {
#pragma unroll
      for (int u = 0; u < 4; ++u) x ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u) dst[i + u * stride] = v[u];
    }
  }
  for (; i < vecs; i += stride) {
    if constexpr (MODE == 0) dst[i] = src[i];
    if constexpr (MODE == 1) x ^= src[i].x ^ src[i].y ^ src[i].z ^ src[i].w;
    if constexpr (MODE == 2) dst[i] = make_uint4(uint32_t(i), 1u, 2u, 3u);
  }
  if constexpr (MODE == 1) {
    __shared__ uint32_t red[4];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x ^= __shfl_xor(x, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0)
      reinterpret_cast<uint32_t*>(dst)[blockIdx.x] = red[0] ^ red[1] ^ red[2] ^ red[3];
  }
}

unsigned grid_for(int64_t items, int threads) {
  int64_t g = (items + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return unsigned(g);
}

}  // namespace

hipError_t launch_probe(int mode, const void* src, void* dst, size_t bytes, hipStream_t s) {
  const size_t vecs = bytes / 16;
  // Eight workgroups of 256 threads per CU on 256 CUs.
  const unsigned grid = 2048;
  const uint4* a = static_cast<const uint4*>(src);
  uint4* b = static_cast<uint4*>(dst);
  if (mode == 0)
    hipLaunchKernelGGL(probe_kernel<0>, dim3(grid), dim3(256), 0, s, a, b, vecs);
  else if (mode == 1)
    hipLaunchKernelGGL(probe_kernel<1>, dim3(grid), dim3(256), 0, s, a, b, vecs);
  else if (mode == 2)
    hipLaunchKernelGGL(probe_kernel<2>, dim3(grid), dim3(256), 0, s, a, b, vecs);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_fill_u32(void* dst, size_t words, uint32_t value, hipStream_t s) {
  if (words == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(int64_t(words), 256)), dim3(256), 0, s,
                     static_cast<uint32_t*>(dst), words, value);
  return hipGetLastError();
}

hipError_t launch_bin_map(int n, int n_bins, int32_t* map, hipStream_t s) {
  hipLaunchKernelGGL(bin_map_kernel, dim3(grid_for(int64_t(n) * (n / 2), 256)), dim3(256), 0, s,
                     n, n_bins, map);
  return hipGetLastError();
}

hipError_t launch_expand_spectrum(int n, const void* ring, int spec, int64_t slot,
                                  int64_t mode_stride, const int32_t* row_width,
                                  const int32_t* tiles, const float2* refspec,
                                  const float4* fscale, float2* out, hipStream_t s) {
  const int64_t mode_bytes = spec == dev::kSpecF32 ? 8 : 4;
  const char* base = static_cast<const char*>(ring) + slot * mode_stride * mode_bytes;
  hipLaunchKernelGGL(expand_kernel, dim3(grid_for(int64_t(n) * (n / 2), 256)), dim3(256), 0, s,
                     n, base, spec, row_width, tiles, refspec, fscale + slot, out);
  return hipGetLastError();
}

hipError_t launch_power_spectra(int n, int n_lags, const float* acc, const int32_t* row_width,
                                const int32_t* tiles, int64_t nyq_slot, const int32_t* lags,
                                int64_t n_frames, float* out, hipStream_t s) {
  hipLaunchKernelGGL(power_kernel,
                     dim3(grid_for(int64_t(n_lags) * n * (n / 2 + 1), 256)), dim3(256), 0, s, n,
                     n_lags, acc, row_width, tiles, nyq_slot, lags, n_frames, out);
  return hipGetLastError();
}

}  // namespace nfs
