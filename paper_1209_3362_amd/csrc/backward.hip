// Differentiation form: gradients of a scalar loss L of D with respect to
// the frames and the per-pixel window, by the adjoint of every step of the
// forward path, taken in reverse (Eq. 1 and the processing section define
// the forward steps; the adjoint of each follows from the chain rule).
//
// With g[l][b] = dL/dD(b, tau_l) / (C_b (N - tau_l)), per batch of frames:
//   grad_spectra_kernel  k-space gradient (dL/dRe + i dL/dIm) of every
//       stored coefficient: G_t(k) = 2 sum_l g[l][b(k)] *
//       ([t + tau < N] (a_t - a_{t+tau}) + [t >= tau] (a_t - a_{t-tau})),
//       from the resident spectra a_t (only their differences enter);
//   inv_col_kernel       Z(y, k_x) = sum_{k_y} G(k_y, k_x) e^{+2 pi i k_y y/n}
//       over the stored modes (the adjoint of the column transform);
//   inv_row_kernel       g'(y, x) = Re sum_{k_x} c_k Z(y, k_x) e^{+2 pi i k_x x/n},
//       c = 1 at k_x = 0 and 2 above (each half-plane mode stands for k and
//       -k), i.e. dL/di' for the mean-normalised image i' = u / m; also the
//       row sums of u = w * i and of g' * u;
//   frame_scal_kernel    per frame 1/m and mean(g' * i') from the row sums;
//   finish_kernel        dL/du = (g' - mean(g' * i')) / m (adjoint of the
//       division by the mean), dL/di = w * dL/du, and the window gradient
//       sum_t i_t * dL/du_t accumulated in FP64 in frame order.
// Inverse transforms are forward DFTs of conjugated data: sum_k x_k
// e^{+2 pi i jk/n} = conj(sum_k conj(x_k) e^{-2 pi i jk/n}).
#include <algorithm>

#include "fft_common.hpp"
#include "nfs_device.hpp"
#include "nfs_kernels.hpp"

namespace nfs {
using namespace dev;

namespace {

__device__ __forceinline__ float2 conjf2(float2 a) { return make_float2(a.x, -a.y); }

__global__ void grad_table_kernel(int n_lags, int n_bins, const double* __restrict__ dL_dD,
                                  const int64_t* __restrict__ bin_count,
                                  const int32_t* __restrict__ lags, int64_t n_frames,
                                  float* __restrict__ gtab) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_lags * n_bins) return;
  const int l = i / n_bins, b = i % n_bins;
  const int64_t tau = lags[l];
  const int64_t np = n_frames - tau;
  const int64_t C = bin_count[b];
  // Lag 0 (every difference is 0) and delays with no pair carry nothing.
  gtab[i] = (tau > 0 && np > 0 && C > 0) ? float(dL_dD[i] / (double(C) * double(np))) : 0.f;
}

// Ring slot of frame t inside the window of frames [tw0, tw0 + capacity)
// that the ring holds during one batch of the backward: slot0 is the slot of
// frame tw0 (tw0 mod capacity), so no 64-bit modulo is taken per load.
__device__ __forceinline__ int64_t window_slot(int64_t t, int64_t tw0, int64_t slot0,
                                               int64_t capacity) {
  const int64_t s = slot0 + (t - tw0);
  return s >= capacity ? s - capacity : s;
}

// Stored value of the frame in `slot` at mode m, as the pair kernel pairs
// it.
template <int SPEC>
__device__ __forceinline__ float2 stored_value(const char* __restrict__ ring,
                                               const float4* __restrict__ fscale,
                                               const float2* __restrict__ refspec,
                                               int64_t mode_stride, int64_t slot, int64_t m) {
  const float4 sc = fscale[slot];
  float2 a;
  if constexpr (SPEC == kSpecF32) {
    a = reinterpret_cast<const float2*>(ring)[slot * mode_stride + m];
  } else {
    const uint32_t w = reinterpret_cast<const uint32_t*>(ring)[slot * mode_stride + m];
    a = SPEC == kSpecBF16 ? unpack_bf16(w) : unpack_f16(w);
    a = make_float2(a.x * sc.z, a.y * sc.z);
  }
  const float2 R = refspec[m];
  return make_float2(fmaf(sc.y, R.x, a.x), fmaf(sc.y, R.y, a.y));
}

// One workgroup: 256 modes of one frame. Workgroups are dispatched
// round-robin over the 8 XCDs; block b is renumbered so that each XCD walks
// whole mode tiles frame by frame, and the spectra of frames t +- lag that
// neighbouring frames share stay in that XCD's L2.
template <int SPEC>
__global__ __launch_bounds__(256) void grad_spectra_kernel(
    const char* __restrict__ ring, const float4* __restrict__ fscale,
    const float2* __restrict__ refspec, int64_t capacity, int64_t mode_stride, int64_t n_modes,
    const int32_t* __restrict__ mode_bin, const float* __restrict__ gtab,
    const int32_t* __restrict__ lags, int n_lags, int n_bins, int64_t n_frames, int64_t t0,
    int nframes, int64_t tw0, int64_t slot0, float2* __restrict__ gk) {
  const int xcd = blockIdx.x % 8, local = blockIdx.x / 8;
  const int tile = xcd + 8 * (local / nframes);
  const int f = local % nframes;
  const int64_t m = int64_t(tile) * 256 + threadIdx.x;
  if (m >= n_modes) return;
  const int64_t t = t0 + f;
  const int b = mode_bin[m];
  if (b < 0) {  // a slot of the tiled layout that holds no stored mode
    gk[int64_t(f) * mode_stride + m] = make_float2(0.f, 0.f);
    return;
  }
  const float2 at = stored_value<SPEC>(ring, fscale, refspec, mode_stride,
                                       window_slot(t, tw0, slot0, capacity), m);
  float gx = 0.f, gy = 0.f;
  for (int l = 0; l < n_lags; ++l) {
    const float c = gtab[l * n_bins + b];
    if (c == 0.f) continue;
    const int64_t tau = lags[l];
    float dx = 0.f, dy = 0.f;
    if (t + tau < n_frames) {
      const float2 o = stored_value<SPEC>(ring, fscale, refspec, mode_stride,
                                          window_slot(t + tau, tw0, slot0, capacity), m);
      dx += at.x - o.x;
      dy += at.y - o.y;
    }
    if (t >= tau) {
      const float2 o = stored_value<SPEC>(ring, fscale, refspec, mode_stride,
                                          window_slot(t - tau, tw0, slot0, capacity), m);
      dx += at.x - o.x;
      dy += at.y - o.y;
    }
    gx = fmaf(c, dx, gx);
    gy = fmaf(c, dy, gy);
  }
  gk[int64_t(f) * mode_stride + m] = make_float2(2.f * gx, 2.f * gy);
}

// Windowed form of grad_spectra_kernel: one workgroup owns KM slots and
// kFB target frames and first copies the spectra of frames [its first
// target - max_lag, its last target + max_lag] of those slots, decoded, to
// LDS (pitch KM + 1 against bank conflicts), so every spectrum is read from
// memory and decoded once per workgroup instead of once per output and lag.
// Thread (j, g): slot m0 + j, targets f0 + g + i (256 / KM) of the window.
constexpr int kFB = 64;
template <int SPEC, int KM>
__global__ __launch_bounds__(256) void grad_spectra_lds_kernel(
    const char* __restrict__ ring, const float4* __restrict__ fscale,
    const float2* __restrict__ refspec, int64_t capacity, int64_t mode_stride, int64_t n_modes,
    const int32_t* __restrict__ mode_bin, const float* __restrict__ gtab,
    const int32_t* __restrict__ lags, int n_lags, int n_bins, int max_lag, int64_t n_frames,
    int64_t t0, int nframes, int64_t tw0, int64_t slot0, float2* __restrict__ gk) {
  constexpr int G = 256 / KM, KP = KM + 1, NO = kFB / G;
  extern __shared__ float2 win[];
  const int fblocks = (nframes + kFB - 1) / kFB;
  const int64_t m0 = int64_t(blockIdx.x / fblocks) * KM;
  const int f0 = (blockIdx.x % fblocks) * kFB;
  const int64_t tfirst = t0 + f0;
  const int64_t tlast = min(t0 + int64_t(nframes), tfirst + kFB);  // exclusive
  const int64_t tlo = max(int64_t(0), tfirst - max_lag);
  const int64_t thi = min(n_frames, tlast + max_lag);
  const int rows = int(thi - tlo);
  const int64_t slot_lo = window_slot(tlo, tw0, slot0, capacity);
  for (int idx = threadIdx.x; idx < rows * KM; idx += 256) {
    const int r = idx / KM, j = idx % KM;
    const int64_t m = m0 + j;
    const int64_t slot = slot_lo + r < capacity ? slot_lo + r : slot_lo + r - capacity;
    win[r * KP + j] = m < n_modes
                          ? stored_value<SPEC>(ring, fscale, refspec, mode_stride, slot, m)
                          : make_float2(0.f, 0.f);
  }
  __syncthreads();
  const int j = threadIdx.x % KM, g = threadIdx.x / KM;
  const int64_t m = m0 + j;
  if (m >= n_modes) return;
  const int b = mode_bin[m];
  float2 acc[NO];
#pragma unroll
  for (int i = 0; i < NO; ++i) acc[i] = make_float2(0.f, 0.f);
  if (b >= 0) {
    for (int l = 0; l < n_lags; ++l) {
      const float c = gtab[l * n_bins + b];
      if (c == 0.f) continue;
      const int tau = lags[l];
#pragma unroll
      for (int i = 0; i < NO; ++i) {
        const int64_t t = tfirst + g + i * G;
        if (t >= tlast) continue;
        const int r = int(t - tlo);
        const float2 at = win[r * KP + j];
        float dx = 0.f, dy = 0.f;
        if (t + tau < n_frames) {
          const float2 o = win[(r + tau) * KP + j];
          dx += at.x - o.x;
          dy += at.y - o.y;
        }
        if (t >= tau) {
          const float2 o = win[(r - tau) * KP + j];
          dx += at.x - o.x;
          dy += at.y - o.y;
        }
        acc[i].x = fmaf(c, dx, acc[i].x);
        acc[i].y = fmaf(c, dy, acc[i].y);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < NO; ++i) {
    const int64_t t = tfirst + g + i * G;
    if (t < tlast)
      gk[(t - t0) * mode_stride + m] = make_float2(2.f * acc[i].x, 2.f * acc[i].y);
  }
}

// One workgroup: CW columns k_x of up to `per_group` frames. Input: the
// stored-mode gradient of each frame (zero at modes that are not stored);
// output Z[f][tile][y][TWD] (tiles of TWD columns, one per workgroup, so
// each workgroup writes one contiguous block). The source offsets of a
// thread's rows are computed once; the next frame is loaded during the
// second half of the current transform.
template <int N>
__global__ __launch_bounds__(ColCfg<N>::THREADS) void inv_col_kernel(
    const float2* __restrict__ gk, int64_t mode_stride, const int32_t* __restrict__ row_width,
    const int32_t* __restrict__ tiles, const float2* __restrict__ tw, int nframes,
    int per_group, float2* __restrict__ z) {
  using C = ColCfg<N>;
  constexpr int CW = C::CW, CP = C::CP, THREADS = C::THREADS, P1 = C::P1, P2 = C::P2;
  constexpr int GROUPS = C::GROUPS, TILES = C::TILES, TWD = C::TWD;
  __shared__ float2 lds[CW * CP];
  __shared__ float2 twl[C::TWL];
  const int grp = blockIdx.x % GROUPS;
  const int f_begin = (blockIdx.x / GROUPS) * per_group;
  const int f_end = min(nframes, f_begin + per_group);
  const int tid = threadIdx.x;
  const int c = tid % CW, j1 = tid / CW;
  const int kx = grp * CW + c;
  load_col_twiddles<N>(twl, tw, tid, THREADS);
  int off[P2];
#pragma unroll
  for (int j2 = 0; j2 < P2; ++j2) {
    const int r = j1 + P1 * j2;
    off[j2] = kx < row_width[r] ? ring_slot(N, tiles, r, kx) : -1;
  }
  auto load = [&](float2 (&v)[P2], int f) {
    const float2* src = gk + int64_t(f) * mode_stride;
#pragma unroll
    for (int j2 = 0; j2 < P2; ++j2)
      v[j2] = off[j2] >= 0 ? conjf2(src[off[j2]]) : make_float2(0.f, 0.f);
  };
  float2 v[P2];
  if (f_begin < f_end) load(v, f_begin);
  __syncthreads();
  float2* vec = lds + c * CP;
  for (int f = f_begin; f < f_end; ++f) {
    dft_first<N>(v, vec, twl, tw, j1);
    __syncthreads();
    if (f + 1 < f_end) load(v, f + 1);
    float2* dst = z + (int64_t(f) * TILES + kx / TWD) * N * TWD + kx % TWD;
    dft_second<N>(vec, j1, [&](int y, float2 X) { dst[int64_t(y) * TWD] = conjf2(X); });
    __syncthreads();
  }
}

// One workgroup: CW rows y of up to `per_group` frames. Reads the rows of
// Z (tiled as inv_col_kernel writes it, so a wave's loads cover whole
// CW-row blocks of tiles), writes g'[f][y][0..n) as floats, and
// rowsums[f][y] = {sum_x u, sum_x g' u} with u = w * i. The next frame's
// rows are loaded during the second half of the current transform.
template <int N, typename T, bool WIN>
__global__ __launch_bounds__(ColCfg<N>::THREADS) void inv_row_kernel(
    const float2* __restrict__ z, float* __restrict__ gprime, const T* __restrict__ frames,
    const float* __restrict__ window, const float2* __restrict__ tw, int nframes,
    int per_group, double2* __restrict__ rowsums) {
  using C = ColCfg<N>;
  constexpr int CW = C::CW, CP = C::CP, THREADS = C::THREADS, P1 = C::P1, P2 = C::P2;
  constexpr int TILES = C::TILES, TWD = C::TWD;
  constexpr int RG = N / CW;  // row groups per frame
  __shared__ float2 lds[CW * CP];
  __shared__ float2 twl[C::TWL];
  __shared__ double2 red[CW][P1];
  const int rg = blockIdx.x % RG;
  const int f_begin = (blockIdx.x / RG) * per_group;
  const int f_end = min(nframes, f_begin + per_group);
  const int tid = threadIdx.x;
  const int c = tid % CW, j1 = tid / CW;
  const int y = rg * CW + c;
  load_col_twiddles<N>(twl, tw, tid, THREADS);
  // Only k = j1 + P1 j2 < n/2 carry data: j2 < P2 / 2.
  constexpr int HALF = P2 / 2;
  auto load = [&](float2 (&v)[P2], int f) {
    const float2* zf = z + int64_t(f) * TILES * N * TWD + int64_t(y) * TWD;
#pragma unroll
    for (int j2 = 0; j2 < P2; ++j2) {
      if (j2 < HALF) {
        const int k = j1 + P1 * j2;
        const float2 a = zf[int64_t(k / TWD) * N * TWD + k % TWD];
        // conj of c_k Z(y, k); at k_x = 0 Z is real (Hermitian column).
        v[j2] = k == 0 ? make_float2(a.x, 0.f) : make_float2(2.f * a.x, -2.f * a.y);
      } else {
        v[j2] = make_float2(0.f, 0.f);
      }
    }
  };
  float2 v[P2];
  if (f_begin < f_end) load(v, f_begin);
  __syncthreads();
  float2* vec = lds + c * CP;
  const float* wr = WIN ? window + int64_t(y) * N : nullptr;
  for (int f = f_begin; f < f_end; ++f) {
    dft_first<N>(v, vec, twl, tw, j1);
    __syncthreads();
    if (f + 1 < f_end) load(v, f + 1);
    const int64_t row = int64_t(f) * N + y;
    float* gr = gprime + row * N;
    const T* ir = frames + row * N;
    double su = 0.0, sgu = 0.0;
    dft_second<N>(vec, j1, [&](int x, float2 X) {
      const float g = X.x;
      float u = float(ir[x]);
      if constexpr (WIN) u *= wr[x];
      su += double(u);
      sgu += double(g) * double(u);
      gr[x] = g;
    });
    red[c][j1] = make_double2(su, sgu);
    __syncthreads();
    if (j1 == 0) {
      double a = 0.0, b = 0.0;
#pragma unroll
      for (int j = 0; j < P1; ++j) {
        a += red[c][j].x;
        b += red[c][j].y;
      }
      rowsums[row] = make_double2(a, b);
    }
  }
}

// Per frame: {1/m, mean(g' * i')} with m = mean(u); a frame with m <= 0
// (degenerate in the forward pass) gets {0, 0}, so its gradient is 0.
__global__ __launch_bounds__(256) void frame_scal_kernel(int n, const double2* __restrict__ rowsums,
                                                         double2* __restrict__ scal) {
  __shared__ double2 red[256];
  const int f = blockIdx.x;
  double a = 0.0, b = 0.0;
  for (int y = threadIdx.x; y < n; y += 256) {
    const double2 v = rowsums[int64_t(f) * n + y];
    a += v.x;
    b += v.y;
  }
  red[threadIdx.x] = make_double2(a, b);
  __syncthreads();
  if (threadIdx.x == 0) {
    double su = 0.0, sgu = 0.0;
    for (int i = 0; i < 256; ++i) {
      su += red[i].x;
      sgu += red[i].y;
    }
    const double px = double(n) * double(n);
    const double m = su / px;
    const bool ok = m > 0.0 && isfinite(m);
    // mean(g' * i') = (sum g' u / m) / n^2
    scal[f] = ok ? make_double2(1.0 / m, sgu / (m * px)) : make_double2(0.0, 0.0);
  }
}

template <typename T, bool WIN>
__global__ __launch_bounds__(256) void finish_kernel(
    int64_t px, int nframes, const float* __restrict__ gprime, const T* __restrict__ frames,
    const float* __restrict__ window, const double2* __restrict__ scal,
    float* __restrict__ dL_dframes, double* __restrict__ gw) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= px) return;
  const float w = WIN ? window[p] : 1.f;
  double acc = 0.0;
  // 16 frames' loads in flight per thread (4: 0.950 ms of backward on the
  // 256 x 512^2 workload, 8: 0.935, 16: 0.928, 32: 1.03 at a lower
  // occupancy).
#pragma unroll 16
  for (int f = 0; f < nframes; ++f) {
    const double2 s = scal[f];
    const double du = (double(gprime[int64_t(f) * px + p]) - s.y) * s.x;
    if (dL_dframes) dL_dframes[int64_t(f) * px + p] = float(double(w) * du);
    acc += double(frames[int64_t(f) * px + p]) * du;
  }
  if (gw) gw[p] += acc;
}

__global__ void window_out_kernel(int64_t px, const double* __restrict__ gw,
                                  float* __restrict__ out) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p < px) out[p] = float(gw[p]);
}

template <int N>
hipError_t inverse_2d(int in_dtype, const float2* gk, int64_t mode_stride,
                      const int32_t* row_width, const int32_t* tiles, const float2* tw,
                      int nframes, float2* z, float* gprime, const void* frames,
                      const float* window, double2* rowsums, hipStream_t s) {
  using C = ColCfg<N>;
  // At least one and at most 8 frames per workgroup, for about `target`
  // workgroups: 1024 for the column transform (its set-up is amortised over
  // more frames; measured faster than 2048 and 512), 2048 for the row
  // transform (measured faster than 1024).
  auto per = [&](int groups, int target) {
    return std::max(1, std::min(8, nframes * groups / target));
  };
  const int pc = per(C::GROUPS, 1024);
  const unsigned col_blocks = unsigned(C::GROUPS * ((nframes + pc - 1) / pc));
  hipLaunchKernelGGL(inv_col_kernel<N>, dim3(col_blocks), dim3(C::THREADS), 0, s, gk,
                     mode_stride, row_width, tiles, tw, nframes, pc, z);
  constexpr int RG = N / C::CW;
  const int pr = per(RG, 2048);
  const dim3 grid(unsigned(RG * ((nframes + pr - 1) / pr)));
#define NFS_INVROW_GO(T, W)                                                                   \
  hipLaunchKernelGGL((inv_row_kernel<N, T, W>), grid, dim3(C::THREADS), 0, s, z, gprime,     \
                     static_cast<const T*>(frames), window, tw, nframes, pr, rowsums)
  if (in_dtype == 0) {
    if (window) NFS_INVROW_GO(uint16_t, true); else NFS_INVROW_GO(uint16_t, false);
  } else {
    if (window) NFS_INVROW_GO(float, true); else NFS_INVROW_GO(float, false);
  }
#undef NFS_INVROW_GO
  return hipGetLastError();
}

}  // namespace

hipError_t launch_grad_table(int n_lags, int n_bins, const double* dL_dD,
                             const int64_t* bin_count, const int32_t* lags, int64_t n_frames,
                             float* gtab, hipStream_t s) {
  const int items = n_lags * n_bins;
  hipLaunchKernelGGL(grad_table_kernel, dim3(unsigned((items + 255) / 256)), dim3(256), 0, s,
                     n_lags, n_bins, dL_dD, bin_count, lags, n_frames, gtab);
  return hipGetLastError();
}

hipError_t launch_grad_spectra(const void* ring, int spec, const float4* fscale,
                               const float2* refspec, int64_t capacity, int64_t mode_stride,
                               int64_t n_modes, const int32_t* mode_bin, const float* gtab,
                               const int32_t* lags, int n_lags, int n_bins, int max_lag,
                               int64_t n_frames, int64_t t0, int nframes, int64_t tw0,
                               int64_t slot0, float2* gk, hipStream_t s) {
  // The windowed kernel when a window of kFB targets plus the lags either
  // side fits 64 KB of LDS with 16 or 8 slots per workgroup (16 measured
  // faster than 32, which holds half as many workgroups per CU, and than 8).
  const int64_t rows = kFB + 2 * int64_t(max_lag);
  const int fblocks = (nframes + kFB - 1) / kFB;
  const char* rr = static_cast<const char*>(ring);
#define NFS_GRADW_GO(SPECV, KMV)                                                              \
  hipLaunchKernelGGL((grad_spectra_lds_kernel<SPECV, KMV>),                                   \
                     dim3(unsigned(((n_modes + KMV - 1) / KMV) * fblocks)), dim3(256),         \
                     size_t(rows) * (KMV + 1) * 8, s, rr, fscale, refspec, capacity,          \
                     mode_stride, n_modes, mode_bin, gtab, lags, n_lags, n_bins, max_lag,      \
                     n_frames, t0, nframes, tw0, slot0, gk)
#define NFS_GRADW_KM(KMV)                                                                     \
  if (rows * (KMV + 1) * 8 <= 64 * 1024) {                                                    \
    if (spec == kSpecF32) NFS_GRADW_GO(kSpecF32, KMV);                                        \
    else if (spec == kSpecBF16) NFS_GRADW_GO(kSpecBF16, KMV);                                 \
    else NFS_GRADW_GO(kSpecF16, KMV);                                                         \
    return hipGetLastError();                                                                 \
  }
  NFS_GRADW_KM(16)
  NFS_GRADW_KM(8)
#undef NFS_GRADW_KM
#undef NFS_GRADW_GO
  // Mode tiles rounded up to a multiple of the 8 XCDs (see the kernel).
  const int64_t tiles = ((n_modes + 255) / 256 + 7) / 8 * 8;
  const dim3 grid(unsigned(tiles * nframes));
  const char* r = static_cast<const char*>(ring);
#define NFS_GRAD_GO(SPECV)                                                                    \
  hipLaunchKernelGGL(grad_spectra_kernel<SPECV>, grid, dim3(256), 0, s, r, fscale, refspec,  \
                     capacity, mode_stride, n_modes, mode_bin, gtab, lags, n_lags, n_bins,   \
                     n_frames, t0, nframes, tw0, slot0, gk)
  if (spec == kSpecF32)
    NFS_GRAD_GO(kSpecF32);
  else if (spec == kSpecBF16)
    NFS_GRAD_GO(kSpecBF16);
  else
    NFS_GRAD_GO(kSpecF16);
#undef NFS_GRAD_GO
  return hipGetLastError();
}

hipError_t launch_inverse_2d(int n, int in_dtype, const float2* gk, int64_t mode_stride,
                             const int32_t* row_width, const int32_t* tiles,
                             const float2* tw, int nframes, float2* z, float* gprime,
                             const void* frames, const float* window, double2* rowsums,
                             hipStream_t s) {
  switch (n) {
#define NFS_INV_CASE(NV)                                                                       \
  case NV:                                                                                     \
    return inverse_2d<NV>(in_dtype, gk, mode_stride, row_width, tiles, tw, nframes, z,       \
                          gprime, frames, window, rowsums, s);
    NFS_INV_CASE(16)
    NFS_INV_CASE(32)
    NFS_INV_CASE(64)
    NFS_INV_CASE(128)
    NFS_INV_CASE(256)
    NFS_INV_CASE(512)
    NFS_INV_CASE(1024)
    NFS_INV_CASE(2048)
    NFS_INV_CASE(4096)
#undef NFS_INV_CASE
  }
  return hipErrorInvalidValue;
}

hipError_t launch_grad_finish(int n, int in_dtype, int nframes, const double2* rowsums,
                              double2* scal, const float* gprime, const void* frames,
                              const float* window, float* dL_dframes, double* gw,
                              hipStream_t s) {
  hipLaunchKernelGGL(frame_scal_kernel, dim3(unsigned(nframes)), dim3(256), 0, s, n, rowsums,
                     scal);
  const int64_t px = int64_t(n) * n;
  const dim3 grid(unsigned((px + 255) / 256));
#define NFS_FIN_GO(T, W)                                                                      \
  hipLaunchKernelGGL((finish_kernel<T, W>), grid, dim3(256), 0, s, px, nframes, gprime,      \
                     static_cast<const T*>(frames), window, scal, dL_dframes, gw)
  if (in_dtype == 0) {
    if (window) NFS_FIN_GO(uint16_t, true); else NFS_FIN_GO(uint16_t, false);
  } else {
    if (window) NFS_FIN_GO(float, true); else NFS_FIN_GO(float, false);
  }
#undef NFS_FIN_GO
  return hipGetLastError();
}

hipError_t launch_window_out(int n, const double* gw, float* out, hipStream_t s) {
  const int64_t px = int64_t(n) * n;
  hipLaunchKernelGGL(window_out_kernel, dim3(unsigned((px + 255) / 256)), dim3(256), 0, s, px,
                     gw, out);
  return hipGetLastError();
}

}  // namespace nfs
