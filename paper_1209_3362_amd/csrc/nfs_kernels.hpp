// Host-side launchers of the library's HIP kernels. Each returns the HIP
// status of its launch; argument shapes are checked by the caller.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace nfs {

// Row pass (per image row: real-to-complex transform of n pixels to the
// n/2 half-plane coefficients k_x = 0..n/2-1) plus per-row sums of what was
// transformed. frames: [nframes][n][n] of u16 (in_dtype 0) or f32 (1);
// ref: [n][n] of the same type subtracted from every frame first, or null;
// window: [n][n] multiplied in after the subtraction, or null. Writes inter
// [nframes][tiles][n][w] complex (tiles of the w columns a column-pass
// workgroup transforms), rowsum [nframes][n] and,
// when rowabs is not null, rowabs [nframes][n]: the rows' sums of |what was
// transformed|.
// nyq: [nframes][n] floats receiving X_y(n/2) (full half-plane plans), or null.
hipError_t launch_row_pass(int n, int in_dtype, const void* frames, const void* ref,
                           const float* window, int nframes, float2* inter, double* rowsum,
                           double* rowabs, float* nyq, const float2* tw, hipStream_t s);

// Fused row and column passes of `nframes` frames (n = 1024 only) in one
// persistent launch of `workers` workgroups: per-XCD task queues, the
// intermediate of a frame handed over inside one XCD through bufA (the
// first `keep` column tiles, 8 x keep x 64 KB) and bufB (the other tiles).
// sched: scheduler state, (8 * 64 + 16 * slots) ints, cleared before the
// launch; slots >= ceil(nframes / 8); frame j is processed on XCD j mod 8,
// so `workers` must be a multiple of 8 (dispatch is round robin over the
// XCDs). Stores exactly what
// launch_row_pass + launch_col_pass store; a wait past spin_limit polls
// sets bit 1 of *status.
hipError_t launch_fused_transform(int n, int in_dtype, int spec, const void* frames,
                                  const void* ref, const float* window, int nframes,
                                  double* rowsum, double* rowabs, float2* bufA, float2* bufB,
                                  int keep, int* sched, int slots, int workers,
                                  unsigned spin_limit, const double* refscal, float4* fscale,
                                  int32_t* status, int64_t t0, int64_t capacity,
                                  int64_t mode_stride, int64_t n_modes, const int32_t* tiles,
                                  const float2* tw, void* ring, unsigned long long* work,
                                  hipStream_t s);

// Column k_x = n/2 of full half-plane plans, after the column pass of the
// same frames: transform of nyq[f][y] over y, stored like the other modes
// (reference: unscaled FP32 into refspec) at slots nyq_slot + r.
hipError_t launch_nyquist_col(int n, bool reference, int spec, const float* nyq, int nframes,
                              int64_t t0, int64_t capacity, int64_t mode_stride,
                              int64_t nyq_slot, const float2* tw, const float4* fscale,
                              void* ring, float2* refspec, hipStream_t s);

// Column pass (per column k_x: complex transform over the n rows), with the
// frame scales formed from the row sums.
// reference == true: the rows are the reference image (one frame); set
// refscal = {S_ref, n^2/S_ref} and store its transform unscaled in refspec
// (FP32, 0 at k = 0).
// reference == false: the rows are (frame - reference); with
// sigma = n^2 / (S_ref + row sums), store sigma * X, 0 at k = 0, for frame f
// in ring slot slot = (t0 + f) mod capacity in the storage type `spec`
// (nfs_desc.spec_dtype: 8 or 4 bytes per mode, mode_stride modes per slot),
// and fscale[slot] = {sigma, sigma - sigma_ref, 2^-e, 0}, with e the FP16
// scale exponent formed from rowabs (FP16 storage) or 0. A frame whose sum
// is not positive and finite sets bit 0 of *status and gets sigma = 0.
// n_modes: slots per spectrum in the tiled layout (tiles, see ring_slot);
// only those are written.
hipError_t launch_col_pass(int n, bool reference, int spec, const float2* inter,
                           const double* rowsum, const double* rowabs, int nframes, int64_t t0,
                           int64_t capacity, int64_t mode_stride, int64_t n_modes,
                           const int32_t* tiles, const float2* tw, void* ring,
                           float2* refspec, double* refscal, float4* fscale, int32_t* status,
                           unsigned long long* work, hipStream_t s);

// Lag-pair accumulation for target frames [T0, T1) and the lags
// lags[0..n_lags): acc[m * acc_pitch + l] += sum_t |I_t(m) - I_{t - lags[l]}(m)|^2
// over t in [T0, T1) with t - lag >= 0 (acc is mode-major; with `assign`
// the sums are stored instead, for modes m < n_modes), where
// I_t = decoded ring slot of t + fscale[slot].y * refspec (refspec has
// mode_stride entries, 0 at k = 0; the ring stores `spec`-typed modes,
// FP16 ones scaled by 1 / fscale[slot].z). Frames [max(0, T0 - max lag), T1)
// must be in the ring. `modes` per workgroup (16 or 8), `hist` LDS rows;
// wave w sums lags of a near-equal contiguous slice (at most per_wave);
// modes 0: the global-memory kernel (at most kGlobalLags lags, any delay);
// kahan: chunk sums added with Kahan compensation, and with comp (laid out
// like acc) not null the window's totals are added to acc with Kahan
// compensation kept in comp across launches (assign clears it). work (or
// null): the (target, lag) pairs summed are added to *work.
hipError_t launch_pairs(const void* ring, int spec, bool kahan, const float2* refspec,
                        const float4* fscale, int64_t n_modes, int64_t mode_stride,
                        int64_t capacity, int64_t T0, int64_t T1, const int32_t* lags,
                        int n_lags, int max_lag, float* acc, int acc_pitch, bool assign,
                        int modes, int hist, int waves, int per_wave, size_t lds,
                        unsigned long long* work, float* comp, hipStream_t s);

// Azimuthal binning from the sums acc [slots][n_lags] (mode-major): segment
// partials over the binning table bin_slots (entries 2 * slot + (k_x > 0),
// ring by ring; segment s covers entries [seg_first[s], seg_first[s + 1])),
// then per ring D[l][b] = sum_{k in ring b} w(k) acc[k][l] / (C_b * pairs_l)
// in double, counts[b] = C_b, pairs[l] = max(0, N - lag_l), status_out[0]
// from *status. pairs_l == 0 gives NaN.
hipError_t launch_bins(int n_bins, const float* acc, int n_lags, const int32_t* bin_slots,
                       const int32_t* seg_first, int n_segs, const int32_t* bin_seg0,
                       double* part, long long* part_cnt, const int32_t* lags,
                       int64_t n_frames, const int32_t* status, double* D, int64_t* counts,
                       int64_t* pairs, int32_t* status_out, hipStream_t s);

// Bandwidth probe over `bytes` (a multiple of 16): mode 0 copies src to
// dst, 1 reads src (dst receives one checksum word per workgroup, 2048
// words), 2 writes dst.
hipError_t launch_probe(int mode, const void* src, void* dst, size_t bytes, hipStream_t s);

// Fills `words` 32-bit words at dst with `value`.
hipError_t launch_fill_u32(void* dst, size_t words, uint32_t value, hipStream_t s);

// Writes the bin of every half-plane mode to map [n][n/2].
hipError_t launch_bin_map(int n, int n_bins, int32_t* map, hipStream_t s);

// Expands ring slot `slot` to the spectrum out [n][n/2] complex: decoded
// stored value + sigma * refspec (sigma = fscale[slot].x), I(0) = n^2,
// zeros where not stored.
hipError_t launch_expand_spectrum(int n, const void* ring, int spec, int64_t slot,
                                  int64_t mode_stride, const int32_t* row_width,
                                  const int32_t* tiles, const float2* refspec,
                                  const float4* fscale, float2* out, hipStream_t s);

// P_tau(k) = acc[mode][l] / (n_frames - lags[l]) written to out
// [n_lags][n][n/2 + 1] (0 at modes that are not stored, NaN for every mode
// of a delay with n_frames - lag <= 0).
hipError_t launch_power_spectra(int n, int n_lags, const float* acc, const int32_t* row_width,
                                const int32_t* tiles, int64_t nyq_slot, const int32_t* lags,
                                int64_t n_frames, float* out, hipStream_t s);

// Differentiation form (nfs_backward). g table: gtab[l][b] =
// dL_dD[l][b] / (C_b (N - lag_l)), 0 for lag 0, delays with no pair and
// empty bins.
hipError_t launch_grad_table(int n_lags, int n_bins, const double* dL_dD,
                             const int64_t* bin_count, const int32_t* lags, int64_t n_frames,
                             float* gtab, hipStream_t s);

// k-space gradient of frames [t0, t0 + nframes) on the stored modes:
// gk[f][m] = 2 sum_l gtab[l][mode_bin[m]] * ([t + lag < N] (a_t - a_{t+lag})
// + [t >= lag] (a_t - a_{t-lag})), a_t decoded as by the pair kernel. The
// frames [max(0, t0 - max_lag), min(N, t0 + nframes + max_lag)) must be in
// the ring, frame tw0 in slot slot0 and frame tw0 + i in slot
// (slot0 + i) mod capacity (a window of at most capacity frames).
hipError_t launch_grad_spectra(const void* ring, int spec, const float4* fscale,
                               const float2* refspec, int64_t capacity, int64_t mode_stride,
                               int64_t n_modes, const int32_t* mode_bin, const float* gtab,
                               const int32_t* lags, int n_lags, int n_bins, int max_lag,
                               int64_t n_frames, int64_t t0, int nframes, int64_t tw0,
                               int64_t slot0, float2* gk, hipStream_t s);

// Adjoint of the 2D transform for nframes frames: inverse column transforms
// of gk (stored modes, [nframes][mode_stride]) into z (n x n/2 complex per
// frame, in tiles of the column transform's workgroup width), then per row
// the real inverse transform with the half-plane weights into gprime
// [nframes][n][n] floats (may alias gk: gk is read before), and rowsums
// [nframes][n] = {sum_x u, sum_x g' u} with u = window * frame (frames: the
// batch's [nframes][n][n] pixels of in_dtype; window may be null).
hipError_t launch_inverse_2d(int n, int in_dtype, const float2* gk, int64_t mode_stride,
                             const int32_t* row_width, const int32_t* tiles,
                             const float2* tw, int nframes, float2* z, float* gprime,
                             const void* frames, const float* window, double2* rowsums,
                             hipStream_t s);

// Adjoint of the normalisation and window product for nframes frames:
// scal[f] = {1/m, mean(g' i')}; dL_dframes[f] = w (g' - mean(g' i')) / m
// (if not null) and gw += sum_f frame_f (g' - mean(g' i')) / m (if not null).
hipError_t launch_grad_finish(int n, int in_dtype, int nframes, const double2* rowsums,
                              double2* scal, const float* gprime, const void* frames,
                              const float* window, float* dL_dframes, double* gw,
                              hipStream_t s);

// out[p] = float(gw[p]) for the n x n pixels.
hipError_t launch_window_out(int n, const double* gw, float* out, hipStream_t s);

// Device address of the library's static scratch array (NFS_STATIC_SCRATCH_BYTES,
// 256-byte aligned) on `device`, looked up once per device and cached.
hipError_t static_scratch(int device, void** addr);

}  // namespace nfs
