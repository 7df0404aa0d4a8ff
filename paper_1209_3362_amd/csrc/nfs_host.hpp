// Host-only planning logic of the structure-function library: descriptor
// validation, the set of stored modes, workspace layout and launch shapes.
// No HIP dependency, so it also builds with a plain C++ compiler for tests.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "nfs.h"
#include "pair_plan.hpp"

namespace nfs {

constexpr int kMinN = 16;
constexpr int kMaxN = 4096;
constexpr size_t kAlign = 256;
// Stored modes summed by one workgroup of the binning pass.
constexpr int kSegModes = 256;
// Target size of the row-transform intermediate of one batch of frames.
constexpr size_t kBatchBytes = size_t(128) << 20;
constexpr int kMaxBatch = 1024;
// Fused transform: workgroups per launch at most (2 per CU on 256 CUs).
constexpr int kFusedMaxWorkers = 512;
// Most ring slots (slot indices are 32-bit in the kernels).
constexpr int64_t kMaxCapacity = 0x7fffffff;
// Per ring slot: {sigma, sigma - sigma_ref, 2^-e (FP16 storage, else 1), 0}.
constexpr size_t kScaleBytes = 16;

inline bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }
inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Exact integer square root: largest s with s*s <= v.
uint64_t isqrt_u64(uint64_t v);
// Smallest s >= 0 with s*s >= v (v >= 0).
int64_t ceil_sqrt_i64(int64_t v);

// Bin of mode (ky, kx): isqrt(|k|^2 nb^2) / (n/2), or -1 when >= nb.
int bin_of(int n, int nb, int ky, int kx);
// Ring b holds the modes with lo <= |k|^2 < hi.
void ring_bounds(int n, int nb, int b, int64_t* lo, int64_t* hi);

struct Layout {
  int n = 0, h = 0, n_bins = 0, n_lags = 0;
  int in_dtype = 0;
  int spec_dtype = 0, accum = 0;
  int mode_bytes = 8;      // bytes per stored mode in the ring
  int64_t modes = 0;       // M: stored modes per spectrum (those in a ring)
  int64_t slots = 0;       // slots per spectrum in the tiled layout (>= M)
  int64_t mode_stride = 0; // slots rounded up to 64: ring slot and sum-row pitch
  int64_t capacity = 0;    // ring slots
  int batch = 0;           // frames per transform launch
  int host_staging = 0;    // two staging buffers of `batch` frames for host pushes
  size_t frame_bytes = 0;  // bytes of one input frame
  int backward = 0;        // nfs_backward buffers reserved
  int full = 0;            // every half-plane mode stored (desc.full_spectra)
  // Full plans: slot of the k_x = n/2 mode of row r is nyq_slot + r (after
  // the tiles); -1 otherwise.
  int64_t nyq_slot = -1;
  int64_t binned = 0;      // modes that land in a ring (every plan bins only these)
  int max_lag = 0;
  std::vector<int32_t> lags;
  std::vector<int32_t> row_width;   // [n] stored modes k_x < n/2 of transform-order row r
  // Tiled slot layout (see ring_slot): {base_0 .. base_T, R_0 .. R_{T-1}},
  // T = n / 16 tiles of 8 columns.
  std::vector<int32_t> tiles;
  std::vector<LagGroup> groups;
  // Binning table: the stored modes of ring 0, then of ring 1, ..., each as
  // 2 * slot + (k_x > 0), rows k_y ascending and k_x ascending within a row
  // (weight 2 for k_x > 0: the mode and its mirror -k; 1 on k_x = 0, where
  // both are stored). Segment s covers entries [seg_first[s],
  // seg_first[s + 1]) (at most kSegModes, of one ring; every ring has at
  // least one segment); ring b owns segments [bin_seg0[b], bin_seg0[b + 1]).
  std::vector<int32_t> bin_slots, seg_first, bin_seg0;
  // Byte offsets into the workspace.
  size_t off_ring = 0, off_inter = 0, off_rowsum = 0, off_rowabs = 0, off_acc = 0;
  size_t off_status = 0, off_tw = 0, off_width = 0, off_tiles = 0;
  size_t off_ref = 0, off_refspec = 0;  // reference frame and its transform
  size_t off_nyq = 0;     // full plans: the row pass's k_x = n/2 values [batch][n]
  size_t off_comp = 0;    // Kahan plans: compensation of the sums, laid out like them
  // Fused transform (n = 1024): scheduler state of one launch, fused_slots
  // job slots per XCD; its two buffers are carved from the intermediate.
  size_t off_sched = 0;
  int fused_slots = 0;
  bool fused_ok = false;   // the intermediate holds the fused buffers (32 MiB)
  size_t off_stage = 0;   // host-push staging: 2 x batch frames (host_staging)
  // nfs_backward (backward): k-space gradients of a batch [batch][mode_stride]
  // complex (the same region later holds its g' images [batch][n][n] floats),
  // per-row sums [batch][n] and per-frame scalars [batch] (two
  // doubles each), window gradient [n][n] FP64, g table [n_lags][n_bins],
  // bin of every stored mode [mode_stride], full-plane modes per bin.
  size_t off_gk = 0, off_brow = 0, off_bscal = 0, off_gw = 0, off_gtab = 0;
  size_t off_mode_bin = 0, off_bin_count = 0;
  std::vector<int32_t> mode_bin;   // [mode_stride], 0 past the stored modes
  std::vector<int64_t> bin_count;  // [n_bins]
  size_t off_fscale = 0;  // after the ring: kScaleBytes per slot
  size_t off_segs = 0, off_bin_slots = 0, off_part = 0, off_part_cnt = 0;
  size_t off_lags = 0, total = 0;
};

// Validates `d`; on failure returns the status and fills `err`.
nfs_status validate_desc(const nfs_desc* d, std::string* err);

// Builds the layout for `d`. With d->capacity == 0 and bytes_available > 0,
// the ring takes every whole spectrum that fits; with both 0 the ring has
// max_lag + 64 slots.
nfs_status make_layout(const nfs_desc* d, size_t bytes_available, Layout* L,
                       std::string* err);

// Host twin of the device ring_slot: slot of (row r, column kx) in the
// tiled layout, or -1 when the row is not kept in kx's tile.
int ring_slot_host(const Layout& L, int r, int kx);

// W_n^j = exp(-2 pi i j / n), j = 0..n-1, evaluated in double and rounded
// once to float; interleaved (re, im).
std::vector<float> twiddle_table(int n);

}  // namespace nfs
