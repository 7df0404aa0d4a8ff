// C ABI of the structure-function library: plan, push, finish, inspect.
//
// A plan carves one caller-owned device workspace (memory planned before
// the run, as in the processing section of the paper) into a ring of
// resident spectra, the row-pass intermediate of one batch of frames, the
// per-lag sums and small tables. Frames are transformed in batches as they
// are pushed; pair sums are accumulated over the window of frames not yet
// paired whenever the ring would otherwise evict a spectrum that a pending
// pair needs, and at the end.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <vector>

#include "nfs.h"
#include "nfs_host.hpp"
#include "nfs_kernels.hpp"

struct nfs_plan_s {
  nfs::Layout L;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  const float* window = nullptr;
  void* ring = nullptr;         // capacity slots of mode_stride stored modes
  float2* inter = nullptr;
  double* rowsum = nullptr;
  double* rowabs = nullptr;     // row sums of |frame - reference| (FP16 storage)
  float* nyq = nullptr;         // full plans: the row pass's k_x = n/2 values
  float* acc = nullptr;
  float* comp = nullptr;        // Kahan plans: compensation of acc across windows
  int32_t* status = nullptr;    // bit 0: a degenerate frame was pushed
  // Work counters: {frames transformed, (target, lag) pairs summed}.
  unsigned long long* work = nullptr;
  double* refscal = nullptr;    // {S_ref, sigma_ref} of the reference frame
  void* ref = nullptr;          // reference frame: first frame of the sequence
  float2* refspec = nullptr;    // its transform on the stored modes
  float4* fscale = nullptr;     // per ring slot: {sigma, sigma - sigma_ref, 2^-e, 0}
  int32_t* seg_first = nullptr;  // binning table and segments (see nfs::Layout)
  int32_t* bin_seg0 = nullptr;
  int32_t* bin_slots = nullptr;
  double* part = nullptr;       // per-segment partial sums [segments][lags]
  long long* part_cnt = nullptr;
  float2* tw = nullptr;
  int32_t* width = nullptr;
  int32_t* tiles = nullptr;     // tiled slot layout (see ring_slot)
  int32_t* lags = nullptr;
  std::vector<nfs::LagGroup> groups;  // pair launch shapes (layout's, or tuned)
  int64_t t_pushed = 0;  // frames pushed
  int64_t t_done = 0;    // frames whose pairs (as the later frame) are summed
  // No pair launch since the sums were reset: the next one stores its sums
  // instead of adding them, so a reset needs no fill of the sums.
  bool sums_fresh = true;
  // Host pushes (host_staging): two device staging buffers of one batch;
  // copies run on `copy`, transforms on `stream`. copied[j] marks batch
  // data in buffer j, freed[j] the end of the transform that read it.
  char* stage[2] = {nullptr, nullptr};
  hipStream_t copy = nullptr;
  hipEvent_t copied[2] = {nullptr, nullptr};
  hipEvent_t freed[2] = {nullptr, nullptr};
  bool freed_recorded[2] = {false, false};
  int next_stage = 0;
  // Fused transform (n = 1024): scheduler state, workgroups per launch and
  // the column tiles kept in the XCD-local buffer; off: the two-pass path.
  bool fused = false;
  int* sched = nullptr;
  int fused_workers = 0;
  int fused_keep = 32;
  // nfs_backward buffers (backward)
  float2* gk = nullptr;
  double2* brow = nullptr;
  double2* bscal = nullptr;
  double* gw = nullptr;
  float* gtab = nullptr;
  int32_t* mode_bin = nullptr;
  int64_t* bin_count = nullptr;
  std::string err;

  ~nfs_plan_s() {
    if (copy) {
      (void)hipStreamSynchronize(copy);
      (void)hipStreamDestroy(copy);
    }
    for (int j = 0; j < 2; ++j) {
      if (copied[j]) (void)hipEventDestroy(copied[j]);
      if (freed[j]) (void)hipEventDestroy(freed[j]);
    }
  }
};

namespace {

std::mutex g_mu;
std::set<nfs_plan_s*>& live() {
  static std::set<nfs_plan_s*> s;
  return s;
}

bool is_live(nfs_plan_s* h) {
  std::lock_guard<std::mutex> lk(g_mu);
  return live().count(h) != 0;
}

nfs_status fail(nfs_plan_s* h, nfs_status s, const std::string& msg) {
  if (h) h->err = msg;
  return s;
}

nfs_status hip_fail(nfs_plan_s* h, hipError_t e, const char* where) {
  return fail(h, NFS_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

// Sum pairs whose later frame is in [t_done, t_pushed).
nfs_status flush_pairs(nfs_plan_s* h) {
  if (h->t_done >= h->t_pushed) return NFS_OK;
  const nfs::Layout& L = h->L;
  for (const nfs::LagGroup& g : h->groups) {
    hipError_t e = nfs::launch_pairs(h->ring, L.spec_dtype, L.accum == NFS_ACC_KAHAN,
                                     h->refspec, h->fscale, L.slots, L.mode_stride,
                                     L.capacity, h->t_done,
                                     h->t_pushed, h->lags + g.first, g.count, g.max_lag,
                                     h->acc + g.first, L.n_lags, h->sums_fresh, g.modes,
                                     g.hist, g.waves, g.per_wave, g.lds, h->work + 1,
                                     h->comp ? h->comp + g.first : nullptr, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "pair kernel launch");
  }
  h->sums_fresh = false;
  h->t_done = h->t_pushed;
  return NFS_OK;
}

// Sums ready for reading: pending pairs summed, and zeros where no pair
// launch has run since the reset (no frames pushed).
nfs_status finish_sums(nfs_plan_s* h) {
  nfs_status st = flush_pairs(h);
  if (st != NFS_OK || !h->sums_fresh) return st;
  const nfs::Layout& L = h->L;
  hipError_t e = nfs::launch_fill_u32(h->acc, size_t(L.n_lags) * L.mode_stride, 0u, h->stream);
  if (e == hipSuccess && h->comp)
    e = nfs::launch_fill_u32(h->comp, size_t(L.n_lags) * L.mode_stride, 0u, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "fill kernel launch");
  h->sums_fresh = false;
  return NFS_OK;
}

nfs_status clear_sums(nfs_plan_s* h) {
  // The status word, the reference scalars (rewritten by the next push) and
  // the work counters: the first 80 bytes of the status block.
  hipError_t e = nfs::launch_fill_u32(h->status, 20, 0u, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "fill kernel launch");
  h->sums_fresh = true;
  h->t_pushed = 0;
  h->t_done = 0;
  return NFS_OK;
}

// Frames of the next transform batch out of `left` still to push: at most
// one batch, and no more than the ring can take beyond the largest lag.
int64_t next_batch(const nfs_plan_s* h, int64_t left) {
  const int64_t room = h->L.capacity - h->L.max_lag;  // >= 1 by construction
  int64_t b = left < h->L.batch ? left : h->L.batch;
  return b < room ? b : room;
}

// Sum the pending pairs if pushing `b` more frames would overwrite a
// spectrum one of them needs: frames [t_pushed, t_pushed + b) evict frames
// up to t_pushed + b - 1 - capacity, and pending pairs need the frames from
// max(0, t_done - max_lag) on.
nfs_status make_room(nfs_plan_s* h, int64_t b) {
  const nfs::Layout& L = h->L;
  const int64_t needed = h->t_done - L.max_lag > 0 ? h->t_done - L.max_lag : 0;
  if (h->t_pushed + b - L.capacity > needed) return flush_pairs(h);
  return NFS_OK;
}

// Normalise, transform and store `b` frames (device memory, b <= the batch
// size, after the reference frame is set) as frames [t, t + b), each in
// ring slot (its frame index) mod capacity.
nfs_status transform_into_ring(nfs_plan_s* h, const char* src, int64_t b, int64_t t) {
  const nfs::Layout& L = h->L;
  if (h->fused) {
    // Bounded waits: about 2^22 polls (seconds) before a stuck wait gives up
    // and reports NFS_E_TIMEOUT through the status word.
    constexpr unsigned kSpinLimit = 1u << 22;
    const int keep = h->fused_keep;
    float2* bufA = h->inter;
    float2* bufB = h->inter + size_t(8) * keep * L.n * 8;
    hipError_t e = nfs::launch_fill_u32(h->sched, size_t(8 * 64 + 16 * L.fused_slots), 0u,
                                        h->stream);
    if (e == hipSuccess)
      e = nfs::launch_fused_transform(L.n, L.in_dtype, L.spec_dtype, src, h->ref, h->window,
                                      int(b), h->rowsum, h->rowabs, bufA, bufB, keep, h->sched,
                                      L.fused_slots, h->fused_workers, kSpinLimit, h->refscal,
                                      h->fscale, h->status, t, L.capacity, L.mode_stride,
                                      L.slots, h->tiles, h->tw, h->ring, h->work, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "fused transform launch");
    return NFS_OK;
  }
  hipError_t e = nfs::launch_row_pass(L.n, L.in_dtype, src, h->ref, h->window, int(b),
                                      h->inter, h->rowsum, h->rowabs, h->nyq, h->tw, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "row pass launch");
  e = nfs::launch_col_pass(L.n, false, L.spec_dtype, h->inter, h->rowsum, h->rowabs, int(b), t,
                           L.capacity, L.mode_stride, L.slots, h->tiles, h->tw, h->ring,
                           h->refspec, h->refscal, h->fscale, h->status, h->work, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "column pass launch");
  if (L.full) {
    e = nfs::launch_nyquist_col(L.n, false, L.spec_dtype, h->nyq, int(b), t, L.capacity,
                                L.mode_stride, L.nyq_slot, h->tw, h->fscale, h->ring,
                                h->refspec, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "Nyquist column launch");
  }
  return NFS_OK;
}

// Normalise, transform and store `b` frames (device memory, b <= the batch
// size) as frames [t_pushed, t_pushed + b); make_room must precede it.
nfs_status transform_batch(nfs_plan_s* h, const char* src, int64_t b) {
  const nfs::Layout& L = h->L;
  hipError_t e = hipSuccess;
  if (h->t_pushed == 0) {
    // The first frame of the sequence becomes the reference subtracted
    // from every frame before its transform; differences of transforms
    // are unchanged, but the stored values no longer carry the static
    // image, whose low-q coefficients would swamp FP32.
    e = hipMemcpyAsync(h->ref, src, L.frame_bytes, hipMemcpyDeviceToDevice, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "reference copy");
    e = nfs::launch_row_pass(L.n, L.in_dtype, h->ref, nullptr, h->window, 1, h->inter,
                             h->rowsum, nullptr, h->nyq, h->tw, h->stream);
    if (e == hipSuccess)
      e = nfs::launch_col_pass(L.n, true, NFS_SPEC_F32, h->inter, h->rowsum, nullptr, 1, 0,
                               L.capacity, L.mode_stride, L.slots, h->tiles, h->tw,
                               h->ring, h->refspec, h->refscal, h->fscale, h->status,
                               nullptr, h->stream);
    if (e == hipSuccess && L.full)
      e = nfs::launch_nyquist_col(L.n, true, NFS_SPEC_F32, h->nyq, 1, 0, L.capacity,
                                  L.mode_stride, L.nyq_slot, h->tw, h->fscale, h->ring,
                                  h->refspec, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "reference transform launch");
  }
  nfs_status st = transform_into_ring(h, src, b, h->t_pushed);
  if (st != NFS_OK) return st;
  h->t_pushed += b;
  return NFS_OK;
}

}  // namespace

extern "C" {

const char* nfs_status_string(nfs_status s) {
  switch (s) {
    case NFS_OK: return "ok";
    case NFS_E_ARG: return "invalid argument";
    case NFS_E_SIZE: return "frame size must be a power of two in [16, 4096]";
    case NFS_E_LAGS: return "invalid lag list";
    case NFS_E_BINS: return "n_bins must be in [1, n/2]";
    case NFS_E_WORKSPACE: return "workspace missing, misaligned or too small";
    case NFS_E_CAPACITY: return "ring capacity must exceed the largest lag";
    case NFS_E_STATE: return "invalid handle or call order";
    case NFS_E_DEGENERATE_FRAME: return "a frame had a non-positive spatial sum";
    case NFS_E_HIP: return "HIP runtime error";
    case NFS_E_UNSUPPORTED: return "option not implemented";
    case NFS_E_SCRATCH:
      return "workspace larger than the library's static scratch (NFS_STATIC_SCRATCH_BYTES)";
    case NFS_E_TIMEOUT: return "a bounded device-side wait gave up; results are incomplete";
  }
  return "unknown status";
}

nfs_status nfs_plan_workspace_size(const nfs_desc* desc, size_t* bytes) {
  if (!bytes) return NFS_E_ARG;
  nfs::Layout L;
  std::string err;
  nfs_status st = nfs::make_layout(desc, 0, &L, &err);
  if (st != NFS_OK) return st;
  *bytes = L.total;
  return NFS_OK;
}

nfs_status nfs_plan(const nfs_desc* desc, void* workspace, size_t bytes, void* stream,
                    nfs_handle* out) {
  if (!out) return NFS_E_ARG;
  *out = nullptr;
  nfs_plan_s* h = new (std::nothrow) nfs_plan_s();
  if (!h) return NFS_E_ARG;
  std::string err;
  nfs_status st = nfs::make_layout(desc, bytes, &h->L, &err);
  if (st == NFS_OK && (!workspace || (reinterpret_cast<uintptr_t>(workspace) % nfs::kAlign)))
    st = NFS_E_WORKSPACE;
  if (st == NFS_OK && bytes < h->L.total) st = NFS_E_WORKSPACE;
  if (st != NFS_OK) {
    delete h;
    return st;
  }
  const nfs::Layout& L = h->L;
  h->groups = L.groups;
  h->stream = static_cast<hipStream_t>(stream);
  h->ws = static_cast<char*>(workspace);
  h->window = desc->window;
  h->ring = h->ws + L.off_ring;
  h->inter = reinterpret_cast<float2*>(h->ws + L.off_inter);
  h->rowsum = reinterpret_cast<double*>(h->ws + L.off_rowsum);
  h->rowabs = L.spec_dtype == NFS_SPEC_F16 ? reinterpret_cast<double*>(h->ws + L.off_rowabs)
                                            : nullptr;
  h->nyq = L.full ? reinterpret_cast<float*>(h->ws + L.off_nyq) : nullptr;
  if (L.fused_ok) {
    // The fused transform is switched off: its first GPU runs did not
    // finish (every wait of its task scheduler ran to its bound), and the
    // cause is not established. Every plan uses the separate row and column
    // passes; the kernel and its host plumbing stay for later work.
    h->fused = false;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
      cus = 256;
    h->fused_workers = std::min(nfs::kFusedMaxWorkers, 2 * cus);
    h->sched = reinterpret_cast<int*>(h->ws + L.off_sched);
  }
  h->acc = reinterpret_cast<float*>(h->ws + L.off_acc);
  h->comp = L.accum == NFS_ACC_KAHAN ? reinterpret_cast<float*>(h->ws + L.off_comp) : nullptr;
  h->status = reinterpret_cast<int32_t*>(h->ws + L.off_status);
  h->work = reinterpret_cast<unsigned long long*>(h->ws + L.off_status + 64);
  h->tw = reinterpret_cast<float2*>(h->ws + L.off_tw);
  h->width = reinterpret_cast<int32_t*>(h->ws + L.off_width);
  h->tiles = reinterpret_cast<int32_t*>(h->ws + L.off_tiles);
  h->lags = reinterpret_cast<int32_t*>(h->ws + L.off_lags);
  h->refscal = reinterpret_cast<double*>(h->ws + L.off_status + 8);
  h->ref = h->ws + L.off_ref;
  h->refspec = reinterpret_cast<float2*>(h->ws + L.off_refspec);
  h->fscale = reinterpret_cast<float4*>(h->ws + L.off_fscale);
  h->seg_first = reinterpret_cast<int32_t*>(h->ws + L.off_segs);
  h->bin_seg0 = h->seg_first + L.seg_first.size();
  h->bin_slots = reinterpret_cast<int32_t*>(h->ws + L.off_bin_slots);
  h->part = reinterpret_cast<double*>(h->ws + L.off_part);
  h->part_cnt = reinterpret_cast<long long*>(h->ws + L.off_part_cnt);
  if (L.backward) {
    h->gk = reinterpret_cast<float2*>(h->ws + L.off_gk);
    h->brow = reinterpret_cast<double2*>(h->ws + L.off_brow);
    h->bscal = reinterpret_cast<double2*>(h->ws + L.off_bscal);
    h->gw = reinterpret_cast<double*>(h->ws + L.off_gw);
    h->gtab = reinterpret_cast<float*>(h->ws + L.off_gtab);
    h->mode_bin = reinterpret_cast<int32_t*>(h->ws + L.off_mode_bin);
    h->bin_count = reinterpret_cast<int64_t*>(h->ws + L.off_bin_count);
  }
  if (L.host_staging) {
    h->stage[0] = h->ws + L.off_stage;
    h->stage[1] = h->stage[0] + size_t(L.batch) * L.frame_bytes;
  }

  const std::vector<float> tw = nfs::twiddle_table(L.n);
  hipError_t e = hipMemcpyAsync(h->tw, tw.data(), tw.size() * sizeof(float),
                                hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h->width, L.row_width.data(), L.row_width.size() * 4,
                       hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h->tiles, L.tiles.data(), L.tiles.size() * 4,
                       hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h->lags, L.lags.data(), L.lags.size() * 4, hipMemcpyHostToDevice,
                       h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h->seg_first, L.seg_first.data(), L.seg_first.size() * 4,
                       hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h->bin_slots, L.bin_slots.data(), L.bin_slots.size() * 4,
                       hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h->bin_seg0, L.bin_seg0.data(), L.bin_seg0.size() * 4,
                       hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess && L.backward)
    e = hipMemcpyAsync(h->mode_bin, L.mode_bin.data(), L.mode_bin.size() * 4,
                       hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess && L.backward)
    e = hipMemcpyAsync(h->bin_count, L.bin_count.data(), L.bin_count.size() * 8,
                       hipMemcpyHostToDevice, h->stream);
  // The pair kernel reads the reference transform in whole workgroup tiles
  // of modes, up to mode_stride; entries past the stored modes stay zero.
  if (e == hipSuccess)
    e = nfs::launch_fill_u32(h->refspec, size_t(L.mode_stride) * 2, 0u, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e == hipSuccess && L.host_staging) {
    // Default priority, like every stream of the library.
    e = hipStreamCreateWithFlags(&h->copy, hipStreamNonBlocking);
    for (int j = 0; j < 2 && e == hipSuccess; ++j) {
      e = hipEventCreateWithFlags(&h->copied[j], hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&h->freed[j], hipEventDisableTiming);
    }
  }
  if (e != hipSuccess) {
    delete h;
    return NFS_E_HIP;
  }
  st = clear_sums(h);
  if (st != NFS_OK) {
    delete h;
    return st;
  }
  {
    std::lock_guard<std::mutex> lk(g_mu);
    live().insert(h);
  }
  *out = h;
  return NFS_OK;
}

nfs_status nfs_push_frames(nfs_handle h, const void* frames, int64_t count) {
  if (!is_live(h)) return NFS_E_STATE;
  if (count < 0) return fail(h, NFS_E_ARG, "count must be >= 0");
  if (count == 0) return NFS_OK;
  if (!frames) return fail(h, NFS_E_ARG, "frames is NULL");
  int64_t i = 0;
  while (i < count) {
    const int64_t b = next_batch(h, count - i);
    nfs_status st = make_room(h, b);
    if (st == NFS_OK)
      st = transform_batch(h, static_cast<const char*>(frames) + size_t(i) * h->L.frame_bytes, b);
    if (st != NFS_OK) return st;
    i += b;
  }
  return NFS_OK;
}

nfs_status nfs_push_host_frames(nfs_handle h, const void* frames, int64_t count) {
  if (!is_live(h)) return NFS_E_STATE;
  if (!h->L.host_staging) return fail(h, NFS_E_STATE, "plan was created without host_staging");
  if (count < 0) return fail(h, NFS_E_ARG, "count must be >= 0");
  if (count == 0) return NFS_OK;
  if (!frames) return fail(h, NFS_E_ARG, "frames is NULL");
  const size_t fb = h->L.frame_bytes;
  int64_t i = 0;
  while (i < count) {
    const int64_t b = next_batch(h, count - i);
    const int j = h->next_stage;
    h->next_stage ^= 1;
    // Copy stream: wait until the transform that last read buffer j is
    // done, upload the batch, mark it. Plan stream: sum pending pairs if
    // needed (overlapping the upload), wait for the upload, transform,
    // mark buffer j free.
    hipError_t e = hipSuccess;
    if (h->freed_recorded[j]) e = hipStreamWaitEvent(h->copy, h->freed[j], 0);
    if (e == hipSuccess)
      e = hipMemcpyAsync(h->stage[j], static_cast<const char*>(frames) + size_t(i) * fb,
                         size_t(b) * fb, hipMemcpyHostToDevice, h->copy);
    if (e == hipSuccess) e = hipEventRecord(h->copied[j], h->copy);
    if (e != hipSuccess) return hip_fail(h, e, "host frame upload");
    nfs_status st = make_room(h, b);
    if (st != NFS_OK) return st;
    e = hipStreamWaitEvent(h->stream, h->copied[j], 0);
    if (e != hipSuccess) return hip_fail(h, e, "host frame upload");
    st = transform_batch(h, h->stage[j], b);
    if (st != NFS_OK) return st;
    e = hipEventRecord(h->freed[j], h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "staging event");
    h->freed_recorded[j] = true;
    i += b;
  }
  return NFS_OK;
}

nfs_status nfs_tune_pairs(nfs_handle h, int32_t* choices, int32_t* groups) {
  if (!is_live(h)) return NFS_E_STATE;
  const nfs::Layout& L = h->L;
  if (h->t_pushed < 2) return fail(h, NFS_E_STATE, "tuning needs at least 2 pushed frames");
  // Target window [T0, T1): every pushed frame when the ring still holds
  // them all (the window a pair flush of the whole stack covers), else the
  // frames whose partners are all still in the ring.
  const int64_t T1 = h->t_pushed;
  const int64_t T0 = T1 <= L.capacity ? 0 : T1 - (L.capacity - L.max_lag);
  // Scratch sums in the row-pass intermediate (dead between pushes): the
  // first slots that fit, in whole workgroup tiles.
  const int64_t inter_bytes = int64_t(L.batch) * L.n * L.h * 8;
  int64_t slots = inter_bytes / (int64_t(L.n_lags) * 4);
  if (slots > L.slots) slots = L.slots;
  slots = slots / 16 * 16;
  if (slots < 16) return fail(h, NFS_E_STATE, "no scratch room for tuning");
  float* scratch = reinterpret_cast<float*>(h->inter);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  for (size_t gi = 0; e == hipSuccess && gi < h->groups.size(); ++gi) {
    const nfs::LagGroup cur = h->groups[gi];
    if (cur.modes == 0) continue;  // long delays: one kernel shape only
    float best_ms = 0.f;
    nfs::LagGroup best = cur;
    for (const nfs::LagGroup& c : nfs::group_candidates(L.lags, cur.first, cur.count)) {
      auto go = [&]() {
        return nfs::launch_pairs(h->ring, L.spec_dtype, L.accum == NFS_ACC_KAHAN, h->refspec,
                                 h->fscale, slots, L.mode_stride, L.capacity, T0, T1,
                                 h->lags + c.first, c.count, c.max_lag, scratch + c.first,
                                 L.n_lags, true, c.modes, c.hist, c.waves, c.per_wave, c.lds,
                                 nullptr, nullptr, h->stream);
      };
      e = go();  // warm-up
      if (e == hipSuccess) e = hipEventRecord(e0, h->stream);
      if (e == hipSuccess) e = go();
      if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) break;
      if (best_ms == 0.f || ms < best_ms) {
        best_ms = ms;
        best = c;
      }
    }
    if (e == hipSuccess) h->groups[gi] = best;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(h, e, "pair tuning");
  if (groups) *groups = int32_t(h->groups.size());
  if (choices)
    for (size_t gi = 0; gi < h->groups.size(); ++gi) {
      choices[2 * gi] = h->groups[gi].modes;
      choices[2 * gi + 1] = h->groups[gi].waves;
    }
  return NFS_OK;
}

nfs_status nfs_set_pair_shapes(nfs_handle h, const int32_t* choices, int32_t groups) {
  if (!is_live(h)) return NFS_E_STATE;
  if (!choices) return fail(h, NFS_E_ARG, "choices is NULL");
  if (groups != int32_t(h->groups.size()))
    return fail(h, NFS_E_ARG, "group count differs from the plan's");
  const nfs::Layout& L = h->L;
  std::vector<nfs::LagGroup> next = h->groups;
  for (size_t gi = 0; gi < next.size(); ++gi) {
    const int modes = choices[2 * gi], waves = choices[2 * gi + 1];
    const nfs::LagGroup& cur = h->groups[gi];
    if (cur.modes == 0) {
      if (modes != 0 || waves != 0)
        return fail(h, NFS_E_ARG, "a long-delay group has one kernel shape (0, 0)");
      continue;
    }
    bool found = false;
    for (const nfs::LagGroup& c : nfs::group_candidates(L.lags, cur.first, cur.count))
      if (c.modes == modes && c.waves == waves) {
        next[gi] = c;
        found = true;
        break;
      }
    if (!found) return fail(h, NFS_E_ARG, "shape not supported for this lag group");
  }
  h->groups = next;
  return NFS_OK;
}

nfs_status nfs_accumulate(nfs_handle h) {
  if (!is_live(h)) return NFS_E_STATE;
  return flush_pairs(h);
}

nfs_status nfs_structure_function(nfs_handle h, double* D, int64_t* bin_counts,
                                  int64_t* lag_pairs, int32_t* status) {
  if (!is_live(h)) return NFS_E_STATE;
  if (!D) return fail(h, NFS_E_ARG, "D is NULL");
  nfs_status st = finish_sums(h);
  if (st != NFS_OK) return st;
  const nfs::Layout& L = h->L;
  hipError_t e = nfs::launch_bins(L.n_bins, h->acc, L.n_lags, h->bin_slots, h->seg_first,
                                  int(L.seg_first.size() - 1), h->bin_seg0, h->part,
                                  h->part_cnt, h->lags, h->t_pushed, h->status, D, bin_counts,
                                  lag_pairs, status, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "bin kernel launch");
  return NFS_OK;
}

nfs_status nfs_power_spectra_2d(nfs_handle h, float* S) {
  if (!is_live(h)) return NFS_E_STATE;
  if (!S) return fail(h, NFS_E_ARG, "S is NULL");
  nfs_status st = finish_sums(h);
  if (st != NFS_OK) return st;
  const nfs::Layout& L = h->L;
  hipError_t e = nfs::launch_power_spectra(L.n, L.n_lags, h->acc, h->width, h->tiles,
                                           L.full ? L.nyq_slot : -1, h->lags,
                                           h->t_pushed, S, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "power spectra launch");
  return NFS_OK;
}

nfs_status nfs_backward(nfs_handle h, const double* dL_dD, const void* frames,
                        float* dL_dframes, float* dL_dwindow) {
  if (!is_live(h)) return NFS_E_STATE;
  const nfs::Layout& L = h->L;
  if (!L.backward) return fail(h, NFS_E_STATE, "plan was created without backward");
  if (!dL_dD) return fail(h, NFS_E_ARG, "dL_dD is NULL");
  if (!frames) return fail(h, NFS_E_ARG, "frames is NULL");
  const int64_t N = h->t_pushed;
  if (N < 1) return fail(h, NFS_E_STATE, "no frame pushed");
  // When the ring no longer holds every frame, the spectra are recomputed
  // from `frames` by the forward passes, window by window: targets
  // [t0, t0 + b) need frames [t0 - max_lag, t0 + b + max_lag), so b is at
  // most capacity - 2 max_lag, and each frame is transformed once more.
  // The last window leaves frames [N - capacity, N) in their slots, as the
  // pushes did, so later pushes and pair sums see the same ring.
  const bool recompute = N > L.capacity;
  int64_t bb = L.batch;
  if (recompute) {
    const int64_t room = L.capacity - 2 * int64_t(L.max_lag);
    if (room < 1)
      return fail(h, NFS_E_CAPACITY,
                  "recomputing spectra for the gradient needs capacity > 2 x the largest lag");
    if (room < bb) bb = room;
  }
  const int64_t px = int64_t(L.n) * L.n;
  hipError_t e = nfs::launch_grad_table(L.n_lags, L.n_bins, dL_dD, h->bin_count, h->lags, N,
                                        h->gtab, h->stream);
  if (e == hipSuccess && dL_dwindow) e = nfs::launch_fill_u32(h->gw, size_t(px) * 2, 0u, h->stream);
  int64_t have = 0;  // frames [0, have) recomputed by this call
  for (int64_t t0 = 0; e == hipSuccess && t0 < N; t0 += bb) {
    const int b = int(N - t0 < bb ? N - t0 : bb);
    const char* fr = static_cast<const char*>(frames) + size_t(t0) * L.frame_bytes;
    if (recompute) {
      const int64_t need = t0 + b + L.max_lag < N ? t0 + b + L.max_lag : N;
      while (have < need) {
        const int64_t c = need - have < L.batch ? need - have : L.batch;
        nfs_status st = transform_into_ring(
            h, static_cast<const char*>(frames) + size_t(have) * L.frame_bytes, c, have);
        if (st != NFS_OK) return st;
        have += c;
      }
    }
    const int64_t tw0 = t0 - L.max_lag > 0 ? t0 - L.max_lag : 0;
    e = nfs::launch_grad_spectra(h->ring, L.spec_dtype, h->fscale, h->refspec, L.capacity,
                                 L.mode_stride, L.slots, h->mode_bin, h->gtab, h->lags,
                                 L.n_lags, L.n_bins, L.max_lag, N, t0, b, tw0,
                                 tw0 % L.capacity, h->gk, h->stream);
    if (e == hipSuccess)
      e = nfs::launch_inverse_2d(L.n, L.in_dtype, h->gk, L.mode_stride, h->width, h->tiles,
                                 h->tw, b, h->inter, reinterpret_cast<float*>(h->gk), fr,
                                 h->window, h->brow, h->stream);
    if (e == hipSuccess)
      e = nfs::launch_grad_finish(L.n, L.in_dtype, b, h->brow, h->bscal,
                                  reinterpret_cast<const float*>(h->gk), fr, h->window,
                                  dL_dframes ? dL_dframes + size_t(t0) * px : nullptr,
                                  dL_dwindow ? h->gw : nullptr, h->stream);
  }
  if (e == hipSuccess && dL_dwindow) e = nfs::launch_window_out(L.n, h->gw, dL_dwindow, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "backward launch");
  return NFS_OK;
}

nfs_status nfs_structure_function_noalloc(const nfs_desc* desc, const void* frames,
                                          int64_t count, double* D, int64_t* bin_counts,
                                          int64_t* lag_pairs, int32_t* status, void* stream) {
  if (!desc || !D || count < 0 || (count > 0 && !frames)) return NFS_E_ARG;
  if (desc->host_staging || desc->backward) return NFS_E_ARG;
  // Size check on the host, before anything touches the device: the layout
  // the plan below will take (capacity 0 = derived from the array's size).
  nfs::Layout L;
  std::string err;
  nfs_status st = nfs::make_layout(desc, NFS_STATIC_SCRATCH_BYTES, &L, &err);
  if (st == NFS_E_WORKSPACE) return NFS_E_SCRATCH;
  if (st != NFS_OK) return st;
  if (L.total > NFS_STATIC_SCRATCH_BYTES) return NFS_E_SCRATCH;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return NFS_E_HIP;
  if (stream) {
    int sdev = -1;
    if (hipStreamGetDevice(static_cast<hipStream_t>(stream), &sdev) != hipSuccess)
      return NFS_E_HIP;
    if (sdev != dev) return NFS_E_ARG;
  }
  void* ws = nullptr;
  if (nfs::static_scratch(dev, &ws) != hipSuccess) return NFS_E_HIP;
  nfs_handle h = nullptr;
  st = nfs_plan(desc, ws, NFS_STATIC_SCRATCH_BYTES, stream, &h);
  if (st != NFS_OK) return st;
  st = nfs_push_frames(h, frames, count);
  if (st == NFS_OK) st = nfs_structure_function(h, D, bin_counts, lag_pairs, status);
  // The enqueued kernels take their arguments by value and the plan owns
  // no stream or event, so the handle can go before the stream passes.
  nfs_status st_destroy = nfs_destroy(h);
  return st != NFS_OK ? st : st_destroy;
}

nfs_status nfs_work_counters(nfs_handle h, int64_t* counters) {
  if (!is_live(h)) return NFS_E_STATE;
  if (!counters) return fail(h, NFS_E_ARG, "counters is NULL");
  hipError_t e = hipMemcpyAsync(counters, h->work, 2 * sizeof(int64_t),
                                hipMemcpyDeviceToDevice, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "work counter copy");
  return NFS_OK;
}

nfs_status nfs_reset(nfs_handle h) {
  if (!is_live(h)) return NFS_E_STATE;
  return clear_sums(h);
}

nfs_status nfs_destroy(nfs_handle h) {
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!live().erase(h)) return NFS_E_STATE;
  }
  delete h;
  return NFS_OK;
}

const char* nfs_last_error(nfs_handle h) {
  if (!is_live(h)) return "invalid handle";
  return h->err.c_str();
}

nfs_status nfs_mode_count(nfs_handle h, int64_t* modes) {
  if (!is_live(h)) return NFS_E_STATE;
  if (!modes) return fail(h, NFS_E_ARG, "modes is NULL");
  *modes = h->L.modes;
  return NFS_OK;
}

nfs_status nfs_bin_map(nfs_handle h, int32_t* map) {
  if (!is_live(h)) return NFS_E_STATE;
  if (!map) return fail(h, NFS_E_ARG, "map is NULL");
  hipError_t e = nfs::launch_bin_map(h->L.n, h->L.n_bins, map, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "bin map launch");
  return NFS_OK;
}

nfs_status nfs_probe_bandwidth(int32_t mode, const void* src, void* dst, size_t bytes,
                               void* stream) {
  if (mode < 0 || mode > 2 || bytes == 0 || bytes % 16 != 0) return NFS_E_ARG;
  if ((mode != 2 && !src) || !dst) return NFS_E_ARG;
  if ((mode != 2 && reinterpret_cast<uintptr_t>(src) % 16) ||
      reinterpret_cast<uintptr_t>(dst) % 16)
    return NFS_E_ARG;
  hipError_t e = nfs::launch_probe(mode, src, dst, bytes, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? NFS_OK : NFS_E_HIP;
}

nfs_status nfs_copy_spectrum(nfs_handle h, int64_t t, float* out) {
  if (!is_live(h)) return NFS_E_STATE;
  if (!out) return fail(h, NFS_E_ARG, "out is NULL");
  if (t < 0 || t >= h->t_pushed || t < h->t_pushed - h->L.capacity)
    return fail(h, NFS_E_STATE, "frame is not in the ring");
  hipError_t e = nfs::launch_expand_spectrum(h->L.n, h->ring, h->L.spec_dtype,
                                             t % h->L.capacity, h->L.mode_stride, h->width,
                                             h->tiles, h->refspec, h->fscale,
                                             reinterpret_cast<float2*>(out), h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "expand launch");
  return NFS_OK;
}

}  // extern "C"
