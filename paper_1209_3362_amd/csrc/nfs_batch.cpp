// Batching form: many image sequences of uneven frame size and length
// analysed together on one GPU.
//
// Each sequence gets its own plan (the per-sequence memory plan of the
// processing section), all carved from one caller-owned workspace. A run
// forks from the caller's stream onto a few worker streams, each sequence
// on the stream with the least work so far (most work first), and joins
// back, so small sequences fill the GPU beside large ones; the whole fork /
// join run can be captured once into a HIP graph and replayed. When the
// spectra of every sequence do not fit a memory budget, rings are shortened
// to time windows (pair sums are then flushed per window).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>
#include <new>
#include <numeric>
#include <set>
#include <string>
#include <vector>

#include "nfs.h"
#include "nfs_host.hpp"

struct nfs_batch_s {
  std::vector<nfs_handle> plans;
  std::vector<hipStream_t> streams;  // worker streams (default priority)
  std::vector<int> order;            // sequences, most work first
  std::vector<int> stream_of;        // worker stream of each sequence
  hipStream_t caller = nullptr;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;

  ~nfs_batch_s() {
    // Let enqueued work finish before its plans and streams go away.
    for (hipStream_t s : streams) (void)hipStreamSynchronize(s);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (nfs_handle p : plans)
      if (p) (void)nfs_destroy(p);
    for (hipStream_t s : streams) (void)hipStreamDestroy(s);
    if (fork) (void)hipEventDestroy(fork);
    for (hipEvent_t e : join)
      if (e) (void)hipEventDestroy(e);
  }
};

namespace {

std::mutex g_bmu;
std::set<nfs_batch_s*>& live_batches() {
  static std::set<nfs_batch_s*> s;
  return s;
}
bool batch_live(nfs_batch_s* b) {
  std::lock_guard<std::mutex> lk(g_bmu);
  return live_batches().count(b) != 0;
}

constexpr int kMaxStreams = 8;

size_t aligned(size_t v) { return nfs::align_up(v, nfs::kAlign); }

// Work of one sequence of `frames` frames: pair terms (the arithmetic of
// the pair kernel) plus pixels transformed, in rough pair-term units.
double sequence_work(const nfs::Layout& L, int64_t frames) {
  double pairs = 0.0;
  for (int32_t t : L.lags) pairs += double(std::max<int64_t>(0, frames - t));
  return pairs * double(L.modes) + 8.0 * double(frames) * L.n * L.n;
}

}  // namespace

extern "C" {

nfs_status nfs_batch_workspace_size(const nfs_desc* descs, int32_t n_seq, size_t* sizes,
                                    size_t* total) {
  if (!descs || n_seq < 1 || !total) return NFS_E_ARG;
  size_t sum = 0;
  for (int32_t j = 0; j < n_seq; ++j) {
    size_t b = 0;
    nfs_status st = nfs_plan_workspace_size(&descs[j], &b);
    if (st != NFS_OK) return st;
    if (sizes) sizes[j] = b;
    sum += aligned(b);
  }
  *total = sum;
  return NFS_OK;
}

nfs_status nfs_batch_capacities(const nfs_desc* descs, const int64_t* frames, int32_t n_seq,
                                size_t budget, int64_t* capacities) {
  if (!descs || !frames || n_seq < 1 || !capacities) return NFS_E_ARG;
  std::vector<int64_t> lo(n_seq), full(n_seq);
  std::string err;
  for (int32_t j = 0; j < n_seq; ++j) {
    if (frames[j] < 1) return NFS_E_ARG;
    nfs_desc d = descs[j];
    d.capacity = 0;
    nfs::Layout L;
    nfs_status st = nfs::make_layout(&d, 0, &L, &err);
    if (st != NFS_OK) return st;
    full[j] = std::max<int64_t>(frames[j], int64_t(L.max_lag) + 1);
    // A window of at least 64 frames (or the whole stack) beyond the lags.
    lo[j] = std::min<int64_t>(full[j], int64_t(L.max_lag) + 64);
  }
  // Workspace of every plan when each ring takes the share s of the frames
  // between its minimal window and its whole stack (exact sizes: a ring's
  // capacity also bounds its transform batch).
  auto caps_at = [&](double s, std::vector<int64_t>* caps) {
    for (int32_t j = 0; j < n_seq; ++j)
      (*caps)[j] = lo[j] + int64_t(double(full[j] - lo[j]) * s);
  };
  auto total_at = [&](const std::vector<int64_t>& caps, size_t* total) {
    size_t sum = 0;
    for (int32_t j = 0; j < n_seq; ++j) {
      nfs_desc d = descs[j];
      d.capacity = caps[j];
      size_t b = 0;
      nfs_status st = nfs_plan_workspace_size(&d, &b);
      if (st != NFS_OK) return st;
      sum += aligned(b);
    }
    *total = sum;
    return NFS_OK;
  };
  std::vector<int64_t> caps(n_seq);
  size_t total = 0;
  caps_at(1.0, &caps);
  nfs_status st = total_at(caps, &total);
  if (st != NFS_OK) return st;
  if (total > budget) {
    caps_at(0.0, &caps);
    if ((st = total_at(caps, &total)) != NFS_OK) return st;
    if (total > budget) return NFS_E_WORKSPACE;
    // The total grows with s: bisect for the largest share that fits.
    double good = 0.0, bad = 1.0;
    std::vector<int64_t> trial(n_seq);
    for (int it = 0; it < 40; ++it) {
      const double mid = 0.5 * (good + bad);
      caps_at(mid, &trial);
      if ((st = total_at(trial, &total)) != NFS_OK) return st;
      if (total <= budget) {
        good = mid;
        caps = trial;
      } else {
        bad = mid;
      }
    }
  }
  for (int32_t j = 0; j < n_seq; ++j) capacities[j] = caps[j];
  return NFS_OK;
}

nfs_status nfs_batch_create(const nfs_desc* descs, int32_t n_seq, int32_t n_streams,
                            void* workspace, size_t bytes, void* stream, nfs_batch_handle* out) {
  if (!out) return NFS_E_ARG;
  *out = nullptr;
  if (!descs || n_seq < 1 || n_streams < 1 || n_streams > kMaxStreams) return NFS_E_ARG;
  if (!workspace || reinterpret_cast<uintptr_t>(workspace) % nfs::kAlign)
    return NFS_E_WORKSPACE;
  std::vector<size_t> sizes(n_seq);
  size_t total = 0;
  nfs_status st = nfs_batch_workspace_size(descs, n_seq, sizes.data(), &total);
  if (st != NFS_OK) return st;
  if (bytes < total) return NFS_E_WORKSPACE;
  nfs_batch_s* b = new (std::nothrow) nfs_batch_s();
  if (!b) return NFS_E_ARG;
  b->caller = static_cast<hipStream_t>(stream);
  const int W = std::min<int32_t>(n_streams, n_seq);
  hipError_t e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
  for (int w = 0; w < W && e == hipSuccess; ++w) {
    hipStream_t s = nullptr;
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) b->streams.push_back(s);
    hipEvent_t ev = nullptr;
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) b->join.push_back(ev);
  }
  if (e != hipSuccess) {
    delete b;
    return NFS_E_HIP;
  }
  // Longest processing time first: most work to the least loaded stream.
  std::vector<double> work(n_seq);
  std::string err;
  for (int32_t j = 0; j < n_seq; ++j) {
    nfs::Layout L;
    st = nfs::make_layout(&descs[j], 0, &L, &err);
    if (st != NFS_OK) {
      delete b;
      return st;
    }
    work[j] = sequence_work(L, descs[j].capacity > 0 ? descs[j].capacity : L.max_lag + 1);
  }
  b->order.resize(n_seq);
  std::iota(b->order.begin(), b->order.end(), 0);
  std::stable_sort(b->order.begin(), b->order.end(),
                   [&](int x, int y) { return work[x] > work[y]; });
  b->stream_of.assign(n_seq, 0);
  std::vector<double> load(W, 0.0);
  for (int j : b->order) {
    const int w = int(std::min_element(load.begin(), load.end()) - load.begin());
    b->stream_of[j] = w;
    load[w] += work[j];
  }
  char* ws = static_cast<char*>(workspace);
  b->plans.assign(n_seq, nullptr);
  for (int32_t j = 0; j < n_seq; ++j) {
    st = nfs_plan(&descs[j], ws, sizes[j], b->streams[b->stream_of[j]], &b->plans[j]);
    if (st != NFS_OK) {
      delete b;
      return st;
    }
    ws += aligned(sizes[j]);
  }
  {
    std::lock_guard<std::mutex> lk(g_bmu);
    live_batches().insert(b);
  }
  *out = b;
  return NFS_OK;
}

nfs_status nfs_batch_plan(nfs_batch_handle b, int32_t j, nfs_handle* plan) {
  if (!batch_live(b)) return NFS_E_STATE;
  if (!plan || j < 0 || j >= int32_t(b->plans.size())) return NFS_E_ARG;
  *plan = b->plans[j];
  return NFS_OK;
}

}  // extern "C"

namespace {

// Enqueue one run: fork onto the worker streams, every sequence's reset,
// push and structure function on its stream, join back to the caller.
nfs_status enqueue_run(nfs_batch_s* b, const void* const* frames, const int64_t* counts,
                       double* const* D, int64_t* const* bin_counts, int64_t* const* lag_pairs,
                       int32_t* const* status) {
  hipError_t e = hipEventRecord(b->fork, b->caller);
  for (size_t w = 0; w < b->streams.size() && e == hipSuccess; ++w)
    e = hipStreamWaitEvent(b->streams[w], b->fork, 0);
  if (e != hipSuccess) return NFS_E_HIP;
  for (int j : b->order) {
    nfs_handle p = b->plans[j];
    nfs_status st = nfs_reset(p);
    if (st == NFS_OK) st = nfs_push_frames(p, frames[j], counts[j]);
    if (st == NFS_OK)
      st = nfs_structure_function(p, D[j], bin_counts ? bin_counts[j] : nullptr,
                                  lag_pairs ? lag_pairs[j] : nullptr,
                                  status ? status[j] : nullptr);
    if (st != NFS_OK) return st;
  }
  for (size_t w = 0; w < b->streams.size() && e == hipSuccess; ++w) {
    e = hipEventRecord(b->join[w], b->streams[w]);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->caller, b->join[w], 0);
  }
  return e == hipSuccess ? NFS_OK : NFS_E_HIP;
}

nfs_status check_run_args(nfs_batch_s* b, const void* const* frames, const int64_t* counts,
                          double* const* D) {
  if (!frames || !counts || !D) return NFS_E_ARG;
  for (size_t j = 0; j < b->plans.size(); ++j)
    if (!frames[j] || !D[j] || counts[j] < 1) return NFS_E_ARG;
  return NFS_OK;
}

}  // namespace

extern "C" {

nfs_status nfs_batch_run(nfs_batch_handle b, const void* const* frames, const int64_t* counts,
                         double* const* D, int64_t* const* bin_counts,
                         int64_t* const* lag_pairs, int32_t* const* status) {
  if (!batch_live(b)) return NFS_E_STATE;
  nfs_status st = check_run_args(b, frames, counts, D);
  if (st != NFS_OK) return st;
  return enqueue_run(b, frames, counts, D, bin_counts, lag_pairs, status);
}

nfs_status nfs_batch_capture(nfs_batch_handle b, const void* const* frames,
                             const int64_t* counts, double* const* D,
                             int64_t* const* bin_counts, int64_t* const* lag_pairs,
                             int32_t* const* status) {
  if (!batch_live(b)) return NFS_E_STATE;
  nfs_status st = check_run_args(b, frames, counts, D);
  if (st != NFS_OK) return st;
  if (!b->caller) return NFS_E_STATE;  // the legacy default stream cannot be captured
  if (b->exec) {
    (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  if (b->graph) {
    (void)hipGraphDestroy(b->graph);
    b->graph = nullptr;
  }
  hipError_t e = hipStreamBeginCapture(b->caller, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) return NFS_E_HIP;
  st = enqueue_run(b, frames, counts, D, bin_counts, lag_pairs, status);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(b->caller, &g);
  if (st != NFS_OK || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return st != NFS_OK ? st : NFS_E_HIP;
  }
  b->graph = g;
  e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
  return e == hipSuccess ? NFS_OK : NFS_E_HIP;
}

nfs_status nfs_batch_replay(nfs_batch_handle b) {
  if (!batch_live(b)) return NFS_E_STATE;
  if (!b->exec) return NFS_E_STATE;
  return hipGraphLaunch(b->exec, b->caller) == hipSuccess ? NFS_OK : NFS_E_HIP;
}

nfs_status nfs_batch_destroy(nfs_batch_handle b) {
  {
    std::lock_guard<std::mutex> lk(g_bmu);
    if (!live_batches().erase(b)) return NFS_E_STATE;
  }
  delete b;
  return NFS_OK;
}

}  // extern "C"
