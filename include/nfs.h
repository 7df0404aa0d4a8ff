/*
 * nfs.h -- C ABI of the MI355X (gfx950) structure-function library.
 *
 * The library computes the structure function of Eq. (1) of Cerchiari,
 * Croccolo, Cardinaux and Scheffold, "Quasi-real-time analysis of dynamic
 * near field scattering data using a graphics processing unit":
 *
 *   D(q, tau) = < |Delta I_m(q, tau)|^2 >,
 *
 * where Delta I_m is the spatial Fourier transform of the difference of two
 * mean-normalised images taken tau frames apart, the average runs over all
 * pairs of frames tau apart (ensemble average taken over time, text after
 * Eq. 1) and the result is averaged azimuthally over rings of |q| (Fig. 1e-f).
 * As in the processing section of the paper, every image is transformed once
 * and only differences of transforms are formed (linearity of the Fourier
 * transform), normalisation divides each transform by its zero-frequency
 * value, and the per-delay averages are accumulated as the images arrive.
 *
 * Conventions (the paper leaves these open):
 *   - forward transform kernel exp(-2*pi*i*k.x/n), unnormalised, applied to
 *     the mean-normalised image, so I(0) = n^2; the library sets I(0) = n^2
 *     exactly in every stored spectrum;
 *   - bins are half-open rings of width pi/n_bins in q = 2*pi*|k|/n,
 *     b(k) = isqrt(|k|^2 * n_bins^2) / (n/2); modes with |k| >= n/2 belong to
 *     no bin;
 *   - D(b, tau) = sum over modes k of bin b of P_tau(k), divided by C_b, the
 *     number of full-plane modes in bin b, with
 *     P_tau(k) = 1/(N - tau) * sum_{t=0}^{N-1-tau} |I_t(k) - I_{t+tau}(k)|^2.
 *
 * Memory: the caller allocates one device workspace (nfs_plan_workspace_size)
 * and every output; the library never allocates or frees device memory.
 * Streams: every call that touches the device only enqueues work on the
 * plan's stream and returns; results are valid once that stream has passed
 * the work. One host thread may use a handle at a time.
 * Errors: every entry point returns an nfs_status; nothing is thrown across
 * the ABI. Argument and state errors are detected on the host before any
 * work is enqueued, and nfs_last_error() then describes them.
 */
#ifndef NFS_H
#define NFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nfs_plan_s* nfs_handle;

typedef enum {
  NFS_OK = 0,
  NFS_E_ARG = 1,              /* null pointer or invalid enum value          */
  NFS_E_SIZE = 2,             /* n not a power of two in [16, 4096]          */
  NFS_E_LAGS = 3,             /* lags empty, negative, unsorted or
                                 duplicated                                  */
  NFS_E_BINS = 4,             /* n_bins outside [1, n/2]                     */
  NFS_E_WORKSPACE = 5,        /* workspace null, misaligned or too small     */
  NFS_E_CAPACITY = 6,         /* ring capacity negative, not larger than the
                                 max lag, or 2^31 or more                    */
  NFS_E_STATE = 7,            /* handle destroyed or used out of order       */
  NFS_E_DEGENERATE_FRAME = 8, /* a frame had a non-positive spatial sum      */
  NFS_E_HIP = 9,              /* a HIP runtime call failed                   */
  NFS_E_UNSUPPORTED = 10,     /* option value not implemented                */
  NFS_E_SCRATCH = 11,         /* problem larger than the static scratch of
                                 nfs_structure_function_noalloc             */
  NFS_E_TIMEOUT = 12          /* a bounded device-side wait of the fused
                                 transform gave up (reported through the
                                 status output); results are incomplete     */
} nfs_status;

/* Pixel type of the frames passed to nfs_push_frames. */
enum { NFS_IN_U16 = 0, NFS_IN_F32 = 1 };
/* Storage type of the resident spectra. Each stored value is
 * sigma_t F[u_t - u_ref] (the frame's transform minus the scaled transform of
 * the first frame of the sequence, fluctuation-sized); the pair kernel adds
 * (sigma_t - sigma_ref) F[u_ref] back in FP32, so differences are those of
 * the normalised transforms.
 *   NFS_SPEC_F32:  FP32 real and imaginary parts, 8 bytes per mode;
 *   NFS_SPEC_BF16: each part rounded to BF16 (nearest, ties to even),
 *                  4 bytes per mode;
 *   NFS_SPEC_F16:  each part multiplied by 2^e_t and rounded to FP16, with
 *                  e_t the largest integer for which
 *                  2^e_t * sigma_t * sum_x |u_t(x) - u_ref(x)| <= 65504 (no
 *                  overflow), 4 bytes per mode.
 * Differences, squares and sums are FP32 in every case (precision form). */
enum { NFS_SPEC_F32 = 0, NFS_SPEC_BF16 = 1, NFS_SPEC_F16 = 2 };
/* Per-mode pair accumulation.
 *   NFS_ACC_PLAIN: FP32 running sums;
 *   NFS_ACC_KAHAN: FP32 sums over each chunk of 32 target frames, added to
 *                  the running sum with Kahan compensation; when a ring
 *                  holds fewer frames than were pushed, each window's totals
 *                  are added to the stored sums with the compensation kept
 *                  per (mode, delay) in the workspace, so it holds over the
 *                  whole average. */
enum { NFS_ACC_PLAIN = 0, NFS_ACC_KAHAN = 1 };

typedef struct {
  int32_t n;            /* frame side; frames are n x n, row-major; power of
                           two in [16, 4096] (the paper processed 32x32 up to
                           4k x 4k images, processing section)                */
  int32_t in_dtype;     /* NFS_IN_U16 or NFS_IN_F32                           */
  int32_t spec_dtype;   /* NFS_SPEC_F32, NFS_SPEC_BF16 or NFS_SPEC_F16        */
  int32_t accum;        /* NFS_ACC_PLAIN or NFS_ACC_KAHAN                     */
  int32_t n_lags;       /* number of delays, >= 1                             */
  const int32_t* lags;  /* host array of n_lags delays in frames, strictly
                           increasing, lags[0] >= 0; copied by nfs_plan. The
                           paper evaluates all N-1 delays and suggests
                           log-spaced ones (discussion section)              */
  int32_t n_bins;       /* number of |q| rings, 1 .. n/2                      */
  int64_t capacity;     /* spectra kept resident (ring slots); must exceed the
                           largest lag and be below 2^31; 0 = as many as the
                           workspace holds (at most 2^31 - 1)                 */
  const float* window;  /* device [n][n] per-pixel weight multiplied into
                           every frame before normalisation, or NULL;
                           borrowed: must stay valid while the plan is used   */
  int32_t host_staging; /* 0, or 1 to accept frames from host memory with
                           nfs_push_host_frames: the workspace then also holds
                           two device staging buffers of one transform batch
                           each, and the plan owns a second (copy) stream    */
  int32_t backward;     /* 0, or 1 to reserve what nfs_backward needs: one
                           batch of k-space gradients, per-row sums, an FP64
                           window-gradient accumulator and per-mode bin
                           tables                                            */
  int32_t full_spectra; /* 0: store and pair only the modes that land in a
                           ring (k_x < n/2, |k| < n/2), enough for D; 1: also
                           the rest of the half plane (the corners |k| >= n/2
                           and the k_x = n/2 column), so nfs_power_spectra_2d
                           returns the entire 2D spectra (discussion section).
                           D is the same either way; 1 costs about 27 % more
                           ring memory, transform stores and pair work        */
} nfs_desc;

/* Bytes of device workspace nfs_plan needs for `desc`. Host only; enqueues
 * nothing. With desc->capacity == 0 the size for a ring of (largest lag + 64)
 * spectra is returned. Memory plan made before any frame is processed, as in
 * the processing section. */
nfs_status nfs_plan_workspace_size(const nfs_desc* desc, size_t* bytes);

/* Create a plan. `workspace` is a device buffer of `bytes` bytes, 256-byte
 * aligned, owned by the caller, that must outlive the handle. `stream` is a
 * hipStream_t (NULL = the default stream) on which all work is enqueued.
 * Initialises the workspace (enqueued) and returns the handle in *out.
 * Synchronises `stream` once, to finish the upload of the plan's tables. */
nfs_status nfs_plan(const nfs_desc* desc, void* workspace, size_t bytes,
                    void* stream, nfs_handle* out);

/* Append `count` frames to the sequence: device array [count][n][n] of the
 * plan's pixel type, borrowed until the stream passes the enqueued work.
 * Each frame is normalised, transformed once and stored in the ring (the
 * per-image transforms of the processing section); pair sums are
 * accumulated whenever the ring would otherwise overwrite a spectrum that a
 * later pair still needs. Frame indices continue across calls. count == 0 is
 * a no-op. */
nfs_status nfs_push_frames(nfs_handle h, const void* frames, int64_t count);

/* Streaming ingest: append `count` frames that are in host memory (array
 * [count][n][n] of the plan's pixel type), for frames that arrive from an
 * acquisition rather than from device memory. The paper processes images
 * as they are acquired and names the host-to-device transfer as the
 * limiting cost (processing and results sections); here each transform
 * batch is copied on the plan's copy stream into one of two staging
 * buffers while the plan's stream transforms the previous batch, so the
 * uploads overlap the transforms and the pair sums. The result is the
 * same as nfs_push_frames on a device copy of the frames, bit for bit.
 * `frames` should be pinned (hipHostMalloc, or a pinned torch tensor) for
 * the copies to run asynchronously; pageable memory is accepted and copied
 * synchronously by the runtime. Borrowed until the plan's stream passes the
 * enqueued work. Needs a plan created with host_staging = 1, else
 * NFS_E_STATE. count == 0 is a no-op. */
nfs_status nfs_push_host_frames(nfs_handle h, const void* frames, int64_t count);

/* Empirical tuning of the pair kernel's launch shape (modes per workgroup
 * and waves summing lags) for each group of lags: times every shape the
 * kernel supports on the frames pushed so far (all of them while the ring
 * holds them all, else the frames whose partners are all still resident;
 * sums go to scratch memory, the plan's sums are not touched) and keeps the
 * fastest for the plan's later pair sums. The choice
 * made at plan time is a fixed rule; tuning can differ from it for unusual
 * lag sets and frame sizes. Synchronises the plan's stream. choices: host
 * int32 [2 * groups] receiving (modes, waves) per group, or NULL; groups:
 * host int32 receiving the number of lag groups, or NULL. NFS_E_STATE when
 * fewer than 2 frames were pushed. Tuned plans give the same D within the
 * FP32 sum tolerance (16 and 8 modes per workgroup split a mode's frames
 * over different lanes), not bit for bit. */
nfs_status nfs_tune_pairs(nfs_handle h, int32_t* choices, int32_t* groups);

/* Apply pair-kernel launch shapes chosen earlier (by nfs_tune_pairs on a
 * plan of the same frame size, lags and storage, e.g. kept in a cache):
 * choices: host int32 [2 * groups] of (modes, waves) per lag group, in the
 * order nfs_tune_pairs reports them. Every pair must be a shape the kernel
 * supports for that group ((0, 0) for a group of delays beyond the LDS
 * history), and groups must equal the plan's group count, else NFS_E_ARG
 * and the plan is unchanged. Host only; enqueues nothing. */
nfs_status nfs_set_pair_shapes(nfs_handle h, const int32_t* choices, int32_t groups);

/* Accumulate the pair sums of every frame pushed so far (enqueued). Needed
 * only to split the work, e.g. to overlap it with acquisition or to time it:
 * nfs_structure_function does it implicitly. */
nfs_status nfs_accumulate(nfs_handle h);

/* Finish the pair sums for every frame pushed so far and write, all on the
 * device:
 *   D          double [n_lags][n_bins]: D(b, tau) as defined above; NaN for a
 *              delay with no pair (N - tau <= 0); exactly 0 for tau = 0;
 *   bin_counts int64 [n_bins]: C_b, full-plane modes per ring (may be NULL);
 *   lag_pairs  int64 [n_lags]: max(0, N - tau) (may be NULL);
 *   status     int32 [1]: NFS_OK, or NFS_E_DEGENERATE_FRAME when some pushed
 *              frame had a spatial sum <= 0 (sticky until nfs_reset; such a
 *              frame's spectrum is stored as zero except I(0) = n^2), or
 *              NFS_E_TIMEOUT when a wait of the fused transform gave up
 *              (sticky; never expected) (may be NULL).
 * May be called again after more pushes; the sums keep growing. */
nfs_status nfs_structure_function(nfs_handle h, double* D, int64_t* bin_counts,
                                  int64_t* lag_pairs, int32_t* status);

/* 2D power spectra, the per-delay "differences area" of the processing
 * section (Fig. 2): finish the pair sums for every frame pushed so far and
 * write, on the device, S float [n_lags][n][n/2 + 1]: entry [l][r][k_x] is
 *   P_tau(k) = (1 / (N - tau)) * sum_t |I_t(k) - I_{t+tau}(k)|^2
 * for tau = lags[l] and the mode (k_y, k_x), r the transform-order row of
 * k_y, at every mode of the half plane for a plan made with
 * desc.full_spectra = 1; otherwise at the stored modes (k_x < n/2,
 * |k| < n/2) and 0 at the others (the k_x = n/2 column and the corners,
 * which belong to no bin); NaN for every mode of a delay with no pair
 * (N - tau <= 0). The sums are FP32 per mode, the division is done in
 * double and rounded once. S is owned by the caller. Enqueued on the
 * plan's stream. */
nfs_status nfs_power_spectra_2d(nfs_handle h, float* S);

/* Differentiation form: gradients of a scalar loss L of D with respect to
 * the frames and the window. D of Eq. (1) is a smooth function of the
 * images and of the per-pixel weight w (desc.window; w = 1 without one), so
 * the adjoint of every step (the azimuthal average, the pair average, the
 * Fourier transform and the division by the image mean) gives
 *   dL_dframes float [N][n][n]: dL/di_t(x) (may be NULL),
 *   dL_dwindow float [n][n]:    dL/dw(x) = sum_t i_t(x) dL/du_t(x), u = w i
 *                               (may be NULL),
 * for the upstream gradient dL_dD, double [n_lags][n_bins] on the device
 * (entries of delays with no pair and of lag 0 are ignored: D does not
 * depend on the frames there). N is the number of frames pushed so far;
 * `frames` must be those frames, device [N][n][n] of the plan's pixel type
 * (the normalisation and window adjoints need the pixels). The k-space
 * gradient is formed from the stored spectra: from the resident ones when
 * the ring still holds every pushed frame (capacity >= N); otherwise they
 * are recomputed from `frames` by the forward transform (one more transform
 * per frame, in windows of targets plus the largest lag either side), which
 * needs capacity > 2 x the largest lag, else NFS_E_CAPACITY. Recomputing
 * leaves the ring as the pushes left it (the last `capacity` frames), so
 * frames can still be pushed afterwards. The plan needs desc.backward = 1,
 * else NFS_E_STATE. FP32 transforms and differences, FP64 sums of pixels
 * and of the window gradient. Enqueued on the plan's stream; the plan's
 * sums are not changed. */
nfs_status nfs_backward(nfs_handle h, const double* dL_dD, const void* frames,
                        float* dL_dframes, float* dL_dwindow);

/* Batching form: many sequences of uneven frame size n and length N
 * analysed together on one GPU. Each sequence has its own plan (desc), all
 * carved from one caller-owned workspace. A run forks from the caller's
 * stream onto up to 8 library streams (default priority), each sequence on
 * the stream with the least work so far, most work first (work estimated
 * from the ring capacity, taken as the expected frame count), and joins back,
 * so small sequences fill the GPU beside large ones. The same run can be
 * captured once into a HIP graph and replayed. Results per sequence are
 * identical, bit for bit, to those of a single plan on the same frames. */
typedef struct nfs_batch_s* nfs_batch_handle;

/* Host only: workspace bytes of each sequence's plan (sizes, may be NULL)
 * and of the whole batch (total, each plan aligned to 256 bytes). */
nfs_status nfs_batch_workspace_size(const nfs_desc* descs, int32_t n_seq, size_t* sizes,
                                    size_t* total);

/* Host only: ring capacities for sequences of frames[j] frames whose
 * workspaces must fit `budget` bytes together. Every ring holds the whole
 * stack (capacity = max(frames, largest lag + 1)) when that fits; otherwise
 * rings become time windows, at least the largest lag + 64 frames, sharing
 * the rest of the budget in proportion to what each would still need
 * (pair sums are then flushed per window). NFS_E_WORKSPACE when even the
 * minimal windows do not fit. The descs' capacity fields are ignored. */
nfs_status nfs_batch_capacities(const nfs_desc* descs, const int64_t* frames, int32_t n_seq,
                                size_t budget, int64_t* capacities);

/* Create a batch of n_seq plans from descs (each with its capacity set),
 * carving `workspace` (device, 256-byte aligned, `bytes` >= the total of
 * nfs_batch_workspace_size, owned by the caller), with n_streams worker
 * streams (1..8); `stream` is the caller's stream runs fork from and join
 * to. */
nfs_status nfs_batch_create(const nfs_desc* descs, int32_t n_seq, int32_t n_streams,
                            void* workspace, size_t bytes, void* stream,
                            nfs_batch_handle* out);

/* The plan of sequence j (owned by the batch; usable with every nfs_ call,
 * its stream is a worker stream of the batch). */
nfs_status nfs_batch_plan(nfs_batch_handle b, int32_t j, nfs_handle* plan);

/* Enqueue one analysis of every sequence: for sequence j, reset, push
 * counts[j] frames from frames[j] (device) and write D[j], bin_counts[j],
 * lag_pairs[j], status[j] as nfs_structure_function does (the last three
 * arrays, and their entries, may be NULL). Host arrays of n_seq entries.
 * The caller's stream waits for all of it. */
nfs_status nfs_batch_run(nfs_batch_handle b, const void* const* frames, const int64_t* counts,
                         double* const* D, int64_t* const* bin_counts,
                         int64_t* const* lag_pairs, int32_t* const* status);

/* Capture the work of nfs_batch_run with these arguments into a HIP graph
 * (nothing is executed; the caller's stream must not be the legacy default
 * stream); nfs_batch_replay launches it on the caller's stream, re-reading
 * the same frame buffers and rewriting the same outputs. Capturing again
 * replaces the graph. */
nfs_status nfs_batch_capture(nfs_batch_handle b, const void* const* frames,
                             const int64_t* counts, double* const* D,
                             int64_t* const* bin_counts, int64_t* const* lag_pairs,
                             int32_t* const* status);
nfs_status nfs_batch_replay(nfs_batch_handle b);

/* Destroy the batch, its plans, streams and graph (the workspace stays the
 * caller's). */
nfs_status nfs_batch_destroy(nfs_batch_handle b);

/* Forget all frames and sums (enqueued); the plan can be reused. */
nfs_status nfs_reset(nfs_handle h);

/* Release the host-side plan. The workspace stays the caller's. Returns
 * NFS_E_STATE when called twice. */
nfs_status nfs_destroy(nfs_handle h);

/* Static description of a status code. */
const char* nfs_status_string(nfs_status s);

/* Description of the last error on this handle ("" if none); valid until
 * the next call on the handle. */
const char* nfs_last_error(nfs_handle h);

/* Work counters of the plan since it was made or last reset, copied to
 * the device buffer `counters`, int64 [2] (enqueued on the plan's stream):
 *   [0] frames transformed (one per pushed frame; a backward that
 *       recomputes spectra adds one per frame it transforms again);
 *   [1] (target, lag) frame pairs whose terms the pair kernels summed, as
 *       counted by each wave of those kernels from its own lag slice and
 *       window bounds (the bounds of its masks); after
 *       nfs_structure_function this equals sum over the lags of
 *       max(0, N - tau) (the processing section's count of differences per
 *       delay), N the frames pushed.
 * Pairs still pending (pushed frames whose sums nfs_accumulate or
 * nfs_structure_function has not yet enqueued) are not counted. */
nfs_status nfs_work_counters(nfs_handle h, int64_t* counters);

/* Allocation-free form, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the whole analysis of one stack in one call, with the plan's
 * workspace taken from a device array inside the library instead of a
 * caller-owned workspace. It plans `desc` (host_staging and backward must be
 * 0, else NFS_E_ARG; capacity 0 = as many ring slots as the array holds),
 * pushes `count` frames from device memory `frames` ([count][n][n] of the
 * plan's pixel type, borrowed until `stream` passes the work), and writes
 * D, bin_counts, lag_pairs and status exactly as nfs_structure_function
 * does (same kernels, same results bit for bit as nfs_plan +
 * nfs_push_frames + nfs_structure_function with the same desc); outputs are
 * caller-owned device buffers. Calls no hipMalloc, hipFree or other
 * device-allocating routine.
 *
 * The array holds NFS_STATIC_SCRATCH_BYTES bytes per GPU (allocated when
 * the library's code is loaded on that GPU, kept until the process ends);
 * a desc whose workspace (nfs_plan_workspace_size) exceeds it returns
 * NFS_E_SCRATCH before any work is enqueued. The array is found for the
 * current device (hipGetDevice); `stream` must belong to that device (NULL
 * = its default stream), else NFS_E_ARG. Every call on a GPU uses that
 * GPU's one array and it keeps the last call's contents: the call clears
 * what must start at zero itself, and calls that overlap on one GPU (on
 * different streams, or from several host threads) race and give wrong
 * results. Work is enqueued on `stream`; the tables are uploaded with
 * ordinary copies from host memory and the call waits once for them, as
 * nfs_plan does. No handle outlives the call, so errors are reported by
 * the status only. */
#define NFS_STATIC_SCRATCH_BYTES (128u << 20)
nfs_status nfs_structure_function_noalloc(const nfs_desc* desc, const void* frames,
                                          int64_t count, double* D, int64_t* bin_counts,
                                          int64_t* lag_pairs, int32_t* status, void* stream);


/* Inspection entry points (tests and tools).
 *
 * nfs_mode_count: number M of modes stored per spectrum. Only the modes
 * that can land in a bin are stored: k_x in [0, n/2) and |k| < n/2 (the
 * half-plane is enough for real images; the k_x = n/2 line and the corners
 * belong to no bin). Host only.
 *
 * nfs_bin_map: device int32 [n][n/2]; entry [r][k_x] is the bin of mode
 * (k_y, k_x), with r the transform-order row of k_y, or -1 when the mode is
 * in no bin; computed by the same device code that bins the sums.
 *
 * nfs_copy_spectrum: device float [n][n/2][2]: the stored spectrum of
 * pushed frame `t` (real, imaginary) on the half plane k_x in [0, n/2), 0 at
 * modes that are not stored. Only frames still in the ring can be copied:
 * NFS_E_STATE otherwise. */
nfs_status nfs_mode_count(nfs_handle h, int64_t* modes);

/* Memory-bandwidth probe (measurement tool, no plan): one kernel over
 * `bytes` bytes (a multiple of 16; src and dst 16-byte aligned device
 * buffers) enqueued on `stream` (NULL = the default stream):
 *   mode 0: copy src to dst (bytes read and bytes written);
 *   mode 1: read src; dst receives 2048 checksum words (8 KB);
 *   mode 2: write dst (src unused, may be NULL).
 * Timing it over buffers that fit the 256 MB Infinity Cache and over larger
 * ones separates the cache-resident rate from the HBM rate.
 * NFS_E_ARG for a bad mode, size or pointer. */
nfs_status nfs_probe_bandwidth(int32_t mode, const void* src, void* dst, size_t bytes,
                               void* stream);
nfs_status nfs_bin_map(nfs_handle h, int32_t* map);
nfs_status nfs_copy_spectrum(nfs_handle h, int64_t t, float* out);

#ifdef __cplusplus
}
#endif

#endif /* NFS_H */
