"""ctypes binding of libnfs.so (include/nfs.h), same names as the C ABI.

PyTorch supplies device memory and the stream; every step of the analysis
runs in the library's HIP kernels. There is no fallback: a missing or
unloadable library raises.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))

STATUS = {
    0: "NFS_OK", 1: "NFS_E_ARG", 2: "NFS_E_SIZE", 3: "NFS_E_LAGS", 4: "NFS_E_BINS",
    5: "NFS_E_WORKSPACE", 6: "NFS_E_CAPACITY", 7: "NFS_E_STATE",
    8: "NFS_E_DEGENERATE_FRAME", 9: "NFS_E_HIP", 10: "NFS_E_UNSUPPORTED",
    11: "NFS_E_SCRATCH", 12: "NFS_E_TIMEOUT",
}
IN_DTYPES = {"u16": 0, "f32": 1}
SPEC_DTYPES = {"f32": 0, "bf16": 1, "f16": 2}
ACCUMS = {"plain": 0, "kahan": 1}
NFS_OK = 0
NFS_E_DEGENERATE_FRAME = 8


class NfsError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__(f"{STATUS.get(status, status)}: {msg}")


def status_name(code):
    return STATUS.get(int(code), str(code))


class NfsDesc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("in_dtype", ctypes.c_int32),
        ("spec_dtype", ctypes.c_int32),
        ("accum", ctypes.c_int32),
        ("n_lags", ctypes.c_int32),
        ("lags", ctypes.POINTER(ctypes.c_int32)),
        ("n_bins", ctypes.c_int32),
        ("capacity", ctypes.c_int64),
        ("window", ctypes.c_void_p),
        ("host_staging", ctypes.c_int32),
        ("backward", ctypes.c_int32),
        ("full_spectra", ctypes.c_int32),
    ]


def library_path():
    return os.environ.get("NFS_LIBRARY", os.path.join(_HERE, "libnfs.so"))


_LIB = None


def load_library():
    """Load libnfs.so once and declare the C signatures."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run `python -m paper_1209_3362_amd.build`")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i32, i64, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    sigs = {
        "nfs_plan_workspace_size": (i32, [ctypes.POINTER(NfsDesc), ctypes.POINTER(sz)]),
        "nfs_plan": (i32, [ctypes.POINTER(NfsDesc), P, sz, P, ctypes.POINTER(P)]),
        "nfs_push_frames": (i32, [P, P, i64]),
        "nfs_push_host_frames": (i32, [P, P, i64]),
        "nfs_accumulate": (i32, [P]),
        "nfs_tune_pairs": (i32, [P, P, ctypes.POINTER(i32)]),
        "nfs_structure_function": (i32, [P, P, P, P, P]),
        "nfs_reset": (i32, [P]),
        "nfs_destroy": (i32, [P]),
        "nfs_status_string": (ctypes.c_char_p, [i32]),
        "nfs_last_error": (ctypes.c_char_p, [P]),
        "nfs_mode_count": (i32, [P, ctypes.POINTER(i64)]),
        "nfs_bin_map": (i32, [P, P]),
        "nfs_copy_spectrum": (i32, [P, i64, P]),
        "nfs_power_spectra_2d": (i32, [P, P]),
        "nfs_backward": (i32, [P, P, P, P, P]),
        "nfs_probe_bandwidth": (i32, [i32, P, P, sz, P]),
        "nfs_work_counters": (i32, [P, P]),
        "nfs_set_pair_shapes": (i32, [P, P, i32]),
        "nfs_structure_function_noalloc": (i32, [ctypes.POINTER(NfsDesc), P, i64, P, P, P, P,
                                                 P]),
        "nfs_batch_workspace_size": (i32, [ctypes.POINTER(NfsDesc), i32, ctypes.POINTER(sz),
                                           ctypes.POINTER(sz)]),
        "nfs_batch_capacities": (i32, [ctypes.POINTER(NfsDesc), ctypes.POINTER(i64), i32, sz,
                                       ctypes.POINTER(i64)]),
        "nfs_batch_create": (i32, [ctypes.POINTER(NfsDesc), i32, i32, P, sz, P,
                                   ctypes.POINTER(P)]),
        "nfs_batch_plan": (i32, [P, i32, ctypes.POINTER(P)]),
        "nfs_batch_run": (i32, [P, ctypes.POINTER(P), ctypes.POINTER(i64), ctypes.POINTER(P),
                                ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P)]),
        "nfs_batch_capture": (i32, [P, ctypes.POINTER(P), ctypes.POINTER(i64),
                                    ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P),
                                    ctypes.POINTER(P)]),
        "nfs_batch_replay": (i32, [P]),
        "nfs_batch_destroy": (i32, [P]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


def _desc(n, lags, n_bins, in_dtype, capacity, window_ptr, spec="f32", accum="plain",
          host_staging=False, backward=False, full_spectra=False):
    arr = (ctypes.c_int32 * len(lags))(*[int(t) for t in lags])
    d = NfsDesc(n=int(n), in_dtype=IN_DTYPES[in_dtype], spec_dtype=SPEC_DTYPES[spec],
                accum=ACCUMS[accum],
                n_lags=len(lags), lags=arr, n_bins=int(n_bins),
                capacity=int(capacity), window=window_ptr, host_staging=int(host_staging),
                backward=int(backward), full_spectra=int(full_spectra))
    return d, arr


def workspace_size(n, lags, n_bins, in_dtype="u16", capacity=0, window=False, spec="f32",
                   accum="plain", host_staging=False, backward=False, full_spectra=False):
    """Workspace bytes for a plan (host only; raises NfsError on a bad desc)."""
    lib = load_library()
    d, _keep = _desc(n, lags, n_bins, in_dtype, capacity, 1 if window else None, spec, accum,
                     host_staging, backward, full_spectra)
    out = ctypes.c_size_t(0)
    st = lib.nfs_plan_workspace_size(ctypes.byref(d), ctypes.byref(out))
    if st != NFS_OK:
        raise NfsError(st, lib.nfs_status_string(st).decode())
    return int(out.value)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def structure_function_noalloc(frames, lags, n_bins, in_dtype="u16", capacity=0,
                                spec="f32", accum="plain", out=None, stream=None):
    """nfs_structure_function_noalloc: D of one stack of device frames
    [N][n][n] with the plan's workspace in the library's static device array
    (no workspace argument). Outputs (D float64 [L][n_bins], counts int64
    [n_bins], pairs int64 [L], status int32 [1]) are allocated here unless
    `out` brings them; enqueued on `stream` (default: the current stream)."""
    lib = load_library()
    if frames.device.type != "cuda":
        raise ValueError("frames must be on a GPU")
    dtype = torch.uint16 if in_dtype == "u16" else torch.float32
    if frames.dtype != dtype or frames.dim() != 3 or frames.shape[1] != frames.shape[2]:
        raise ValueError(f"frames must be {dtype} [count][n][n]")
    frames = frames.contiguous()
    n = int(frames.shape[-1])
    lags = [int(t) for t in lags]
    if out is None:
        out = (torch.empty((len(lags), int(n_bins)), dtype=torch.float64, device=frames.device),
               torch.empty(int(n_bins), dtype=torch.int64, device=frames.device),
               torch.empty(len(lags), dtype=torch.int64, device=frames.device),
               torch.empty(1, dtype=torch.int32, device=frames.device))
    D, counts, pairs, status = out
    d, _keep = _desc(n, lags, n_bins, in_dtype, capacity, None, spec, accum)
    stream = stream or torch.cuda.current_stream(frames.device)
    with torch.cuda.device(frames.device):
        st = lib.nfs_structure_function_noalloc(
            ctypes.byref(d), _ptr(frames), ctypes.c_int64(frames.shape[0]), _ptr(D),
            _ptr(counts), _ptr(pairs), _ptr(status), ctypes.c_void_p(stream.cuda_stream))
    if st != NFS_OK:
        raise NfsError(st, lib.nfs_status_string(st).decode())
    return D, counts, pairs, status


def check_backward_frames(pushed, n, shape):
    """nfs_backward reads N frames and writes N frame gradients, N the number
    of frames pushed: the stack handed to it must be exactly [N][n][n]."""
    if pushed < 1:
        raise ValueError("no frame pushed: nothing to differentiate")
    if tuple(shape) != (pushed, n, n):
        raise ValueError(f"frames must be the {pushed} pushed frames, [{pushed}][{n}][{n}]; "
                         f"got {list(shape)}")


class Plan:
    """A structure-function plan on one GPU.

    Plan(n, lags, n_bins, in_dtype="u16"|"f32", capacity=N, window=None,
         spec="f32"|"bf16"|"f16", accum="plain"|"kahan", host_staging=False,
         backward=False, full_spectra=False)
    .push(frames)            frames: [count][n][n] uint16/float32 on the device, or in
                             host memory (pinned for overlap) with host_staging=True
    .structure_function()    -> (D float64 [L][n_bins], counts int64 [n_bins],
                                 pairs int64 [L], status int) on the device
    .backward(dL_dD, frames) -> (dL/dframes, dL/dwindow) (plans made with backward=True)
    """

    def __init__(self, n, lags, n_bins, in_dtype="u16", capacity=0, window=None,
                 device=None, stream=None, spec="f32", accum="plain", host_staging=False,
                 backward=False, full_spectra=False):
        self.lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the structure-function library needs one")
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        self.n, self.lags, self.n_bins = int(n), [int(t) for t in lags], int(n_bins)
        self.in_dtype = in_dtype
        self.spec, self.accum = spec, accum
        self.torch_dtype = torch.uint16 if in_dtype == "u16" else torch.float32
        self.window = None
        wptr = None
        if window is not None:
            w = window.to(device=self.device, dtype=torch.float32).contiguous()
            if tuple(w.shape) != (self.n, self.n):
                raise ValueError("window must be [n][n]")
            self.window = w
            wptr = w.data_ptr()
        self.stream = stream or torch.cuda.current_stream(self.device)
        self.host_staging = bool(host_staging)
        self._borrowed = []  # host frames the copy stream may still read
        self.pushed = 0      # frames pushed since the plan was made or reset
        d, self._lags_keep = _desc(self.n, self.lags, self.n_bins, in_dtype, capacity, wptr,
                                   spec, accum, self.host_staging, backward, full_spectra)
        size = ctypes.c_size_t(0)
        st = self.lib.nfs_plan_workspace_size(ctypes.byref(d), ctypes.byref(size))
        self._check(st, None)
        self.workspace = torch.empty(int(size.value), dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            st = self.lib.nfs_plan(ctypes.byref(d), _ptr(self.workspace),
                                   ctypes.c_size_t(self.workspace.numel()),
                                   ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        self._check(st, None)
        self.handle = h
        m = ctypes.c_int64(0)
        self._check(self.lib.nfs_mode_count(self.handle, ctypes.byref(m)))
        self.modes = int(m.value)

    def _check(self, st, handle=True):
        if st != NFS_OK:
            msg = ""
            if handle and getattr(self, "handle", None):
                msg = self.lib.nfs_last_error(self.handle).decode()
            raise NfsError(st, msg or self.lib.nfs_status_string(st).decode())

    def push(self, frames):
        """Append frames [count][n][n] of the plan's pixel type: a device
        tensor (nfs_push_frames), or a host tensor on a plan made with
        host_staging=True (nfs_push_host_frames; pinned memory lets the
        uploads overlap the transforms)."""
        host = frames.device.type == "cpu"
        if not host and frames.device != self.device:
            raise ValueError(f"frames must be on {self.device} or in host memory")
        if host and not self.host_staging:
            raise ValueError("host frames need a plan made with host_staging=True")
        if frames.dtype != self.torch_dtype:
            raise ValueError(f"frames must be {self.torch_dtype}")
        if frames.dim() != 3 or tuple(frames.shape[1:]) != (self.n, self.n):
            raise ValueError("frames must be [count][n][n]")
        frames = frames.contiguous()
        if host:
            self._check(self.lib.nfs_push_host_frames(self.handle, _ptr(frames),
                                                      ctypes.c_int64(frames.shape[0])))
            # Borrowed until the plan's stream has passed the uploads.
            self._borrowed.append(frames)
        else:
            self._check(self.lib.nfs_push_frames(self.handle, _ptr(frames),
                                                 ctypes.c_int64(frames.shape[0])))
        self.pushed += int(frames.shape[0])
        return self

    def synchronize(self):
        """Wait for the plan's stream; releases borrowed host frames."""
        self.stream.synchronize()
        self._borrowed.clear()

    def tune_pairs(self, cache=True):
        """Pair-kernel launch shapes per lag group, [(modes, waves)]: taken
        from the tuning cache (tune_cache.py; key: GPU architecture, n, lags,
        storage, accumulation) through nfs_set_pair_shapes when it holds this
        plan's key, else timed by nfs_tune_pairs on the frames pushed so far
        (synchronises the plan's stream) and stored in the cache."""
        from . import tune_cache
        path = tune_cache.cache_path() if cache else None
        key = None
        if path is not None:
            arch = torch.cuda.get_device_properties(self.device).gcnArchName
            key = tune_cache.cache_key(arch, self.n, self.lags, self.spec, self.accum)
            shapes = None if tune_cache.refresh() else tune_cache.lookup(path, key)
            if shapes is not None and self.set_pair_shapes(shapes, strict=False):
                self.tuned_from_cache = True
                return shapes
        n = ctypes.c_int32(0)
        self._check(self.lib.nfs_tune_pairs(self.handle, None, ctypes.byref(n)))
        arr = (ctypes.c_int32 * (2 * n.value))()
        self._check(self.lib.nfs_tune_pairs(self.handle, arr, ctypes.byref(n)))
        shapes = [(arr[2 * i], arr[2 * i + 1]) for i in range(n.value)]
        self.tuned_from_cache = False
        if key is not None:
            tune_cache.store(path, key, shapes)
        return shapes

    def set_pair_shapes(self, shapes, strict=True):
        """nfs_set_pair_shapes: apply [(modes, waves)] per lag group. With
        strict=False a rejected list returns False instead of raising."""
        flat = [int(v) for pair in shapes for v in pair]
        arr = (ctypes.c_int32 * max(1, len(flat)))(*flat)
        st = self.lib.nfs_set_pair_shapes(self.handle, arr, ctypes.c_int32(len(shapes)))
        if st != NFS_OK and not strict:
            return False
        self._check(st)
        return True

    def accumulate(self):
        """Sum the pairs of every frame pushed so far (enqueued)."""
        self._check(self.lib.nfs_accumulate(self.handle))
        return self

    def empty_outputs(self):
        L, nb = len(self.lags), self.n_bins
        return (torch.empty((L, nb), dtype=torch.float64, device=self.device),
                torch.empty(nb, dtype=torch.int64, device=self.device),
                torch.empty(L, dtype=torch.int64, device=self.device),
                torch.empty(1, dtype=torch.int32, device=self.device))

    def structure_function(self, sync=True, out=None):
        if out is None:
            out = self.empty_outputs()
        D, counts, pairs, status = out
        self._check(self.lib.nfs_structure_function(self.handle, _ptr(D), _ptr(counts),
                                                    _ptr(pairs), _ptr(status)))
        if sync:
            self.synchronize()
        return D, counts, pairs, status

    def work_counters(self, sync=True):
        """nfs_work_counters: (frames transformed, frame pairs summed) as a
        device int64 [2] tensor (synchronised and returned as two ints by
        default)."""
        out = torch.empty(2, dtype=torch.int64, device=self.device)
        self._check(self.lib.nfs_work_counters(self.handle, _ptr(out)))
        if not sync:
            return out
        self.stream.synchronize()
        return int(out[0].item()), int(out[1].item())

    def power_spectra(self, sync=True):
        """P_tau(k) as float32 [n_lags][n][n/2 + 1] (nfs_power_spectra_2d):
        every mode for a plan made with full_spectra=True, else the modes
        that land in a ring and 0 elsewhere."""
        out = torch.empty((len(self.lags), self.n, self.n // 2 + 1), dtype=torch.float32,
                          device=self.device)
        self._check(self.lib.nfs_power_spectra_2d(self.handle, _ptr(out)))
        if sync:
            self.stream.synchronize()
        return out

    def backward(self, dL_dD, frames, frames_grad=True, window_grad=True, sync=True):
        """nfs_backward: gradients of a loss with upstream gradient dL_dD
        [L][n_bins] with respect to `frames` (the frames pushed so far, on the
        device) and the window. Returns (float32 [N][n][n] or None,
        float32 [n][n] or None)."""
        g = dL_dD.to(device=self.device, dtype=torch.float64).contiguous()
        if tuple(g.shape) != (len(self.lags), self.n_bins):
            raise ValueError("dL_dD must be [n_lags][n_bins]")
        if frames.device != self.device or frames.dtype != self.torch_dtype:
            raise ValueError(f"frames must be {self.torch_dtype} on {self.device}")
        check_backward_frames(self.pushed, self.n, tuple(frames.shape))
        frames = frames.contiguous()
        gf = torch.empty(frames.shape, dtype=torch.float32, device=self.device) \
            if frames_grad else None
        gw = torch.empty((self.n, self.n), dtype=torch.float32, device=self.device) \
            if window_grad else None
        self._check(self.lib.nfs_backward(self.handle, _ptr(g), _ptr(frames),
                                          _ptr(gf) if gf is not None else None,
                                          _ptr(gw) if gw is not None else None))
        if sync:
            self.synchronize()
        return gf, gw

    def bin_map(self):
        out = torch.empty((self.n, self.n // 2), dtype=torch.int32, device=self.device)
        self._check(self.lib.nfs_bin_map(self.handle, _ptr(out)))
        self.stream.synchronize()
        return out

    def spectrum(self, t):
        out = torch.empty((self.n, self.n // 2, 2), dtype=torch.float32, device=self.device)
        self._check(self.lib.nfs_copy_spectrum(self.handle, ctypes.c_int64(t), _ptr(out)))
        self.stream.synchronize()
        return torch.view_as_complex(out)

    def reset(self):
        self._check(self.lib.nfs_reset(self.handle))
        self.pushed = 0

    def close(self):
        if getattr(self, "handle", None):
            self.synchronize()
            self.lib.nfs_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _StructureFunction(torch.autograd.Function):
    """D(q, tau) of a frame stack as a differentiable function of the frames
    and the window: the forward pushes the stack through a plan, the
    backward calls nfs_backward on the same plan."""

    @staticmethod
    def forward(ctx, frames, window, lags, n_bins, spec, accum, capacity):
        in_dtype = "u16" if frames.dtype == torch.uint16 else "f32"
        N, n = frames.shape[0], frames.shape[-1]
        if not capacity:
            capacity = max(N, max(lags) + 1)
        plan = Plan(n, lags, n_bins, in_dtype=in_dtype, capacity=capacity,
                    window=None if window is None else window.detach(), spec=spec,
                    accum=accum, backward=True, device=frames.device)
        frames = frames.detach().contiguous()
        plan.push(frames)
        D, _, _, st = plan.structure_function()
        if int(st.item()) != NFS_OK:
            plan.close()
            raise NfsError(int(st.item()), "a frame had a non-positive spatial sum")
        ctx.plan = plan
        ctx.save_for_backward(frames)
        return D

    @staticmethod
    def backward(ctx, dD):
        (frames,) = ctx.saved_tensors
        plan = ctx.plan
        want_f, want_w = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        gf, gw = plan.backward(dD, frames, frames_grad=want_f, window_grad=want_w)
        plan.close()
        ctx.plan = None
        return gf, gw, None, None, None, None, None


def structure_function(frames, lags, n_bins, window=None, spec="f32", accum="plain",
                       capacity=None):
    """D [L][n_bins] (float64) of a device frame stack [N][n][n], differentiable
    with respect to float32 frames and the window (torch autograd).
    `capacity` is the plan's ring size in frames (default: the whole stack);
    with fewer slots than frames the spectra are not kept for the backward
    but recomputed there (needs capacity > 2 x the largest lag)."""
    return _StructureFunction.apply(frames, window, [int(t) for t in lags], int(n_bins), spec,
                                    accum, int(capacity or 0))


def probe_bandwidth(mode, src, dst, nbytes, stream=None):
    """nfs_probe_bandwidth: enqueue one copy (0), read (1) or write (2) pass
    over `nbytes` bytes of device tensors on `stream` (torch's current one by
    default)."""
    lib = load_library()
    s = stream or torch.cuda.current_stream()
    st = lib.nfs_probe_bandwidth(int(mode), None if src is None else _ptr(src), _ptr(dst),
                                 ctypes.c_size_t(int(nbytes)), ctypes.c_void_p(s.cuda_stream))
    if st != NFS_OK:
        raise NfsError(st, lib.nfs_status_string(st).decode())


def batch_capacities(seqs, budget):
    """Ring capacities for sequences [(n, lags, n_bins, in_dtype, frames, spec)]
    whose plans must fit `budget` bytes together (nfs_batch_capacities)."""
    lib = load_library()
    descs = (NfsDesc * len(seqs))()
    keep = []
    for j, (n, lags, nb, dt, _frames, spec) in enumerate(seqs):
        d, arr = _desc(n, lags, nb, dt, 0, None, spec)
        descs[j] = d
        keep.append(arr)
    frames = (ctypes.c_int64 * len(seqs))(*[int(q[4]) for q in seqs])
    caps = (ctypes.c_int64 * len(seqs))()
    st = lib.nfs_batch_capacities(descs, frames, len(seqs), ctypes.c_size_t(int(budget)), caps)
    if st != NFS_OK:
        raise NfsError(st, lib.nfs_status_string(st).decode())
    return [int(c) for c in caps]


class Batch:
    """Many sequences analysed together (nfs_batch_*).

    Batch(seqs, streams=4) with seqs = [dict(n=, lags=, n_bins=, in_dtype=,
    capacity=, spec=)]; .run(frames_list) -> [(D, counts, pairs, status)] on
    the device; .capture(frames_list) then .replay() for a HIP graph of the
    same run."""

    def __init__(self, seqs, streams=4, device=None, stream=None):
        self.lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the structure-function library needs one")
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        self.seqs = [dict(q) for q in seqs]
        n_seq = len(seqs)
        self._descs = (NfsDesc * n_seq)()
        self._keep = []
        for j, q in enumerate(self.seqs):
            d, arr = _desc(q["n"], q["lags"], q["n_bins"], q.get("in_dtype", "u16"),
                           q.get("capacity", 0), None, q.get("spec", "f32"),
                           q.get("accum", "plain"))
            self._descs[j] = d
            self._keep.append(arr)
        total = ctypes.c_size_t(0)
        st = self.lib.nfs_batch_workspace_size(self._descs, n_seq, None, ctypes.byref(total))
        if st != NFS_OK:
            raise NfsError(st, self.lib.nfs_status_string(st).decode())
        self.workspace = torch.empty(int(total.value), dtype=torch.uint8, device=self.device)
        # A stream of its own: graphs cannot be captured on the legacy stream.
        self.stream = stream or torch.cuda.Stream(self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            st = self.lib.nfs_batch_create(self._descs, n_seq, int(streams),
                                           _ptr(self.workspace),
                                           ctypes.c_size_t(self.workspace.numel()),
                                           ctypes.c_void_p(self.stream.cuda_stream),
                                           ctypes.byref(h))
        if st != NFS_OK:
            raise NfsError(st, self.lib.nfs_status_string(st).decode())
        self.handle = h
        self._outs = None
        self._args = None

    def _arrays(self, frames_list):
        n_seq = len(self.seqs)
        if len(frames_list) != n_seq:
            raise ValueError("one frame stack per sequence")
        P = ctypes.c_void_p
        outs = []
        for q, f in zip(self.seqs, frames_list):
            dt = torch.uint16 if q.get("in_dtype", "u16") == "u16" else torch.float32
            if f.device != self.device or f.dtype != dt or f.dim() != 3 or \
                    tuple(f.shape[1:]) != (q["n"], q["n"]) or not f.is_contiguous():
                raise ValueError("frames must be contiguous [count][n][n] of the sequence's "
                                 "pixel type on the batch's device")
            L, nb = len(q["lags"]), q["n_bins"]
            outs.append((torch.empty((L, nb), dtype=torch.float64, device=self.device),
                         torch.empty(nb, dtype=torch.int64, device=self.device),
                         torch.empty(L, dtype=torch.int64, device=self.device),
                         torch.empty(1, dtype=torch.int32, device=self.device)))
        fr = (P * n_seq)(*[f.data_ptr() for f in frames_list])
        cn = (ctypes.c_int64 * n_seq)(*[f.shape[0] for f in frames_list])
        arrs = [(P * n_seq)(*[o[i].data_ptr() for o in outs]) for i in range(4)]
        return outs, (fr, cn, *arrs)

    def _after_current(self):
        """Order the batch's stream after the work already enqueued on the
        current stream (which may still be producing the frames)."""
        self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def _before_current(self):
        """Order later work on the current stream (reads of the outputs,
        reuse of the frames' or outputs' memory) after the batch's run."""
        torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def tune(self, frames_list, cache=True):
        """Every sequence's pair-kernel launch shapes: from the tuning cache
        (tune_cache.py) when it holds the sequence's key, else timed on its
        frames (push, nfs_tune_pairs, reset per plan) and cached; returns the
        shapes."""
        from . import tune_cache
        self._arrays(frames_list)  # validates shapes and types
        # The plans' pushes run on the batch's worker streams: let the
        # frames be complete first.
        torch.cuda.current_stream(self.device).synchronize()
        path = tune_cache.cache_path() if cache else None
        arch = torch.cuda.get_device_properties(self.device).gcnArchName
        shapes = []
        for j, f in enumerate(frames_list):
            q = self.seqs[j]
            key = tune_cache.cache_key(arch, q["n"], q["lags"], q.get("spec", "f32"),
                                       q.get("accum", "plain"))
            p = ctypes.c_void_p()
            st = self.lib.nfs_batch_plan(self.handle, j, ctypes.byref(p))
            if st != NFS_OK:
                raise NfsError(st, self.lib.nfs_status_string(st).decode())
            cached = None if tune_cache.refresh() else tune_cache.lookup(path, key)
            if cached is not None:
                flat = [int(v) for pair in cached for v in pair]
                arr = (ctypes.c_int32 * max(1, len(flat)))(*flat)
                if self.lib.nfs_set_pair_shapes(p, arr, ctypes.c_int32(len(cached))) == NFS_OK:
                    shapes.append(cached)
                    continue
            st = self.lib.nfs_push_frames(p, _ptr(f), ctypes.c_int64(f.shape[0]))
            n = ctypes.c_int32(0)
            arr = (ctypes.c_int32 * 64)()
            if st == NFS_OK:
                st = self.lib.nfs_tune_pairs(p, arr, ctypes.byref(n))
            if st == NFS_OK:
                st = self.lib.nfs_reset(p)
            if st != NFS_OK:
                raise NfsError(st, self.lib.nfs_last_error(p).decode())
            found = [(arr[2 * i], arr[2 * i + 1]) for i in range(n.value)]
            tune_cache.store(path, key, found)
            shapes.append(found)
        return shapes

    def run(self, frames_list, sync=True):
        outs, args = self._arrays(frames_list)
        self._after_current()
        st = self.lib.nfs_batch_run(self.handle, *args)
        if st != NFS_OK:
            raise NfsError(st, self.lib.nfs_status_string(st).decode())
        self._before_current()
        if sync:
            self.stream.synchronize()
        return outs

    def capture(self, frames_list):
        """Capture one run into a graph; returns the output tensors every
        replay rewrites."""
        outs, args = self._arrays(frames_list)
        # Nothing is executed by the capture; replays order themselves after
        # the current stream. Make the batch's stream idle before capturing.
        self._after_current()
        self.stream.synchronize()
        st = self.lib.nfs_batch_capture(self.handle, *args)
        if st != NFS_OK:
            raise NfsError(st, self.lib.nfs_status_string(st).decode())
        self._outs, self._args, self._frames = outs, args, list(frames_list)
        return outs

    def replay(self, sync=True):
        self._after_current()
        st = self.lib.nfs_batch_replay(self.handle)
        if st != NFS_OK:
            raise NfsError(st, self.lib.nfs_status_string(st).decode())
        self._before_current()
        if sync:
            self.stream.synchronize()
        return self._outs

    def close(self):
        if getattr(self, "handle", None):
            self.stream.synchronize()
            self.lib.nfs_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
