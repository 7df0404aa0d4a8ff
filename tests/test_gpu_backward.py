"""Differentiation form on the GPU (nfs_backward): gradients of a loss of D
with respect to the frames and the window against the FP64 oracle adjoint
(oracle/backward.py, itself pinned by central differences and torch
autograd).

Tolerance: the GPU forms the k-space gradient from FP32 spectra and runs
FP32 inverse transforms, so each gradient entry carries an error of a few
FP32 roundings of the largest entries of its frame; the bar is a maximum
absolute error of 1e-4 of the largest gradient entry (of the frame
gradient, and of the window gradient)."""
import numpy as np
import pytest
import torch

import gen
import oracle
from gpu_util import require_gpu, say

pytestmark = pytest.mark.gpu


def _hann(n):
    return np.outer(np.hanning(n), np.hanning(n))


def _check(name, got, want, tol=1e-4):
    scale = np.abs(want).max()
    err = np.abs(got - want).max()
    print(f"{name}: max |err| / max |grad| = {err / scale:.2e}")
    assert err <= tol * scale, (name, err / scale)


def _run(frames, lags, n_bins, G, window, in_dtype="f32", spec="f32", chunk=None,
         capacity=None, full_spectra=False):
    import paper_1209_3362_amd as nfs
    N, n = frames.shape[0], frames.shape[-1]
    t = frames.to("cuda")
    w = None if window is None else torch.from_numpy(window.astype(np.float32)).cuda()
    cap = capacity or max(N, max(lags) + 1)
    plan = nfs.Plan(n, lags, n_bins, in_dtype=in_dtype, capacity=cap, window=w, spec=spec,
                    backward=True, full_spectra=full_spectra)
    if chunk:
        for i in range(0, N, chunk):
            plan.push(t[i:i + chunk])
    else:
        plan.push(t)
    gf, gw = plan.backward(torch.from_numpy(G), t)
    out = gf.cpu().numpy(), gw.cpu().numpy()
    plan.close()
    return out


def test_backward_matches_oracle_windowed_f32():
    require_gpu()
    cfg = gen.config("c1", N=40)
    lags = [0, 1, 2, 4, 8, 16, 39, 40]
    say("backward: 40 frames 128x128 f32, Hann window, lags 0..40, 64 bins, seed 41")
    f = gen.make_stack(cfg, 41)
    w = _hann(128)
    G = np.random.default_rng(41).standard_normal((len(lags), 64))
    want = oracle.structure_function_grad(f.numpy(), lags, 64, G, window=w)
    gf, gw = _run(f, lags, 64, G, w, chunk=13)
    _check("frames", gf, want["frames"])
    _check("window", gw, want["window"])


def test_backward_matches_oracle_u16_without_window():
    require_gpu()
    cfg = gen.config("c2", n=64, N=50, lags=[1, 3, 7, 20], n_bins=32)
    say("backward: 50 frames 64x64 u16, no window, lags 1,3,7,20, 32 bins, seed 42")
    f = gen.make_stack(cfg, 42)
    G = np.random.default_rng(42).standard_normal((4, 32))
    want = oracle.structure_function_grad(f.numpy().astype(np.float64), cfg["lags"], 32, G)
    gf, gw = _run(f, cfg["lags"], 32, G, None, in_dtype="u16")
    _check("frames", gf, want["frames"])
    _check("window", gw, want["window"])


@pytest.mark.parametrize("n", [16, 256, 2048])
def test_backward_other_sizes(n):
    require_gpu()
    N = {16: 12, 256: 24, 2048: 5}[n]
    cfg = gen.config("c1", n=n, N=N, n_bins=n // 2)
    lags = [1, 2, 5]
    say(f"backward: {N} frames {n}x{n} f32, Hann window, lags 1,2,5, seed 43")
    f = gen.make_stack(cfg, 43)
    w = _hann(n) + 0.1
    G = np.random.default_rng(43).standard_normal((3, n // 2))
    want = oracle.structure_function_grad(f.numpy(), lags, n // 2, G, window=w)
    gf, gw = _run(f, lags, n // 2, G, w)
    _check("frames", gf, want["frames"])
    _check("window", gw, want["window"])


@pytest.mark.parametrize("lags", [[1, 3, 60], [2, 450]])
def test_backward_window_and_global_gradient_kernels(lags):
    """Short lags take the LDS-windowed k-space gradient kernel; a largest
    lag of 450 needs more history than its LDS holds and takes the
    global-memory kernel."""
    require_gpu()
    N = lags[-1] + 30
    cfg = gen.config("c1", n=32, N=N, n_bins=16)
    say(f"backward: {N} frames 32x32 f32, lags {lags}, seed 45")
    f = gen.make_stack(cfg, 45)
    G = np.random.default_rng(45).standard_normal((len(lags), 16))
    want = oracle.structure_function_grad(f.numpy(), lags, 16, G)
    gf, gw = _run(f, lags, 16, G, None, chunk=97)
    _check("frames", gf, want["frames"])
    _check("window", gw, want["window"])


@pytest.mark.parametrize("spec,tol", [("bf16", 3e-2), ("f16", 3e-3)])
def test_backward_from_16bit_spectra(spec, tol):
    """With 16-bit resident spectra the k-space gradient uses the decoded
    stored values (the gradient of the D computed from them); against the
    exact adjoint the error is set by the storage rounding (8 or 11
    significant bits of fluctuation-sized values), orders of magnitude below
    what a wrong decode, scale or reference correction would give."""
    require_gpu()
    cfg = gen.config("c1", N=40)
    lags = [1, 2, 4, 8, 16]
    say(f"backward from {spec} spectra: 40 frames 128x128 f32, Hann window, seed 47")
    f = gen.make_stack(cfg, 47)
    w = _hann(128) + 0.1
    G = np.random.default_rng(47).standard_normal((len(lags), 64))
    want = oracle.structure_function_grad(f.numpy(), lags, 64, G, window=w)
    gf, gw = _run(f, lags, 64, G, w, spec=spec)
    _check("frames", gf, want["frames"], tol=tol)
    _check("window", gw, want["window"], tol=tol)


def test_backward_differentiation_workload():
    """256 float32 frames of 512x512, Hann window, lags 1, 2, 4, ..., 64,
    256 bins: with every spectrum resident and with a 160-slot ring (spectra
    recomputed in the backward, 32 targets per window), against the oracle
    on every pixel, and the scale invariance of D (sum_x i_t dL/di_t = 0 for
    every frame, sum_x w dL/dw = 0)."""
    require_gpu()
    cfg = gen.config("c5")
    lags = cfg["lags"]
    assert lags == [1, 2, 4, 8, 16, 32, 64] and cfg["n_bins"] == 256
    say("backward: 256 frames 512x512 f32 drawn on the GPU, Hann window, seed 5")
    f = gen.make_stack(cfg, 5, device="cuda")
    w = _hann(512)
    G = np.random.default_rng(5).standard_normal((len(lags), 256))
    gf, gw = _run(f, lags, 256, G, w)
    say("backward: same stack, 160-slot ring, spectra recomputed")
    rf, rw = _run(f, lags, 256, G, w, capacity=160)
    host = f.cpu().numpy()
    for t in (0, 100, 255):
        dot = float((host[t].astype(np.float64) * gf[t]).sum())
        assert abs(dot) <= 1e-4 * float(np.abs(host[t] * gf[t]).sum()), t
    dot = float((w * gw).sum())
    assert abs(dot) <= 1e-4 * float(np.abs(w * gw).sum())
    say("backward: FP64 oracle adjoint of the 256 x 512^2 stack")
    want = oracle.structure_function_grad(host, lags, 256, G, window=w)
    _check("frames", gf, want["frames"])
    _check("window", gw, want["window"])
    _check("frames, recomputed", rf, want["frames"])
    _check("window, recomputed", rw, want["window"])
    # Recomputed spectra are the pushed ones bit for bit (same kernels on the
    # same pixels), and each target's k-space gradient sums the same terms in
    # the same order: the frame gradients agree exactly.
    assert np.array_equal(rf, gf)


@pytest.mark.parametrize("spec,tol", [("f32", 1e-4), ("f16", 3e-3)])
def test_backward_recompute_matches_oracle(spec, tol):
    """A ring of 20 slots under 40 frames (lags 0..8: windows of 4 targets,
    spectra recomputed from the frames), chunked pushes, Hann window."""
    require_gpu()
    cfg = gen.config("c1", N=40)
    lags = [0, 1, 2, 4, 8]
    say(f"backward recompute ({spec}): 40 frames 128x128 f32, ring 20, lags 0..8, seed 48")
    f = gen.make_stack(cfg, 48)
    w = _hann(128) + 0.1
    G = np.random.default_rng(48).standard_normal((len(lags), 64))
    want = oracle.structure_function_grad(f.numpy(), lags, 64, G, window=w)
    gf, gw = _run(f, lags, 64, G, w, spec=spec, chunk=7, capacity=20)
    _check("frames", gf, want["frames"], tol=tol)
    _check("window", gw, want["window"], tol=tol)


@pytest.mark.parametrize("capacity", [None, 24])
def test_backward_of_full_spectra_plans(capacity):
    """A plan that stores the entire half plane (its extra modes lie in no
    ring, so they carry no gradient) gives the gradient of the plan that
    stores the ring modes only, resident and with the spectra recomputed
    (a 24-slot ring for 60 frames, largest lag 9), and both match the
    oracle adjoint."""
    require_gpu()
    cfg = gen.config("c1", n=64, N=60, n_bins=32)
    lags = [1, 4, 9]
    say(f"backward, full spectra: 60 frames 64x64 f32, Hann window, lags 1,4,9, ring {capacity}")
    f = gen.make_stack(cfg, 47)
    w = _hann(64) + 0.05
    G = np.random.default_rng(47).standard_normal((3, 32))
    want = oracle.structure_function_grad(f.numpy(), lags, 32, G, window=w)
    got = {}
    for full in (False, True):
        got[full] = _run(f, lags, 32, G, w, chunk=17, capacity=capacity, full_spectra=full)
        _check(f"frames (full={full})", got[full][0], want["frames"])
        _check(f"window (full={full})", got[full][1], want["window"])
    _check("frames, full vs ring-modes plan", got[True][0], got[False][0], tol=1e-6)
    _check("window, full vs ring-modes plan", got[True][1], got[False][1], tol=1e-6)


def test_backward_after_host_pushes():
    """Frames pushed from pinned host memory through the staging buffers,
    then the gradient (resident and recomputed): the same as after device
    pushes, bit for bit."""
    import paper_1209_3362_amd as nfs
    require_gpu()
    cfg = gen.config("c1", n=64, N=50, n_bins=32)
    lags = [1, 3, 8]
    say("backward after host pushes: 50 frames 64x64 f32, lags 1,3,8, rings 50 and 20")
    f = gen.make_stack(cfg, 48)
    G = torch.from_numpy(np.random.default_rng(48).standard_normal((3, 32)))
    t = f.cuda()
    for cap in (50, 20):
        out = []
        for host in (False, True):
            plan = nfs.Plan(64, lags, 32, in_dtype="f32", capacity=cap, backward=True,
                            host_staging=True)
            for i in range(0, 50, 12):
                part = f[i:i + 12]
                plan.push(part.pin_memory() if host else part.cuda())
            gf, gw = plan.backward(G, t)
            out.append((gf.cpu().numpy(), gw.cpu().numpy()))
            plan.close()
        assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1]), cap


def test_backward_recompute_long_lags_u16():
    """Recompute with a largest lag of 450 (the global-memory gradient
    kernel) over 1000 u16 frames in a 905-slot ring: windows of 5 targets."""
    require_gpu()
    lags = [1, 7, 450]
    cfg = gen.config("c2", n=32, N=1000, n_bins=16)
    say("backward recompute: 1000 frames 32x32 u16, ring 905, lags 1,7,450, seed 49")
    f = gen.make_stack(cfg, 49)
    G = np.random.default_rng(49).standard_normal((len(lags), 16))
    want = oracle.structure_function_grad(f.numpy().astype(np.float64), lags, 16, G)
    gf, gw = _run(f, lags, 16, G, None, in_dtype="u16", capacity=905)
    _check("frames", gf, want["frames"])
    _check("window", gw, want["window"])


def test_backward_recompute_leaves_the_ring_as_pushed():
    """After a recomputing backward the ring holds the last `capacity` frames
    exactly as the pushes stored them: more pushes give the same D, bit for
    bit, as a plan that never ran the backward."""
    import paper_1209_3362_amd as nfs
    require_gpu()
    cfg = gen.config("c1", n=64, N=70, n_bins=32)
    lags = [1, 2, 5, 9]
    say("backward recompute: 50 + 20 frames 64x64 f32, ring 30, lags 1..9, seed 50")
    f = gen.make_stack(cfg, 50).cuda()
    G = torch.from_numpy(np.random.default_rng(50).standard_normal((len(lags), 32)))
    out = []
    for run_backward in (False, True):
        plan = nfs.Plan(64, lags, 32, in_dtype="f32", capacity=30, backward=True)
        plan.push(f[:50])
        plan.structure_function()
        before = [torch.empty(64, 32, 2, device="cuda") for _ in range(30)]
        for i, t in enumerate(range(20, 50)):
            plan._check(plan.lib.nfs_copy_spectrum(plan.handle, t,
                                                   nfs.nfs._ptr(before[i])))
        if run_backward:
            plan.backward(G, f[:50])
            for i, t in enumerate(range(20, 50)):
                after = torch.empty(64, 32, 2, device="cuda")
                plan._check(plan.lib.nfs_copy_spectrum(plan.handle, t, nfs.nfs._ptr(after)))
                torch.cuda.synchronize()
                assert torch.equal(after, before[i]), t
        plan.push(f[50:])
        D, C, P, st = plan.structure_function()
        out.append(D.cpu().numpy())
        plan.close()
    assert np.array_equal(out[0], out[1])
    ref = oracle.structure_function(f.cpu().numpy(), lags, 32)
    assert np.allclose(out[1], ref["D"], rtol=1e-4, atol=0)


def test_autograd_recompute():
    """The autograd wrapper with a ring smaller than the stack."""
    import paper_1209_3362_amd as nfs
    require_gpu()
    cfg = gen.config("c1", N=30)
    lags = [1, 3, 6]
    say("autograd recompute: 30 frames 128x128 f32, ring 16, learnable window, seed 51")
    f = gen.make_stack(cfg, 51).cuda().requires_grad_(True)
    w = torch.from_numpy(_hann(128).astype(np.float32) + 0.05).cuda().requires_grad_(True)
    D = nfs.structure_function(f, lags, 64, window=w, capacity=16)
    G = torch.randn(D.shape, dtype=torch.float64, generator=torch.Generator().manual_seed(51))
    (D * G.cuda()).sum().backward()
    wn = w.detach().cpu().numpy().astype(np.float64)
    want = oracle.structure_function_grad(f.detach().cpu().numpy(), lags, 64, G.numpy(),
                                          window=wn)
    _check("frames", f.grad.cpu().numpy(), want["frames"])
    _check("window", w.grad.cpu().numpy(), want["window"])


def test_autograd_function():
    import paper_1209_3362_amd as nfs
    require_gpu()
    cfg = gen.config("c1", N=24)
    lags = [1, 2, 4, 8]
    say("autograd: 24 frames 128x128 f32 with a learnable window, seed 44")
    f = gen.make_stack(cfg, 44).cuda().requires_grad_(True)
    w = torch.from_numpy(_hann(128).astype(np.float32) + 0.05).cuda().requires_grad_(True)
    D = nfs.structure_function(f, lags, 64, window=w)
    G = torch.randn(D.shape, dtype=torch.float64, generator=torch.Generator().manual_seed(44))
    (D * G.cuda()).sum().backward()
    ref = oracle.structure_function(f.detach().cpu().numpy(), lags, 64,
                                    window=w.detach().cpu().numpy().astype(np.float64))
    assert np.allclose(D.detach().cpu().numpy(), ref["D"], rtol=1e-4, atol=0)
    want = oracle.structure_function_grad(f.detach().cpu().numpy(), lags, 64, G.numpy(),
                                          window=w.detach().cpu().numpy().astype(np.float64))
    _check("frames", f.grad.cpu().numpy(), want["frames"])
    _check("window", w.grad.cpu().numpy(), want["window"])


def test_backward_state_errors():
    import paper_1209_3362_amd as nfs
    require_gpu()
    say("backward: plan without backward buffers, ring smaller than the stack")
    f = torch.ones(6, 64, 64, device="cuda") + torch.rand(6, 64, 64, device="cuda")
    G = torch.zeros(1, 8, dtype=torch.float64)
    plan = nfs.Plan(64, [1], 8, in_dtype="f32", capacity=6)
    plan.push(f)
    with pytest.raises(nfs.NfsError) as e:
        plan.backward(G, f)
    assert e.value.status == 7
    plan.close()
    # A ring of 2 slots under 6 frames cannot hold a target and its partners
    # either side (capacity must exceed 2 x the largest lag to recompute).
    plan = nfs.Plan(64, [1], 8, in_dtype="f32", capacity=2, backward=True)
    plan.push(f)
    with pytest.raises(nfs.NfsError) as e:
        plan.backward(G, f)
    assert e.value.status == 6 and "capacity" in str(e.value)
    plan.close()
