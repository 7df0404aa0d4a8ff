"""The fused transform (row and column passes in one persistent launch, the
intermediate handed over inside one XCD) against the two-pass path and the
FP64 oracle at n = 1024: stored spectra and D bit for bit equal to the
two-pass path (same arithmetic in the same order), for every storage type,
with a window, with f32 and u16 input, for each split of the column tiles
between the XCD-local buffer and memory, and over a ring shorter than the
stack."""
import numpy as np
import pytest
import torch

import gen
import oracle
from gpu_util import assert_D_close, require_gpu, say

pytestmark = [
    pytest.mark.gpu,
    pytest.mark.skip(reason="fused transform switched off: its first GPU runs did not finish "
                            "(scheduler waits ran to their bound); cause not established"),
]


def _run(monkeypatch, mode, frames, lags, n_bins, in_dtype, capacity, keep=None, spec="f32",
         window=None, chunk=None, copy=()):
    import paper_1209_3362_amd as nfs
    monkeypatch.setenv("NFS_TRANSFORM", mode)
    if keep is None:
        monkeypatch.delenv("NFS_FUSED_KEEP", raising=False)
    else:
        monkeypatch.setenv("NFS_FUSED_KEEP", str(keep))
    plan = nfs.Plan(1024, lags, n_bins, in_dtype=in_dtype, capacity=capacity, spec=spec,
                    window=window)
    N = frames.shape[0]
    step = chunk or N
    for i in range(0, N, step):
        plan.push(frames[i:i + step])
    spectra = []
    for t in copy:
        out = torch.empty(1024, 512, 2, device="cuda")
        plan._check(plan.lib.nfs_copy_spectrum(plan.handle, t, nfs.nfs._ptr(out)))
        spectra.append(out)
    D, C, P, st = plan.structure_function()
    counts = plan.work_counters()
    res = (D.cpu().numpy(), int(st.item()), [s.cpu().numpy() for s in spectra], counts)
    plan.close()
    return res


@pytest.mark.parametrize("keep", [None, 0, 64])
def test_fused_equals_two_pass_u16(monkeypatch, keep):
    require_gpu()
    cfg = gen.config("c2", N=40)
    lags = [0, 1, 2, 5, 13, 39, 40]
    say(f"fused transform: 40 frames 1024x1024 u16, keep {keep}, seed 21")
    f = gen.make_stack(cfg, 21, device="cuda")
    a = _run(monkeypatch, "fused", f, lags, 512, "u16", 48, keep=keep, copy=(0, 17, 39))
    b = _run(monkeypatch, "two_pass", f, lags, 512, "u16", 48, copy=(0, 17, 39))
    assert a[1] == 0 and b[1] == 0
    for x, y in zip(a[2], b[2]):
        assert np.array_equal(x, y)
    assert np.array_equal(a[0], b[0], equal_nan=True)
    assert a[3] == b[3] == (40, sum(max(0, 40 - t) for t in lags))
    if keep is None:
        say("fused transform: FP64 oracle on the 40 x 1024^2 stack")
        ref = oracle.structure_function(f.cpu().numpy().astype(np.float64), lags, 512)
        assert_D_close(a[0], ref["D"], rtol=1e-4)


@pytest.mark.parametrize("spec", ["bf16", "f16"])
def test_fused_equals_two_pass_16bit_window_f32(monkeypatch, spec):
    require_gpu()
    cfg = gen.config("c1", n=1024, N=20, n_bins=512)
    lags = [1, 3, 7]
    say(f"fused transform: 20 frames 1024x1024 f32, Hann window, {spec}, seed 22")
    f = gen.make_stack(cfg, 22, device="cuda")
    w = torch.from_numpy(np.outer(np.hanning(1024), np.hanning(1024)).astype(np.float32) + 0.1)
    a = _run(monkeypatch, "fused", f, lags, 512, "f32", 20, spec=spec, window=w, copy=(3, 19))
    b = _run(monkeypatch, "two_pass", f, lags, 512, "f32", 20, spec=spec, window=w, copy=(3, 19))
    assert a[1] == 0 and b[1] == 0
    for x, y in zip(a[2], b[2]):
        assert np.array_equal(x, y)
    assert np.array_equal(a[0], b[0], equal_nan=True)


def test_fused_ring_wrap_and_chunks(monkeypatch):
    """A 30-slot ring under 70 frames pushed in chunks of 9: several fused
    launches, frames wrapping the ring, pair windows flushed in between."""
    require_gpu()
    cfg = gen.config("c2", N=70)
    lags = [1, 4, 11, 20]
    say("fused transform: 70 frames 1024x1024 u16, ring 30, chunks of 9, seed 23")
    f = gen.make_stack(cfg, 23, device="cuda")
    a = _run(monkeypatch, "fused", f, lags, 512, "u16", 30, chunk=9)
    b = _run(monkeypatch, "two_pass", f, lags, 512, "u16", 30, chunk=9)
    assert a[1] == 0 and np.array_equal(a[0], b[0], equal_nan=True)
    assert a[3] == (70, sum(max(0, 70 - t) for t in lags))
