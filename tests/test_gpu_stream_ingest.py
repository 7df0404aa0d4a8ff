"""Streaming ingest (nfs_push_host_frames): frames pushed from host memory
through the plan's two staging buffers and copy stream give the same D,
counts and pairs as the same frames pushed from device memory, bit for bit
(the same kernels see the same bytes), and match the FP64 oracle."""
import numpy as np
import pytest
import torch

import gen
import oracle
from gpu_util import assert_D_close, require_gpu, say

pytestmark = pytest.mark.gpu


def _run(frames, lags, n_bins, in_dtype, capacity, chunks, host, pinned=True, **opts):
    import paper_1209_3362_amd as nfs
    plan = nfs.Plan(frames.shape[-1], lags, n_bins, in_dtype=in_dtype, capacity=capacity,
                    host_staging=True, **opts)
    i = 0
    for k, c in enumerate(chunks):
        part = frames[i:i + c]
        if host is True or (host == "mixed" and k % 2 == 0):
            part = part.cpu()
            if pinned:
                part = part.pin_memory()
        else:
            part = part.cuda()
        plan.push(part)
        i += c
    assert i == frames.shape[0]
    D, C, P, st = plan.structure_function()
    out = (D.cpu().numpy(), C.cpu().numpy(), P.cpu().numpy(), int(st.item()))
    plan.close()
    return out


@pytest.mark.parametrize("host", [True, "mixed"])
def test_host_push_equals_device_push_with_ring_wrap(host):
    require_gpu()
    cfg = gen.config("c1")
    lags = cfg["lags"]
    say(f"host ingest ({host}): 64 frames 128x128 f32, capacity 30, uneven chunks")
    f = gen.make_stack(cfg, 21)
    chunks = [7, 13, 1, 20, 23]
    ref = _run(f, lags, 64, "f32", 30, chunks, host=False)
    got = _run(f, lags, 64, "f32", 30, chunks, host=host)
    for a, b in zip(ref[:3], got[:3]):
        assert np.array_equal(a, b, equal_nan=True)
    assert got[3] == ref[3] == 0
    exact = oracle.structure_function(f.numpy(), lags, 64)
    assert_D_close(got[0], exact["D"], rtol=1e-4)
    assert np.array_equal(got[1], exact["counts"])


@pytest.mark.parametrize("spec,accum", [("bf16", "kahan"), ("f16", "plain")])
def test_host_push_16bit_storage_windowed(spec, accum):
    """Host pushes into plans with 16-bit spectra, Kahan sums and a window,
    with ring wrap: the same bytes as device pushes."""
    require_gpu()
    cfg = gen.config("c1", n=64, N=70, n_bins=32)
    lags = [1, 2, 5, 11, 23]
    say(f"host ingest: 70 frames 64x64 f32, {spec}/{accum}, Hann window, capacity 40")
    f = gen.make_stack(cfg, 23)
    w = torch.from_numpy((np.outer(np.hanning(64), np.hanning(64)) + 0.1).astype(np.float32))
    opts = dict(spec=spec, accum=accum, window=w.cuda())
    chunks = [9, 17, 30, 14]
    ref = _run(f, lags, 32, "f32", 40, chunks, host=False, **opts)
    got = _run(f, lags, 32, "f32", 40, chunks, host=True, **opts)
    for a, b in zip(ref[:3], got[:3]):
        assert np.array_equal(a, b, equal_nan=True)
    assert got[3] == ref[3] == 0


def test_host_push_pageable_u16():
    require_gpu()
    cfg = gen.config("c2", n=128, N=80, lags=[1, 2, 3, 5, 8, 13, 21, 34, 55, 79], n_bins=64)
    say("host ingest: 80 frames 128x128 u16 from pageable memory, capacity 100")
    f = gen.make_stack(cfg, 22)
    ref = _run(f, cfg["lags"], 64, "u16", 100, [80], host=False)
    got = _run(f, cfg["lags"], 64, "u16", 100, [33, 47], host=True, pinned=False)
    for a, b in zip(ref[:3], got[:3]):
        assert np.array_equal(a, b, equal_nan=True)


def test_host_push_full_size_equals_device_push():
    """The benchmark workload (1000 uint16 frames 1024x1024, 50 lags, 512
    rings) pushed from pinned host memory in one call."""
    require_gpu()
    cfg = gen.config("c2")
    say("host ingest: 1000 frames 1024x1024 u16 drawn on the GPU, seed 2, pinned host copy")
    f = gen.make_stack(cfg, 2, device="cuda")
    ref = _run(f, cfg["lags"], 512, "u16", 1000, [1000], host=False)
    got = _run(f, cfg["lags"], 512, "u16", 1000, [1000], host=True)
    for a, b in zip(ref[:3], got[:3]):
        assert np.array_equal(a, b, equal_nan=True)
    assert got[3] == 0


def test_host_push_needs_a_staging_plan():
    import paper_1209_3362_amd as nfs
    require_gpu()
    say("host ingest: plan without staging rejects host frames")
    plan = nfs.Plan(64, [1], 8, in_dtype="f32", capacity=4)
    with pytest.raises(ValueError):
        plan.push(torch.ones(2, 64, 64))
    lib = nfs.load_library()
    import ctypes
    x = torch.ones(2, 64, 64).pin_memory()
    st = lib.nfs_push_host_frames(plan.handle, ctypes.c_void_p(x.data_ptr()), 2)
    assert nfs.status_name(st) == "NFS_E_STATE"
    assert b"host_staging" in lib.nfs_last_error(plan.handle)
    plan.close()
