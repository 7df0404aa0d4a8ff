"""The allocation-free entry point (nfs_structure_function_noalloc) against
the workspace entry points (nfs_plan + nfs_push_frames +
nfs_structure_function) on the same frames, and both against the FP64
oracle: two calls in a row on the one static array, the second smaller,
so the second must not see anything the first left behind."""
import numpy as np
import pytest
import torch

import gen
import oracle
import paper_1209_3362_amd as nfs
from tests.gpu_util import assert_D_close, require_gpu, run_plan, say

pytestmark = pytest.mark.gpu


def noalloc(frames, lags, n_bins, in_dtype, capacity):
    require_gpu()
    t = torch.as_tensor(frames)
    t = t.to(torch.uint16 if in_dtype == "u16" else torch.float32).to("cuda").contiguous()
    D, C, P, st = nfs.structure_function_noalloc(t, lags, n_bins, in_dtype=in_dtype,
                                                 capacity=capacity)
    torch.cuda.current_stream().synchronize()
    return D.cpu().numpy(), C.cpu().numpy(), P.cpu().numpy(), int(st.item())


def check_case(frames, lags, n_bins, in_dtype, capacity, tag):
    ref = oracle.structure_function(np.asarray(frames, dtype=np.float64), lags, n_bins)
    say(f"noalloc {tag}: static-scratch entry point")
    Dn, Cn, Pn, stn = noalloc(frames, lags, n_bins, in_dtype, capacity)
    say(f"noalloc {tag}: workspace entry points")
    Dw, Cw, Pw, stw = run_plan(frames, lags, n_bins, in_dtype, capacity=capacity)
    assert stn == 0 and stw == 0
    # Same kernels and layout: identical bit for bit (NaN where no pair).
    assert np.array_equal(Dn, Dw, equal_nan=True)
    assert np.array_equal(Cn, Cw) and np.array_equal(Pn, Pw)
    assert np.array_equal(Cn, ref["counts"]) and np.array_equal(Pn, ref["pairs"])
    return assert_D_close(Dn, ref["D"], rtol=1e-4)


def test_noalloc_two_calls_second_smaller():
    cfg = gen.config("c1")
    big = gen.make_stack(cfg, 1).numpy()                     # 64 x 128^2 f32
    check_case(big, cfg["lags"], cfg["n_bins"], "f32", 64, "64x128^2 f32")
    # Second call: fewer, smaller u16 frames, lag 0 and a ring shorter than
    # the stack (windowed sums): the array still holds the first call's
    # spectra, sums and tables.
    small_cfg = gen.config("c2", n=64, N=20)
    small = gen.make_stack(small_cfg, 5).numpy()
    check_case(small, [0, 1, 3, 7, 11], 32, "u16", 12, "20x64^2 u16, ring 12")


def test_noalloc_derived_capacity_and_oversize():
    """capacity 0 takes as many ring slots as the array holds; a plan larger
    than the array is refused with NFS_E_SCRATCH and leaves the outputs
    untouched."""
    cfg = gen.config("c1", N=40)
    frames = gen.make_stack(cfg, 3).numpy()
    lags = [1, 2, 4, 8, 16, 45]  # 45 >= N: no pair, D NaN
    check_case(frames, lags, cfg["n_bins"], "f32", 0, "40x128^2 f32, capacity 0")
    t = torch.zeros((4, 1024, 1024), dtype=torch.uint16, device="cuda")
    out = (torch.full((3, 512), 7.0, dtype=torch.float64, device="cuda"),
           torch.zeros(512, dtype=torch.int64, device="cuda"),
           torch.zeros(3, dtype=torch.int64, device="cuda"),
           torch.zeros(1, dtype=torch.int32, device="cuda"))
    say("noalloc: oversize plan refused")
    with pytest.raises(nfs.NfsError) as e:
        nfs.structure_function_noalloc(t, [1, 2, 3], 512, in_dtype="u16", capacity=200,
                                       out=out)
    assert nfs.status_name(e.value.status) == "NFS_E_SCRATCH"
    torch.cuda.synchronize()
    assert bool((out[0] == 7.0).all())
