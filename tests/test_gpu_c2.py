"""The throughput workload at full size, in the benchmark's launch
configuration, checked on bins the oracle can afford and by properties that
hold everywhere."""
import numpy as np
import pytest

import gen
import oracle
from gpu_util import assert_D_close, require_gpu, say

pytestmark = pytest.mark.gpu


def test_c2_full_size_sampled_bins():
    import paper_1209_3362_amd as nfs
    require_gpu()
    cfg = gen.config("c2")
    say("c2 full size: 1000 frames 1024x1024 u16 drawn on the GPU, seed 2, 50 lags, 512 bins")
    frames = gen.make_stack(cfg, 2, device="cuda")
    plan = nfs.Plan(1024, cfg["lags"], 512, in_dtype="u16", capacity=1000)
    plan.push(frames)
    D, C, P, st = plan.structure_function()
    plan.close()
    D, C, P = D.cpu().numpy(), C.cpu().numpy(), P.cpu().numpy()
    assert int(st.item()) == 0
    assert np.all(np.isfinite(D)) and np.all(D >= 0.0)
    assert np.all(D[:, 0] == 0.0)
    assert np.array_equal(C, oracle.bin_counts(oracle.bin_index(1024, 512), 512))
    assert P.tolist() == [1000 - t for t in cfg["lags"]]
    bins = [1, 2, 7, 60, 255, 511]
    say("c2 oracle on sampled bins " + str(bins))
    ref = oracle.structure_function_bins(frames.cpu().numpy(), cfg["lags"], 512, bins,
                                         workers=16)
    worst = assert_D_close(D[:, bins], ref["D"], rtol=1e-4)
    print("c2 sampled bins worst relative error", worst)


def test_n1024_all_bins_in_benchmark_shapes():
    """Every one of the 512 rings at n = 1024 against the full FP64 oracle:
    64 uint16 frames of the throughput model, its 50 lags (those >= 64 have
    no pair and must come out NaN), the benchmark's launch shapes (32-frame
    transform batches, the 16-mode, 8-wave pair launch of lags up to 500;
    the ring holds the largest lag plus one batch, so the whole stack is one
    pair window)."""
    import paper_1209_3362_amd as nfs
    require_gpu()
    cfg = gen.config("c2")
    N = 64
    say("n=1024 all bins: 64 frames 1024x1024 u16 drawn on the GPU, seed 21, 50 lags, 512 bins")
    frames = gen.make_stack(cfg, 21, device="cuda", N=N)
    plan = nfs.Plan(1024, cfg["lags"], 512, in_dtype="u16", capacity=cfg["lags"][-1] + 32)
    plan.push(frames)
    D, C, P, st = plan.structure_function()
    plan.close()
    D, C, P = D.cpu().numpy(), C.cpu().numpy(), P.cpu().numpy()
    assert int(st.item()) == 0
    say("n=1024 all bins: FP64 oracle on the whole plane")
    ref = oracle.structure_function(frames.cpu().numpy().astype(np.float64), cfg["lags"], 512)
    assert np.array_equal(C, ref["counts"]) and np.array_equal(P, ref["pairs"])
    assert np.array_equal(np.isnan(D), np.isnan(ref["D"]))
    assert np.all(np.isnan(D[[t >= N for t in cfg["lags"]]]))
    assert np.all(D[[t < N for t in cfg["lags"]], 0] == 0.0)
    worst = assert_D_close(D, ref["D"], rtol=1e-4)
    print("n=1024 all bins worst relative error", worst)
