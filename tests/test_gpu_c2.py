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
