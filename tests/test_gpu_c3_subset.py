"""Precision workload (4000 x 1024^2 u16, every lag 1..400) on its first 256
frames, in every storage / accumulation form, against the FP64 oracle on
sampled bins and against the plain FP32 run on all bins.

Forms in the plain FP32 storage meet the 1e-4 bar against the exact
definition; 16-bit forms meet it against the oracle's storage model, and
their per-bin error against the exact definition and against the plain run
is printed (max and median over lags) for the record."""
import numpy as np
import pytest

import gen
import oracle
from gpu_util import assert_D_close, require_gpu, say

pytestmark = pytest.mark.gpu

BINS = [1, 2, 7, 60, 255, 511]


def _table(name, D, ref):
    ok = ~np.isnan(ref) & (ref != 0)
    rel = np.where(ok, np.abs(D - ref) / np.where(ok, np.abs(ref), 1), np.nan)
    cells = ", ".join(f"b{b}: max {np.nanmax(rel[:, j]):.1e} med {np.nanmedian(rel[:, j]):.1e}"
                      for j, b in enumerate(BINS))
    print(f"{name}: {cells}")


def test_c3_subset_all_forms():
    import torch
    import paper_1209_3362_amd as nfs
    require_gpu()
    cfg = gen.config("c3", N=256)
    lags = cfg["lags"]
    say("c3 subset: 256 frames 1024x1024 u16 drawn on the GPU, seed 3, lags 1..400, 512 bins")
    frames = gen.make_stack(cfg, 3, device="cuda")
    host = frames.cpu().numpy().astype(np.float64)
    results = {}
    for spec, accum in (("f32", "plain"), ("f32", "kahan"), ("bf16", "kahan"),
                        ("f16", "kahan")):
        say(f"c3 subset on the GPU: spectra {spec}, sums {accum}")
        plan = nfs.Plan(1024, lags, 512, in_dtype="u16", capacity=401, spec=spec, accum=accum)
        plan.push(frames)
        D, C, P, st = plan.structure_function()
        plan.close()
        assert int(st.item()) == 0
        results[(spec, accum)] = D.cpu().numpy()
        assert P.cpu().numpy().tolist() == [max(0, 256 - t) for t in lags]
    say("c3 subset: FP64 oracle on sampled bins " + str(BINS))
    exact = oracle.structure_function_bins(host, lags, 512, BINS, workers=16)["D"]
    plain = results[("f32", "plain")]
    for key, D in results.items():
        spec, accum = key
        sub = D[:, BINS]
        if spec == "f32":
            worst = assert_D_close(sub, exact, rtol=1e-4)
            print(f"{spec}/{accum} vs FP64 oracle worst {worst:.2e}")
        else:
            say(f"c3 subset: FP64 storage model {spec} on sampled bins")
            model = oracle.structure_function_stored_bins(host, lags, 512, BINS, spec,
                                                         workers=16)["D"]
            worst = assert_D_close(sub, model, rtol=1e-4)
            print(f"{spec}/{accum} vs its storage model worst {worst:.2e}")
        _table(f"{spec}/{accum} vs FP64 oracle", sub, exact)
        if key != ("f32", "plain"):
            _table(f"{spec}/{accum} vs plain FP32 run", sub, plain[:, BINS])
            ok = ~np.isnan(plain) & (plain != 0)
            rel = np.abs(D[ok] - plain[ok]) / np.abs(plain[ok])
            print(f"{spec}/{accum} vs plain FP32 run, all bins: max {rel.max():.2e} "
                  f"median {np.median(rel):.2e}")
