"""Helpers shared by the GPU parity tests (no test functions here)."""
import sys

import numpy as np
import torch


def say(msg):
    """Name the case before GPU work so a failed run can be traced."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def require_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("GPU test run without a visible GPU")


def run_plan(frames, lags, n_bins, in_dtype, capacity=None, window=None, chunk=None,
             spec="f32", accum="plain"):
    """Push `frames` (torch or numpy [N][n][n]) through a plan; return numpy results."""
    import paper_1209_3362_amd as nfs
    require_gpu()
    t = torch.as_tensor(frames)
    t = t.to(torch.uint16 if in_dtype == "u16" else torch.float32).to("cuda").contiguous()
    N, n = t.shape[0], t.shape[-1]
    cap = capacity if capacity is not None else max(N, max(lags) + 1)
    plan = nfs.Plan(n, lags, n_bins, in_dtype=in_dtype, capacity=cap, window=window,
                    spec=spec, accum=accum)
    if chunk:
        for i in range(0, N, chunk):
            plan.push(t[i:i + chunk])
    else:
        plan.push(t)
    D, C, P, st = plan.structure_function()
    out = (D.cpu().numpy(), C.cpu().numpy(), P.cpu().numpy(), int(st.item()))
    plan.close()
    return out


def assert_D_close(Dg, Do, rtol=1e-4, atol=0.0):
    """NaN pattern equal; exact zeros of the oracle exact on the GPU too;
    elsewhere |Dg - Do| <= rtol*|Do| + atol."""
    Dg = np.asarray(Dg)
    Do = np.asarray(Do)
    assert Dg.shape == Do.shape
    assert np.array_equal(np.isnan(Dg), np.isnan(Do))
    ok = ~np.isnan(Do)
    zero = ok & (Do == 0.0)
    assert np.all(Dg[zero] == 0.0), "exact zeros differ"
    nz = ok & ~zero
    err = np.abs(Dg[nz] - Do[nz])
    bound = rtol * np.abs(Do[nz]) + atol
    worst = float(np.max(err / np.maximum(np.abs(Do[nz]), 1e-300))) if nz.any() else 0.0
    assert np.all(err <= bound), f"max relative error {worst:.3e}"
    return worst
