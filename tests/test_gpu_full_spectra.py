"""Plans that store the entire half plane (desc.full_spectra = 1): the 2D
power spectra P_tau(k) of the paper's differences area (Fig. 2; the
discussion section stores the entire 2D power spectra) on every mode,
including the corners |k| >= n/2 and the k_x = n/2 column, against the FP64
oracle's full-plane P; D is the same as from a plan that stores only the
modes that land in a ring."""
import numpy as np
import pytest
import torch

import gen
import oracle
from gpu_util import require_gpu, say

pytestmark = pytest.mark.gpu


def _check_power(S, P_full, N, lags, n):
    """S [L][n][n/2+1] from the GPU against the oracle's full-plane P
    [L][n][n] restricted to k_x = 0..n/2: 1e-4 relative plus 1e-6 of the
    delay's largest value; tau = 0 exactly 0; no pair: NaN."""
    worst = 0.0
    for i, tau in enumerate(lags):
        if N - tau <= 0:
            assert np.all(np.isnan(S[i])), tau
            continue
        if tau == 0:
            assert np.all(S[i] == 0), tau
            continue
        o = np.asarray(P_full[i])[:, : n // 2 + 1]
        err = np.abs(S[i] - o)
        bound = 1e-4 * np.abs(o) + 1e-6 * np.abs(o).max()
        assert np.all(err <= bound), (tau, float((err / np.maximum(o, 1e-30)).max()))
        big = o > 1e-3 * o.max()
        worst = max(worst, float((err[big] / o[big]).max()))
    return worst


@pytest.mark.parametrize("n,N,in_dtype,cap,chunk", [
    (16, 12, "f32", 12, None),
    (128, 20, "f32", 32, None),
    (64, 40, "u16", 24, 7),      # ring shorter than the stack, chunked pushes
    (256, 10, "f32", 10, None),
])
def test_full_power_spectra_match_oracle(n, N, in_dtype, cap, chunk):
    import paper_1209_3362_amd as nfs
    require_gpu()
    lags = [0, 1, 3, 7, N - 1, N, N + 5] if cap > N + 5 else [0, 1, 3, 7]
    cfg = gen.config("c2" if in_dtype == "u16" else "c1", n=n, N=N, n_bins=n // 2)
    say(f"full spectra: {N} frames {n}x{n} {in_dtype}, ring {cap}, lags {lags}, seed 6")
    f = gen.make_stack(cfg, 6)
    ref = oracle.structure_function(f.numpy().astype(np.float64), lags, n // 2,
                                    return_power=True)
    t = f.cuda()
    out = {}
    for full in (False, True):
        plan = nfs.Plan(n, lags, n // 2, in_dtype=in_dtype, capacity=cap, full_spectra=full)
        assert plan.modes == (n * (n // 2 + 1) if full else plan.modes)
        for i in range(0, N, chunk or N):
            plan.push(t[i:i + (chunk or N)])
        D, C, P, st = plan.structure_function()
        S = plan.power_spectra().cpu().numpy()
        plan.close()
        out[full] = (D.cpu().numpy(), C.cpu().numpy(), S)
        assert int(st.item()) == 0
    # D comes from the same ring modes with the same per-mode arithmetic.
    assert np.array_equal(out[True][0], out[False][0], equal_nan=True)
    assert np.array_equal(out[True][1], ref["counts"])
    S = out[True][2]
    assert S.shape == (len(lags), n, n // 2 + 1)
    worst = _check_power(S, ref["P"], N, lags, n)
    print(f"full power spectra n={n}: worst relative error {worst:.2e}")
    # The stored-modes plan agrees with the full one where it stores a mode
    # and is 0 elsewhere.
    part = out[False][2]
    stored = part != 0
    assert np.array_equal(part[stored], S[stored], equal_nan=True)


def test_full_spectra_16bit_storage():
    """BF16 and FP16 storage of the full half plane: within the storage
    rounding of the FP32 full plan (8 / 11 significant bits of
    fluctuation-sized values), and D unchanged by the extra modes."""
    import paper_1209_3362_amd as nfs
    require_gpu()
    n, N, lags = 64, 24, [1, 2, 5]
    cfg = gen.config("c2", n=n, N=N, n_bins=32)
    say("full spectra, 16-bit storage: 24 frames 64x64 u16, lags 1,2,5, seed 7")
    t = gen.make_stack(cfg, 7).cuda()
    res = {}
    for spec in ("f32", "bf16", "f16"):
        for full in (False, True):
            plan = nfs.Plan(n, lags, 32, in_dtype="u16", capacity=N, spec=spec,
                            full_spectra=full)
            plan.push(t)
            D, _, _, _ = plan.structure_function()
            res[(spec, full)] = (D.cpu().numpy(), plan.power_spectra().cpu().numpy())
            plan.close()
        assert np.array_equal(res[(spec, True)][0], res[(spec, False)][0])
    ref = res[("f32", True)][1]
    for spec, tol in (("bf16", 3e-2), ("f16", 3e-3)):
        S = res[(spec, True)][1]
        err = np.abs(S - ref).max(axis=(1, 2)) / np.abs(ref).max(axis=(1, 2))
        print(f"{spec}: max |P - P_f32| / max P per lag {err}")
        assert np.all(err <= tol), (spec, err)
