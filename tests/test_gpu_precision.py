"""Precision form on the GPU: 16-bit resident spectra and Kahan-compensated
pair sums.

16-bit storage is checked against the oracle's storage model
(oracle/precision.py: the same values rounded the same way, everything else
FP64) at the 1e-4 bar of the FP32 path; its cost against the exact
definition is printed, not asserted, since it is a property of the storage
type. Kahan sums are checked against the exact definition."""
import numpy as np
import pytest

import gen
import oracle
from gpu_util import assert_D_close, run_plan, say

pytestmark = pytest.mark.gpu


def _rel(a, b):
    ok = ~np.isnan(b) & (b != 0)
    return float(np.max(np.abs(a[ok] - b[ok]) / np.abs(b[ok])))


@pytest.mark.parametrize("spec", ["bf16", "f16"])
def test_16bit_storage_matches_the_storage_model_f32_frames(spec):
    cfg = gen.config("c1", N=48)
    lags = [0, 1, 2, 4, 8, 16, 47, 48]
    say(f"{spec} storage: 48 frames 128x128 f32, lags 0..48, 64 bins, seed 11")
    f = gen.make_stack(cfg, 11)
    model = oracle.structure_function_stored(f.numpy(), lags, 64, spec)
    exact = oracle.structure_function(f.numpy(), lags, 64)
    D, C, P, st = run_plan(f, lags, 64, "f32", spec=spec)
    assert st == 0 and np.array_equal(C, model["counts"])
    assert np.array_equal(P, model["pairs"])
    worst = assert_D_close(D, model["D"], rtol=1e-4)
    print(f"{spec}: GPU vs storage model {worst:.2e}, storage model vs exact "
          f"{_rel(model['D'], exact['D']):.2e}, GPU vs exact {_rel(D, exact['D']):.2e}")


@pytest.mark.parametrize("spec", ["bf16", "f16"])
def test_16bit_storage_u16_poisson_frames(spec):
    cfg = gen.config("c2", n=128, N=80, lags=[1, 2, 3, 5, 8, 13, 21, 34, 55, 79], n_bins=64)
    say(f"{spec} storage: 80 frames 128x128 u16 Poisson, 10 lags, 64 bins, seed 12")
    f = gen.make_stack(cfg, 12)
    model = oracle.structure_function_stored(f.numpy().astype(np.float64), cfg["lags"], 64, spec)
    exact = oracle.structure_function(f.numpy().astype(np.float64), cfg["lags"], 64)
    D, C, P, st = run_plan(f, cfg["lags"], 64, "u16", spec=spec, chunk=13)
    assert st == 0
    worst = assert_D_close(D, model["D"], rtol=1e-4)
    print(f"{spec} u16: GPU vs storage model {worst:.2e}, storage model vs exact "
          f"{_rel(model['D'], exact['D']):.2e}")


def test_f16_storage_with_window_and_ring_wrap():
    cfg = gen.config("c1", n=64, N=60, n_bins=32)
    lags = [1, 3, 7, 20]
    say("f16 storage: 60 frames 64x64 f32, Hann window, capacity 30, chunks of 7")
    f = gen.make_stack(cfg, 13)
    w = np.outer(np.hanning(64), np.hanning(64)).astype(np.float32)
    import torch
    model = oracle.structure_function_stored(f.numpy(), lags, 32, "f16", window=w)
    D, C, P, st = run_plan(f, lags, 32, "f32", capacity=30, window=torch.from_numpy(w),
                           chunk=7, spec="f16")
    assert st == 0
    assert_D_close(D, model["D"], rtol=1e-4)


@pytest.mark.parametrize("spec", ["bf16", "f16"])
def test_16bit_spectra_copy(spec):
    """nfs_copy_spectrum of 16-bit slots (I_t = paired value + I_0) against the
    storage model's a_t + I_0: equal up to the FP32 transform's error and,
    where the FP32 value sits next to a rounding boundary, one unit in the
    last place of the storage type relative to the stored fluctuation s_t."""
    import paper_1209_3362_amd as nfs
    from gpu_util import require_gpu
    require_gpu()
    cfg = gen.config("c1", N=5)
    say(f"{spec} stored spectra: 5 frames 128x128 f32, seed 14")
    f = gen.make_stack(cfg, 14)
    a, exps = oracle.stored_spectra(f.numpy(), spec)
    norm, means = oracle.normalise(f.numpy())
    I = oracle.spectra(norm)
    plan = nfs.Plan(128, [1], 64, in_dtype="f32", capacity=5, spec=spec)
    plan.push(f.cuda())
    stored = oracle.bin_index(128, 64)[:, :64] >= 0
    for t in range(5):
        g = plan.spectrum(t).cpu().numpy()
        o = (a[t] + I[0])[:, :64]
        o[0, 0] = 128 * 128
        st = (I[t] - means[0] / means[t] * I[0])[:, :64]
        if spec == "bf16":
            ulp = 2.0 ** -7 * np.abs(st)
        else:
            e = int(exps[t])
            ulp = np.maximum(2.0 ** -10 * np.abs(st), 2.0 ** (-24 - e))
        assert g[0, 0] == 128 * 128
        assert np.all(g[~stored] == 0)
        err = np.abs(g - o)[stored]
        lim = 1.01 * ulp[stored] + 2e-6 * np.abs(I[t]).max()
        assert np.all(err <= lim), (t, float((err - lim).max()))
    plan.close()


def test_kahan_matches_the_definition():
    cfg = gen.config("c1")
    say("kahan sums: c1 64 frames 128x128 f32, lags 1,2,4,8,16")
    f = gen.make_stack(cfg, 1)
    ref = oracle.structure_function(f.numpy(), cfg["lags"], 64)
    D, C, P, st = run_plan(f, cfg["lags"], 64, "f32", accum="kahan")
    assert st == 0
    worst = assert_D_close(D, ref["D"], rtol=1e-4)
    print("kahan c1 worst relative error", worst)


def test_kahan_long_sum_of_equal_terms():
    """One cosine mode: every pair of lag tau contributes the same
    (eps n^2)^2 (1 - cos(omega tau)) / 2 per stored mode, so a long plain FP32
    running sum drifts while the compensated one stays at the transform's
    precision."""
    n, N = 16, 4000
    modes = [(3, 2, 0.05, 0.7)]
    say("kahan long sum: 4000 frames 16x16 cosine, lags 1, 5")
    f = gen.cosine_stack(n, N, modes, dtype=np.float32)
    lags = [1, 5]
    bidx = oracle.bin_index(n, 8)
    b0 = bidx[3, 2]
    C0 = oracle.bin_counts(bidx, 8)[b0]
    want = np.array([(0.05 * n * n) ** 2 * (1 - np.cos(0.7 * t)) / C0 for t in lags])
    Dp, _, _, _ = run_plan(f, lags, 8, "f32", capacity=N)
    Dk, _, _, _ = run_plan(f, lags, 8, "f32", capacity=N, accum="kahan")
    ep = np.abs(Dp[:, b0] / want - 1).max()
    ek = np.abs(Dk[:, b0] / want - 1).max()
    print(f"long sum: plain relative error {ep:.2e}, kahan {ek:.2e}")
    assert ek < 1e-5
    assert ek <= ep


def test_kahan_long_sum_across_many_windows():
    """The one-cosine stack of 4000 frames through a 16-slot ring (about 360
    pair windows, pushes of 7 frames): window totals are added with Kahan
    compensation kept across windows, so the compensated sum stays at the
    transform's precision while the plain one drifts."""
    n, N = 16, 4000
    modes = [(3, 2, 0.05, 0.7)]
    say("kahan long sum, 16-slot ring: 4000 frames 16x16 cosine, lags 1, 5, pushes of 7")
    f = gen.cosine_stack(n, N, modes, dtype=np.float32)
    lags = [1, 5]
    bidx = oracle.bin_index(n, 8)
    b0 = bidx[3, 2]
    C0 = oracle.bin_counts(bidx, 8)[b0]
    want = np.array([(0.05 * n * n) ** 2 * (1 - np.cos(0.7 * t)) / C0 for t in lags])
    Dp, _, _, _ = run_plan(f, lags, 8, "f32", capacity=16, chunk=7)
    Dk, _, _, _ = run_plan(f, lags, 8, "f32", capacity=16, chunk=7, accum="kahan")
    ep = np.abs(Dp[:, b0] / want - 1).max()
    ek = np.abs(Dk[:, b0] / want - 1).max()
    print(f"long sum over many windows: plain relative error {ep:.2e}, kahan {ek:.2e}")
    assert ek < 1e-5
    assert ek <= ep


def test_kahan_across_ring_windows():
    """Kahan sums over several pair windows (ring smaller than the stack,
    uneven pushes) against the exact definition."""
    cfg = gen.config("c1", N=90)
    lags = [1, 3, 10, 25]
    say("kahan sums with ring wrap: 90 frames 128x128 f32, capacity 40, chunks of 11")
    f = gen.make_stack(cfg, 15)
    ref = oracle.structure_function(f.numpy(), lags, 64)
    D, C, P, st = run_plan(f, lags, 64, "f32", capacity=40, chunk=11, accum="kahan")
    assert st == 0 and np.array_equal(P, ref["pairs"])
    assert_D_close(D, ref["D"], rtol=1e-4)
