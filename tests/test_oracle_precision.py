"""Pins of the oracle's 16-bit storage model (oracle/precision.py), CPU only.

The rounding functions are pinned by hand-computed values, by the library
conversions they must agree with, and by their error bounds; the stored
spectra by the exact identity they reduce to without rounding."""
import math

import numpy as np
import pytest
import torch

import gen
import oracle


def test_round_bf16_hand_values():
    x = np.array([1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, math.pi, 1 + 2.0 ** -8 + 2.0 ** -20,
                  0.0, 2.0 ** 40, 3.0 * 2.0 ** -30])
    want = np.array([1.0, 1.0, 1 + 2.0 ** -6, 3.140625, 1 + 2.0 ** -7,
                     0.0, 2.0 ** 40, 3.0 * 2.0 ** -30])
    assert np.array_equal(oracle.round_bf16(x), want)
    assert np.array_equal(oracle.round_bf16(-x), -want)


def test_round_bf16_matches_torch_on_float32_values():
    rng = np.random.default_rng(7)
    x = (rng.standard_normal(20000) * np.exp(rng.uniform(-20, 20, 20000))).astype(np.float32)
    t = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(oracle.round_bf16(x.astype(np.float64)), t)


def test_round_bf16_error_bound_and_idempotence():
    rng = np.random.default_rng(8)
    x = rng.standard_normal(10000) * 1e3
    r = oracle.round_bf16(x)
    assert np.all(np.abs(r - x) <= 2.0 ** -8 * np.abs(x))
    assert np.array_equal(oracle.round_bf16(r), r)


def test_f16_exponent():
    assert oracle.f16_exponent(65504.0) == 0
    assert oracle.f16_exponent(65505.0) == -1
    assert oracle.f16_exponent(1.0) == 15
    assert oracle.f16_exponent(0.0) == 0
    rng = np.random.default_rng(9)
    for b in np.exp(rng.uniform(-30, 30, 500)):
        e = oracle.f16_exponent(b)
        assert b * 2.0 ** e <= 65504.0 < b * 2.0 ** (e + 1)


def test_round_f16_matches_numpy_half_and_its_bound():
    rng = np.random.default_rng(10)
    x = rng.standard_normal(5000) * 50.0
    for e in (-3, 0, 7):
        r = oracle.round_f16_scaled(x, e)
        assert np.array_equal(r, (x * 2.0 ** e).astype(np.float16).astype(np.float64) / 2.0 ** e)
        # 11 significant bits in the normal range, absolute 2^-25 below it
        assert np.all(np.abs(r - x) <= np.maximum(2.0 ** -11 * np.abs(x), 2.0 ** (-25 - e)))


def _small_stack(N=14, n=32, seed=3):
    cfg = gen.config("c1", n=n, N=N, n_bins=n // 2)
    return gen.make_stack(cfg, seed).numpy()


def test_stored_without_rounding_is_the_plain_definition():
    f = _small_stack()
    lags = [0, 1, 2, 5, 13, 14]
    ref = oracle.structure_function(f, lags, 16, return_power=True)
    got = oracle.structure_function_stored(f, lags, 16, "none", return_power=True)
    ok = ~np.isnan(ref["D"])
    assert np.array_equal(np.isnan(ref["D"]), np.isnan(got["D"]))
    assert np.allclose(got["D"][ok], ref["D"][ok], rtol=1e-12, atol=0)
    fin = ~np.isnan(ref["P"])
    assert np.abs(got["P"][fin] - ref["P"][fin]).max() <= 1e-12 * np.abs(ref["P"][fin]).max()


@pytest.mark.parametrize("store", ["bf16", "f16"])
def test_stored_values_keep_their_rounding_bound(store):
    f = _small_stack(N=10, n=16, seed=4)
    a, exps = oracle.stored_spectra(f, store)
    exact, _ = oracle.stored_spectra(f, "none")
    norm, means = oracle.normalise(f)
    I = oracle.spectra(norm)
    ratio = means[0] / means
    for t in range(len(f)):
        s = I[t] - ratio[t] * I[0]
        err = a[t] - exact[t]
        err[0, 0] = 0.0
        s[0, 0] = 0.0
        if store == "bf16":
            lim_re = 2.0 ** -8 * np.abs(s.real)
            lim_im = 2.0 ** -8 * np.abs(s.imag)
        else:
            e = int(exps[t])
            # the exponent's bound covers every coefficient (|F[v](k)| <= sum |v|)
            assert np.abs(s).max() * 2.0 ** e <= 65504.0
            lim_re = np.maximum(2.0 ** -11 * np.abs(s.real), 2.0 ** (-25 - e))
            lim_im = np.maximum(2.0 ** -11 * np.abs(s.imag), 2.0 ** (-25 - e))
        assert np.all(np.abs(err.real) <= lim_re * (1 + 1e-9) + 1e-12)
        assert np.all(np.abs(err.imag) <= lim_im * (1 + 1e-9) + 1e-12)
    # the reference frame stores exactly zero fluctuation
    assert np.all(a[0] == exact[0])


@pytest.mark.parametrize("store", ["bf16", "f16"])
def test_bins_version_matches_full_version(store):
    f = _small_stack(N=12, n=32, seed=5)
    lags = [1, 3, 11, 12]
    full = oracle.structure_function_stored(f, lags, 16, store)
    bins = [0, 1, 7, 15]
    part = oracle.structure_function_stored_bins(f, lags, 16, bins, store, workers=2)
    ok = ~np.isnan(full["D"][:, bins])
    assert np.array_equal(np.isnan(part["D"]), ~ok)
    assert np.allclose(part["D"][ok], full["D"][:, bins][ok], rtol=1e-12, atol=0)
    assert np.array_equal(part["counts"], full["counts"][bins])
