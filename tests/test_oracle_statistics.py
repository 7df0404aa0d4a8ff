"""Statistical pins of the oracle: Eq. (1) recovered from a known model.

Frames come from the synthetic generator with a flat beam of c counts, a
fluctuation amplitude eps, Ornstein-Uhlenbeck modes with f(q, tau) =
exp(-Gamma(q) tau) and additive white noise of sigma counts. For that model
every mode k != 0 has

  E[P_tau(k)] = eps^2 c_s^2 n^4 A(k)^2 (1 - exp(-Gamma(k) tau)) + 2 n^2 sigma^2 / c^2,

the form of Eq. (1) with T(q) I_s(q) ~ A(q)^2 and a flat noise floor B. The
tests are seeded, so they are deterministic; the tolerances sit several
standard errors from the observed deviations.
"""
import numpy as np
import pytest
from scipy.optimize import least_squares

import gen
import oracle

OU = dict(name="ou", n=32, N=1500, dtype="f32", peak=1000.0, eps=0.05,
          gamma_a=0.05, gamma_b=1.0, noise="gauss", noise_sigma=2.0,
          lags=[1, 2, 4, 8, 16, 32, 64], n_bins=16)


def _model_terms(cfg):
    amp, gam, c_s = gen.frames.field_model(cfg)
    return amp.numpy(), gam.numpy(), float(c_s)


def test_bin_averages_match_the_model_expectation():
    cfg = dict(OU)
    f = gen.make_stack(cfg, 21, flat_beam=True).numpy()
    r = oracle.structure_function(f, cfg["lags"], cfg["n_bins"])
    amp, gam, c_s = _model_terms(cfg)
    n, c, eps, sig = cfg["n"], cfg["peak"], cfg["eps"], cfg["noise_sigma"]
    bidx = oracle.bin_index(n, cfg["n_bins"])
    B = 2.0 * n * n * sig ** 2 / c ** 2
    for i, tau in enumerate(cfg["lags"]):
        Pk = eps ** 2 * c_s ** 2 * n ** 4 * amp ** 2 * (1.0 - np.exp(-gam * tau)) + B
        Pk[0, 0] = 0.0
        E = oracle.azimuthal_average(Pk[None], bidx, cfg["n_bins"])[0]
        z = r["D"][i, 1:] / E[1:] - 1.0
        assert np.abs(z).max() < 0.08
        assert np.abs(z).mean() < 0.015
    assert np.all(r["D"][:, 0] == 0.0)


def test_gamma_of_q_and_noise_floor_are_recovered_by_a_fit():
    cfg = dict(OU, lags=list(range(1, 81)))
    f = gen.make_stack(cfg, 22, flat_beam=True).numpy()
    r = oracle.structure_function(f, cfg["lags"], cfg["n_bins"])
    amp, _, _ = _model_terms(cfg)
    n = cfg["n"]
    bidx = oracle.bin_index(n, cfg["n_bins"])
    ks = np.fft.fftfreq(n) * n
    q2 = (2 * np.pi / n) ** 2 * (ks[:, None] ** 2 + ks[None, :] ** 2)
    tau = np.array(cfg["lags"], dtype=float)
    D = r["D"][:, 1:]

    def model(p):
        s, ga, gb, B = p
        out = np.empty_like(D)
        for b in range(1, cfg["n_bins"]):
            m = bidx == b
            a2 = amp[m] ** 2
            g = ga + gb * q2[m]
            out[:, b - 1] = s * (a2[None, :] * (1 - np.exp(-g[None, :] * tau[:, None]))).mean(axis=1) + B
        return out

    fit = least_squares(lambda p: ((model(p) - D) / D).ravel(),
                        x0=[D.max() / amp.max() ** 2, 0.1, 0.5, 1e-3], x_scale="jac")
    s, ga, gb, B = fit.x
    B_true = 2.0 * n * n * cfg["noise_sigma"] ** 2 / cfg["peak"] ** 2
    assert abs(ga / cfg["gamma_a"] - 1) < 0.12
    assert abs(gb / cfg["gamma_b"] - 1) < 0.05
    assert abs(B / B_true - 1) < 0.05


def test_pure_noise_gives_a_flat_floor():
    cfg = dict(OU, eps=0.0, lags=[1, 2, 5, 13, 40])
    f = gen.make_stack(cfg, 23, flat_beam=True).numpy()
    r = oracle.structure_function(f, cfg["lags"], cfg["n_bins"])
    n = cfg["n"]
    B = 2.0 * n * n * cfg["noise_sigma"] ** 2 / cfg["peak"] ** 2
    ratio = r["D"][:, 1:] / B
    assert abs(ratio.mean() - 1.0) < 0.01
    assert np.abs(ratio - 1.0).max() < 0.1
