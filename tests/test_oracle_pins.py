"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test targets one step (O1-O6 in the oracle's docstring) and is chosen so
that a plausible slip there (a dropped normalisation, a wrong sign or index,
a wrong pair set, an off-by-one ring) fails it.
"""
import cmath
import math

import numpy as np
import pytest

import gen
import oracle


def brute_dft2(img):
    """Explicit double sum of exp(-2*pi*i*(ky*y + kx*x)/n), Python complex."""
    n = img.shape[0]
    out = np.empty((n, n), dtype=np.complex128)
    for ky in range(n):
        for kx in range(n):
            s = 0j
            for y in range(n):
                for x in range(n):
                    s += img[y, x] * cmath.exp(-2j * math.pi * ((ky * y + kx * x) % n) / n)
            out[ky, kx] = s
    return out


def dft_matrix(n):
    """W[k, j] = exp(-2*pi*i*k*j/n), built from math.cos/math.sin."""
    W = np.empty((n, n), dtype=np.complex128)
    for k in range(n):
        for j in range(n):
            a = -2.0 * math.pi * ((k * j) % n) / n
            W[k, j] = complex(math.cos(a), math.sin(a))
    return W


def rand_frames(rng, N, n, lo=0.5, hi=2.0):
    return rng.uniform(lo, hi, size=(N, n, n))


@pytest.mark.parametrize("n", [4, 8, 16])
def test_spectra_match_brute_force_dft(n):
    rng = np.random.default_rng(100 + n)
    frames = rand_frames(rng, 2, n)
    norm, _ = oracle.normalise(frames)
    spec = oracle.spectra(norm)
    for t in range(2):
        ref = brute_dft2(norm[t])
        scale = np.abs(ref).max()
        assert np.abs(spec[t] - ref).max() <= 1e-12 * scale
        # the mean-normalised image sums to n^2
        assert abs(ref[0, 0] - n * n) <= 1e-12 * n * n
        assert spec[t][0, 0] == n * n


def test_divide_by_dc_equals_mean_normalisation():
    # Processing section: dividing each image transform by its zero-frequency
    # value replaces the spatial-mean normalisation; n^2 F[u]/F[u](0) must
    # equal the transform of u/<u>.
    rng = np.random.default_rng(7)
    n = 8
    u = rand_frames(rng, 3, n, 10.0, 4000.0)
    spec = oracle.spectra(oracle.normalise(u)[0])
    for t in range(3):
        Fu = brute_dft2(u[t])
        lhs = n * n * Fu / Fu[0, 0]
        assert np.abs(lhs - spec[t]).max() <= 1e-13 * np.abs(lhs).max()


def test_normalisation_makes_frame_scale_irrelevant():
    rng = np.random.default_rng(8)
    f = rand_frames(rng, 9, 16)
    a = oracle.structure_function(f, [1, 2, 5], 8)["D"]
    b = oracle.structure_function(f * 1234.5, [1, 2, 5], 8)["D"]
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=0)


def test_linearity_fft_of_differences():
    # Processing section: transforming single images and differencing the
    # transforms replaces transforming each of the N(N-1)/2 image differences.
    rng = np.random.default_rng(12)
    N, n = 12, 16
    frames = rand_frames(rng, N, n)
    norm, _ = oracle.normalise(frames)
    W = dft_matrix(n)
    lags = list(range(0, N + 2))
    P, pairs = oracle.pair_power(oracle.spectra(norm), lags)
    for i, tau in enumerate(lags):
        if tau >= N:
            assert pairs[i] == 0 and np.all(np.isnan(P[i]))
            continue
        acc = np.zeros((n, n))
        for t in range(N - tau):
            d = W @ (norm[t] - norm[t + tau]) @ W.T
            acc += np.abs(d) ** 2
        acc /= (N - tau)
        assert pairs[i] == N - tau
        scale = max(acc.max(), 1e-300)
        # the DC term of a difference is zero mathematically; both sides agree
        assert np.abs(P[i] - acc).max() <= 1e-12 * scale + 1e-18


def test_parseval_against_real_space():
    rng = np.random.default_rng(3)
    N, n = 20, 32
    frames = rand_frames(rng, N, n)
    norm, _ = oracle.normalise(frames)
    lags = [1, 3, 7, 19]
    P, _ = oracle.pair_power(oracle.spectra(norm), lags)
    for i, tau in enumerate(lags):
        real = sum(((norm[t] - norm[t + tau]) ** 2).sum() for t in range(N - tau))
        real *= n * n / (N - tau)
        assert abs(P[i].sum() - real) <= 1e-12 * real


def test_lag_zero_is_exactly_zero():
    c = gen.config("c1", N=10)
    f = gen.make_stack(c, 5).numpy()
    r = oracle.structure_function(f, [0, 1], 64)
    assert np.all(r["D"][0] == 0.0)
    assert np.all(r["D"][1, 1:] > 0.0)
    # with n_bins = n/2, bin 0 holds only k = 0, whose coefficient is n^2 in
    # every frame, so its differences vanish exactly
    assert r["D"][1, 0] == 0.0
    assert r["pairs"].tolist() == [10, 9]


def test_power_is_symmetric_under_k_to_minus_k():
    rng = np.random.default_rng(4)
    N, n = 6, 16
    P, _ = oracle.pair_power(oracle.spectra(oracle.normalise(rand_frames(rng, N, n))[0]), [1, 2])
    neg = (-np.arange(n)) % n
    for i in range(2):
        mirrored = P[i][np.ix_(neg, neg)]
        assert np.abs(P[i] - mirrored).max() <= 1e-12 * P[i].max()


def test_bin_counts_by_hand():
    # Rings of unit width when n_bins = n/2. Ring 0: only k = 0. Ring 1
    # (1 <= |k| < 2): (+-1,0),(0,+-1),(+-1,+-1). Ring 2 (4 <= |k|^2 < 9):
    # (+-2,0),(0,+-2), |k|^2=5: 8 modes, |k|^2=8: 4 modes. Ring 3 (9..15):
    # |k|^2 = 9: 4, 10: 8, 13: 8. Ring 4 (16..24): 16: 4, 17: 8, 18: 4,
    # 20: 8. Ring 5 (25..35): 25: 12, 26: 8, 29: 8, 32: 4, 34: 8.
    C = oracle.bin_counts(oracle.bin_index(64, 32), 32)
    assert C[:6].tolist() == [1, 8, 16, 20, 24, 40]


@pytest.mark.parametrize("n", [8, 16, 64, 128])
def test_bins_cover_exactly_the_disc(n):
    # Whatever the bin count, the binned modes are the lattice points with
    # |k| < n/2, counted here by brute force.
    half = n // 2
    ks = [j if j < n // 2 else j - n for j in range(n)]
    inside = sum(1 for a in ks for b in ks if a * a + b * b < half * half)
    for nb in sorted({1, 3, max(1, n // 4), n // 2}):
        C = oracle.bin_counts(oracle.bin_index(n, nb), nb)
        assert C.sum() == inside
        assert np.all(C > 0)


@pytest.mark.parametrize("n,nb", [(16, 8), (16, 3), (64, 32), (64, 5), (128, 64)])
def test_bin_index_is_the_ring_of_q(n, nb):
    # Bins are rings of width dq = pi/nb in q = 2*pi*|k|/n; checked with
    # floating point away from ring edges and exactly with integers.
    b = oracle.bin_index(n, nb)
    half = n // 2
    dq = math.pi / nb
    for iy in range(n):
        ky = iy if iy < n // 2 else iy - n
        for ix in range(n):
            kx = ix if ix < n // 2 else ix - n
            r2 = kx * kx + ky * ky
            if r2 >= half * half:
                assert b[iy, ix] == -1
                continue
            x = (2 * math.pi * math.sqrt(r2) / n) / dq
            if abs(x - round(x)) > 1e-9:
                assert b[iy, ix] == int(math.floor(x))
            bb = b[iy, ix]
            assert (bb * half) ** 2 <= r2 * nb * nb < ((bb + 1) * half) ** 2


def test_c1_bin_totals_match_lattice_count():
    n, nb = 128, 64
    C = oracle.bin_counts(oracle.bin_index(n, nb), nb)
    inside = sum(1 for a in range(-64, 64) for b in range(-64, 64) if a * a + b * b < 64 * 64)
    assert C.sum() == inside == 12849
    assert n * n - inside == 3535


def _single_mode_expect(n, nb, eps, omega, tau, C):
    return (eps * n * n) ** 2 * (1.0 - math.cos(omega * tau)) / C


@pytest.mark.parametrize("ky,kx", [(3, 5), (-7, 2), (0, 9), (11, 0)])
def test_closed_form_single_cosine(ky, kx):
    n, N, nb = 32, 24, 16
    eps, omega = 0.05, 0.37
    f = gen.cosine_stack(n, N, [(ky, kx, eps, omega)])
    lags = [1, 2, 5, 11, 23]
    r = oracle.structure_function(f, lags, nb)
    bidx = oracle.bin_index(n, nb)
    b0 = bidx[ky % n, kx % n]
    C = r["counts"]
    for i, tau in enumerate(lags):
        want = _single_mode_expect(n, nb, eps, omega, tau, C[b0])
        assert abs(r["D"][i, b0] - want) <= 1e-12 * want
        others = np.delete(r["D"][i], b0)
        assert np.abs(others).max() <= 1e-12 * want


def test_closed_form_multi_cosine():
    n, N, nb = 32, 30, 16
    modes = [(1, 2, 0.03, 0.2), (4, -3, 0.02, 1.1), (0, 7, 0.05, 2.5),
             (-6, -6, 0.01, 0.05), (9, 1, 0.04, 0.7)]
    f = gen.cosine_stack(n, N, modes)
    lags = [1, 3, 4, 9, 17, 29]
    r = oracle.structure_function(f, lags, nb)
    bidx = oracle.bin_index(n, nb)
    C = r["counts"]
    want = np.zeros((len(lags), nb))
    for (ky, kx, eps, om) in modes:
        b = bidx[ky % n, kx % n]
        for i, tau in enumerate(lags):
            want[i, b] += (eps * n * n) ** 2 * (1 - math.cos(om * tau)) / C[b]
    scale = want.max()
    assert np.abs(r["D"] - want).max() <= 1e-12 * scale


def test_lag_beyond_stack_gives_nan_and_no_pairs():
    rng = np.random.default_rng(9)
    f = rand_frames(rng, 5, 8)
    r = oracle.structure_function(f, [1, 4, 5, 9], 4)
    assert r["pairs"].tolist() == [4, 1, 0, 0]
    assert np.all(np.isnan(r["D"][2:])) and np.all(np.isfinite(r["D"][:2]))


def test_degenerate_frame_is_rejected():
    f = np.ones((3, 8, 8))
    f[1] = 0.0
    with pytest.raises(ValueError):
        oracle.structure_function(f, [1], 4)


def test_bins_subset_matches_full():
    c = gen.config("c1", N=20)
    f = gen.make_stack(c, 11).numpy()
    full = oracle.structure_function(f, c["lags"], c["n_bins"])
    bins = [0, 1, 7, 40, 63]
    sub = oracle.structure_function_bins(f, c["lags"], c["n_bins"], bins)
    np.testing.assert_allclose(sub["D"], full["D"][:, bins], rtol=1e-12, atol=0)
    assert sub["counts"].tolist() == full["counts"][bins].tolist()
    assert sub["pairs"].tolist() == full["pairs"].tolist()
