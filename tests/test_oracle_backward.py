"""Pins of the oracle's gradient (oracle/backward.py), CPU only.

The adjoint is checked against central differences of the plain FP64
definition, against reverse-mode automatic differentiation of a separate
torch float64 implementation of the definition, and against two exact
invariances of D: every frame may be scaled (each image is divided by its
own mean) and so may the window."""
import numpy as np
import pytest
import torch

import gen
import oracle

LAGS = [0, 1, 2, 5, 9, 10, 12]


def _case(n=16, N=10, n_bins=8, seed=31):
    cfg = gen.config("c1", n=n, N=N, n_bins=n_bins)
    f = gen.make_stack(cfg, seed).numpy().astype(np.float64)
    rng = np.random.default_rng(seed)
    w = rng.uniform(0.5, 1.5, (n, n))
    G = rng.standard_normal((len(LAGS), n_bins))
    return f, w, G


def _loss(f, w, G, n_bins):
    D = oracle.structure_function(f, LAGS, n_bins, window=w)["D"]
    ok = ~np.isnan(D)
    return float((G[ok] * D[ok]).sum())


def test_matches_central_differences():
    f, w, G = _case()
    grad = oracle.structure_function_grad(f, LAGS, 8, G, window=w)
    rng = np.random.default_rng(5)
    scale = max(np.abs(grad["frames"]).max(), 1e-300)
    for _ in range(32):
        t, y, x = rng.integers(0, f.shape[0]), rng.integers(0, 16), rng.integers(0, 16)
        h = 1e-5 * abs(f[t, y, x])
        fp, fm = f.copy(), f.copy()
        fp[t, y, x] += h
        fm[t, y, x] -= h
        fd = (_loss(fp, w, G, 8) - _loss(fm, w, G, 8)) / (2 * h)
        assert abs(fd - grad["frames"][t, y, x]) <= 1e-6 * scale, (t, y, x)
    wscale = np.abs(grad["window"]).max()
    for _ in range(32):
        y, x = rng.integers(0, 16), rng.integers(0, 16)
        h = 1e-5 * abs(w[y, x])
        wp, wm = w.copy(), w.copy()
        wp[y, x] += h
        wm[y, x] -= h
        fd = (_loss(f, wp, G, 8) - _loss(f, wm, G, 8)) / (2 * h)
        assert abs(fd - grad["window"][y, x]) <= 1e-6 * wscale, (y, x)


def _torch_D(f, w, n_bins):
    """The definition again, in torch float64, for autograd."""
    N, n = f.shape[0], f.shape[1]
    u = f * w
    m = u.mean(dim=(1, 2), keepdim=True)
    I = torch.fft.fft2(u / m)
    keep = torch.ones((n, n), dtype=torch.float64)
    keep[0, 0] = 0.0
    I = I * keep + float(n * n) * (1.0 - keep)
    bidx = torch.from_numpy(oracle.bin_index(n, n_bins))
    onehot = torch.zeros((n * n, n_bins), dtype=torch.float64)
    inside = (bidx >= 0).reshape(-1)
    onehot[inside.nonzero().squeeze(1), bidx.reshape(-1)[inside]] = 1.0
    C = onehot.sum(0)
    rows = []
    for tau in LAGS:
        if N - tau <= 0:
            rows.append(torch.full((n_bins,), float("nan"), dtype=torch.float64))
            continue
        d = I[: N - tau] - I[tau:]
        P = (d.real ** 2 + d.imag ** 2).mean(0).reshape(-1)
        rows.append((P @ onehot) / C)
    return torch.stack(rows)


def test_matches_torch_autograd():
    f, w, G = _case(n=32, N=14, n_bins=16, seed=32)
    ft = torch.tensor(f, requires_grad=True)
    wt = torch.tensor(w, requires_grad=True)
    D = _torch_D(ft, wt, 16)
    ok = ~torch.isnan(D)
    L = (torch.from_numpy(G)[ok] * D[ok]).sum()
    L.backward()
    grad = oracle.structure_function_grad(f, LAGS, 16, G, window=w)
    D0 = oracle.structure_function(f, LAGS, 16, window=w)["D"]
    assert np.allclose(D.detach().numpy(), D0, rtol=1e-12, atol=0, equal_nan=True)
    gf, gw = ft.grad.numpy(), wt.grad.numpy()
    assert np.abs(grad["frames"] - gf).max() <= 1e-10 * np.abs(gf).max()
    assert np.abs(grad["window"] - gw).max() <= 1e-10 * np.abs(gw).max()


def test_scale_invariance():
    """D does not change when one frame, or the window, is multiplied by a
    constant, so the gradient is orthogonal to each frame and to the window
    (Euler's identity for functions homogeneous of degree 0)."""
    f, w, G = _case(n=32, N=12, n_bins=16, seed=33)
    grad = oracle.structure_function_grad(f, LAGS, 16, G, window=w)
    for t in range(f.shape[0]):
        dot = (f[t] * grad["frames"][t]).sum()
        assert abs(dot) <= 1e-11 * np.abs(f[t] * grad["frames"][t]).sum()
    dot = (w * grad["window"]).sum()
    assert abs(dot) <= 1e-11 * np.abs(w * grad["window"]).sum()


def test_zero_cases():
    f, w, G = _case()
    z = oracle.structure_function_grad(f, LAGS, 8, np.zeros_like(G), window=w)
    assert not z["frames"].any() and not z["window"].any()
    # Lag 0 (d = 0 exactly) and delays with no pair carry no gradient.
    G2 = np.zeros_like(G)
    G2[LAGS.index(0)] = 1.0
    G2[LAGS.index(10)] = 1.0
    G2[LAGS.index(12)] = 1.0
    z = oracle.structure_function_grad(f, LAGS, 8, G2, window=w)
    assert not z["frames"].any() and not z["window"].any()


def test_rejects_bad_upstream_shape():
    f, w, G = _case()
    with pytest.raises(ValueError):
        oracle.structure_function_grad(f, LAGS, 8, G[:, :4], window=w)
