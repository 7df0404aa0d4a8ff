"""Plain FP64 definition of the structure function of Eq. (1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Notation: frames i_t(x), t = 0..N-1, of n x n pixels; k = (k_y, k_x) are
signed integer frequencies in transform order; tau is a lag in frames;
n_bins is the number of |q| bins. The steps are, in the paper's order:

  O1-O2  divide every image by its spatial average (method section, the
         paragraph that introduces the image differences Delta i_m);
  O3     spatial Fourier transform of each normalised image, once per image
         (linearity of the transform, processing section);
  O4     for each lag tau, average |I_t(k) - I_{t+tau}(k)|^2 over all pairs
         (t, t+tau): the time average that replaces the ensemble average of
         Eq. (1) for stationary dynamics (text after Eq. (1)), stored per
         delay as in the "differences area" of Fig. 2;
  O5-O6  azimuthal average over rings of |q| (text after Eq. (1), Fig. 1e-f).

Readings where the paper is silent: the forward transform is unnormalised
with kernel exp(-2*pi*i*k.x/n), so a mean-normalised image has
I(0) = n^2 exactly (dividing the transform by its zero-frequency value, as in
the processing section, is the same thing up to that constant); I_t(0) is set
to n^2 exactly; every pair (t, t+tau) counts with equal weight; bins are
half-open rings of equal width in q = 2*pi*|k|/n over [0, pi), bin
b(k) = isqrt(|k|^2 * n_bins^2) // (n/2), and modes with b >= n_bins are left
out.

Everything is computed directly: a full-plane complex transform (never a
half-plane real transform), an explicit loop over pairs and a Python-integer
bin index.
"""
import math

import numpy as np


def normalise(frames, window=None):
    """O1-O2: u_t = w * i_t, then i'_t = u_t / mean_x(u_t).

    Returns (normalised frames float64 [N][n][n], means float64 [N]).
    Raises ValueError when a frame's mean is not positive and finite.
    """
    u = np.asarray(frames, dtype=np.float64)
    if u.ndim != 3 or u.shape[1] != u.shape[2]:
        raise ValueError("frames must be [N][n][n]")
    if window is not None:
        u = u * np.asarray(window, dtype=np.float64)[None, :, :]
    n = u.shape[1]
    means = u.reshape(u.shape[0], -1).sum(axis=1) / float(n * n)
    if not np.all(np.isfinite(means)) or np.any(means <= 0.0):
        raise ValueError("a frame has a non-positive or non-finite mean")
    return u / means[:, None, None], means


def spectra(norm_frames):
    """O3: I_t(k) = sum_x i'_t(x) exp(-2*pi*i*(k_y*y + k_x*x)/n), full plane.

    The zero-frequency coefficient of a mean-normalised image equals n^2; it
    is set to exactly n^2.
    """
    x = np.asarray(norm_frames, dtype=np.float64)
    n = x.shape[-1]
    out = np.fft.fft2(x, axes=(-2, -1))
    out[..., 0, 0] = float(n * n)
    return out


def pair_power(spec, lags):
    """O4: P_tau(k) = 1/(N - tau) * sum_{t=0}^{N-1-tau} |I_t(k) - I_{t+tau}(k)|^2.

    `spec` is [N][...] complex (any trailing shape of modes). Returns
    (P float64 [L][...], pairs int64 [L]). A lag with N - tau <= 0 has no
    pair: its row is NaN and its pair count 0. Lag 0 gives exactly 0.
    """
    spec = np.asarray(spec)
    N = spec.shape[0]
    P = np.empty((len(lags),) + spec.shape[1:], dtype=np.float64)
    pairs = np.zeros(len(lags), dtype=np.int64)
    for i, tau in enumerate(lags):
        tau = int(tau)
        if tau < 0:
            raise ValueError("lags must be non-negative")
        npair = N - tau
        if npair <= 0:
            P[i] = np.nan
            continue
        acc = np.zeros(spec.shape[1:], dtype=np.float64)
        for t in range(npair):
            d = spec[t] - spec[t + tau]
            acc += d.real * d.real + d.imag * d.imag
        P[i] = acc / npair
        pairs[i] = npair
    return P, pairs


def bin_index(n, n_bins):
    """O5: bin of every full-plane mode, -1 for modes outside every bin.

    b(k) = isqrt((k_x^2 + k_y^2) * n_bins^2) // (n/2), with k in transform
    order; bins are half-open rings of width pi/n_bins in q = 2*pi*|k|/n.
    """
    n = int(n)
    n_bins = int(n_bins)
    half = n // 2
    ks = [j if j < (n + 1) // 2 else j - n for j in range(n)]
    b = np.empty((n, n), dtype=np.int64)
    nb2 = n_bins * n_bins
    for iy, ky in enumerate(ks):
        for ix, kx in enumerate(ks):
            v = math.isqrt((kx * kx + ky * ky) * nb2) // half
            b[iy, ix] = v if v < n_bins else -1
    return b


def bin_counts(bidx, n_bins):
    """C_b = number of full-plane modes with b(k) = b."""
    flat = np.asarray(bidx).ravel()
    return np.bincount(flat[flat >= 0], minlength=n_bins).astype(np.int64)


def azimuthal_average(P, bidx, n_bins):
    """O6: D(b, tau) = (1/C_b) * sum_{k : b(k) = b} P_tau(k); NaN for empty bins.

    P is [L][modes...] with the same trailing shape as `bidx`.
    """
    P = np.asarray(P, dtype=np.float64)
    flat_b = np.asarray(bidx).ravel()
    flat_P = P.reshape(P.shape[0], -1)
    D = np.full((P.shape[0], n_bins), np.nan, dtype=np.float64)
    counts = np.bincount(flat_b[flat_b >= 0], minlength=n_bins)
    for b in range(n_bins):
        if counts[b] == 0:
            continue
        sel = flat_b == b
        D[:, b] = flat_P[:, sel].sum(axis=1) / float(counts[b])
    return D


def structure_function(frames, lags, n_bins, window=None, return_power=False):
    """Steps O1-O6 on a whole stack.

    Returns a dict with D float64 [L][n_bins], counts int64 [n_bins],
    pairs int64 [L], and with return_power the 2D spectra P [L][n][n].
    """
    norm, _ = normalise(frames, window)
    n = norm.shape[1]
    spec = spectra(norm)
    P, pairs = pair_power(spec, lags)
    bidx = bin_index(n, n_bins)
    out = dict(D=azimuthal_average(P, bidx, n_bins),
               counts=bin_counts(bidx, n_bins), pairs=pairs)
    if return_power:
        out["P"] = P
    return out


def structure_function_bins(frames, lags, n_bins, bins, window=None, workers=1):
    """Steps O1-O6 for a few bins only, for stacks too large to hold in FP64.

    Frames are normalised and transformed one at a time (by `workers`
    threads, each doing whole frames) and only the modes of the requested
    bins are kept. Returns D float64 [L][len(bins)], counts int64
    [len(bins)] and pairs int64 [L], equal to the matching columns of
    structure_function().
    """
    N = len(frames)
    n = int(np.asarray(frames[0]).shape[-1])
    bidx = bin_index(n, n_bins)
    bins = [int(b) for b in bins]
    sel = np.isin(bidx, bins)
    keep = np.empty((N, int(sel.sum())), dtype=np.complex128)
    w = None if window is None else np.asarray(window, dtype=np.float64)

    def one(t):
        norm, _ = normalise(np.asarray(frames[t])[None], w)
        keep[t] = spectra(norm)[0][sel]

    if workers > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max_workers=workers) as ex:
            list(ex.map(one, range(N)))
    else:
        for t in range(N):
            one(t)
    P, pairs = pair_power(keep, lags)
    sub_b = bidx[sel]
    counts_all = bin_counts(bidx, n_bins)
    D = np.empty((len(lags), len(bins)), dtype=np.float64)
    for j, b in enumerate(bins):
        m = sub_b == b
        D[:, j] = P[:, m].sum(axis=1) / float(counts_all[b]) if counts_all[b] else np.nan
    return dict(D=D, counts=counts_all[bins], pairs=pairs)
