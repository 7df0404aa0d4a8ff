"""16-bit storage of the resident spectra, FP64 (precision form).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The method keeps one transform per image and differences stored transforms
(processing section, the store of image FFTs of Fig. 2). Storing them in a
16-bit type keeps 8 (BF16) or 11 (FP16) significant bits, so the static
illumination, whose low-q coefficients are orders of magnitude larger than
the fluctuations, would leave nothing of the fluctuations. A fixed
reference spectrum is therefore subtracted before rounding, which leaves
every difference I_t - I_t' unchanged in exact arithmetic:

  u_t = w * i_t, m_t = mean_x(u_t), I_t = F[u_t / m_t] (with I_t(0) = n^2);
  the first frame u_0 is the reference;
  s_t = F[u_t - u_0] / m_t = I_t - (m_0 / m_t) * I_0          (stored value)
  a_t = R(s_t) + (m_0 / m_t - 1) * I_0                       (paired value)

where R rounds the real and imaginary parts to the storage type: BF16
directly (round to nearest, ties to even, 8 significant bits), FP16 after
scaling by 2^e_t, with e_t the largest integer such that
2^e_t * B_t <= 65504 for the bound B_t = sum_x |u_t - u_0| / m_t >= |s_t(k)|
(so no value overflows; e_t = 0 when B_t = 0). With R the identity, a_t =
I_t exactly. The zero-frequency coefficient, whose differences are zero,
is set to n^2 in every a_t.

D(b, tau) then follows steps O4-O6 of the plain definition on a_t.
"""
import math

import numpy as np

from .dda import azimuthal_average, bin_counts, bin_index, normalise, pair_power, spectra

F16_MAX = 65504.0


def round_bf16(x):
    """Round float64 values to the nearest BF16 value (8 significant bits,
    ties to even); zeros, infinities and NaN pass through."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)  # x = m * 2^e, 0.5 <= |m| < 1
    # 8 significant bits: scale the mantissa to [128, 256), round half to even.
    r = np.ldexp(np.rint(np.ldexp(m, 8)), e - 8)
    return np.where(np.isfinite(x), r, x)


def f16_exponent(bound):
    """Largest integer e with bound * 2^e <= 65504 (0 for bound <= 0),
    clamped to [-100, 100]."""
    b = float(bound)
    if not (b > 0.0) or not math.isfinite(b):
        return 0
    # 65504 / b = f * 2^k with 0.5 <= f < 1, so floor(log2(65504 / b)) = k - 1.
    _, k = math.frexp(F16_MAX / b)
    e = k - 1
    while e > -100 and b * 2.0 ** e > F16_MAX:
        e -= 1
    while e < 100 and b * 2.0 ** (e + 1) <= F16_MAX:
        e += 1
    return max(-100, min(100, e))


def round_f16_scaled(x, e):
    """Round x * 2^e to FP16 (numpy's round to nearest even) and scale back."""
    x = np.asarray(x, dtype=np.float64)
    return np.ldexp(np.ldexp(x, e).astype(np.float16).astype(np.float64), -e)


def _round_complex(s, store, e=0):
    if store == "none":
        return s
    if store == "bf16":
        return round_bf16(s.real) + 1j * round_bf16(s.imag)
    if store == "f16":
        return round_f16_scaled(s.real, e) + 1j * round_f16_scaled(s.imag, e)
    raise ValueError("store must be 'none', 'bf16' or 'f16'")


def stored_spectra(frames, store, window=None):
    """a_t of the module docstring for every frame, full plane complex128
    [N][n][n]; also returns the FP16 exponents e_t (zeros unless f16)."""
    u = np.asarray(frames, dtype=np.float64)
    if window is not None:
        u = u * np.asarray(window, dtype=np.float64)[None, :, :]
    norm, means = normalise(u)
    n = u.shape[1]
    I = spectra(norm)
    ratio = means[0] / means
    exps = np.zeros(len(u), dtype=np.int64)
    a = np.empty_like(I)
    for t in range(len(u)):
        s = I[t] - ratio[t] * I[0]
        if store == "f16":
            exps[t] = f16_exponent(np.abs(u[t] - u[0]).sum() / means[t])
        a[t] = _round_complex(s, store, int(exps[t])) + (ratio[t] - 1.0) * I[0]
        a[t, 0, 0] = float(n * n)
    return a, exps


def structure_function_stored(frames, lags, n_bins, store, window=None, return_power=False):
    """Steps O4-O6 on the 16-bit stored spectra a_t. Returns the same dict as
    structure_function (D, counts, pairs, optional P) plus the exponents."""
    a, exps = stored_spectra(frames, store, window)
    n = a.shape[-1]
    P, pairs = pair_power(a, lags)
    bidx = bin_index(n, n_bins)
    out = dict(D=azimuthal_average(P, bidx, n_bins), counts=bin_counts(bidx, n_bins),
               pairs=pairs, exponents=exps)
    if return_power:
        out["P"] = P
    return out


def structure_function_stored_bins(frames, lags, n_bins, bins, store, window=None, workers=1):
    """structure_function_stored for a few bins only, one frame at a time (for
    stacks too large to hold in FP64); equal to the matching columns of
    structure_function_stored()."""
    N = len(frames)
    n = int(np.asarray(frames[0]).shape[-1])
    bidx = bin_index(n, n_bins)
    bins = [int(b) for b in bins]
    sel = np.isin(bidx, bins)
    w = None if window is None else np.asarray(window, dtype=np.float64)

    def weighted(t):
        f = np.asarray(frames[t], dtype=np.float64)
        return f if w is None else f * w

    u0 = weighted(0)
    norm0, m0 = normalise(u0[None])
    I0 = spectra(norm0)[0][sel]
    keep = np.empty((N, int(sel.sum())), dtype=np.complex128)

    def one(t):
        ut = weighted(t)
        norm, mt = normalise(ut[None])
        It = spectra(norm)[0][sel]
        ratio = m0[0] / mt[0]
        e = f16_exponent(np.abs(ut - u0).sum() / mt[0]) if store == "f16" else 0
        keep[t] = _round_complex(It - ratio * I0, store, e) + (ratio - 1.0) * I0

    if workers > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max_workers=workers) as ex:
            list(ex.map(one, range(N)))
    else:
        for t in range(N):
            one(t)
    # The zero-frequency mode (first in row-major order when selected) has
    # a_t(0) = n^2, as in stored_spectra.
    if sel[0, 0]:
        keep[:, 0] = float(n * n)
    P, pairs = pair_power(keep, lags)
    sub_b = bidx[sel]
    counts_all = bin_counts(bidx, n_bins)
    D = np.empty((len(lags), len(bins)), dtype=np.float64)
    for j, b in enumerate(bins):
        m = sub_b == b
        D[:, j] = P[:, m].sum(axis=1) / float(counts_all[b]) if counts_all[b] else np.nan
    return dict(D=D, counts=counts_all[bins], pairs=pairs)
