"""Gradients of a scalar loss of D with respect to the frames and the window,
FP64 (differentiation form).

TEST INFRASTRUCTURE ONLY (see the package docstring).

D(b, tau) of Eq. (1) is a smooth function of the images and of a per-pixel
weight w applied to them, so a loss L(D) can be minimised over either (for
example to fit an apodisation window, or to propagate D into a learned
model). Given G[l][b] = dL/dD(b, tau_l), the adjoint runs the steps of the
definition (module dda) backwards:

  B6  dL/dP_tau(k) = G[l][b(k)] / C_b on every full-plane mode of bin b(k);
      0 on modes outside every bin and for delays with no pair (N <= tau),
      where D does not depend on the frames.
  B4  P_tau(k) = 1/(N - tau) * sum_t |I_t(k) - I_{t+tau}(k)|^2: for every
      pair (t, t + tau), with d = I_t(k) - I_{t+tau}(k) and
      c = dL/dP_tau(k) / (N - tau), the gradient (dL/dRe + i dL/dIm) of
      I_t(k) gains 2 c d and that of I_{t+tau}(k) loses 2 c d.
  B3  I_t = F[i'_t] with I_t(0) set to n^2: the zero-frequency coefficient
      does not depend on i'_t, so its gradient is dropped; then
      dL/di'_t(x) = Re sum_k conj(g_t(k)) exp(-2 pi i k.x / n).
  B2  i'_t = u_t / m_t with m_t = mean_x u_t:
      dL/du_t = (dL/di'_t - mean_x(dL/di'_t * i'_t)) / m_t.
  B1  u_t = w * i_t: dL/di_t = w * dL/du_t, dL/dw = sum_t i_t * dL/du_t.
"""
import numpy as np

from .dda import bin_counts, bin_index, normalise, spectra


def structure_function_grad(frames, lags, n_bins, G, window=None):
    """dL/d(frames) [N][n][n] and dL/dw [n][n] (w = 1 when window is None)
    for the upstream gradient G [L][n_bins] of D; returns a dict with keys
    "frames" and "window", float64."""
    i = np.asarray(frames, dtype=np.float64)
    N, n = i.shape[0], i.shape[1]
    w = np.ones((n, n)) if window is None else np.asarray(window, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64)
    if G.shape != (len(lags), n_bins):
        raise ValueError("G must be [n_lags][n_bins]")
    norm, means = normalise(i, w)
    I = spectra(norm)
    bidx = bin_index(n, n_bins)
    counts = bin_counts(bidx, n_bins)
    inside = bidx >= 0

    # B6 and B4
    g = np.zeros_like(I)
    for l, tau in enumerate(lags):
        tau = int(tau)
        if N - tau <= 0:
            continue
        dP = np.zeros((n, n))
        dP[inside] = G[l, bidx[inside]] / counts[bidx[inside]]
        c = dP / float(N - tau)
        for t in range(N - tau):
            d = I[t] - I[t + tau]
            g[t] += 2.0 * c * d
            g[t + tau] -= 2.0 * c * d

    # B3
    g[:, 0, 0] = 0.0
    dnorm = np.fft.fft2(np.conj(g), axes=(-2, -1)).real

    # B2
    proj = (dnorm * norm).reshape(N, -1).mean(axis=1)
    du = (dnorm - proj[:, None, None]) / means[:, None, None]

    # B1
    return dict(frames=du * w[None, :, :], window=(i * du).sum(axis=0))
