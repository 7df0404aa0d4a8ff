"""Seeded synthetic frame stacks.

The paper's data (shadowgraph images of non-equilibrium concentration
fluctuations under a static beam, test-experiment section) are not available,
so frames are synthesised with the same structure: a static Gaussian beam
profile modulated by a small fluctuating field whose Fourier modes follow
independent Ornstein-Uhlenbeck processes, plus camera noise.

Draw order (fixed, per frame t = 0..N-1): complex normals for every mode
(real parts then imaginary parts), then the noise draw for every pixel.
Frames are a function of (config, seed, device): torch's CPU and GPU random
generators differ, so a test that feeds both the oracle and the HIP path
draws the stack once and hands the same array to both.
"""
import math

import numpy as np
import torch


def signed_freqs(n, device="cpu"):
    """Integer frequencies in transform order: 0, 1, ..., n/2-1, -n/2, ..., -1."""
    j = torch.arange(n, device=device, dtype=torch.float64)
    return torch.where(j < (n + 1) // 2, j, j - n)


def field_model(cfg, device="cpu"):
    """Per-mode amplitude A(q), decay rate Gamma(q) and field scale c_s.

    q = 2*pi*|k|/n in rad/px. A(q) = max(q, 2*pi/64)^-2 with A(0) = 0, so the
    field has zero spatial mean; Gamma(q) = gamma_a + gamma_b * q^2 per frame.
    c_s scales the field to unit stationary variance per pixel.
    """
    n = cfg["n"]
    f = signed_freqs(n, device)
    ky, kx = f[:, None], f[None, :]
    q = 2.0 * math.pi * torch.sqrt(kx * kx + ky * ky) / n
    amp = torch.clamp(q, min=2.0 * math.pi / 64.0) ** -2
    amp[0, 0] = 0.0
    gamma = cfg["gamma_a"] + cfg["gamma_b"] * q * q
    c_s = (amp.pow(2).sum() / 2.0).rsqrt()
    return amp, gamma, c_s


def beam_profile(cfg, device="cpu", flat=False):
    """Static beam: Gaussian of width 40 px per 128 px of frame side, or flat."""
    n = cfg["n"]
    if flat:
        return torch.full((n, n), float(cfg["peak"]), dtype=torch.float64,
                          device=device)
    sigma_b = 40.0 * n / 128.0
    c = (n - 1) / 2.0
    y = torch.arange(n, device=device, dtype=torch.float64) - c
    r2 = y[:, None] ** 2 + y[None, :] ** 2
    return cfg["peak"] * torch.exp(-r2 / (2.0 * sigma_b * sigma_b))


def make_stack(cfg, seed, device="cpu", N=None, flat_beam=False, noise=None):
    """Draw a [N][n][n] frame stack for workload `cfg` with random seed `seed`.

    Returns a torch tensor on `device`: uint16 for cfg["dtype"] == "u16"
    (Poisson counts clipped to the 12-bit range), float32 otherwise
    (additive Gaussian noise of cfg["noise_sigma"] counts, or none).
    """
    n = int(cfg["n"])
    N = int(cfg["N"] if N is None else N)
    noise = cfg["noise"] if noise is None else noise
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    amp, gamma, c_s = field_model(cfg, device)
    rho = torch.exp(-gamma)
    drive = torch.sqrt(1.0 - rho * rho) * amp
    beam = beam_profile(cfg, device, flat=flat_beam)
    eps = float(cfg["eps"])

    def xi():
        re = torch.randn((n, n), generator=gen, device=device, dtype=torch.float64)
        im = torch.randn((n, n), generator=gen, device=device, dtype=torch.float64)
        return torch.complex(re, im) * math.sqrt(0.5)

    out_dtype = torch.uint16 if cfg["dtype"] == "u16" else torch.float32
    frames = torch.empty((N, n, n), dtype=out_dtype, device=device)
    z = amp * xi()
    for t in range(N):
        if t:
            z = rho * z + drive * xi()
        s = c_s * torch.fft.ifft2(z).real * float(n * n)
        lam = beam * (1.0 + eps * s)
        if noise == "poisson":
            cnt = torch.poisson(torch.clamp(lam, min=0.0), generator=gen)
            frames[t] = torch.clamp(cnt, 0.0, 4095.0).to(torch.int32).to(out_dtype)
        elif noise == "gauss":
            e = torch.randn((n, n), generator=gen, device=device, dtype=torch.float64)
            frames[t] = (lam + float(cfg["noise_sigma"]) * e).to(out_dtype)
        elif noise == "none":
            frames[t] = lam.to(out_dtype)
        else:
            raise ValueError(f"unknown noise model {noise!r}")
    return frames


def cosine_stack(n, N, modes, dtype=np.float64):
    """Frames 1 + sum_j eps_j * cos(2*pi*(ky_j*y + kx_j*x)/n + omega_j*t).

    `modes` is a list of (ky, kx, eps, omega). With no mode at k = 0 every
    frame has spatial mean exactly 1, which gives closed forms for the
    structure function.
    """
    y = np.arange(n, dtype=np.float64)[:, None]
    x = np.arange(n, dtype=np.float64)[None, :]
    out = np.ones((N, n, n), dtype=np.float64)
    for (ky, kx, eps, omega) in modes:
        ph = 2.0 * np.pi * ((ky * y + kx * x) % n) / n
        for t in range(N):
            out[t] += eps * np.cos(ph + omega * t)
    return out.astype(dtype)
