"""Named synthetic workloads.

Each entry fixes the frame size n, the frame count N, the input type, the
field/beam/noise parameters of the generator and the analysis inputs (lags,
number of |q| bins). The shapes follow the ranges the paper processed
(32 to 2048 images of 32x32 up to 4k x 4k pixels, processing section) and a
12-bit camera for the integer workload.
"""
from .lags import log_spaced_lags, power_of_two_lags

CONFIGS = {
    # 64 float frames of 128x128: the small case the oracle finishes in
    # well under a second.
    "c1": dict(name="c1", n=128, N=64, dtype="f32", peak=1000.0, eps=0.01,
               gamma_a=0.05, gamma_b=2.0, noise="gauss", noise_sigma=2.0,
               lags=[1, 2, 4, 8, 16], n_bins=64),
    # 1000 uint16 frames of 1024x1024 (12-bit camera, Poisson shot noise),
    # 50 log-spaced lags from 1 to 500, 512 |q| bins: the throughput workload.
    "c2": dict(name="c2", n=1024, N=1000, dtype="u16", peak=3000.0, eps=0.005,
               gamma_a=0.002, gamma_b=0.5, noise="poisson", noise_sigma=0.0,
               lags=log_spaced_lags(500, 50), n_bins=512),
    # The precision workload: 4000 frames of the same uint16 model, every lag
    # from 1 to 400, 512 |q| bins.
    "c3": dict(name="c3", n=1024, N=4000, dtype="u16", peak=3000.0, eps=0.005,
               gamma_a=0.002, gamma_b=0.5, noise="poisson", noise_sigma=0.0,
               lags=list(range(1, 401)), n_bins=512),
    # 256 float frames of 512x512, power-of-two lags up to 64.
    "c5": dict(name="c5", n=512, N=256, dtype="f32", peak=1000.0, eps=0.01,
               gamma_a=0.05, gamma_b=2.0, noise="gauss", noise_sigma=2.0,
               lags=power_of_two_lags(64), n_bins=256),
}


def config(name, **overrides):
    """A copy of a named workload with some fields replaced."""
    c = dict(CONFIGS[name])
    c["lags"] = list(c["lags"])
    c.update(overrides)
    return c


def batch_workload(master_seed=4, count=16, sizes=(256, 512, 1024, 2048), frames=(200, 2000),
                   lag_count=32):
    """The batching workload: `count` sequences of the uint16 camera model
    with frame size drawn from `sizes`, frame count uniform in `frames`,
    decay-rate parameters gamma_a in [0.001, 0.01] and gamma_b in [0.1, 2]
    (Gamma = gamma_a + gamma_b q^2) drawn from `master_seed`; `lag_count`
    log-spaced lags up to N/2 and n/2 |q| bins per sequence. Sequence j is
    drawn with seed 40 + j (entry "seed")."""
    import numpy as np
    rng = np.random.default_rng(int(master_seed))
    out = []
    for j in range(int(count)):
        n = int(rng.choice(np.asarray(sizes)))
        N = int(rng.integers(frames[0], frames[1] + 1))
        ga = float(rng.uniform(0.001, 0.01))
        gb = float(rng.uniform(0.1, 2.0))
        tmax = max(1, N // 2)
        c = config("c2", n=n, N=N, gamma_a=ga, gamma_b=gb,
                   lags=log_spaced_lags(tmax, min(int(lag_count), tmax)), n_bins=n // 2)
        c["name"] = f"c4/{j}"
        c["seed"] = 40 + j
        out.append(c)
    return out
